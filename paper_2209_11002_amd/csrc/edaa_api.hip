// C ABI of the EDAA library (declared in include/edaa.h): argument checks,
// workspace, the run sequence of Algorithm 1 for a batch of runs, optional
// HIP-graph capture, and the selection of Algorithm 2.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <stdlib.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "edaa.h"
#include "edaa_internal.h"

using namespace edaa;

namespace {

thread_local std::string g_last_error;

edaa_status fail(edaa_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

struct GraphEntry {
    std::string key;
    hipGraphExec_t exec = nullptr;
    long long launches = 0;
};

// Event pairs recorded around pass launches (EDAA_FLAG_TIME_PASSES).
struct PassTimer {
    std::vector<hipEvent_t> ev;     // 2 per timed launch
    std::vector<int> kind;          // 0 A-pass, 1 B-pass, 2 closing pass
    int used = 0;
    bool enabled = false;
    hipError_t mark(hipStream_t st, int k, bool end) {
        if (!enabled) return hipSuccess;
        const size_t slot = (size_t)used * 2 + (end ? 1 : 0);
        while (ev.size() <= slot) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            ev.push_back(e);
        }
        if ((size_t)used >= kind.size()) kind.resize(used + 1);
        kind[used] = k;
        hipError_t r = hipEventRecord(ev[slot], st);
        if (end) ++used;
        return r;
    }
};

}  // namespace

// Device memory of the no-allocation entry point (edaa_fit_noalloc): one
// copy of this array on every GPU the library runs on, held until the process
// ends.  Host code never passes the array's name to a kernel or a copy (on
// the host it is only a stand-in): it uses the device address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device by edaa_create and kept in g_scratch_ptr.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current); null and
// a HIP error on failure.
hipError_t scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

struct edaa_ctx {
    int device = 0;
    void* scratch = nullptr;           // this device's copy of `scratch` (device address)
    hipStream_t stream = nullptr;      // the caller's stream
    hipStream_t cap_stream = nullptr;  // private stream used for graph capture
    bool poisoned = false;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    long long last_launches = 0;
    std::vector<GraphEntry> graphs;    // most recent last
    size_t graph_cap = 16;
    PassTimer timer;
};

#define EDAA_HIP(ctx, call)                                                                         \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) {                                                                     \
            (ctx)->poisoned = true;                                                                 \
            return fail(EDAA_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));               \
        }                                                                                           \
    } while (0)

#define EDAA_REQUIRE(cond, ...)                                                                     \
    do {                                                                                            \
        if (!(cond)) return fail(EDAA_EINVAL, __VA_ARGS__);                                         \
    } while (0)

namespace {

struct Arena {
    size_t off = 0;
    template <typename T>
    size_t take(size_t n) {
        off = (off + 255) & ~(size_t)255;
        const size_t o = off;
        off += n * sizeof(T);
        return o;
    }
};

edaa_status ensure_ws(edaa_ctx* ctx, size_t bytes) {
    if (bytes <= ctx->ws_bytes) return EDAA_OK;
    // Graphs hold pointers into the workspace: drop them before reallocating.
    for (auto& ge : ctx->graphs) (void)hipGraphExecDestroy(ge.exec);
    ctx->graphs.clear();
    if (ctx->ws) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    const size_t want = std::max(bytes, (size_t)(1 << 20));
    if (hipMalloc(&ctx->ws, want) != hipSuccess) {
        (void)hipGetLastError();
        ctx->ws = nullptr;
        return fail(EDAA_ENOMEM, "could not allocate %zu bytes of device workspace", want);
    }
    ctx->ws_bytes = want;
    return EDAA_OK;
}

edaa_status check_ctx(edaa_ctx* ctx) {
    if (!ctx) return fail(EDAA_EINVAL, "null context");
    if (ctx->poisoned) return fail(EDAA_EDEVICE, "context is poisoned by an earlier device error");
    if (hipSetDevice(ctx->device) != hipSuccess) {
        ctx->poisoned = true;
        return fail(EDAA_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    }
    return EDAA_OK;
}

edaa_status check_params(const edaa_params* P) {
    EDAA_REQUIRE(P != nullptr, "params is null");
    EDAA_REQUIRE(P->T >= 0 && P->K1 >= 0 && P->K2 >= 0, "T, K1, K2 must be >= 0 (got %d, %d, %d)", P->T, P->K1,
                 P->K2);
    EDAA_REQUIRE(P->T <= 1000000, "T too large");
    EDAA_REQUIRE(isfinite(P->init_scale), "init_scale must be finite");
    EDAA_REQUIRE(isfinite(P->eta1) && P->eta1 >= 0.0 && isfinite(P->eta2) && P->eta2 >= 0.0,
                 "eta1/eta2 must be finite and >= 0 (0 selects the paper's rule)");
    EDAA_REQUIRE(isfinite(P->select_threshold) && P->select_threshold >= 1.0, "select_threshold must be >= 1");
    EDAA_REQUIRE(P->x_dtype == EDAA_X_F32 || P->x_dtype == EDAA_X_BF16, "x_dtype must be EDAA_X_F32 or EDAA_X_BF16");
    EDAA_REQUIRE(P->runs_per_chunk >= 0 && P->pixel_groups >= 0 && P->tiles_per_item >= 0,
                 "runs_per_chunk, pixel_groups and tiles_per_item must be >= 0");
    EDAA_REQUIRE(P->coherence_mode == EDAA_COHERENCE_COSINE || P->coherence_mode == EDAA_COHERENCE_RAW,
                 "coherence_mode must be EDAA_COHERENCE_COSINE or EDAA_COHERENCE_RAW");
    return EDAA_OK;
}

edaa_status check_shape(int L, int N, int p, int M) {
    EDAA_REQUIRE(L >= 1 && L <= kMaxL, "L must be in [1, %d] (got %d)", kMaxL, L);
    EDAA_REQUIRE(p >= 1 && p <= kMaxP, "p must be in [1, %d] (got %d)", kMaxP, p);
    EDAA_REQUIRE(N >= p, "N must be >= p (got N=%d, p=%d)", N, p);
    EDAA_REQUIRE(M >= 1, "M must be >= 1 (got %d)", M);
    EDAA_REQUIRE((double)M * p * N < 2147483647.0 && (double)L * N < 2147483647.0, "problem too large");
    return EDAA_OK;
}

// ---------------------------------------------------------------------------
// Launch shapes chosen by the autotuner (edaa_autotune, edaa_autotune_ragged),
// per problem class: for an ensemble (L, p, M, X dtype and the tile count
// rounded up to a power of two) the runs per chunk and pixel groups, for a
// ragged batch (image count, total tiles rounded up to a power of two,
// largest p, X dtype) the tiles per work item.  Kept for the process; when
// the environment variable EDAA_TUNE_CACHE names a file, entries are read
// from it on first use and appended to it when tuned, one per line:
//   edaa-tune-v1 <class> <value1> <value2> <microseconds per outer iteration>
// (later lines win).
// ---------------------------------------------------------------------------
struct TuneTable {
    std::mutex mu;
    bool loaded = false;
    std::map<std::string, std::pair<int, int>> shapes;
};

TuneTable& tune_table() {
    static TuneTable t;
    return t;
}

int log2_ceil(long long v) {
    int b = 0;
    while ((1ll << b) < v) ++b;
    return b;
}

std::string ensemble_class(int L, int N, int p, int M, int x_dtype) {
    char buf[96];
    snprintf(buf, sizeof(buf), "ens:%d:%d:%d:%d:%d", L, p, M, x_dtype, log2_ceil((N + kTile - 1) / kTile));
    return buf;
}

std::string ragged_class(int n, const edaa_image_desc* images, int x_dtype) {
    long long tiles = 0;
    int pmax = 0;
    for (int k = 0; k < n; ++k) {
        tiles += (images[k].N + kTile - 1) / kTile;
        pmax = std::max(pmax, images[k].p);
    }
    char buf[96];
    snprintf(buf, sizeof(buf), "rag:%d:%d:%d:%d", n, log2_ceil(tiles), pmax, x_dtype);
    return buf;
}

void tune_load_locked(TuneTable& t) {
    if (t.loaded) return;
    t.loaded = true;
    const char* path = getenv("EDAA_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char tag[32], cls[96];
    int v1, v2;
    double us;
    while (fscanf(f, "%31s %95s %d %d %lf", tag, cls, &v1, &v2, &us) == 5)
        if (strcmp(tag, "edaa-tune-v1") == 0) t.shapes[cls] = std::make_pair(v1, v2);
    fclose(f);
}

bool tune_lookup(const std::string& cls, int* v1, int* v2) {
    TuneTable& t = tune_table();
    std::lock_guard<std::mutex> lk(t.mu);
    tune_load_locked(t);
    auto it = t.shapes.find(cls);
    if (it == t.shapes.end()) return false;
    *v1 = it->second.first;
    *v2 = it->second.second;
    return true;
}

void tune_store(const std::string& cls, int v1, int v2, double us) {
    TuneTable& t = tune_table();
    std::lock_guard<std::mutex> lk(t.mu);
    tune_load_locked(t);
    t.shapes[cls] = std::make_pair(v1, v2);
    const char* path = getenv("EDAA_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "edaa-tune-v1 %s %d %d %.3f\n", cls.c_str(), v1, v2, us);
    fclose(f);
}

// Launch shape of an M-run problem: the caller's requests, else a tuned
// shape of its class, else the default (EDAA_PLAN_* in *source).
edaa_status plan_geom(int L, int N, int p, int M, const edaa_params* P, Geom* g, int* source) {
    if (P->runs_per_chunk > 0 && !runs_fit(p, P->runs_per_chunk, L))
        return fail(EDAA_EUNSUPPORTED, "runs_per_chunk=%d has no pass kernels for p=%d, L=%d", P->runs_per_chunk, p,
                    L);
    int R = P->runs_per_chunk, npg = P->pixel_groups, src = EDAA_PLAN_REQUESTED;
    if (R == 0 && npg == 0) {
        src = EDAA_PLAN_DEFAULT;
        int tR = 0, tn = 0;
        if (tune_lookup(ensemble_class(L, N, p, M, P->x_dtype), &tR, &tn) && runs_fit(p, tR, L) &&
            (M > 1 || tR == 1)) {
            R = tR;
            npg = tn;
            src = EDAA_PLAN_TUNED;
        }
    }
    *g = make_geom(L, N, M, p, R, npg);
    if (!geom_valid(*g))
        return fail(EDAA_EUNSUPPORTED, "no pass kernels fit L=%d with p=%d (runs per chunk %d, LDS limit %zu bytes)",
                    L, p, g->R, kMaxLdsBytes);
    if (source) *source = src;
    return EDAA_OK;
}

// Device buffers of one batched run, carved out of the context workspace.
struct RunBuffers {
    State s;
    uint64_t* seeds;
    double* gammas;
};

// x_bytes: bytes per element of X (4 or 2) for the padded copy.
size_t layout(const Geom& g, int T, int x_bytes, char* base, RunBuffers* rb) {
    Arena a;
    const size_t Q = (size_t)g.M * g.p;
    const size_t ldx = (size_t)g.ntiles * kTile;
    const size_t o_Xp = a.take<char>((size_t)g.L * ldx * x_bytes);
    const size_t o_Bst = a.take<float>(Q * (size_t)g.ntiles * kTile);   // rows padded to whole tiles
    const size_t o_tsh = a.take<float>((size_t)g.ntiles * g.Qp);
    const size_t o_colm = a.take<float>(g.Qp);
    const size_t o_cols = a.take<float>(g.Qp);
    const size_t o_E = a.take<float>((size_t)(g.L + kPadRows) * g.Qp);
    const size_t o_Ed = a.take<double>((size_t)g.L * g.Qp);
    const size_t o_W = a.take<float>((size_t)(g.L + kPadRows) * g.Qp);
    const size_t o_XAt = a.take<double>((size_t)g.L * g.Qp);
    const size_t o_AAt = a.take<double>((size_t)g.M * g.p * g.p);
    const size_t o_eta = a.take<float>(2 * (size_t)g.M);
    const size_t o_etad = a.take<double>(2 * (size_t)g.M);
    const size_t o_trace = a.take<double>((size_t)g.M * (T + 1));
    const size_t o_fit = a.take<double>(g.M);
    const size_t o_mu = a.take<double>(g.M);
    const size_t o_V = a.take<float>((size_t)g.npg * g.nqc * g.L * g.QC);
    const size_t o_mp = a.take<float>((size_t)g.npg * g.Qp);
    const size_t o_sp = a.take<float>((size_t)g.npg * g.Qp);
    const size_t o_AA = a.take<float>((size_t)g.npg * g.nqc * g.R * g.p * g.p);
    const size_t o_lp = a.take<double>((size_t)g.npg * g.M);
    const size_t o_fp = a.take<double>((size_t)g.npg * g.M);
    const size_t o_seed = a.take<uint64_t>(g.M);
    const size_t o_gam = a.take<double>(g.M);
    if (rb) {
        State& s = rb->s;
        s.X = base + o_Xp;
        s.ldx = ldx;
        s.x_bf16 = x_bytes == 2 ? 1 : 0;
        s.Bst = (float*)(base + o_Bst);
        s.tshift = (float*)(base + o_tsh);
        s.colm = (float*)(base + o_colm);
        s.cols = (float*)(base + o_cols);
        s.E = (float*)(base + o_E);
        s.Ed = (double*)(base + o_Ed);
        s.W = (float*)(base + o_W);
        s.XAtd = (double*)(base + o_XAt);
        s.AAtd = (double*)(base + o_AAt);
        s.eta = (float*)(base + o_eta);
        s.etad = (double*)(base + o_etad);
        s.trace = (double*)(base + o_trace);
        s.fit = (double*)(base + o_fit);
        s.mu = (double*)(base + o_mu);
        s.Vpart = (float*)(base + o_V);
        s.mpart = (float*)(base + o_mp);
        s.spart = (float*)(base + o_sp);
        s.AApart = (float*)(base + o_AA);
        s.lpart = (double*)(base + o_lp);
        s.fpart = (double*)(base + o_fp);
        s.T = T;
        rb->seeds = (uint64_t*)(base + o_seed);
        rb->gammas = (double*)(base + o_gam);
    }
    return a.off + 256;
}

// Enqueue the whole sequence of Algorithm 1 for g.M runs.  Returns the number
// of kernel launches, or a negative HIP error.
struct Seq {
    PassTimer* timer;   // mutable: capture switches timing off
    const Geom* g;
    const State* s;
    const void* X;      // the caller's X [L][N], copied into s->X (padded)
    RunInit ri;
    int mode;          // kModeInitRng or kModeInitB0
    const float* A0;
    int T, K1, K2;
    float* B_out;
    float* E_out;
    int coherence_mode;
    const float* E_given;   // abundance estimation with E fixed (A-passes only), else null
};

hipError_t enqueue_sequence(const Seq& q, hipStream_t st, long long* launches) {
    const Geom& g = *q.g;
    const State& s = *q.s;
    long long n = 0;
    hipError_t e;
#define EDAA_L(call)                          \
    do {                                      \
        e = (call);                           \
        if (e != hipSuccess) return e;        \
        ++n;                                  \
    } while (0)
    EDAA_L(launch_pad_x(q.X, const_cast<void*>(s.X), g.L, g.N, s.ldx, s.x_bf16, st));
    // zero the padded [L][Qp] arrays (pad columns must read as zero)
    EDAA_L(launch_fill(s.E, (size_t)(g.L + kPadRows) * g.Qp, 0.f, st));
    EDAA_L(launch_fill(s.W, (size_t)(g.L + kPadRows) * g.Qp, 0.f, st));
    EDAA_L(launch_fill((float*)s.XAtd, 2 * (size_t)g.L * g.Qp, 0.f, st));
    EDAA_L(launch_fill((float*)s.Ed, 2 * (size_t)g.L * g.Qp, 0.f, st));
    EDAA_L(launch_init_A(g, s, q.A0, st));
    PassTimer* tm = q.timer;
    if (q.E_given) {
        // A-phase only with the given endmembers: eq. update_A with E fixed
        EDAA_L(launch_set_e(q.E_given, g, s, st));
        EDAA_L(launch_eta(g, s, q.ri, st));
        for (int t = 0; t < q.T; ++t) {
            if ((e = tm->mark(st, 0, false)) != hipSuccess) return e;
            EDAA_L(launch_apass(g, s, q.K1, t, st));
            if ((e = tm->mark(st, 0, true)) != hipSuccess) return e;
            EDAA_L(launch_reduce_aa(g, s, t, st));
        }
        EDAA_L(launch_close(g, s, st));
        EDAA_L(launch_reduce_close(g, s, st));
        *launches = n;
        return hipSuccess;
    }
    EDAA_L(launch_bpass(g, s, q.mode, q.ri, st));
    EDAA_L(launch_reduce_b(g, s, 0, st));
    EDAA_L(launch_eta(g, s, q.ri, st));
    for (int t = 0; t < q.T; ++t) {
        if ((e = tm->mark(st, 0, false)) != hipSuccess) return e;
        EDAA_L(launch_apass(g, s, q.K1, t, st));
        if ((e = tm->mark(st, 0, true)) != hipSuccess) return e;
        EDAA_L(launch_reduce_a(g, s, t, st));
        ++n;   // launch_reduce_a enqueues two kernels
        for (int k = 0; k < q.K2; ++k) {
            if ((e = tm->mark(st, 1, false)) != hipSuccess) return e;
            EDAA_L(launch_bpass(g, s, kModeStep, q.ri, st));
            if ((e = tm->mark(st, 1, true)) != hipSuccess) return e;
            EDAA_L(launch_reduce_b(g, s, k + 1 < q.K2 ? 1 : 0, st));
        }
    }
    if ((e = tm->mark(st, 2, false)) != hipSuccess) return e;
    EDAA_L(launch_close(g, s, st));
    if ((e = tm->mark(st, 2, true)) != hipSuccess) return e;
    EDAA_L(launch_reduce_close(g, s, st));
    EDAA_L(launch_finalize(g, s, q.B_out, q.E_out, q.coherence_mode, st));
    n += (q.B_out ? 1 : 0);
#undef EDAA_L
    *launches = n;
    return hipSuccess;
}

std::string graph_key(const Seq& q, const void* X, const void* ws) {
    char buf[640];
    const Geom& g = *q.g;
    snprintf(buf, sizeof(buf),
             "%d,%d,%d,%d,%d,%d,%d,%d,%d|%d,%d,%d|%p,%p,%p,%p,%p,%p,%p|%a,%a,%a|%d,%d", g.L, g.N, g.M, g.p, g.R,
             g.npg, g.nqc, q.mode, q.coherence_mode, q.T, q.K1, q.K2, X, (const void*)q.s->A, (const void*)q.B_out,
             (const void*)q.E_out, (const void*)q.A0, (const void*)(q.E_given ? q.E_given : q.ri.B0), ws,
             (double)q.ri.init_scale, q.ri.eta1,
             q.ri.eta2, q.s->x_bf16 + 2 * q.s->x_mfma, q.timer->enabled ? 1 : 0);
    return buf;
}

// Run an enqueue function eagerly, or capture it once into a HIP graph kept
// under `key` and replay that graph.
template <typename F>
edaa_status run_captured(edaa_ctx* ctx, const std::string& key, bool use_graph, F&& enqueue) {
    if (!use_graph) {
        long long n = 0;
        hipError_t e = enqueue(ctx->stream, &n);
        if (e != hipSuccess) {
            ctx->poisoned = true;
            return fail(EDAA_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
        }
        ctx->last_launches = n;
        return EDAA_OK;
    }
    for (size_t i = 0; i < ctx->graphs.size(); ++i) {
        if (ctx->graphs[i].key == key) {
            EDAA_HIP(ctx, hipGraphLaunch(ctx->graphs[i].exec, ctx->stream));
            ctx->last_launches = ctx->graphs[i].launches;
            return EDAA_OK;
        }
    }
    if (!ctx->cap_stream) EDAA_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    EDAA_HIP(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    long long n = 0;
    hipError_t e = enqueue(ctx->cap_stream, &n);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        ctx->poisoned = true;
        return fail(EDAA_EDEVICE, "graph capture failed: %s / %s", hipGetErrorString(e), hipGetErrorString(e2));
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        ctx->poisoned = true;
        return fail(EDAA_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    while (!ctx->graphs.empty() && ctx->graphs.size() >= ctx->graph_cap) {
        (void)hipGraphExecDestroy(ctx->graphs.front().exec);
        ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back(GraphEntry{key, exec, n});
    EDAA_HIP(ctx, hipGraphLaunch(exec, ctx->stream));
    ctx->last_launches = n;
    return EDAA_OK;
}

// Run (or replay) the sequence on the caller's stream.
edaa_status run_sequence(edaa_ctx* ctx, const Seq& q, const void* X, int use_graph) {
    ctx->timer.used = 0;
    // Events recorded inside a captured graph carry no timestamps on this
    // runtime: pass timing is taken in eager mode only.
    if (use_graph) q.timer->enabled = false;
    const std::string key = use_graph ? graph_key(q, X, ctx->ws) : std::string();
    return run_captured(ctx, key, use_graph != 0,
                        [&](hipStream_t st, long long* n) { return enqueue_sequence(q, st, n); });
}

// bf16 X runs the B-pass (bit 0) and the A-pass (bit 1) on the bf16 matrix
// cores unless the caller asks for the float32 ones or the chunk does not
// fit the pass's LDS layout.  float32 X runs its passes there (three-term
// products; the A-pass where xas_chunk allows) when the chunk has at least
// two column blocks, over which the split of each X value is shared (with one
// column block the float32 matrix-core passes are faster), unless
// EDAA_FLAG_F32_MFMA asks for the float32 (and float64) matrix cores.
int use_xb(const Geom& g, int x_bytes, int flags) {
    if (x_bytes == 4) {
        if ((flags & EDAA_FLAG_F32_MFMA) || (g.p * g.R + 15) / 16 < 2) return 0;
        return (xs_fits(g.p, g.R, g.L) ? 1 : 0) | (xas_fits(g.p, g.R, g.L) ? 2 : 0);
    }
    if (flags & EDAA_FLAG_BF16_WIDEN) return 0;
    return (xb_fits(g.p, g.R, g.L) ? 1 : 0) | (xa_fits(g.p, g.R, g.L) ? 2 : 0);
}

// Shared implementation of edaa_fit (M = 1) and edaa_ensemble.
edaa_status run_batch(edaa_ctx* ctx, const void* X, int L, int N, int p, const edaa_params* P, int M,
                      const uint64_t* seeds, const double* gammas, const float* A0, const float* B0, float* A_all,
                      float* B_all, float* E_all, double* loss, double* fit, double* mu, double* eta_out,
                      const float* E_given = nullptr) {
    Geom g;
    edaa_status st0 = plan_geom(L, N, p, M, P, &g, nullptr);
    if (st0 != EDAA_OK) return st0;
    const int x_bytes = P->x_dtype == EDAA_X_BF16 ? 2 : 4;
    const size_t need = layout(g, P->T, x_bytes, nullptr, nullptr);
    edaa_status st = ensure_ws(ctx, need);
    if (st != EDAA_OK) return st;
    RunBuffers rb;
    memset(&rb, 0, sizeof(rb));
    layout(g, P->T, x_bytes, (char*)ctx->ws, &rb);
    State& s = rb.s;
    s.A = A_all;
    s.x_mfma = use_xb(g, x_bytes, P->flags);

    // Host -> device copies of the per-run scalars happen outside any graph.
    EDAA_HIP(ctx, hipMemcpyAsync(rb.seeds, seeds, sizeof(uint64_t) * M, hipMemcpyHostToDevice, ctx->stream));
    EDAA_HIP(ctx, hipMemcpyAsync(rb.gammas, gammas, sizeof(double) * M, hipMemcpyHostToDevice, ctx->stream));

    Seq q;
    q.timer = &ctx->timer;
    ctx->timer.enabled = (P->flags & EDAA_FLAG_TIME_PASSES) != 0;
    q.g = &g;
    q.s = &s;
    q.X = X;
    q.ri.seeds = rb.seeds;
    q.ri.gammas = rb.gammas;
    q.ri.init_scale = (float)P->init_scale;
    q.ri.B0 = B0;
    q.ri.A0 = A0;
    q.ri.eta1 = P->eta1;
    q.ri.eta2 = P->eta2;
    q.mode = B0 ? kModeInitB0 : kModeInitRng;
    q.A0 = A0;
    q.T = P->T;
    q.K1 = P->K1;
    q.K2 = P->K2;
    q.B_out = B_all;
    q.E_out = E_all;
    q.coherence_mode = P->coherence_mode;
    q.E_given = E_given;
    st = run_sequence(ctx, q, X, (P->flags & EDAA_FLAG_GRAPH) ? 1 : 0);
    if (st != EDAA_OK) return st;

    if (loss) EDAA_HIP(ctx, hipMemcpyAsync(loss, s.trace, sizeof(double) * M * (P->T + 1), hipMemcpyDeviceToHost,
                                          ctx->stream));
    if (fit) EDAA_HIP(ctx, hipMemcpyAsync(fit, s.fit, sizeof(double) * M, hipMemcpyDeviceToHost, ctx->stream));
    if (mu) EDAA_HIP(ctx, hipMemcpyAsync(mu, s.mu, sizeof(double) * M, hipMemcpyDeviceToHost, ctx->stream));
    if (eta_out)
        EDAA_HIP(ctx, hipMemcpyAsync(eta_out, s.etad, sizeof(double) * 2 * M, hipMemcpyDeviceToHost, ctx->stream));
    if (loss || fit || mu || eta_out) EDAA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return EDAA_OK;
}

// ---------------------------------------------------------------------------
// Ragged batch: single runs on images of different (L, N, p).  Images of equal
// p form a group; every kernel of Algorithm 1 is one launch per group, whose
// workgroups look up their image in a device table (ImageJob) through a map
// workgroup -> (image, workgroup within the image).
// ---------------------------------------------------------------------------
struct RaggedGroup {
    int p;
    int nb[kMapKinds];
    const int2* map[kMapKinds];   // device
    size_t lds_a, lds_b, lds_c;
};

// Padded copy of one ragged image's X.
struct PadJob {
    const void* X;
    void* Xp;
    int L, N;
    size_t ldx;
    int bf16;
};

hipError_t enqueue_ragged(const std::vector<RaggedGroup>& groups, const std::vector<PadJob>& pads,
                          const ImageJob* jobs, const PersistPlan* plan, size_t plan_lds, int plan_wgs, int T, int K1,
                          int K2, int cosine, hipStream_t st, long long* launches) {
    long long n = 0;
    hipError_t e;
    for (const PadJob& pj : pads) {
        if ((e = launch_pad_x(pj.X, pj.Xp, pj.L, pj.N, pj.ldx, pj.bf16, st)) != hipSuccess) return e;
        ++n;
    }
    if (plan) {
        // every image of p <= kPersistMaxP: one persistent launch (after the start-state kernel)
        if ((e = launch_ragged_persistent(*plan, plan_lds, plan_wgs, st)) != hipSuccess) return e;
        n += 2;
    }
    if (groups.empty()) {
        *launches = n;
        return hipSuccess;
    }
    auto L_ = [&](int kernel, int mapk, size_t lds, int arg) -> hipError_t {
        for (const RaggedGroup& G : groups) {
            hipError_t r = launch_multi(kernel, G.p, jobs, G.map[mapk], G.nb[mapk], lds ? lds : 0, arg, st);
            if (r != hipSuccess) return r;
            ++n;
        }
        return hipSuccess;
    };
    // the LDS size differs per group: pass it per group through a second loop
    auto Lp = [&](int kernel, size_t RaggedGroup::*lds, int arg) -> hipError_t {
        for (const RaggedGroup& G : groups) {
            hipError_t r = launch_multi(kernel, G.p, jobs, G.map[kMapPass], G.nb[kMapPass], G.*lds, arg, st);
            if (r != hipSuccess) return r;
            ++n;
        }
        return hipSuccess;
    };
    if ((e = L_(kMultiPrep, kMapElem, 0, 0)) != hipSuccess) return e;
    if ((e = Lp(kMultiBpassInit, &RaggedGroup::lds_b, 0)) != hipSuccess) return e;
    if ((e = L_(kMultiRedB, kMapRows, 0, 0)) != hipSuccess) return e;
    if ((e = L_(kMultiEta, kMapOne, 0, 0)) != hipSuccess) return e;
    for (int t = 0; t < T; ++t) {
        if ((e = Lp(kMultiApass, &RaggedGroup::lds_a, K1)) != hipSuccess) return e;
        if ((e = L_(kMultiRedAA, kMapAA, 0, t)) != hipSuccess) return e;
        if ((e = L_(kMultiRedA, kMapRows, 0, t)) != hipSuccess) return e;
        for (int k = 0; k < K2; ++k) {
            if ((e = Lp(kMultiBpassStep, &RaggedGroup::lds_b, 0)) != hipSuccess) return e;
            if ((e = L_(kMultiRedB, kMapRows, 0, k + 1 < K2 ? 1 : 0)) != hipSuccess) return e;
        }
    }
    if ((e = Lp(kMultiClose, &RaggedGroup::lds_c, 0)) != hipSuccess) return e;
    if ((e = L_(kMultiCloseReduce, kMapOne, 0, 0)) != hipSuccess) return e;
    if ((e = L_(kMultiFinal, kMapElem, 0, cosine)) != hipSuccess) return e;
    *launches = n;
    return hipSuccess;
}

// Host tables of a persistent launch over the images `idx` (see PersistPlan).
struct PersistTables {
    int sub_stride = 0;
    int nsub[3] = {0, 0, 0};
    long long seg_len[3] = {0, 0, 0};
    std::vector<int> kind, arg;           // [3][sub_stride]
    std::vector<long long> base;          // [3][sub_stride]
    std::vector<int> cnt;                 // [kPkKinds][n]
    std::vector<long long> pre;           // [kPkKinds][n + 1]
    std::vector<long long> need0, iter;   // [3][n], [n]
};

PersistTables persist_tables(const std::vector<Geom>& geoms, const std::vector<int>& idx, int T, int K2) {
    PersistTables pt;
    const int n = (int)idx.size();
    pt.sub_stride = std::max(3, 3 + 2 * K2);
    pt.kind.assign(3 * pt.sub_stride, 0);
    pt.arg.assign(3 * pt.sub_stride, 0);
    pt.base.assign(3 * pt.sub_stride, 0);
    auto add = [&](int g, int kind, int arg) {
        pt.kind[g * pt.sub_stride + pt.nsub[g]] = kind;
        pt.arg[g * pt.sub_stride + pt.nsub[g]] = arg;
        ++pt.nsub[g];
    };
    add(0, kPkBpassInit, 0);
    add(0, kPkRowsB, 0);
    add(0, kPkEta, 0);
    add(1, kPkApass, 0);
    add(1, kPkAA, 0);
    add(1, kPkRowsA, 0);
    for (int k = 0; k < K2; ++k) {
        add(1, kPkBpassStep, 0);
        add(1, kPkRowsB, k + 1 < K2 ? 1 : 0);
    }
    add(2, kPkClose, 0);
    add(2, kPkCloseRed, 0);
    add(2, kPkFinal, 0);
    pt.cnt.assign((size_t)kPkKinds * n, 0);
    pt.pre.assign((size_t)kPkKinds * (n + 1), 0);
    for (int k = 0; k < n; ++k) {
        const Geom& g = geoms[idx[k]];
        const int rows = (g.L + kPersistRows - 1) / kPersistRows;
        const int c[kPkKinds] = {g.npg, g.npg, g.npg, rows, (g.p * g.p + 1 + 7) / 8, rows, 1, g.npg, 1,
                                 kPersistFinal};
        for (int kd = 0; kd < kPkKinds; ++kd) pt.cnt[(size_t)kd * n + k] = c[kd];
    }
    for (int kd = 0; kd < kPkKinds; ++kd)
        for (int k = 0; k < n; ++k)
            pt.pre[(size_t)kd * (n + 1) + k + 1] = pt.pre[(size_t)kd * (n + 1) + k] + pt.cnt[(size_t)kd * n + k];
    for (int g = 0; g < 3; ++g) {
        long long b = 0;
        for (int j = 0; j < pt.nsub[g]; ++j) {
            pt.base[g * pt.sub_stride + j] = b;
            b += pt.pre[(size_t)pt.kind[g * pt.sub_stride + j] * (n + 1) + n];
        }
        pt.seg_len[g] = b;
    }
    pt.need0.assign(3 * (size_t)n, 0);
    pt.iter.assign(n, 0);
    for (int k = 0; k < n; ++k) {
        long long pro = 0, it = 0;
        for (int j = 0; j < pt.nsub[0]; ++j) pro += pt.cnt[(size_t)pt.kind[j] * n + k];
        for (int j = 0; j < pt.nsub[1]; ++j) it += pt.cnt[(size_t)pt.kind[pt.sub_stride + j] * n + k];
        pt.need0[k] = 0;
        pt.need0[n + k] = pro;
        pt.need0[2 * n + k] = pro + (long long)T * it;
        pt.iter[k] = it;
    }
    return pt;
}

// Tiles per work item of the persistent kernel: tuned for the batch's class,
// else kDefaultTilesPerItem.
int tiles_per_item_default(int n, const edaa_image_desc* images, int x_dtype) {
    int v1 = 0, v2 = 0;
    if (tune_lookup(ragged_class(n, images, x_dtype), &v1, &v2) && v1 > 0) return v1;
    return kDefaultTilesPerItem;
}

edaa_status run_ragged(edaa_ctx* ctx, int n, edaa_image_desc* images, const edaa_params* P) {
    const int T = P->T, K1 = P->K1, K2 = P->K2;
    const int x_bytes = P->x_dtype == EDAA_X_BF16 ? 2 : 4;
    const bool grouped_only = (P->flags & EDAA_FLAG_RAGGED_GROUPED) != 0;
    const int tpi = P->tiles_per_item > 0 ? P->tiles_per_item : tiles_per_item_default(n, images, P->x_dtype);
    // images for the persistent kernel, and groups of equal p (order of first
    // appearance) for the launch-per-kernel path
    std::vector<int> pidx;
    std::vector<int> ps;
    std::vector<std::vector<int>> members;
    for (int k = 0; k < n; ++k) {
        if (!grouped_only && images[k].p <= kPersistMaxP) {
            pidx.push_back(k);
            continue;
        }
        size_t gi = 0;
        while (gi < ps.size() && ps[gi] != images[k].p) ++gi;
        if (gi == ps.size()) {
            ps.push_back(images[k].p);
            members.emplace_back();
        }
        members[gi].push_back(k);
    }
    // geometry: a persistent image has one item per pixel group of about
    // `tpi` tiles; an image's own pixel_groups > 0 pins its item count
    std::vector<Geom> geoms(n);
    std::vector<char> is_p(n, 0);
    for (int k : pidx) is_p[k] = 1;
    for (int k = 0; k < n; ++k) {
        const edaa_image_desc& d = images[k];
        const int ntiles = (d.N + kTile - 1) / kTile;
        const int req = d.pixel_groups > 0 ? d.pixel_groups : (is_p[k] ? (ntiles + tpi - 1) / tpi : 0);
        geoms[k] = make_geom(d.L, d.N, 1, d.p, 1, req);
        images[k].pixel_groups = geoms[k].npg;
    }
    // workspace: per-image state, the job tables, the maps, the persistent tables
    std::vector<size_t> off(n);
    Arena a;
    for (int k = 0; k < n; ++k) off[k] = a.take<char>(layout(geoms[k], T, x_bytes, nullptr, nullptr));
    const size_t o_jobs = a.take<ImageJob>(n);
    const size_t o_pjobs = a.take<ImageJob>(std::max<size_t>(pidx.size(), 1));
    std::vector<std::vector<int2>> maps(ps.size() * kMapKinds);
    for (size_t gi = 0; gi < ps.size(); ++gi)
        for (int k : members[gi]) {
            const Geom& g = geoms[k];
            for (int b = 0; b < g.npg * g.nqc; ++b) maps[gi * kMapKinds + kMapPass].push_back(make_int2(k, b));
            for (int b = 0; b < g.L; ++b) maps[gi * kMapKinds + kMapRows].push_back(make_int2(k, b));
            maps[gi * kMapKinds + kMapOne].push_back(make_int2(k, 0));
            for (int b = 0; b < kElemBlocks; ++b) maps[gi * kMapKinds + kMapElem].push_back(make_int2(k, b));
            for (int b = 0; b < aa_blocks(g.p); ++b) maps[gi * kMapKinds + kMapAA].push_back(make_int2(k, b));
        }
    std::vector<size_t> o_maps(maps.size());
    for (size_t i = 0; i < maps.size(); ++i) o_maps[i] = a.take<int2>(maps[i].size());
    PersistTables pt;
    size_t o_kind = 0, o_arg = 0, o_base = 0, o_cnt = 0, o_pre = 0, o_need = 0, o_iter = 0, o_ctr = 0;
    if (!pidx.empty()) {
        pt = persist_tables(geoms, pidx, T, K2);
        o_kind = a.take<int>(pt.kind.size());
        o_arg = a.take<int>(pt.arg.size());
        o_base = a.take<long long>(pt.base.size());
        o_cnt = a.take<int>(pt.cnt.size());
        o_pre = a.take<long long>(pt.pre.size());
        o_need = a.take<long long>(pt.need0.size());
        o_iter = a.take<long long>(pt.iter.size());
        o_ctr = a.take<unsigned long long>(pidx.size() + 2);
    }
    edaa_status st = ensure_ws(ctx, a.off + 256);
    if (st != EDAA_OK) return st;
    char* base = (char*)ctx->ws;

    std::vector<ImageJob> jobs(n);
    std::vector<PadJob> pads(n);
    std::vector<uint64_t> seeds(n);
    std::vector<double> gammas(n);
    std::vector<RunBuffers> rbs(n);
    for (int k = 0; k < n; ++k) {
        const edaa_image_desc& d = images[k];
        RunBuffers& rb = rbs[k];
        memset(&rb, 0, sizeof(rb));
        layout(geoms[k], T, x_bytes, base + off[k], &rb);
        rb.s.A = d.A;
        ImageJob& J = jobs[k];
        memset(&J, 0, sizeof(J));
        J.g = geoms[k];
        J.s = rb.s;
        J.ri.seeds = rb.seeds;
        J.ri.gammas = rb.gammas;
        J.ri.init_scale = (float)P->init_scale;
        J.ri.B0 = nullptr;
        J.ri.A0 = nullptr;
        J.ri.eta1 = P->eta1;
        J.ri.eta2 = P->eta2;
        J.B_out = d.B;
        J.E_out = d.E;
        pads[k] = PadJob{d.X, const_cast<void*>(rb.s.X), d.L, d.N, rb.s.ldx, rb.s.x_bf16};
        seeds[k] = d.seed;
        gammas[k] = d.gamma;
    }
    std::vector<ImageJob> pjobs;
    for (int k : pidx) pjobs.push_back(jobs[k]);
    // host -> device copies happen outside any graph
    for (int k = 0; k < n; ++k) {
        EDAA_HIP(ctx, hipMemcpyAsync(rbs[k].seeds, &seeds[k], sizeof(uint64_t), hipMemcpyHostToDevice, ctx->stream));
        EDAA_HIP(ctx, hipMemcpyAsync(rbs[k].gammas, &gammas[k], sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    }
    const ImageJob* jobs_dev = (const ImageJob*)(base + o_jobs);
    EDAA_HIP(ctx, hipMemcpyAsync(base + o_jobs, jobs.data(), sizeof(ImageJob) * n, hipMemcpyHostToDevice, ctx->stream));
    std::vector<RaggedGroup> groups(ps.size());
    for (size_t gi = 0; gi < ps.size(); ++gi) {
        RaggedGroup& G = groups[gi];
        G.p = ps[gi];
        for (int mk = 0; mk < kMapKinds; ++mk) {
            const std::vector<int2>& m = maps[gi * kMapKinds + mk];
            G.nb[mk] = (int)m.size();
            G.map[mk] = (const int2*)(base + o_maps[gi * kMapKinds + mk]);
            EDAA_HIP(ctx, hipMemcpyAsync(base + o_maps[gi * kMapKinds + mk], m.data(), sizeof(int2) * m.size(),
                                         hipMemcpyHostToDevice, ctx->stream));
        }
        G.lds_a = G.lds_b = G.lds_c = 0;
        for (int k : members[gi]) {
            const Geom& g = geoms[k];
            G.lds_a = std::max(G.lds_a, launch_lds_bytes(g, 0));
            G.lds_b = std::max(G.lds_b, launch_lds_bytes(g, 1));
            G.lds_c = std::max(G.lds_c, launch_lds_bytes(g, 2));
        }
    }
    PersistPlan plan;
    memset(&plan, 0, sizeof(plan));
    size_t plan_lds = 0;
    int plan_wgs = 0;
    const int cosine = P->coherence_mode == EDAA_COHERENCE_COSINE ? 1 : 0;
    if (!pidx.empty()) {
        auto up = [&](size_t o, const void* src, size_t bytes) -> hipError_t {
            return hipMemcpyAsync(base + o, src, bytes, hipMemcpyHostToDevice, ctx->stream);
        };
        EDAA_HIP(ctx, up(o_pjobs, pjobs.data(), sizeof(ImageJob) * pjobs.size()));
        EDAA_HIP(ctx, up(o_kind, pt.kind.data(), sizeof(int) * pt.kind.size()));
        EDAA_HIP(ctx, up(o_arg, pt.arg.data(), sizeof(int) * pt.arg.size()));
        EDAA_HIP(ctx, up(o_base, pt.base.data(), sizeof(long long) * pt.base.size()));
        EDAA_HIP(ctx, up(o_cnt, pt.cnt.data(), sizeof(int) * pt.cnt.size()));
        EDAA_HIP(ctx, up(o_pre, pt.pre.data(), sizeof(long long) * pt.pre.size()));
        EDAA_HIP(ctx, up(o_need, pt.need0.data(), sizeof(long long) * pt.need0.size()));
        EDAA_HIP(ctx, up(o_iter, pt.iter.data(), sizeof(long long) * pt.iter.size()));
        plan.jobs = (const ImageJob*)(base + o_pjobs);
        plan.n_images = (int)pidx.size();
        plan.T = T;
        plan.K1 = K1;
        plan.cosine = cosine;
        for (int g = 0; g < 3; ++g) {
            plan.seg_len[g] = pt.seg_len[g];
            plan.nsub[g] = pt.nsub[g];
        }
        plan.sub_stride = pt.sub_stride;
        plan.seg_kind = (const int*)(base + o_kind);
        plan.seg_arg = (const int*)(base + o_arg);
        plan.seg_base = (const long long*)(base + o_base);
        plan.cnt = (const int*)(base + o_cnt);
        plan.pre = (const long long*)(base + o_pre);
        plan.need0 = (const long long*)(base + o_need);
        plan.iter = (const long long*)(base + o_iter);
        unsigned long long* ctr = (unsigned long long*)(base + o_ctr);
        plan.ticket = ctr;
        plan.status = (int*)(ctr + 1);
        plan.done = ctr + 2;
        plan_lds = (size_t)4 * 512 * sizeof(double);
        for (int k : pidx) {
            const Geom& g = geoms[k];
            plan_lds = std::max({plan_lds, launch_lds_bytes(g, 0), launch_lds_bytes(g, 1), launch_lds_bytes(g, 2)});
        }
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus <= 0)
            cus = 256;
        plan_wgs = cus;
    }
    // the copies read host vectors of this frame: finish them before any
    // return path releases those vectors
    EDAA_HIP(ctx, hipStreamSynchronize(ctx->stream));

    std::string key = "ragged";
    {
        char buf[192];
        snprintf(buf, sizeof(buf), "|%d,%d,%d,%d,%d,%a,%p,%d", T, K1, K2, P->coherence_mode, P->x_dtype,
                 P->init_scale, ctx->ws, P->flags & EDAA_FLAG_RAGGED_GROUPED);
        key += buf;
        for (int k = 0; k < n; ++k) {
            const edaa_image_desc& d = images[k];
            snprintf(buf, sizeof(buf), "|%d,%d,%d,%d,%p,%p,%p,%p", d.L, d.N, d.p, geoms[k].npg, d.X, (void*)d.A,
                     (void*)d.B, (void*)d.E);
            key += buf;
        }
    }
    const PersistPlan* planp = pidx.empty() ? nullptr : &plan;
    st = run_captured(ctx, key, (P->flags & EDAA_FLAG_GRAPH) != 0, [&](hipStream_t s, long long* nl) {
        return enqueue_ragged(groups, pads, jobs_dev, planp, plan_lds, plan_wgs, T, K1, K2, cosine, s, nl);
    });
    if (st != EDAA_OK) return st;
    for (int k = 0; k < n; ++k)
        if (images[k].loss_trace)
            EDAA_HIP(ctx, hipMemcpyAsync(images[k].loss_trace, rbs[k].s.trace, sizeof(double) * (T + 1),
                                         hipMemcpyDeviceToHost, ctx->stream));
    if (planp) {
        int status = 0;
        EDAA_HIP(ctx, hipMemcpyAsync(&status, plan.status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        EDAA_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (status != 0) {
            ctx->poisoned = true;
            return fail(EDAA_EDEVICE, "persistent ragged kernel: a wait for earlier items exceeded its bound");
        }
    } else {
        EDAA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    return EDAA_OK;
}

}  // namespace

namespace {
// Outer iterations of the autotuner's trial runs: the time of one outer
// iteration is the difference of the two, divided by their difference.
constexpr int kTuneShortT = 2, kTuneLongT = 6;

// Milliseconds of `call` (enqueued on the context stream), from HIP events.
template <typename F>
edaa_status time_call(edaa_ctx* ctx, F&& call, double* ms) {
    hipEvent_t e0, e1;
    EDAA_HIP(ctx, hipEventCreate(&e0));
    EDAA_HIP(ctx, hipEventCreate(&e1));
    EDAA_HIP(ctx, hipEventRecord(e0, ctx->stream));
    edaa_status st = call();
    if (st == EDAA_OK) {
        EDAA_HIP(ctx, hipEventRecord(e1, ctx->stream));
        EDAA_HIP(ctx, hipEventSynchronize(e1));
        float f = 0.f;
        EDAA_HIP(ctx, hipEventElapsedTime(&f, e0, e1));
        *ms = f;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}
}  // namespace

extern "C" {

void edaa_default_params(edaa_params* P) {
    if (!P) return;
    memset(P, 0, sizeof(*P));
    P->T = 100;
    P->K1 = 5;
    P->K2 = 5;
    P->gamma = 1.0;
    P->eta1 = 0.0;
    P->eta2 = 0.0;
    P->init_scale = 0.1;
    P->select_threshold = 1.05;
    P->x_dtype = EDAA_X_F32;
    P->coherence_mode = EDAA_COHERENCE_COSINE;
    P->flags = 0;
    P->runs_per_chunk = 0;
    P->pixel_groups = 0;
    P->tiles_per_item = 0;
}

const char* edaa_last_error(void) { return g_last_error.c_str(); }

edaa_status edaa_create(edaa_ctx** out, int device, void* stream) {
    if (!out) return fail(EDAA_EINVAL, "out is null");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return fail(EDAA_EDEVICE, "no HIP device available");
    }
    if (device < 0 || device >= n) return fail(EDAA_EINVAL, "device %d out of range [0, %d)", device, n);
    if (hipSetDevice(device) != hipSuccess) return fail(EDAA_EDEVICE, "hipSetDevice(%d) failed", device);
    void* sp = nullptr;
    const hipError_t se = scratch_address(device, &sp);
    if (se != hipSuccess) {
        (void)hipGetLastError();
        return fail(EDAA_EDEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", device,
                    hipGetErrorString(se));
    }
    edaa_ctx* ctx = new edaa_ctx();
    ctx->device = device;
    ctx->scratch = sp;
    ctx->stream = (hipStream_t)stream;
    *out = ctx;
    return EDAA_OK;
}

void edaa_destroy(edaa_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& ge : ctx->graphs) (void)hipGraphExecDestroy(ge.exec);
    for (auto& e : ctx->timer.ev) (void)hipEventDestroy(e);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->ws) (void)hipFree(ctx->ws);
    delete ctx;
}

long long edaa_last_launch_count(edaa_ctx* ctx) { return ctx ? ctx->last_launches : -1; }

edaa_status edaa_set_graph_cache(edaa_ctx* ctx, int n) {
    edaa_status st = check_ctx(ctx);
    if (st != EDAA_OK) return st;
    EDAA_REQUIRE(n >= 1, "graph cache capacity must be >= 1 (got %d)", n);
    ctx->graph_cap = (size_t)n;
    while (ctx->graphs.size() > ctx->graph_cap) {
        (void)hipGraphExecDestroy(ctx->graphs.front().exec);
        ctx->graphs.erase(ctx->graphs.begin());
    }
    return EDAA_OK;
}

edaa_status edaa_plan(int L, int N, int p, int M, const edaa_params* params, edaa_launch_plan* out) {
    edaa_status st = check_params(params);
    if (st != EDAA_OK) return st;
    if ((st = check_shape(L, N, p, M)) != EDAA_OK) return st;
    EDAA_REQUIRE(out != nullptr, "out is null");
    Geom g;
    int source = 0;
    if ((st = plan_geom(L, N, p, M, params, &g, &source)) != EDAA_OK) return st;
    out->runs_per_chunk = g.R;
    out->chunks = g.nqc;
    out->pixel_groups = g.npg;
    out->double_buffer = g.dbuf;
    out->source = source;
    out->bf16_passes = use_xb(g, params->x_dtype == EDAA_X_BF16 ? 2 : 4, params->flags);
    return EDAA_OK;
}

edaa_status edaa_pass_times(edaa_ctx* ctx, int kind, int* count, double* total_ms) {
    edaa_status st = check_ctx(ctx);
    if (st != EDAA_OK) return st;
    EDAA_REQUIRE(kind >= 0 && kind <= 2 && count && total_ms, "kind must be 0, 1 or 2; count/total_ms non-null");
    EDAA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    int n = 0;
    double tot = 0.0;
    for (int i = 0; i < ctx->timer.used; ++i) {
        if (ctx->timer.kind[i] != kind) continue;
        float ms = 0.f;
        EDAA_HIP(ctx, hipEventElapsedTime(&ms, ctx->timer.ev[2 * i], ctx->timer.ev[2 * i + 1]));
        tot += ms;
        ++n;
    }
    *count = n;
    *total_ms = tot;
    return EDAA_OK;
}

edaa_status edaa_normalize_pixels(edaa_ctx* ctx, const float* X_in, void* X_out, int L, int N, int out_dtype,
                                  int* n_zero) {
    edaa_status st = check_ctx(ctx);
    if (st != EDAA_OK) return st;
    EDAA_REQUIRE(X_in && X_out, "X_in and X_out must not be null");
    EDAA_REQUIRE(L >= 1 && N >= 1, "L and N must be >= 1 (got %d, %d)", L, N);
    EDAA_REQUIRE((double)L * N < 2147483647.0, "image too large");
    EDAA_REQUIRE(out_dtype == EDAA_X_F32 || out_dtype == EDAA_X_BF16, "out_dtype must be EDAA_X_F32 or EDAA_X_BF16");
    EDAA_REQUIRE(out_dtype == EDAA_X_F32 || (const void*)X_in != X_out, "bf16 output cannot overwrite the input");
    int* dz = nullptr;
    if (n_zero) {
        st = ensure_ws(ctx, 256);
        if (st != EDAA_OK) return st;
        dz = (int*)ctx->ws;
        EDAA_HIP(ctx, hipMemsetAsync(dz, 0, sizeof(int), ctx->stream));
    }
    EDAA_HIP(ctx, launch_normalize(X_in, X_out, L, N, out_dtype == EDAA_X_BF16, dz, ctx->stream));
    if (n_zero) {
        EDAA_HIP(ctx, hipMemcpyAsync(n_zero, dz, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        EDAA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    return EDAA_OK;
}

edaa_status edaa_fit(edaa_ctx* ctx, const void* X, int L, int N, int p, const edaa_params* params, uint64_t seed,
                     const float* A0, const float* B0, float* A, float* B, float* E, double* loss_trace,
                     double* eta_out) {
    edaa_status st = check_ctx(ctx);
    if (st != EDAA_OK) return st;
    if ((st = check_params(params)) != EDAA_OK) return st;
    if ((st = check_shape(L, N, p, 1)) != EDAA_OK) return st;
    EDAA_REQUIRE(X && A && B, "X, A and B must not be null");
    EDAA_REQUIRE(params->eta1 > 0.0 || (isfinite(params->gamma) && params->gamma > 0.0),
                 "gamma must be finite and > 0 (got %g)", params->gamma);
    const double gamma = params->gamma;
    st = run_batch(ctx, X, L, N, p, params, 1, &seed, &gamma, A0, B0, A, B, E, loss_trace, nullptr, nullptr,
                   eta_out);
    if (st != EDAA_OK) return st;
    if (loss_trace && !isfinite(loss_trace[params->T]))
        return fail(EDAA_ENUMERIC, "the objective is not finite after %d outer iterations", params->T);
    return EDAA_OK;
}

edaa_status edaa_fit_noalloc(edaa_ctx* ctx, const void* X, int L, int N, int p, const edaa_params* params,
                             uint64_t seed, const float* A0, const float* B0, float* A, float* B, float* E,
                             double* loss_trace_dev, double* eta_dev) {
    edaa_status st = check_ctx(ctx);
    if (st != EDAA_OK) return st;
    if ((st = check_params(params)) != EDAA_OK) return st;
    if ((st = check_shape(L, N, p, 1)) != EDAA_OK) return st;
    EDAA_REQUIRE(X && A && B, "X, A and B must not be null");
    EDAA_REQUIRE(params->eta1 > 0.0 || (isfinite(params->gamma) && params->gamma > 0.0),
                 "gamma must be finite and > 0 (got %g)", params->gamma);
    EDAA_REQUIRE((params->flags & (EDAA_FLAG_GRAPH | EDAA_FLAG_TIME_PASSES)) == 0,
                 "edaa_fit_noalloc takes neither EDAA_FLAG_GRAPH nor EDAA_FLAG_TIME_PASSES (both allocate)");
    EDAA_REQUIRE(ctx->scratch != nullptr, "context has no scratch memory");
    Geom g;
    if ((st = plan_geom(L, N, p, 1, params, &g, nullptr)) != EDAA_OK) return st;
    const int x_bytes = params->x_dtype == EDAA_X_BF16 ? 2 : 4;
    const size_t need = layout(g, params->T, x_bytes, nullptr, nullptr);
    if (need > kScratchBytes)
        return fail(EDAA_EUNSUPPORTED,
                    "L=%d, N=%d, p=%d needs %zu bytes of scratch; edaa_fit_noalloc holds at most %zu (use edaa_fit)",
                    L, N, p, need, kScratchBytes);
    RunBuffers rb;
    memset(&rb, 0, sizeof(rb));
    layout(g, params->T, x_bytes, (char*)ctx->scratch, &rb);
    State& s = rb.s;
    s.A = A;
    s.x_mfma = use_xb(g, x_bytes, params->flags);
    if (loss_trace_dev) s.trace = loss_trace_dev;     // [1][T+1]: the caller's array is the trace
    if (eta_dev) s.etad = eta_dev;
    EDAA_HIP(ctx, launch_set_run(rb.seeds, rb.gammas, seed, params->gamma, ctx->stream));

    Seq q;
    PassTimer off;
    q.timer = &off;
    q.g = &g;
    q.s = &s;
    q.X = X;
    q.ri.seeds = rb.seeds;
    q.ri.gammas = rb.gammas;
    q.ri.init_scale = (float)params->init_scale;
    q.ri.B0 = B0;
    q.ri.A0 = A0;
    q.ri.eta1 = params->eta1;
    q.ri.eta2 = params->eta2;
    q.mode = B0 ? kModeInitB0 : kModeInitRng;
    q.A0 = A0;
    q.T = params->T;
    q.K1 = params->K1;
    q.K2 = params->K2;
    q.B_out = B;
    q.E_out = E;
    q.coherence_mode = params->coherence_mode;
    q.E_given = nullptr;
    long long n = 0;
    const hipError_t e = enqueue_sequence(q, ctx->stream, &n);
    if (e != hipSuccess) {
        ctx->poisoned = true;
        return fail(EDAA_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    }
    ctx->last_launches = n + 1;
    return EDAA_OK;
}

edaa_status edaa_abundances(edaa_ctx* ctx, const void* X, int L, int N, int p, const edaa_params* params,
                            const float* E, const float* A0, float* A, double* loss_trace, double* eta_out) {
    edaa_status st = check_ctx(ctx);
    if (st != EDAA_OK) return st;
    if ((st = check_params(params)) != EDAA_OK) return st;
    if ((st = check_shape(L, N, p, 1)) != EDAA_OK) return st;
    EDAA_REQUIRE(X && E && A, "X, E and A must not be null");
    EDAA_REQUIRE(params->eta1 > 0.0 || (isfinite(params->gamma) && params->gamma > 0.0),
                 "gamma must be finite and > 0 (got %g)", params->gamma);
    const double gamma = params->gamma;
    const uint64_t seed = 0;
    st = run_batch(ctx, X, L, N, p, params, 1, &seed, &gamma, A0, nullptr, A, nullptr, nullptr, loss_trace, nullptr,
                   nullptr, eta_out, E);
    if (st != EDAA_OK) return st;
    if (loss_trace && !isfinite(loss_trace[params->T]))
        return fail(EDAA_ENUMERIC, "the objective is not finite after %d outer iterations", params->T);
    return EDAA_OK;
}

int edaa_select(const double* fit, const double* mu, int M, double threshold) {
    if (!fit || !mu || M <= 0) return -1;
    double fmin = INFINITY;
    bool any = false;
    for (int m = 0; m < M; ++m)
        if (isfinite(fit[m])) {
            fmin = any ? fmin < fit[m] ? fmin : fit[m] : fit[m];
            any = true;
        }
    if (!any) return -1;
    int best = -1;
    double bmu = 0.0;
    for (int m = 0; m < M; ++m) {
        if (!isfinite(fit[m]) || !(fit[m] <= threshold * fmin)) continue;
        if (best < 0 || (isnan(bmu) && !isnan(mu[m])) || mu[m] < bmu) {
            best = m;
            bmu = mu[m];
        }
    }
    return best;
}

edaa_status edaa_ensemble(edaa_ctx* ctx, const void* X, int L, int N, int p, const edaa_params* params, int M,
                          const uint64_t* seeds, const double* gammas, float* A_all, float* B_all, float* E_all,
                          double* loss, double* fit, double* mu, int* run_status, int* selected) {
    edaa_status st = check_ctx(ctx);
    if (st != EDAA_OK) return st;
    if ((st = check_params(params)) != EDAA_OK) return st;
    if ((st = check_shape(L, N, p, M)) != EDAA_OK) return st;
    EDAA_REQUIRE(X && A_all && B_all && seeds && gammas, "X, A_all, B_all, seeds and gammas must not be null");
    if (params->eta1 <= 0.0)
        for (int m = 0; m < M; ++m)
            EDAA_REQUIRE(isfinite(gammas[m]) && gammas[m] > 0.0, "gammas[%d] must be finite and > 0 (got %g)", m,
                         gammas[m]);
    std::vector<double> tr((size_t)M * (params->T + 1)), f(M), u(M);
    st = run_batch(ctx, X, L, N, p, params, M, seeds, gammas, nullptr, nullptr, A_all, B_all, E_all, tr.data(),
                   f.data(), u.data(), nullptr);
    if (st != EDAA_OK) return st;
    int n_ok = 0;
    for (int m = 0; m < M; ++m) {
        const bool ok = isfinite(tr[(size_t)m * (params->T + 1) + params->T]) && isfinite(f[m]);
        if (!ok) f[m] = INFINITY;
        if (run_status) run_status[m] = ok ? EDAA_OK : EDAA_ENUMERIC;
        n_ok += ok;
    }
    const int sel = edaa_select(f.data(), u.data(), M, params->select_threshold);
    if (loss) memcpy(loss, tr.data(), sizeof(double) * tr.size());
    if (fit) memcpy(fit, f.data(), sizeof(double) * M);
    if (mu) memcpy(mu, u.data(), sizeof(double) * M);
    if (selected) *selected = sel;
    if (n_ok == 0) return fail(EDAA_ENUMERIC, "no run of the ensemble has a finite objective");
    return EDAA_OK;
}

edaa_status edaa_fit_ragged(edaa_ctx* ctx, int n_images, edaa_image_desc* images, const edaa_params* params) {
    edaa_status st = check_ctx(ctx);
    if (st != EDAA_OK) return st;
    if ((st = check_params(params)) != EDAA_OK) return st;
    EDAA_REQUIRE(n_images >= 1 && images, "n_images must be >= 1 and images non-null");
    for (int k = 0; k < n_images; ++k) {
        const edaa_image_desc& d = images[k];
        if ((st = check_shape(d.L, d.N, d.p, 1)) != EDAA_OK) return st;
        EDAA_REQUIRE(d.X && d.A && d.B, "image %d: X, A and B must not be null", k);
        EDAA_REQUIRE(params->eta1 > 0.0 || (isfinite(d.gamma) && d.gamma > 0.0), "image %d: gamma must be > 0", k);
        EDAA_REQUIRE(d.pixel_groups >= 0, "image %d: pixel_groups must be >= 0", k);
        if (!runs_fit(d.p, 1, d.L))
            return fail(EDAA_EUNSUPPORTED, "image %d: no pass kernels fit L=%d with p=%d (LDS limit %zu bytes)", k,
                        d.L, d.p, kMaxLdsBytes);
    }
    return run_ragged(ctx, n_images, images, params);
}


edaa_status edaa_autotune(edaa_ctx* ctx, const void* X, int L, int N, int p, int M, const edaa_params* params,
                          edaa_launch_plan* best, double* best_us) {
    edaa_status st = check_ctx(ctx);
    if (st != EDAA_OK) return st;
    if ((st = check_params(params)) != EDAA_OK) return st;
    if ((st = check_shape(L, N, p, M)) != EDAA_OK) return st;
    EDAA_REQUIRE(X != nullptr, "X must not be null");
    // candidate shapes: every compiled chunk size that fits (one run per
    // chunk only for single runs), each with half, the default and twice
    // the default pixel groups rounded to multiples of 8, and the default
    // itself (one workgroup per CU over all chunks, not rounded)
    std::vector<std::pair<int, int>> cand;
    int rc[4] = {0, 0, 0, 0};
    const int nr = run_choices(p, rc);
    for (int i = 0; i < nr; ++i) {
        const int R = rc[i];
        if (!runs_fit(p, R, L) || (M == 1) != (R == 1)) continue;
        const Geom g0 = make_geom(L, N, M, p, R, 0);
        const int base = g0.npg;
        for (int f : {1, 2, 4, 0}) {
            int npg = base * f / 2;
            if (npg >= 8) npg &= ~7;
            if (f == 0) npg = kTargetWorkgroups / g0.nqc;     // one workgroup per CU, not rounded
            npg = std::max(1, std::min(npg, (N + kTile - 1) / kTile));
            bool dup = false;
            for (auto& c : cand) dup |= (c.first == R && c.second == npg);
            if (!dup) cand.emplace_back(R, npg);
        }
    }
    if (cand.empty()) return fail(EDAA_EUNSUPPORTED, "no pass kernels fit L=%d with p=%d", L, p);
    // outputs and per-run inputs of the trial runs
    float* buf = nullptr;
    const size_t na = (size_t)M * p * N, ne = (size_t)M * L * p;
    if (hipMalloc(&buf, sizeof(float) * (2 * na + ne)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(EDAA_ENOMEM, "could not allocate the trial outputs");
    }
    std::vector<uint64_t> seeds(M);
    std::vector<double> gammas(M, isfinite(params->gamma) && params->gamma > 0.0 ? params->gamma : 1.0);
    for (int m = 0; m < M; ++m) seeds[m] = (uint64_t)m;
    edaa_params P = *params;
    P.flags &= ~(EDAA_FLAG_GRAPH | EDAA_FLAG_TIME_PASSES);
    double bus = -1.0;
    int bi = 0;
    for (size_t i = 0; i < cand.size() && st == EDAA_OK; ++i) {
        P.runs_per_chunk = cand[i].first;
        P.pixel_groups = cand[i].second;
        // the time of one outer iteration: ((T = 6) - (T = 2)) / 4, each the
        // best of two after a warm-up
        double t[2] = {1e30, 1e30};
        for (int rep = 0; rep < 5 && st == EDAA_OK; ++rep) {
            P.T = (rep == 0 || rep % 2 == 1) ? kTuneShortT : kTuneLongT;
            double ms = 0.0;
            st = time_call(ctx,
                           [&]() {
                               return run_batch(ctx, X, L, N, p, &P, M, seeds.data(), gammas.data(), nullptr,
                                                nullptr, buf, buf + na, buf + 2 * na, nullptr, nullptr, nullptr,
                                                nullptr);
                           },
                           &ms);
            if (rep > 0) t[(rep - 1) % 2] = std::min(t[(rep - 1) % 2], ms);
        }
        const double us = 1e3 * (t[1] - t[0]) / (kTuneLongT - kTuneShortT);
        if (st == EDAA_OK && (bus < 0.0 || us < bus)) {
            bus = us;
            bi = (int)i;
        }
    }
    (void)hipFree(buf);
    if (st != EDAA_OK) return st;
    tune_store(ensemble_class(L, N, p, M, params->x_dtype), cand[bi].first, cand[bi].second, bus);
    if (best) {
        const Geom g = make_geom(L, N, M, p, cand[bi].first, cand[bi].second);
        best->runs_per_chunk = g.R;
        best->chunks = g.nqc;
        best->pixel_groups = g.npg;
        best->double_buffer = g.dbuf;
        best->source = EDAA_PLAN_TUNED;
        best->bf16_passes = use_xb(g, params->x_dtype == EDAA_X_BF16 ? 2 : 4, params->flags);
    }
    if (best_us) *best_us = bus;
    return EDAA_OK;
}

edaa_status edaa_autotune_ragged(edaa_ctx* ctx, int n_images, edaa_image_desc* images, const edaa_params* params,
                                 int* best_tiles_per_item, double* best_us) {
    edaa_status st = check_ctx(ctx);
    if (st != EDAA_OK) return st;
    if ((st = check_params(params)) != EDAA_OK) return st;
    EDAA_REQUIRE(n_images >= 1 && images, "n_images must be >= 1 and images non-null");
    std::vector<edaa_image_desc> d(n_images);
    edaa_params P = *params;
    P.flags &= ~(EDAA_FLAG_GRAPH | EDAA_FLAG_TIME_PASSES | EDAA_FLAG_RAGGED_GROUPED);
    double bus = -1.0;
    int bt = kDefaultTilesPerItem;
    for (int tpi : {1, 2, 4, 8, 16, 32, 64, 128}) {
        P.tiles_per_item = tpi;
        double t[2] = {1e30, 1e30};
        for (int rep = 0; rep < 5; ++rep) {
            // a fit writes the item counts it used into the descriptors:
            // start every trial from unpinned copies
            for (int k = 0; k < n_images; ++k) {
                d[k] = images[k];
                d[k].loss_trace = nullptr;
                d[k].pixel_groups = 0;
            }
            P.T = (rep == 0 || rep % 2 == 1) ? kTuneShortT : kTuneLongT;
            double ms = 0.0;
            st = time_call(ctx, [&]() { return edaa_fit_ragged(ctx, n_images, d.data(), &P); }, &ms);
            if (st != EDAA_OK) return st;
            if (rep > 0) t[(rep - 1) % 2] = std::min(t[(rep - 1) % 2], ms);
        }
        const double us = 1e3 * (t[1] - t[0]) / (kTuneLongT - kTuneShortT);
        if (bus < 0.0 || us < bus) {
            bus = us;
            bt = tpi;
        }
    }
    tune_store(ragged_class(n_images, images, params->x_dtype), bt, 0, bus);
    if (best_tiles_per_item) *best_tiles_per_item = bt;
    if (best_us) *best_us = bus;
    return EDAA_OK;
}

namespace {
edaa_status grad_work(edaa_ctx* ctx, int L, int N, int p, GradWork* w) {
    Arena a;
    const int nblk = grad_blocks(N);
    const size_t oE = a.take<float>((size_t)L * p), oEd = a.take<double>((size_t)L * p),
                 oW = a.take<double>((size_t)L * p), oV = a.take<double>((size_t)nblk * L * p),
                 oL = a.take<double>(nblk), oCm = a.take<float>((size_t)nblk * p),
                 oCs = a.take<float>((size_t)nblk * p), oSt = a.take<float>(2 * (size_t)p);
    edaa_status st = ensure_ws(ctx, a.off + 256);
    if (st != EDAA_OK) return st;
    char* b = (char*)ctx->ws;
    w->E = (float*)(b + oE);
    w->Ed = (double*)(b + oEd);
    w->Wd = (double*)(b + oW);
    w->Vpart = (double*)(b + oV);
    w->lpart = (double*)(b + oL);
    w->cm = (float*)(b + oCm);
    w->cs = (float*)(b + oCs);
    w->colstat = (float*)(b + oSt);
    w->nblk = nblk;
    return EDAA_OK;
}
}  // namespace

edaa_status edaa_loss_fwd(edaa_ctx* ctx, const float* X, const float* A, const float* B, int L, int N, int p,
                          float* loss_dev) {
    edaa_status st = check_ctx(ctx);
    if (st != EDAA_OK) return st;
    if ((st = check_shape(L, N, p, 1)) != EDAA_OK) return st;
    EDAA_REQUIRE(X && A && B && loss_dev, "X, A, B and loss_dev must not be null");
    GradWork w;
    if ((st = grad_work(ctx, L, N, p, &w)) != EDAA_OK) return st;
    EDAA_HIP(ctx, launch_loss_fwd(X, A, B, L, N, p, w, loss_dev, ctx->stream));
    return EDAA_OK;
}

edaa_status edaa_loss_bwd(edaa_ctx* ctx, const float* X, const float* A, const float* B, int L, int N, int p,
                          const float* grad_out, float* gA, float* gB) {
    edaa_status st = check_ctx(ctx);
    if (st != EDAA_OK) return st;
    if ((st = check_shape(L, N, p, 1)) != EDAA_OK) return st;
    EDAA_REQUIRE(X && A && B && grad_out, "X, A, B and grad_out must not be null");
    EDAA_REQUIRE(gA || gB, "at least one of gA, gB must be non-null");
    GradWork w;
    if ((st = grad_work(ctx, L, N, p, &w)) != EDAA_OK) return st;
    EDAA_HIP(ctx, launch_loss_bwd(X, A, B, L, N, p, grad_out, w, gA, gB, ctx->stream));
    return EDAA_OK;
}

edaa_status edaa_mirror_step_A(edaa_ctx* ctx, float* A, const float* gA, int p, int N, float eta) {
    edaa_status st = check_ctx(ctx);
    if (st != EDAA_OK) return st;
    EDAA_REQUIRE(A && gA, "A and gA must not be null");
    EDAA_REQUIRE(p >= 1 && p <= kMaxP && N >= 1, "need 1 <= p <= %d and N >= 1", kMaxP);
    EDAA_REQUIRE(isfinite(eta), "eta must be finite");
    EDAA_HIP(ctx, launch_mirror_A(A, gA, p, N, eta, ctx->stream));
    return EDAA_OK;
}

edaa_status edaa_mirror_step_B(edaa_ctx* ctx, float* B, const float* gB, int N, int p, float eta) {
    edaa_status st = check_ctx(ctx);
    if (st != EDAA_OK) return st;
    EDAA_REQUIRE(B && gB, "B and gB must not be null");
    EDAA_REQUIRE(p >= 1 && p <= kMaxP && N >= 1, "need 1 <= p <= %d and N >= 1", kMaxP);
    EDAA_REQUIRE(isfinite(eta), "eta must be finite");
    GradWork w;
    if ((st = grad_work(ctx, 1, N, p, &w)) != EDAA_OK) return st;
    EDAA_HIP(ctx, launch_mirror_B(B, gB, N, p, eta, w, ctx->stream));
    return EDAA_OK;
}

}  // extern "C"
