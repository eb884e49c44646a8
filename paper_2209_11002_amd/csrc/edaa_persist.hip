// Persistent execution of a ragged batch: single EDAA runs (Algorithm 1) on
// images of different (L, N, p), all advanced by one launch of one kernel.
//
// Work is cut into items: a pass over X (init B-pass, A-pass, B-step pass,
// closing pass) is npg items per image, each one pixel group (tiles i,
// i + npg, ...); a reduction of the per-item partials is one item per block
// of rows (or per eight entries of A A^T); step sizes, the final objective
// and the outputs are single items.  The sequence of an image is
// prologue (init B-pass, column statistics and E, step sizes), T times the
// outer iteration (A-pass, A A^T and objective, X A^T and W, then K2 times a
// B-step pass and its reduction) and epilogue (closing pass and its sum,
// outputs), exactly the launch sequence of a single fit.
//
// Items are handed out by one ticket counter in a fixed order: sub-stage by
// sub-stage, and within a sub-stage image by image.  An item may start once
// its image has completed every item of the earlier sub-stages, counted by a
// per-image counter that each finished item increments (agent-scope release;
// the waiting workgroup acquires).  Every item an item waits for holds a
// smaller ticket, already taken by a running workgroup, so the smallest
// unfinished ticket can always proceed: the scheme cannot deadlock, whatever
// the number of resident workgroups.  A wait that exceeds a generous bound
// (far beyond any legitimate wait) sets an error flag and lets the workgroup
// leave, so the kernel always ends.
#include "edaa_device.h"

namespace edaa {
namespace {

constexpr int kPersistThreads = 512;
constexpr unsigned long long kSpinLimit = 1ull << 22;   // polls of ~1 us: a few seconds

__device__ __forceinline__ long long ld_relaxed(const unsigned long long* p) {
    return (long long)__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Item (sub-stage kind, image k, index i, outer iteration it, argument) of
// ticket t, and the number of items of image k that must be done before it.
struct Item {
    int kind, k, i, it, arg;
    long long need;
};

__device__ Item decode(const PersistPlan& P, long long t) {
    Item it{};
    int g;
    long long r;
    if (t < P.seg_len[0]) {
        g = 0;
        r = t;
        it.it = 0;
    } else if (t < P.seg_len[0] + (long long)P.T * P.seg_len[1]) {
        g = 1;
        const long long u = t - P.seg_len[0];
        it.it = (int)(u / P.seg_len[1]);
        r = u % P.seg_len[1];
    } else {
        g = 2;
        r = t - P.seg_len[0] - (long long)P.T * P.seg_len[1];
        it.it = P.T;
    }
    const int* kinds = P.seg_kind + g * P.sub_stride;
    const int* args = P.seg_arg + g * P.sub_stride;
    const long long* base = P.seg_base + g * P.sub_stride;
    int j = 0;
    while (j + 1 < P.nsub[g] && base[j + 1] <= r) ++j;
    it.kind = kinds[j];
    it.arg = args[j];
    const long long r2 = r - base[j];
    const long long* pre = P.pre + (size_t)it.kind * (P.n_images + 1);
    int lo = 0, hi = P.n_images;                  // largest k with pre[k] <= r2
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= r2) lo = mid; else hi = mid;
    }
    it.k = lo;
    it.i = (int)(r2 - pre[lo]);
    long long need = P.need0[g * P.n_images + lo] + (g == 1 ? (long long)it.it * P.iter[lo] : 0);
    for (int jj = 0; jj < j; ++jj) need += P.cnt[kinds[jj] * P.n_images + lo];
    it.need = need;
    return it;
}

// One item of an image with p = PP.  Not inlined: each p gets its own
// register allocation (inlining all nine into the kernel made the allocator
// spill).
template <int PP>
__device__ __noinline__ void run_item(const PersistPlan& P, const ImageJob& J, const Item& it, float* smem) {
    const Geom& g = J.g;
    const State& s = J.s;
    double* scratch = (double*)smem;
    switch (it.kind) {
        case kPkBpassInit:
            bpass_body<PP, 1, false>(g, s, it.i, s.W, kModeInitRng, J.ri);
            break;
        case kPkBpassStep:
            bpass_body<PP, 1, true>(g, s, it.i, s.W, kModeStep, J.ri);
            break;
        case kPkApass:
            apass_body<PP, 1>(g, s, it.i, s.E, P.K1);
            break;
        case kPkRowsB: {
            const int l0 = it.i * kPersistRows;
            reduce_b_rows<PP, 1>(g, s, l0, min(kPersistRows, g.L - l0), 0, it.arg, scratch);
            break;
        }
        case kPkAA: {
            const int n = P.cnt[kPkAA * P.n_images + it.k];
            reduce_aa_body<PP, 1>(g, s, 0, 8 * it.i, 8 * n, it.it);
            break;
        }
        case kPkRowsA: {
            const int l0 = it.i * kPersistRows;
            reduce_a_rows<PP, 1>(g, s, l0, min(kPersistRows, g.L - l0), 0, scratch);
            break;
        }
        case kPkEta:
            eta_body<PP>(g, s, 0, J.ri, scratch);
            break;
        case kPkClose:
            close_body<PP, 1, 8>(g, s, it.i, s.E);
            break;
        case kPkCloseRed:
            reduce_close_body(g, s, threadIdx.x, kPersistThreads);
            break;
        case kPkFinal:
            final_B_body<PP>(g, s, it.i, 0, kPersistFinal, J.B_out);
            if (it.i == 0) {
                __syncthreads();
                final_E_body<PP>(g, s, 0, J.E_out, P.cosine, scratch);
            }
            break;
        default:
            break;
    }
}

__global__ __launch_bounds__(kPersistThreads, 1) void k_ragged_persistent(PersistPlan P) {
    // Dynamic LDS only (the bodies expect it 16-byte aligned); the item of
    // the workgroup is handed from thread 0 to the others in its first bytes.
    extern __shared__ float smem[];
    Item& s_it = *(Item*)smem;
    const long long total = P.seg_len[0] + (long long)P.T * P.seg_len[1] + P.seg_len[2];
    for (;;) {
        if (threadIdx.x == 0) {
            const long long t = (long long)atomicAdd(P.ticket, 1ull);
            Item it;
            if (t >= total) {
                it.kind = -1;
            } else {
                it = decode(P, t);
                unsigned long long spins = 0;
                while (ld_relaxed(P.done + it.k) < it.need) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > kSpinLimit) {
                        atomicExch(P.status, 1);
                        it.kind = -1;
                        break;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            s_it = it;
        }
        __syncthreads();
        const Item it = s_it;
        __syncthreads();                           // every thread holds the item before a body writes LDS
        if (it.kind < 0) break;
        const ImageJob& J = P.jobs[it.k];
        switch (J.g.p) {
            case 1: run_item<1>(P, J, it, smem); break;
            case 2: run_item<2>(P, J, it, smem); break;
            case 3: run_item<3>(P, J, it, smem); break;
            case 4: run_item<4>(P, J, it, smem); break;
            case 5: run_item<5>(P, J, it, smem); break;
            case 6: run_item<6>(P, J, it, smem); break;
            case 7: run_item<7>(P, J, it, smem); break;
            case 8: run_item<8>(P, J, it, smem); break;
            case 9: run_item<9>(P, J, it, smem); break;
            default: break;
        }
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_fetch_add(P.done + it.k, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Start state of every image: E, W, X A^T, E (float64) zero and A = 1/p;
// the ticket, the per-image counters and the status flag zero.
__global__ __launch_bounds__(kThreads) void k_persist_prep(PersistPlan P) {
    const int k = blockIdx.y;
    const ImageJob& J = P.jobs[k];
    const Geom& g = J.g;
    const State& s = J.s;
    const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, st = (size_t)gridDim.x * blockDim.x;
    const size_t nf = (size_t)(g.L + kPadRows) * g.Qp, nd = (size_t)g.L * g.Qp;
    for (size_t i = i0; i < nf; i += st) {
        s.E[i] = 0.f;
        s.W[i] = 0.f;
    }
    for (size_t i = i0; i < nd; i += st) {
        s.XAtd[i] = 0.0;
        s.Ed[i] = 0.0;
    }
    const size_t na = (size_t)g.p * g.N;
    for (size_t i = i0; i < na; i += st) s.A[i] = 1.f / (float)g.p;
    if (i0 == 0) P.done[k] = 0ull;
    if (k == 0 && i0 == 0) {
        *P.ticket = 0ull;
        *P.status = 0;
    }
}

}  // namespace

hipError_t launch_ragged_persistent(const PersistPlan& P, size_t lds_bytes, int n_workgroups, hipStream_t st) {
    hipLaunchKernelGGL(k_persist_prep, dim3(kElemBlocks, P.n_images), dim3(kThreads), 0, st, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    set_max_lds((const void*)k_ragged_persistent, (int)lds_bytes);
    hipLaunchKernelGGL(k_ragged_persistent, dim3(n_workgroups), dim3(kPersistThreads), lds_bytes, st, P);
    return hipGetLastError();
}

}  // namespace edaa
