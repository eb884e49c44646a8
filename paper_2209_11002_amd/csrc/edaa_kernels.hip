// Common kernels and host-side geometry of the EDAA library: the padded copy
// of X, fills, normalisation, the closing reduction, and the dispatch of the
// per-p pass launchers (edaa_inst.hip) by p.
#include <algorithm>

#include "edaa_device.h"

namespace edaa {
namespace {

__global__ void k_reduce_close(Geom g, State s) {
    reduce_close_body(g, s, threadIdx.x + blockIdx.x * blockDim.x, blockDim.x * gridDim.x);
}

// The padded copy of X the pass kernels read: [L][ldx], pixels >= N zero.
__global__ void k_pad_x(const void* __restrict__ X, void* __restrict__ Xp, int L, int N, size_t ldx, int bf16) {
    const size_t n = (size_t)L * ldx;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t l = i / ldx, pix = i % ldx;
        if (bf16)
            ((uint16_t*)Xp)[i] = pix < (size_t)N ? ((const uint16_t*)X)[l * N + pix] : (uint16_t)0;
        else
            ((float*)Xp)[i] = pix < (size_t)N ? ((const float*)X)[l * N + pix] : 0.f;
    }
}

__global__ void k_fill(float* __restrict__ dst, size_t n, float v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) dst[i] = v;
}

__global__ void k_init_A(float* __restrict__ A, const float* __restrict__ A0, size_t n, float v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        A[i] = A0 ? A0[i] : v;
}

__global__ __launch_bounds__(kThreads) void k_normalize(const float* __restrict__ Xin, void* Xout, int L, int N,
                                                        int out_bf16, int* n_zero) {
    const int pix = blockIdx.x * kThreads + threadIdx.x;
    if (pix >= N) return;
    float ss = 0.f;
    for (int l = 0; l < L; ++l) {
        const float x = Xin[(size_t)l * N + pix];
        ss = fmaf(x, x, ss);
    }
    const bool zero = !(ss > 0.f);
    const float inv = zero ? 0.f : 1.f / sqrtf(ss);
    if (zero && n_zero) atomicAdd(n_zero, 1);
    if (out_bf16) {
        uint16_t* Xh = (uint16_t*)Xout;
        for (int l = 0; l < L; ++l) Xh[(size_t)l * N + pix] = f32_to_bf16_rne(Xin[(size_t)l * N + pix] * inv);
    } else {
        float* Xf = (float*)Xout;
        for (int l = 0; l < L; ++l) Xf[(size_t)l * N + pix] = Xin[(size_t)l * N + pix] * inv;
    }
}

// Given endmembers (abundance estimation with E fixed): E [L][p] of run 0
// into the padded float and float64 state arrays.
__global__ void k_set_e(const float* __restrict__ Eg, float* __restrict__ E, double* __restrict__ Ed, int L, int p,
                        int Qp) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < L * p; e += gridDim.x * blockDim.x) {
        const int l = e / p, j = e % p;
        E[(size_t)l * Qp + j] = Eg[e];
        Ed[(size_t)l * Qp + j] = (double)Eg[e];
    }
}

// Seed and gamma of a single run into device memory (used where no host copy
// may be enqueued).
__global__ void k_set_run(uint64_t* __restrict__ seeds, double* __restrict__ gammas, uint64_t seed, double gamma) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        seeds[0] = seed;
        gammas[0] = gamma;
    }
}

}  // namespace

#define EDAA_DECL_OPS(P) const PassOps* ops_p##P();
EDAA_DECL_OPS(1) EDAA_DECL_OPS(2) EDAA_DECL_OPS(3) EDAA_DECL_OPS(4) EDAA_DECL_OPS(5) EDAA_DECL_OPS(6)
EDAA_DECL_OPS(7) EDAA_DECL_OPS(8) EDAA_DECL_OPS(9) EDAA_DECL_OPS(10) EDAA_DECL_OPS(11) EDAA_DECL_OPS(12)
EDAA_DECL_OPS(13) EDAA_DECL_OPS(14) EDAA_DECL_OPS(15) EDAA_DECL_OPS(16)
#undef EDAA_DECL_OPS

const PassOps* pass_ops(int p) {
    static const PassOps* (*const table[kMaxP + 1])() = {nullptr,  ops_p1,  ops_p2,  ops_p3,  ops_p4,  ops_p5,
                                                          ops_p6,  ops_p7,  ops_p8,  ops_p9,  ops_p10, ops_p11,
                                                          ops_p12, ops_p13, ops_p14, ops_p15, ops_p16};
    return (p >= 1 && p <= kMaxP) ? table[p]() : nullptr;
}

size_t launch_lds_bytes(const Geom& g, int kind) {
    if (kind == 2) return pass_lds_bytes(g.p, g.R, g.L, 2);
    return (size_t)pass_lds(g.p, g.R, g.L, g.dbuf, g.ecs, g.gf).total * sizeof(float);
}

size_t pass_lds_bytes(int PP, int R, int L, int kind) {
    if (kind == 2) return ((size_t)L * kXS + 16 * kTile) * sizeof(float);
    const int QCP = (PP * R + 15) & ~15;
    return (size_t)pass_lds(PP, R, L, 0, QCP + 1, 0).total * sizeof(float);
}

bool xb_fits(int p, int R, int L) {
    return L <= kXbMaxL && (size_t)xb_lds(p, R, L).total <= kMaxLdsBytes;
}

bool xs_fits(int p, int R, int L) {
    return L <= kXbMaxL && (size_t)xs_lds(p, R, L).total <= kMaxLdsBytes;
}

bool xas_fits(int p, int R, int L) {
    return xas_chunk(p, R) && L <= kXbMaxL && (size_t)xa_lds(p, R, L, 0).total <= kMaxLdsBytes;
}

// (above p = 12 the bf16 A-pass kernels spill registers to scratch: the
// float64 A-pass serves those)
bool xa_fits(int p, int R, int L) {
    return p <= 12 && L <= kXbMaxL && (size_t)xa_lds(p, R, L, 0).total <= kMaxLdsBytes;
}

bool runs_fit(int p, int R, int L) {
    if (!has_runs(p, R) || L > max_bands(p, R)) return false;
    for (int kind = 0; kind < 3; ++kind)
        if (pass_lds_bytes(p, R, L, kind) > kMaxLdsBytes) return false;
    return true;
}

// Default chunk size: among the compiled sizes whose kernels fit (LDS and the
// accumulators' band capacity), the one with the least padded column work
// plus a per-chunk cost of one column block for the chunk's own X stream.
int runs_per_chunk(int p, int M, int L) {
    if (M <= 1) return 1;
    int c[4] = {0, 0, 0, 0};
    const int n = run_choices(p, c);
    int best = 1;
    long best_cost = -1;
    for (int i = 0; i < n; ++i) {
        const int R = c[i];
        if (!runs_fit(p, R, L)) continue;
        const long nqc = (M + R - 1) / R, qcp = ((long)p * R + 15) & ~15L;
        const long cost = nqc * (qcp + 16);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = R;
        }
    }
    return best;
}

Geom make_geom(int L, int N, int M, int p, int R, int npg_req) {
    Geom g;
    g.L = L; g.N = N; g.M = M; g.p = p;
    g.R = R > 0 ? R : runs_per_chunk(p, M, L);
    g.QC = g.R * p;
    g.nqc = (M + g.R - 1) / g.R;
    g.Qp = g.nqc * g.QC;
    g.ntiles = (N + kTile - 1) / kTile;
    // default: one workgroup per CU over all chunks.  The pass kernels' LDS
    // holds one workgroup per CU at a time, and a second round only repeats
    // the per-workgroup set-up (measured: single runs over 94k and 314k
    // pixels 5-16% faster than with two rounds, the headline ensemble 1.4%)
    int npg = npg_req > 0 ? npg_req : kTargetWorkgroups / g.nqc;
    npg = std::max(1, std::min(npg, g.ntiles));
    g.npg = npg;
    // prefer the double-buffered X tile, then the conflict-free operand pitch
    const int QCP = (g.QC + 15) & ~15;
    auto fits = [&](int db, int ecs, int gf = 0) {
        return (size_t)pass_lds(p, g.R, L, db, ecs, gf).total * sizeof(float) <= kMaxLdsBytes;
    };
    if (fits(1, QCP + 4)) {
        g.dbuf = 1; g.ecs = QCP + 4;
    } else if (fits(1, QCP + 1)) {
        g.dbuf = 1; g.ecs = QCP + 1;
    } else if (fits(0, QCP + 4)) {
        g.dbuf = 0; g.ecs = QCP + 4;
    } else {
        g.dbuf = 0; g.ecs = QCP + 1;
    }
    g.gf = fits(g.dbuf, g.ecs, 1) ? 1 : 0;
    return g;
}

bool geom_valid(const Geom& g) { return runs_fit(g.p, g.R, g.L) && g.npg >= 1 && g.npg <= g.ntiles; }

hipError_t launch_multi(int kernel, int p, const ImageJob* jobs, const int2* map, int nblocks, size_t lds_bytes,
                        int arg, hipStream_t st) {
    if (nblocks <= 0) return hipSuccess;
    const PassOps* o = pass_ops(p);
    return o ? o->multi(kernel, jobs, map, nblocks, lds_bytes, arg, st) : hipErrorInvalidValue;
}

hipError_t launch_pad_x(const void* X, void* Xp, int L, int N, size_t ldx, int bf16, hipStream_t st) {
    const size_t n = (size_t)L * ldx;
    const int bx = (int)std::min<size_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_pad_x, dim3(bx), dim3(256), 0, st, X, Xp, L, N, ldx, bf16);
    return hipGetLastError();
}

hipError_t launch_fill(float* dst, size_t n, float value, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int bx = (int)std::min<size_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fill, dim3(bx), dim3(256), 0, st, dst, n, value);
    return hipGetLastError();
}

hipError_t launch_init_A(const Geom& g, const State& s, const float* A0, hipStream_t st) {
    const size_t n = (size_t)g.M * g.p * g.N;
    const int bx = (int)std::min<size_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_init_A, dim3(bx), dim3(256), 0, st, s.A, A0, n, 1.0f / (float)g.p);
    return hipGetLastError();
}

#define EDAA_OPS_OR_FAIL(g)                            \
    const PassOps* o = pass_ops((g).p);                \
    if (!o) return hipErrorInvalidValue;

hipError_t launch_bpass(const Geom& g, const State& s, int mode, const RunInit& ri, hipStream_t st) {
    EDAA_OPS_OR_FAIL(g);
    return o->bpass(g, s, mode, ri, st);
}
hipError_t launch_reduce_b(const Geom& g, const State& s, int need_w, hipStream_t st) {
    EDAA_OPS_OR_FAIL(g);
    return o->reduce_b(g, s, need_w, st);
}
hipError_t launch_apass(const Geom& g, const State& s, int K1, int t, hipStream_t st) {
    (void)t;
    EDAA_OPS_OR_FAIL(g);
    return o->apass(g, s, K1, st);
}
hipError_t launch_reduce_a(const Geom& g, const State& s, int t, hipStream_t st) {
    EDAA_OPS_OR_FAIL(g);
    return o->reduce_a(g, s, t, st);
}
hipError_t launch_reduce_aa(const Geom& g, const State& s, int t, hipStream_t st) {
    EDAA_OPS_OR_FAIL(g);
    return o->reduce_aa(g, s, t, st);
}
hipError_t launch_close(const Geom& g, const State& s, hipStream_t st) {
    EDAA_OPS_OR_FAIL(g);
    return o->close(g, s, st);
}
hipError_t launch_eta(const Geom& g, const State& s, const RunInit& ri, hipStream_t st) {
    EDAA_OPS_OR_FAIL(g);
    return o->eta(g, s, ri, st);
}
hipError_t launch_finalize(const Geom& g, const State& s, float* B_out, float* E_out, int coherence_mode,
                           hipStream_t st) {
    EDAA_OPS_OR_FAIL(g);
    return o->finalize(g, s, B_out, E_out, coherence_mode == 0 ? 1 : 0, st);
}
#undef EDAA_OPS_OR_FAIL

hipError_t launch_set_e(const float* E_given, const Geom& g, const State& s, hipStream_t st) {
    const int n = g.L * g.p;
    hipLaunchKernelGGL(k_set_e, dim3(std::max(1, std::min((n + 255) / 256, 1024))), dim3(256), 0, st, E_given, s.E,
                       s.Ed, g.L, g.p, g.Qp);
    return hipGetLastError();
}
hipError_t launch_set_run(uint64_t* seeds, double* gammas, uint64_t seed, double gamma, hipStream_t st) {
    hipLaunchKernelGGL(k_set_run, dim3(1), dim3(64), 0, st, seeds, gammas, seed, gamma);
    return hipGetLastError();
}
hipError_t launch_reduce_close(const Geom& g, const State& s, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_close, dim3((g.M + 255) / 256), dim3(256), 0, st, g, s);
    return hipGetLastError();
}
hipError_t launch_normalize(const float* Xin, void* Xout, int L, int N, int out_bf16, int* n_zero_dev,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_normalize, dim3((N + kThreads - 1) / kThreads), dim3(kThreads), 0, st, Xin, Xout, L, N,
                       out_bf16, n_zero_dev);
    return hipGetLastError();
}

}  // namespace edaa
