// HIP kernels for the modular (autograd) path of EDAA (float32 inputs and
// outputs, float64 arithmetic inside):
//   loss  f(A, B) = 1/2 ||X - X B A||_F^2            (eq. AA)
//   dA    = (X B)^T (X B A - X)  = G A - E^T X        (E = X B, G = E^T E)
//   dB    = X^T (X B A - X) A^T  = X^T W,  W = E (A A^T) - X A^T
//   mirror steps of eq. update_softmax on the columns of A (over p) and of B
//   (over all N pixels).
// X is [L][N] float32, A [p][N], B [N][p].  The pixel axis is split over
// workgroups; cross-workgroup sums are per-workgroup partials reduced in a
// fixed order.
#include <math.h>

#include "edaa_internal.h"

namespace edaa {
namespace {

constexpr int kPad = kTile + 1;

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Cross-pixel sums, per workgroup, in float64:
//   MODE 0:  V[l][j] = sum_i X[l][i] B[i][j]                       (E = X B)
//   MODE 1:  V[l][j] = sum_i (X[l][i] - sum_k E[l][k] A[k][i]) A[j][i]   (R A^T)
template <int PP, int MODE>
__global__ __launch_bounds__(kThreads) void k_xw(const float* __restrict__ X, const float* __restrict__ Wt,
                                                 const double* __restrict__ Ed, int L, int N,
                                                 double* __restrict__ Vpart) {
    extern __shared__ float smem[];
    float* Xs = smem;                  // [L][kPad]
    float* Ws = Xs + L * kPad;         // [kTile][PP]
    const int tid = threadIdx.x, lane = tid & 63, r0 = tid >> 6;
    const int ntiles = (N + kTile - 1) / kTile;
    double V[2][PP], Er[2][PP];
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
        const int l = tid + rr * kThreads;
#pragma unroll
        for (int j = 0; j < PP; ++j) {
            V[rr][j] = 0.0;
            Er[rr][j] = (MODE == 1 && l < L) ? Ed[l * PP + j] : 0.0;
        }
    }
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        __syncthreads();
        const int pix = tile * kTile + lane;
        const bool ok = pix < N;
        for (int l = r0; l < L; l += 4) Xs[l * kPad + lane] = ok ? X[(size_t)l * N + pix] : 0.f;
        if (r0 == 0)
#pragma unroll
            for (int j = 0; j < PP; ++j)
                Ws[lane * PP + j] = ok ? (MODE == 0 ? Wt[(size_t)pix * PP + j] : Wt[(size_t)j * N + pix]) : 0.f;
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            const int l = tid + rr * kThreads;
            if (l < L)
                for (int i = 0; i < kTile; ++i) {
                    double v = (double)Xs[l * kPad + i];
                    if (MODE == 1) {
#pragma unroll
                        for (int k = 0; k < PP; ++k) v = fma(-Er[rr][k], (double)Ws[i * PP + k], v);
                    }
#pragma unroll
                    for (int j = 0; j < PP; ++j) V[rr][j] = fma(v, (double)Ws[i * PP + j], V[rr][j]);
                }
        }
    }
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
        const int l = tid + rr * kThreads;
        if (l < L)
#pragma unroll
            for (int j = 0; j < PP; ++j) Vpart[((size_t)blockIdx.x * L + l) * PP + j] = V[rr][j];
    }
}

// out[e] = sign * sum_b part[b][e] for e < n (fixed order); out32 optional.
__global__ void k_sum_parts(const double* __restrict__ part, int nblk, int n, double sign, double* __restrict__ out,
                            float* __restrict__ out32) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += part[(size_t)b * n + e];
    acc *= sign;
    out[e] = acc;
    if (out32) out32[e] = (float)acc;
}

// Per-pixel residual ||x_i - E a_i||^2 in float64, summed per block.
template <int PP>
__global__ __launch_bounds__(kThreads) void k_resid(const float* __restrict__ X, const double* __restrict__ E,
                                                    const float* __restrict__ A, int L, int N,
                                                    double* __restrict__ lpart) {
    __shared__ double red[kThreads / 64];
    double acc = 0.0;
    for (int pix = blockIdx.x * kThreads + threadIdx.x; pix < N; pix += gridDim.x * kThreads) {
        double a[PP];
#pragma unroll
        for (int j = 0; j < PP; ++j) a[j] = (double)A[(size_t)j * N + pix];
        for (int l = 0; l < L; ++l) {
            double r = (double)X[(size_t)l * N + pix];
#pragma unroll
            for (int j = 0; j < PP; ++j) r = fma(-E[l * PP + j], a[j], r);
            acc = fma(r, r, acc);
        }
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) lpart[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_loss_final(const double* __restrict__ lpart, int nblk, float* __restrict__ loss) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double acc = 0.0;
        for (int b = 0; b < nblk; ++b) acc += lpart[b];
        *loss = (float)(0.5 * acc);
    }
}

// gA[:, i] = go * E^T (E a_i - x_i), from the per-band residual, in float64.
template <int PP>
__global__ __launch_bounds__(kThreads) void k_grad_a(const float* __restrict__ X, const double* __restrict__ E,
                                                     const float* __restrict__ A, int L, int N,
                                                     const float* __restrict__ go, float* __restrict__ gA) {
    const double s = (double)*go;
    for (int pix = blockIdx.x * kThreads + threadIdx.x; pix < N; pix += gridDim.x * kThreads) {
        double a[PP], g[PP];
#pragma unroll
        for (int j = 0; j < PP; ++j) {
            a[j] = (double)A[(size_t)j * N + pix];
            g[j] = 0.0;
        }
        for (int l = 0; l < L; ++l) {
            double r = -(double)X[(size_t)l * N + pix];
#pragma unroll
            for (int j = 0; j < PP; ++j) r = fma(E[l * PP + j], a[j], r);
#pragma unroll
            for (int j = 0; j < PP; ++j) g[j] = fma(E[l * PP + j], r, g[j]);
        }
#pragma unroll
        for (int j = 0; j < PP; ++j) gA[(size_t)j * N + pix] = (float)(s * g[j]);
    }
}

// gB[i][:] = go * W^T x_i with W = (X B A - X) A^T, in float64.
template <int PP>
__global__ __launch_bounds__(kThreads) void k_grad_b(const float* __restrict__ X, const double* __restrict__ W,
                                                     int L, int N, const float* __restrict__ go,
                                                     float* __restrict__ gB) {
    const double s = (double)*go;
    for (int pix = blockIdx.x * kThreads + threadIdx.x; pix < N; pix += gridDim.x * kThreads) {
        double g[PP];
#pragma unroll
        for (int j = 0; j < PP; ++j) g[j] = 0.0;
        for (int l = 0; l < L; ++l) {
            const double x = (double)X[(size_t)l * N + pix];
#pragma unroll
            for (int j = 0; j < PP; ++j) g[j] = fma(W[l * PP + j], x, g[j]);
        }
#pragma unroll
        for (int j = 0; j < PP; ++j) gB[(size_t)pix * PP + j] = (float)(s * g[j]);
    }
}

// Mirror step on the columns of A (over the p entries of each pixel).
__global__ __launch_bounds__(kThreads) void k_mirror_a(float* __restrict__ A, const float* __restrict__ gA, int p,
                                                       int N, float eta) {
    const int pix = blockIdx.x * kThreads + threadIdx.x;
    if (pix >= N) return;
    float v[kMaxP];
    float mx = -INFINITY;
    for (int j = 0; j < p; ++j) {
        v[j] = logf(A[(size_t)j * N + pix]) - eta * gA[(size_t)j * N + pix];
        mx = fmaxf(mx, v[j]);
    }
    float s = 0.f;
    for (int j = 0; j < p; ++j) {
        v[j] = expf(v[j] - mx);
        s += v[j];
    }
    const float inv = 1.f / s;
    for (int j = 0; j < p; ++j) A[(size_t)j * N + pix] = v[j] * inv;
}

// Mirror step on the columns of B (over all N pixels), pass 1: per-block
// column (max, sum exp) of v = log b - eta g with an online merge.
__global__ __launch_bounds__(kThreads) void k_mirror_b1(const float* __restrict__ B, const float* __restrict__ gB,
                                                        int N, int p, float eta, float* __restrict__ cm,
                                                        float* __restrict__ cs) {
    __shared__ float sm[kThreads / 64], ss[kThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int j = 0; j < p; ++j) {
        float m = -INFINITY, s = 0.f;
        for (int pix = blockIdx.x * kThreads + threadIdx.x; pix < N; pix += gridDim.x * kThreads) {
            const float v = logf(B[(size_t)pix * p + j]) - eta * gB[(size_t)pix * p + j];
            if (v == -INFINITY) continue;
            if (v > m) {
                s = s * expf(m - v) + 1.f;
                m = v;
            } else {
                s += expf(v - m);
            }
        }
        const float wm = wave_max(m);
        const float sc = (m == -INFINITY) ? 0.f : s * expf(m - wm);
        const float wsum = wave_sum(sc);
        if (lane == 0) {
            sm[w] = wm;
            ss[w] = wsum;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            float bm = -INFINITY;
            for (int k = 0; k < kThreads / 64; ++k) bm = fmaxf(bm, sm[k]);
            float bs = 0.f;
            for (int k = 0; k < kThreads / 64; ++k)
                if (sm[k] != -INFINITY) bs += ss[k] * expf(sm[k] - bm);
            cm[(size_t)blockIdx.x * p + j] = bm;
            cs[(size_t)blockIdx.x * p + j] = bs;
        }
        __syncthreads();
    }
}

__global__ void k_mirror_b2(const float* __restrict__ cm, const float* __restrict__ cs, int nblk, int p,
                            float* __restrict__ colstat) {
    const int j = threadIdx.x;
    if (j >= p) return;
    float m = -INFINITY;
    for (int b = 0; b < nblk; ++b) m = fmaxf(m, cm[(size_t)b * p + j]);
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) {
        const float bm = cm[(size_t)b * p + j];
        if (bm != -INFINITY) s += cs[(size_t)b * p + j] * expf(bm - m);
    }
    colstat[j] = m;
    colstat[p + j] = logf(s);
}

__global__ __launch_bounds__(kThreads) void k_mirror_b3(float* __restrict__ B, const float* __restrict__ gB, int N,
                                                        int p, float eta, const float* __restrict__ colstat) {
    const size_t n = (size_t)N * p;
    for (size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += (size_t)gridDim.x * kThreads) {
        const int j = (int)(e % p);
        const float v = logf(B[e]) - eta * gB[e];
        B[e] = (v == -INFINITY) ? 0.f : expf(v - colstat[j] - colstat[p + j]);
    }
}

template <int PP>
struct GradOps {
    static hipError_t make_e(const float* X, const float* B, int L, int N, const GradWork& w, hipStream_t st) {
        const size_t lds = ((size_t)L * kPad + (size_t)kTile * PP) * sizeof(float);
        set_max_lds((const void*)k_xw<PP, 0>, (int)lds);
        hipLaunchKernelGGL((k_xw<PP, 0>), dim3(w.nblk), dim3(kThreads), lds, st, X, B, (const double*)nullptr, L, N,
                           w.Vpart);
        const int n = L * PP;
        hipLaunchKernelGGL(k_sum_parts, dim3((n + 255) / 256), dim3(256), 0, st, (const double*)w.Vpart, w.nblk, n,
                           1.0, w.Ed, w.E);
        return hipGetLastError();
    }
    static hipError_t fwd(const float* X, const float* A, const float* B, int L, int N, const GradWork& w,
                          float* loss, hipStream_t st) {
        hipError_t e = make_e(X, B, L, N, w, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_resid<PP>), dim3(w.nblk), dim3(kThreads), 0, st, X, (const double*)w.Ed, A, L, N,
                           w.lpart);
        hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, st, w.lpart, w.nblk, loss);
        return hipGetLastError();
    }
    static hipError_t bwd(const float* X, const float* A, const float* B, int L, int N, const float* go,
                          const GradWork& w, float* gA, float* gB, hipStream_t st) {
        hipError_t e = make_e(X, B, L, N, w, st);
        if (e != hipSuccess) return e;
        if (gA)
            hipLaunchKernelGGL((k_grad_a<PP>), dim3(w.nblk), dim3(kThreads), 0, st, X, (const double*)w.Ed, A, L, N,
                               go, gA);
        if (gB) {
            const size_t lds = ((size_t)L * kPad + (size_t)kTile * PP) * sizeof(float);
            set_max_lds((const void*)k_xw<PP, 1>, (int)lds);
            hipLaunchKernelGGL((k_xw<PP, 1>), dim3(w.nblk), dim3(kThreads), lds, st, X, A, (const double*)w.Ed, L,
                               N, w.Vpart);
            const int n = L * PP;
            // W = E A A^T - X A^T = -(X - E A) A^T
            hipLaunchKernelGGL(k_sum_parts, dim3((n + 255) / 256), dim3(256), 0, st, (const double*)w.Vpart,
                               w.nblk, n, -1.0, w.Wd, (float*)nullptr);
            hipLaunchKernelGGL((k_grad_b<PP>), dim3(w.nblk), dim3(kThreads), 0, st, X, (const double*)w.Wd, L, N,
                               go, gB);
        }
        return hipGetLastError();
    }
};

template <template <int> class Op, typename F>
hipError_t with_p(int p, F&& f) {
    switch (p) {
#define EDAA_GCASE(PPV) case PPV: return f(Op<PPV>());
        EDAA_GCASE(1) EDAA_GCASE(2) EDAA_GCASE(3) EDAA_GCASE(4) EDAA_GCASE(5) EDAA_GCASE(6) EDAA_GCASE(7)
        EDAA_GCASE(8) EDAA_GCASE(9) EDAA_GCASE(10) EDAA_GCASE(11) EDAA_GCASE(12) EDAA_GCASE(13) EDAA_GCASE(14)
        EDAA_GCASE(15) EDAA_GCASE(16)
#undef EDAA_GCASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int grad_blocks(int N) {
    const int ntiles = (N + kTile - 1) / kTile;
    return std::max(1, std::min(ntiles, 512));
}

hipError_t launch_loss_fwd(const float* X, const float* A, const float* B, int L, int N, int p, const GradWork& w,
                           float* loss_dev, hipStream_t st) {
    return with_p<GradOps>(p, [&](auto op) { return decltype(op)::fwd(X, A, B, L, N, w, loss_dev, st); });
}

hipError_t launch_loss_bwd(const float* X, const float* A, const float* B, int L, int N, int p,
                           const float* grad_out, const GradWork& w, float* gA, float* gB, hipStream_t st) {
    return with_p<GradOps>(p, [&](auto op) { return decltype(op)::bwd(X, A, B, L, N, grad_out, w, gA, gB, st); });
}

hipError_t launch_mirror_A(float* A, const float* gA, int p, int N, float eta, hipStream_t st) {
    hipLaunchKernelGGL(k_mirror_a, dim3((N + kThreads - 1) / kThreads), dim3(kThreads), 0, st, A, gA, p, N, eta);
    return hipGetLastError();
}

hipError_t launch_mirror_B(float* B, const float* gB, int N, int p, float eta, const GradWork& w, hipStream_t st) {
    const int nblk = w.nblk;
    hipLaunchKernelGGL(k_mirror_b1, dim3(nblk), dim3(kThreads), 0, st, B, gB, N, p, eta, w.cm, w.cs);
    hipLaunchKernelGGL(k_mirror_b2, dim3(1), dim3(64), 0, st, w.cm, w.cs, nblk, p, w.colstat);
    const size_t n = (size_t)N * p;
    const int bx = (int)std::min<size_t>((n + kThreads - 1) / kThreads, 8192);
    hipLaunchKernelGGL(k_mirror_b3, dim3(bx), dim3(kThreads), 0, st, B, gB, N, p, eta, w.colstat);
    return hipGetLastError();
}

}  // namespace edaa
