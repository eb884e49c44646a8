// HIP kernels (gfx950, wave64) for the EDAA hot path.
//
// The method (arXiv 2209.11002, Algorithm 1) alternates K1 entropic steps on
// the abundances A (eq. update_A) and K2 entropic steps on the pixel weights B
// (eq. update_B).  Written per pixel i with E = X B (L x p):
//
//   A-step:  a_i <- softmax(log a_i - eta1 (G a_i - E^T x_i)),  G = E^T E
//            (the A-subproblem separates over pixels once E is fixed, so one
//            pass over X serves all K1 steps);
//   B-step:  b_j <- softmax over all N pixels of (log b_j - eta2 X^T w_j),
//            W = E (A A^T) - X A^T, followed by E <- X B_new
//            (the new E is accumulated in the same pass over X).
//
// Every pass streams X once in tiles of 64 pixels x L bands staged in LDS; the
// tile serves both contractions of the pass (the per-pixel projection with E or
// W, and the accumulation X_tile * weights^T over the tile's pixels).  Runs of
// an ensemble are stacked along the endmember axis, R runs per workgroup
// column, so that one X tile serves every run.  Cross-workgroup sums go
// through per-workgroup partials reduced in a fixed order (deterministic); the
// column softmax over N uses per-tile shifts and an online (max, sum) merge.
#include <math.h>

#include "edaa_internal.h"

namespace edaa {
namespace {

constexpr int kPad = kTile + 1;   // LDS row stride of the X tile (no bank conflicts)

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

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

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Philox4x64-10 (Salmon et al., SC'11): 10 rounds of two 64x64->128
// multiplies with a Weyl key schedule.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += W0; k1 += W1; }
        const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
        const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}

// u[i][j] in [0,1): word j%4 of the block for counter (i, j/4, 0, 0), key
// (seed, 0), top 24 bits.
__device__ __forceinline__ float uniform_u(uint64_t seed, int i, int j) {
    uint64_t c[4] = {(uint64_t)i, (uint64_t)(j >> 2), 0ull, 0ull};
    philox4x64_10(c, seed, 0ull);
    const uint64_t w = c[j & 3];
    return (float)(uint32_t)(w >> 40) * 5.9604644775390625e-08f;   // 2^-24
}

// Workgroup -> (pixel group, chunk).  Blocks are dispatched round-robin over
// the 8 XCDs (block b runs on XCD b % 8); all chunks of one pixel group are
// placed on one XCD, at consecutive dispatch slots, so they share the X tiles
// in that XCD's L2.
__device__ __forceinline__ void wg_coords(const Geom& g, int& pg, int& c) {
    const int b = blockIdx.x;
    if ((g.npg & 7) == 0) {
        const int xcd = b & 7, k = b >> 3;
        c = k % g.nqc;
        pg = (k / g.nqc) * 8 + xcd;
    } else {
        c = b % g.nqc;
        pg = b / g.nqc;
    }
}

// Stage X[:, tile*64 : tile*64+64] in LDS as float (zero past N).
__device__ __forceinline__ void load_tile(const void* X, int x_bf16, int L, int N, int tile, float* Xs) {
    const int i = threadIdx.x & 63, r0 = threadIdx.x >> 6;
    const int pix = tile * kTile + i;
    const bool ok = pix < N;
    if (x_bf16) {
        const uint16_t* Xh = (const uint16_t*)X;
#pragma unroll 8
        for (int l = r0; l < L; l += 4) Xs[l * kPad + i] = ok ? bf16_to_f32(Xh[(size_t)l * N + pix]) : 0.f;
    } else {
        const float* Xf = (const float*)X;
#pragma unroll 8
        for (int l = r0; l < L; l += 4) Xs[l * kPad + i] = ok ? Xf[(size_t)l * N + pix] : 0.f;
    }
}

// K1 entropic steps of eq. update_A for one pixel: a <- softmax(log a -
// eta1 (G a - P)), P = E^T x.  The logarithm is carried between steps.
template <int PP>
__device__ __forceinline__ void a_steps(float (&a)[PP], const float (&P)[PP], const float* G, float eta1, int K1) {
    float la[PP];
#pragma unroll
    for (int j = 0; j < PP; ++j) la[j] = logf(a[j]);
    for (int k = 0; k < K1; ++k) {
        float v[PP];
        float mx = -INFINITY;
#pragma unroll
        for (int j = 0; j < PP; ++j) {
            float gj = -P[j];
#pragma unroll
            for (int kk = 0; kk < PP; ++kk) gj = fmaf(G[j * PP + kk], a[kk], gj);
            v[j] = fmaf(-eta1, gj, la[j]);
            mx = fmaxf(mx, v[j]);
        }
        float ssum = 0.f;
#pragma unroll
        for (int j = 0; j < PP; ++j) {
            v[j] -= mx;
            a[j] = expf(v[j]);
            ssum += a[j];
        }
        const float inv = 1.f / ssum, lsum = logf(ssum);
#pragma unroll
        for (int j = 0; j < PP; ++j) {
            a[j] *= inv;
            la[j] = v[j] - lsum;
        }
    }
}

template <int PP, int R>
struct Shape {
    static constexpr int QC = PP * R;                          // columns per chunk
    static constexpr int QCs = (QC + 3) & ~3;                  // LDS row stride of weights
    static constexpr int RW = (R == 1) ? 1 : R / 4;            // runs per wave (R > 1)
    static constexpr int AAN = R * PP * PP;                    // A A^T entries per chunk
    static constexpr int AAT = (AAN + kThreads - 1) / kThreads;
    static constexpr int CPW = (R == 1) ? (PP + 3) / 4 : RW * PP;   // softmax columns per wave
};

// Accumulate V[l][q] += sum_i Xs[l][i] * Ws[i][q] for the rows of this thread.
template <int QC, int QCs>
__device__ __forceinline__ void accumulate_rows(float (&V)[2][QC], const float* Xs, const float* Ws, int L) {
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
        const int l = threadIdx.x + rr * kThreads;
        if (l < L) {
            const float* xr = Xs + l * kPad;
            for (int i = 0; i < kTile; ++i) {
                const float x = xr[i];
                const float* wr = Ws + i * QCs;
#pragma unroll
                for (int q = 0; q < QC; ++q) V[rr][q] = fmaf(x, wr[q], V[rr][q]);
            }
        }
    }
}

// --------------------------------------------------------------------------
// A-pass: per tile, residual at the incoming (A, E) for the objective trace,
// P = E^T x, K1 A-steps, write A, accumulate X A^T and A A^T partials.
// --------------------------------------------------------------------------
template <int PP, int R>
__global__ __launch_bounds__(kThreads, 2) void k_apass(Geom g, State s, const float* __restrict__ E, int K1) {
    using S = Shape<PP, R>;
    constexpr int QC = S::QC, QCs = S::QCs, RW = S::RW, AAN = S::AAN, AAT = S::AAT;
    extern __shared__ float smem[];
    float* Xs = smem;                         // [L][kPad]
    float* As = Xs + g.L * kPad;              // [kTile][QCs]
    float* Gs = As + kTile * QCs;             // [R][PP][PP]
    float* Ps = Gs + AAN;                     // R == 1: [4][kTile][PP]
    float* Ls = Ps + 4 * kTile * PP;          // R == 1: [4][kTile]

    int pg, c;
    wg_coords(g, pg, c);
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = uniform_int(tid >> 6);
    const int L = g.L, N = g.N;
    const int col0 = c * QC;
    float* __restrict__ A = s.A;

    // Gram matrices G_m = E_m^T E_m of this chunk's runs, from the E chunk
    // staged in the (not yet used) X tile buffer.
    for (int e = tid; e < L * QC; e += kThreads) {
        const int l = e / QC, q = e % QC;
        Xs[e] = E[(size_t)l * g.Qp + col0 + q];
    }
    __syncthreads();
    for (int e = tid; e < AAN; e += kThreads) {
        const int r = e / (PP * PP), jk = e % (PP * PP), j = jk / PP, k = jk % PP;
        const float* Ec = Xs + r * PP;
        float acc = 0.f;
        for (int l = 0; l < L; ++l) acc = fmaf(Ec[l * QC + j], Ec[l * QC + k], acc);
        Gs[e] = acc;
    }

    float V[2][QC];
#pragma unroll
    for (int rr = 0; rr < 2; ++rr)
#pragma unroll
        for (int q = 0; q < QC; ++q) V[rr][q] = 0.f;
    float aa[AAT];
#pragma unroll
    for (int e = 0; e < AAT; ++e) aa[e] = 0.f;
    double lacc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) lacc[r] = 0.0;

    for (int tile = pg; tile < g.ntiles; tile += g.npg) {
        __syncthreads();
        load_tile(s.X, s.x_bf16, L, N, tile, Xs);
        const int pix = tile * kTile + lane;
        const bool pok = pix < N;
        __syncthreads();
        if constexpr (R == 1) {
            const int m = c;   // single run
            float a[PP], P[PP];
#pragma unroll
            for (int j = 0; j < PP; ++j) {
                a[j] = pok ? A[(size_t)(m * PP + j) * N + pix] : 0.f;
                P[j] = 0.f;
            }
            float ls = 0.f;
            const int Lq = (L + 3) >> 2, l0 = w * Lq, l1 = min(L, l0 + Lq);
            for (int l = l0; l < l1; ++l) {
                const float x = Xs[l * kPad + lane];
                const float* El = E + (size_t)l * g.Qp + col0;
                float r = x;
#pragma unroll
                for (int j = 0; j < PP; ++j) {
                    const float e = El[j];
                    P[j] = fmaf(e, x, P[j]);
                    r = fmaf(-e, a[j], r);
                }
                ls = fmaf(r, r, ls);
            }
#pragma unroll
            for (int j = 0; j < PP; ++j) Ps[(w * kTile + lane) * PP + j] = P[j];
            Ls[w * kTile + lane] = ls;
            __syncthreads();
            if (w == 0) {
#pragma unroll
                for (int j = 0; j < PP; ++j)
                    P[j] = Ps[lane * PP + j] + Ps[(kTile + lane) * PP + j] + Ps[(2 * kTile + lane) * PP + j] +
                           Ps[(3 * kTile + lane) * PP + j];
                const float lsum = Ls[lane] + Ls[kTile + lane] + Ls[2 * kTile + lane] + Ls[3 * kTile + lane];
                if (pok) lacc[0] += (double)lsum;
                a_steps<PP>(a, P, Gs, s.eta[2 * m], K1);
#pragma unroll
                for (int j = 0; j < PP; ++j) {
                    if (pok) A[(size_t)(m * PP + j) * N + pix] = a[j];
                    As[lane * QCs + j] = pok ? a[j] : 0.f;
                }
            }
        } else {
            float a[RW][PP], P[RW][PP], ls[RW];
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const int m = c * R + w * RW + r;
                const bool rok = pok && m < g.M;
#pragma unroll
                for (int j = 0; j < PP; ++j) {
                    a[r][j] = rok ? A[(size_t)(m * PP + j) * N + pix] : 0.f;
                    P[r][j] = 0.f;
                }
                ls[r] = 0.f;
            }
            const float* Ew = E + col0 + w * RW * PP;
            for (int l = 0; l < L; ++l) {
                const float x = Xs[l * kPad + lane];
                const float* El = Ew + (size_t)l * g.Qp;
#pragma unroll
                for (int r = 0; r < RW; ++r) {
                    float rv = x;
#pragma unroll
                    for (int j = 0; j < PP; ++j) {
                        const float e = El[r * PP + j];
                        P[r][j] = fmaf(e, x, P[r][j]);
                        rv = fmaf(-e, a[r][j], rv);
                    }
                    ls[r] = fmaf(rv, rv, ls[r]);
                }
            }
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const int m = c * R + w * RW + r;
                const bool mok = m < g.M;
                if (mok) {
                    if (pok) lacc[r] += (double)ls[r];
                    a_steps<PP>(a[r], P[r], Gs + (w * RW + r) * PP * PP, s.eta[2 * m], K1);
                }
#pragma unroll
                for (int j = 0; j < PP; ++j) {
                    if (mok && pok) A[(size_t)(m * PP + j) * N + pix] = a[r][j];
                    As[lane * QCs + (w * RW + r) * PP + j] = (mok && pok) ? a[r][j] : 0.f;
                }
            }
        }
        __syncthreads();
        accumulate_rows<QC, QCs>(V, Xs, As, L);
#pragma unroll
        for (int e = 0; e < AAT; ++e) {
            const int idx = tid + e * kThreads;
            if (idx < AAN) {
                const int r = idx / (PP * PP), jk = idx % (PP * PP), j = jk / PP, k = jk % PP;
                float acc = aa[e];
                for (int i = 0; i < kTile; ++i) acc = fmaf(As[i * QCs + r * PP + j], As[i * QCs + r * PP + k], acc);
                aa[e] = acc;
            }
        }
    }

    const size_t wgi = (size_t)pg * g.nqc + c;
    float* Vp = s.Vpart + wgi * (size_t)L * QC;
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
        const int l = tid + rr * kThreads;
        if (l < L)
#pragma unroll
            for (int q = 0; q < QC; ++q) Vp[(size_t)l * QC + q] = V[rr][q];
    }
#pragma unroll
    for (int e = 0; e < AAT; ++e) {
        const int idx = tid + e * kThreads;
        if (idx < AAN) s.AApart[wgi * AAN + idx] = aa[e];
    }
    if constexpr (R == 1) {
        if (w == 0) {
            const double tot = wave_sum(lacc[0]);
            if (lane == 0) s.lpart[(size_t)pg * g.M + c] = tot;
        }
    } else {
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int m = c * R + w * RW + r;
            const double tot = wave_sum(lacc[r]);
            if (lane == 0 && m < g.M) s.lpart[(size_t)pg * g.M + m] = tot;
        }
    }
}

// --------------------------------------------------------------------------
// B-pass: per tile, g = W^T x (STEP) and v = log b - eta2 g, or the start
// values (INIT: 0.1 u, or log B0); per-tile column max and online merge into
// the workgroup's running (max, sum); write the shifted weights and the
// tile's shift; accumulate X * weights^T.
// --------------------------------------------------------------------------
template <int PP, int R>
__global__ __launch_bounds__(kThreads, 2) void k_bpass(Geom g, State s, const float* __restrict__ W, int mode,
                                                        RunInit ri) {
    using S = Shape<PP, R>;
    constexpr int QC = S::QC, QCs = S::QCs, RW = S::RW, CPW = S::CPW;
    extern __shared__ float smem[];
    float* Xs = smem;                         // [L][kPad]
    float* Ws = Xs + g.L * kPad;              // [kTile][QCs]
    float* Fs = Ws + kTile * QCs;             // [QCs]
    float* Ps = Fs + QCs;                     // R == 1: [4][kTile][PP]

    int pg, c;
    wg_coords(g, pg, c);
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = uniform_int(tid >> 6);
    const int L = g.L, N = g.N;
    const int col0 = c * QC;

    // Columns owned by this wave for the softmax part: local column index
    // (within the chunk), run and endmember.
    int qloc[CPW], mrun_idx[CPW], jend[CPW];
    bool qok[CPW];
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
        if constexpr (R == 1) {
            const int j = w + 4 * k;
            qloc[k] = j; mrun_idx[k] = c; jend[k] = j;
            qok[k] = j < PP;
        } else {
            const int r = k / PP, j = k % PP;
            qloc[k] = (w * RW + r) * PP + j; mrun_idx[k] = c * R + w * RW + r; jend[k] = j;
            qok[k] = mrun_idx[k] < g.M;
        }
    }
    float mrun[CPW], srun[CPW], lzc[CPW], eta2[CPW];
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
        mrun[k] = -INFINITY; srun[k] = 0.f; lzc[k] = 0.f; eta2[k] = 0.f;
        if (qok[k] && mode == kModeStep) {
            const int qp = col0 + qloc[k];
            lzc[k] = -s.colm[qp] - logf(s.cols[qp]);
            eta2[k] = s.eta[2 * mrun_idx[k] + 1];
        }
    }

    float V[2][QC];
#pragma unroll
    for (int rr = 0; rr < 2; ++rr)
#pragma unroll
        for (int q = 0; q < QC; ++q) V[rr][q] = 0.f;

    for (int tile = pg; tile < g.ntiles; tile += g.npg) {
        __syncthreads();
        load_tile(s.X, s.x_bf16, L, N, tile, Xs);
        const int pix = tile * kTile + lane;
        const bool pok = pix < N;
        __syncthreads();

        float gv[CPW];
#pragma unroll
        for (int k = 0; k < CPW; ++k) gv[k] = 0.f;
        if (mode == kModeStep) {
            if constexpr (R == 1) {
                float P[PP];
#pragma unroll
                for (int j = 0; j < PP; ++j) P[j] = 0.f;
                const int Lq = (L + 3) >> 2, l0 = w * Lq, l1 = min(L, l0 + Lq);
                for (int l = l0; l < l1; ++l) {
                    const float x = Xs[l * kPad + lane];
                    const float* Wl = W + (size_t)l * g.Qp + col0;
#pragma unroll
                    for (int j = 0; j < PP; ++j) P[j] = fmaf(Wl[j], x, P[j]);
                }
#pragma unroll
                for (int j = 0; j < PP; ++j) Ps[(w * kTile + lane) * PP + j] = P[j];
                __syncthreads();
#pragma unroll
                for (int k = 0; k < CPW; ++k)
                    if (qok[k]) {
                        const int j = jend[k];
                        gv[k] = Ps[lane * PP + j] + Ps[(kTile + lane) * PP + j] + Ps[(2 * kTile + lane) * PP + j] +
                                Ps[(3 * kTile + lane) * PP + j];
                    }
            } else {
                const float* Ww = W + col0 + w * RW * PP;
                for (int l = 0; l < L; ++l) {
                    const float x = Xs[l * kPad + lane];
                    const float* Wl = Ww + (size_t)l * g.Qp;
#pragma unroll
                    for (int k = 0; k < CPW; ++k) gv[k] = fmaf(Wl[k], x, gv[k]);
                }
            }
        }

#pragma unroll
        for (int k = 0; k < CPW; ++k) {
            if (!qok[k]) {
                if constexpr (R != 1) {
                    Ws[lane * QCs + qloc[k]] = 0.f;
                    if (lane == 0) Fs[qloc[k]] = 0.f;
                }
                continue;
            }
            const int m = mrun_idx[k], j = jend[k], q = m * PP + j, qp = col0 + qloc[k];
            float v = -INFINITY;
            if (pok) {
                if (mode == kModeStep) {
                    const float b = s.Bst[(size_t)q * N + pix];
                    v = logf(b) + (s.tshift[(size_t)tile * g.Qp + qp] + lzc[k]) - eta2[k] * gv[k];
                } else if (mode == kModeInitRng) {
                    v = ri.init_scale * uniform_u(ri.seeds[m], pix, j);
                } else {
                    v = logf(ri.B0[(size_t)pix * PP + j]);
                }
            }
            const float mt = wave_max(v);
            const float mnew = fmaxf(mrun[k], mt);
            const float f = (mrun[k] == -INFINITY) ? 0.f : expf(mrun[k] - mnew);
            const float wv = (v == -INFINITY) ? 0.f : expf(v - mnew);
            srun[k] = srun[k] * f + wave_sum(wv);
            mrun[k] = mnew;
            if (pok) s.Bst[(size_t)q * N + pix] = wv;
            if (lane == 0) {
                s.tshift[(size_t)tile * g.Qp + qp] = mnew;
                Fs[qloc[k]] = f;
            }
            Ws[lane * QCs + qloc[k]] = wv;
        }
        __syncthreads();
        // rescale the running accumulation to the new shifts, then add the tile
#pragma unroll
        for (int rr = 0; rr < 2; ++rr)
#pragma unroll
            for (int q = 0; q < QC; ++q) V[rr][q] *= Fs[q];
        accumulate_rows<QC, QCs>(V, Xs, Ws, L);
    }

    const size_t wgi = (size_t)pg * g.nqc + c;
    float* Vp = s.Vpart + wgi * (size_t)L * QC;
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
        const int l = tid + rr * kThreads;
        if (l < L)
#pragma unroll
            for (int q = 0; q < QC; ++q) Vp[(size_t)l * QC + q] = V[rr][q];
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < CPW; ++k) {
            if (!qok[k] && R == 1) continue;
            const int qp = col0 + qloc[k];
            s.mpart[(size_t)pg * g.Qp + qp] = qok[k] ? mrun[k] : -INFINITY;
            s.spart[(size_t)pg * g.Qp + qp] = qok[k] ? srun[k] : 0.f;
        }
    }
}

// --------------------------------------------------------------------------
// Closing pass: objective and l1 fit of every run at the final (A, E).
// --------------------------------------------------------------------------
template <int PP, int R>
__global__ __launch_bounds__(kThreads, 2) void k_close(Geom g, State s, const float* __restrict__ E) {
    using S = Shape<PP, R>;
    constexpr int QC = S::QC, RW = S::RW;
    extern __shared__ float smem[];
    float* Xs = smem;                 // [L][kPad]
    float* Ls = Xs + g.L * kPad;      // R == 1: [2][4][kTile]

    int pg, c;
    wg_coords(g, pg, c);
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = uniform_int(tid >> 6);
    const int L = g.L, N = g.N, col0 = c * QC;
    double lacc[RW], facc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) lacc[r] = facc[r] = 0.0;

    for (int tile = pg; tile < g.ntiles; tile += g.npg) {
        __syncthreads();
        load_tile(s.X, s.x_bf16, L, N, tile, Xs);
        const int pix = tile * kTile + lane;
        const bool pok = pix < N;
        __syncthreads();
        if constexpr (R == 1) {
            const int m = c;
            float a[PP];
#pragma unroll
            for (int j = 0; j < PP; ++j) a[j] = pok ? s.A[(size_t)(m * PP + j) * N + pix] : 0.f;
            float ls = 0.f, fs = 0.f;
            const int Lq = (L + 3) >> 2, l0 = w * Lq, l1 = min(L, l0 + Lq);
            for (int l = l0; l < l1; ++l) {
                const float* El = E + (size_t)l * g.Qp + col0;
                float r = Xs[l * kPad + lane];
#pragma unroll
                for (int j = 0; j < PP; ++j) r = fmaf(-El[j], a[j], r);
                ls = fmaf(r, r, ls);
                fs += fabsf(r);
            }
            Ls[w * kTile + lane] = ls;
            Ls[(4 + w) * kTile + lane] = fs;
            __syncthreads();
            if (w == 0 && pok) {
                lacc[0] += (double)(Ls[lane] + Ls[kTile + lane] + Ls[2 * kTile + lane] + Ls[3 * kTile + lane]);
                facc[0] += (double)(Ls[4 * kTile + lane] + Ls[5 * kTile + lane] + Ls[6 * kTile + lane] +
                                    Ls[7 * kTile + lane]);
            }
        } else {
            float a[RW][PP], ls[RW], fs[RW];
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const int m = c * R + w * RW + r;
                const bool rok = pok && m < g.M;
#pragma unroll
                for (int j = 0; j < PP; ++j) a[r][j] = rok ? s.A[(size_t)(m * PP + j) * N + pix] : 0.f;
                ls[r] = fs[r] = 0.f;
            }
            const float* Ew = E + col0 + w * RW * PP;
            for (int l = 0; l < L; ++l) {
                const float x = Xs[l * kPad + lane];
                const float* El = Ew + (size_t)l * g.Qp;
#pragma unroll
                for (int r = 0; r < RW; ++r) {
                    float rv = x;
#pragma unroll
                    for (int j = 0; j < PP; ++j) rv = fmaf(-El[r * PP + j], a[r][j], rv);
                    ls[r] = fmaf(rv, rv, ls[r]);
                    fs[r] += fabsf(rv);
                }
            }
            if (pok)
#pragma unroll
                for (int r = 0; r < RW; ++r) {
                    lacc[r] += (double)ls[r];
                    facc[r] += (double)fs[r];
                }
        }
    }
    if constexpr (R == 1) {
        if (w == 0) {
            const double lt = wave_sum(lacc[0]), ft = wave_sum(facc[0]);
            if (lane == 0) {
                s.lpart[(size_t)pg * g.M + c] = lt;
                s.fpart[(size_t)pg * g.M + c] = ft;
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int m = c * R + w * RW + r;
            const double lt = wave_sum(lacc[r]), ft = wave_sum(facc[r]);
            if (lane == 0 && m < g.M) {
                s.lpart[(size_t)pg * g.M + m] = lt;
                s.fpart[(size_t)pg * g.M + m] = ft;
            }
        }
    }
}

// --------------------------------------------------------------------------
// Reductions of the per-workgroup partials, in a fixed order.  Grid:
// (row blocks, chunks); a workgroup owns whole rows of its chunk.
// --------------------------------------------------------------------------
// The cross-workgroup sums, E and W = E (A A^T) - X A^T are formed in float64:
// E A A^T and X A^T are both of order N/p while W is of the order of the
// residual, so forming the difference in float32 would lose most digits.
template <int PP, int R>
__global__ __launch_bounds__(kThreads) void k_reduce_b(Geom g, State s, int need_w) {
    constexpr int QC = PP * R;
    constexpr int ROWS = kThreads / QC;
    constexpr int FCH = 64;                        // partial groups per factor chunk
    __shared__ float Ms[QC];
    __shared__ double Ss[QC];
    __shared__ float Fac[FCH][QC];
    __shared__ double Es[ROWS][QC];
    const int rb = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
    const int col0 = c * QC, L = g.L;

    for (int q = tid; q < QC; q += kThreads) {
        const int m = c * R + q / PP;
        float mx = -INFINITY;
        for (int pg = 0; pg < g.npg; ++pg) mx = fmaxf(mx, s.mpart[(size_t)pg * g.Qp + col0 + q]);
        double sm = 0.0;
        if (mx != -INFINITY)
            for (int pg = 0; pg < g.npg; ++pg) {
                const float mp = s.mpart[(size_t)pg * g.Qp + col0 + q];
                if (mp != -INFINITY) sm += (double)s.spart[(size_t)pg * g.Qp + col0 + q] * (double)expf(mp - mx);
            }
        Ms[q] = mx;
        Ss[q] = sm;
        if (rb == 0 && m < g.M) {
            s.colm[col0 + q] = mx;
            s.cols[col0 + q] = (float)sm;
        }
    }
    const int lr = tid / QC, q = tid % QC;
    const int l = rb * ROWS + lr;
    const bool act = tid < ROWS * QC && l < L;
    const int m = c * R + q / PP;
    double acc = 0.0;
    for (int pb = 0; pb < g.npg; pb += FCH) {
        __syncthreads();
        for (int e = tid; e < FCH * QC; e += kThreads) {
            const int pp = e / QC, qq = e % QC, pg = pb + pp;
            float f = 0.f;
            if (pg < g.npg) {
                const float mp = s.mpart[(size_t)pg * g.Qp + col0 + qq];
                f = (mp == -INFINITY) ? 0.f : expf(mp - Ms[qq]);
            }
            Fac[pp][qq] = f;
        }
        __syncthreads();
        if (act) {
            const int pe = min(FCH, g.npg - pb);
            for (int pp = 0; pp < pe; ++pp)
                acc += (double)s.Vpart[(((size_t)(pb + pp) * g.nqc + c) * L + l) * QC + q] * (double)Fac[pp][q];
        }
    }
    double e = 0.0;
    if (act && m < g.M) e = acc / Ss[q];
    if (act) {
        s.E[(size_t)l * g.Qp + col0 + q] = (float)e;
        s.Ed[(size_t)l * g.Qp + col0 + q] = e;
        Es[lr][q] = e;
    }
    __syncthreads();
    if (need_w && act) {
        double wv = 0.0;
        if (m < g.M) {
            const int ml = q / PP, j = q % PP;
            wv = -s.XAtd[(size_t)l * g.Qp + col0 + q];
            const double* aat = s.AAtd + (size_t)m * PP * PP;
#pragma unroll
            for (int k = 0; k < PP; ++k) wv = fma(Es[lr][ml * PP + k], aat[k * PP + j], wv);
        }
        s.W[(size_t)l * g.Qp + col0 + q] = (float)wv;
    }
}

template <int PP, int R>
__global__ __launch_bounds__(kThreads) void k_reduce_a(Geom g, State s, int t) {
    constexpr int QC = PP * R;
    constexpr int ROWS = kThreads / QC;
    constexpr int AAN = R * PP * PP;
    __shared__ double AAs[AAN];
    const int rb = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
    const int col0 = c * QC, L = g.L;

    for (int e = tid; e < AAN; e += kThreads) {
        double acc = 0.0;
        for (int pg = 0; pg < g.npg; ++pg) acc += (double)s.AApart[((size_t)pg * g.nqc + c) * AAN + e];
        AAs[e] = acc;
        const int m = c * R + e / (PP * PP);
        if (rb == 0 && m < g.M) s.AAtd[(size_t)m * PP * PP + e % (PP * PP)] = acc;
    }
    if (rb == 0 && tid < R) {
        const int m = c * R + tid;
        if (m < g.M) {
            double acc = 0.0;
            for (int pg = 0; pg < g.npg; ++pg) acc += s.lpart[(size_t)pg * g.M + m];
            s.trace[(size_t)m * (s.T + 1) + t] = 0.5 * acc;
        }
    }
    __syncthreads();
    const int lr = tid / QC, q = tid % QC;
    const int l = rb * ROWS + lr;
    if (tid < ROWS * QC && l < L) {
        const int m = c * R + q / PP, ml = q / PP, j = q % PP;
        double xa = 0.0;
        for (int pg = 0; pg < g.npg; ++pg) xa += (double)s.Vpart[(((size_t)pg * g.nqc + c) * L + l) * QC + q];
        double wv = 0.0;
        if (m < g.M) {
            wv = -xa;
            const double* El = s.Ed + (size_t)l * g.Qp + col0 + ml * PP;
#pragma unroll
            for (int k = 0; k < PP; ++k) wv = fma(El[k], AAs[ml * PP * PP + k * PP + j], wv);
        } else {
            xa = 0.0;
        }
        s.XAtd[(size_t)l * g.Qp + col0 + q] = xa;
        s.W[(size_t)l * g.Qp + col0 + q] = (float)wv;
    }
}

__global__ void k_reduce_close(Geom g, State s) {
    for (int m = threadIdx.x + blockIdx.x * blockDim.x; m < g.M; m += blockDim.x * gridDim.x) {
        double la = 0.0, fa = 0.0;
        for (int pg = 0; pg < g.npg; ++pg) {
            la += s.lpart[(size_t)pg * g.M + m];
            fa += s.fpart[(size_t)pg * g.M + m];
        }
        s.trace[(size_t)m * (s.T + 1) + s.T] = 0.5 * la;
        s.fit[m] = fa;
    }
}

// --------------------------------------------------------------------------
// Step sizes (eq. eta0A, eq. eta0B): sigma_max^2(X B0) is the largest
// eigenvalue of the p x p Gram matrix E0^T E0, found by cyclic Jacobi
// rotations in float64 by one thread per run.
// --------------------------------------------------------------------------
__device__ double jacobi_max_eig(double* a, int n) {
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int i = 0; i < n; ++i) {
            dia += a[i * n + i] * a[i * n + i];
            for (int j = i + 1; j < n; ++j) off += a[i * n + j] * a[i * n + j];
        }
        if (off <= 1e-32 * dia || off == 0.0) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[p * n + q];
                if (apq == 0.0) continue;
                const double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < n; ++k) {
                    const double akp = a[k * n + p], akq = a[k * n + q];
                    a[k * n + p] = cs * akp - sn * akq;
                    a[k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = a[p * n + k], aqk = a[q * n + k];
                    a[p * n + k] = cs * apk - sn * aqk;
                    a[q * n + k] = sn * apk + cs * aqk;
                }
            }
    }
    double mx = a[0];
    for (int i = 1; i < n; ++i) mx = fmax(mx, a[i * n + i]);
    return mx;
}

template <int PP>
__global__ __launch_bounds__(kThreads) void k_eta(Geom g, State s, RunInit ri) {
    __shared__ double Gd[PP * PP];
    const int m = blockIdx.x, tid = threadIdx.x;
    const int c = m / g.R, col0 = c * g.QC + (m % g.R) * PP;
    for (int e = tid; e < PP * PP; e += kThreads) {
        const int j = e / PP, k = e % PP;
        double acc = 0.0;
        for (int l = 0; l < g.L; ++l)
            acc += s.Ed[(size_t)l * g.Qp + col0 + j] * s.Ed[(size_t)l * g.Qp + col0 + k];
        Gd[e] = acc;
    }
    __syncthreads();
    if (tid == 0) {
        const double lam = jacobi_max_eig(Gd, PP);
        const double e1 = ri.eta1 > 0.0 ? ri.eta1 : ri.gammas[m] / lam;
        const double e2 = ri.eta2 > 0.0 ? ri.eta2 : sqrt((double)PP / (double)g.N) * e1;
        s.eta[2 * m] = (float)e1;
        s.eta[2 * m + 1] = (float)e2;
        s.etad[2 * m] = e1;
        s.etad[2 * m + 1] = e2;
    }
}

// --------------------------------------------------------------------------
// Outputs: normalised B in [M][N][p], E in [M][L][p], coherence per run.
// --------------------------------------------------------------------------
template <int PP>
__global__ __launch_bounds__(kThreads) void k_final_B(Geom g, State s, float* B_out) {
    const int m = blockIdx.y;
    const size_t n = (size_t)g.N * PP;
    const int c = m / g.R, base = c * g.QC + (m % g.R) * PP;
    for (size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += (size_t)gridDim.x * kThreads) {
        const int pix = (int)(e / PP), j = (int)(e % PP);
        const int qp = base + j, tile = pix / kTile;
        const float b = s.Bst[(size_t)(m * PP + j) * g.N + pix];
        B_out[(size_t)m * n + e] = b * expf(s.tshift[(size_t)tile * g.Qp + qp] - s.colm[qp] - logf(s.cols[qp]));
    }
}

template <int PP>
__global__ __launch_bounds__(kThreads) void k_final_E(Geom g, State s, float* E_out, int cosine) {
    __shared__ double Gd[PP * PP];
    const int m = blockIdx.x, tid = threadIdx.x;
    const int c = m / g.R, base = c * g.QC + (m % g.R) * PP;
    if (E_out)
        for (int e = tid; e < g.L * PP; e += kThreads) {
            const int l = e / PP, j = e % PP;
            E_out[(size_t)m * g.L * PP + e] = s.E[(size_t)l * g.Qp + base + j];
        }
    for (int e = tid; e < PP * PP; e += kThreads) {
        const int j = e / PP, k = e % PP;
        double acc = 0.0;
        for (int l = 0; l < g.L; ++l)
            acc += s.Ed[(size_t)l * g.Qp + base + j] * s.Ed[(size_t)l * g.Qp + base + k];
        Gd[e] = acc;
    }
    __syncthreads();
    if (tid == 0) {
        double mu = -INFINITY;
        for (int j = 0; j < PP; ++j)
            for (int k = 0; k < PP; ++k) {
                if (j == k) continue;
                double v = Gd[j * PP + k];
                if (cosine) {
                    const double nj = sqrt(Gd[j * PP + j]), nk = sqrt(Gd[k * PP + k]);
                    v = v / ((nj > 0.0 ? nj : 1.0) * (nk > 0.0 ? nk : 1.0));
                }
                mu = fmax(mu, v);
            }
        s.mu[m] = mu;
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

// --------------------------------------------------------------------------
// Host-side dispatch over the (p, runs-per-chunk) instantiations.
// --------------------------------------------------------------------------
}  // namespace

size_t pass_lds_bytes(int PP, int R, int L, int kind) {
    const int QC = PP * R, QCs = (QC + 3) & ~3;
    size_t b = (size_t)L * kPad;
    // the [4][kTile][PP] band-split scratch exists only in the single-run kernels
    const size_t split = (R == 1) ? (size_t)4 * kTile * PP : 0;
    if (kind == 0) b += (size_t)kTile * QCs + (size_t)R * PP * PP + split + (R == 1 ? 4 * kTile : 0);   // A-pass
    if (kind == 1) b += (size_t)kTile * QCs + QCs + split;                                            // B-pass
    if (kind == 2) b += (size_t)8 * kTile;                                                            // close
    return b * sizeof(float);
}

namespace {

template <int PP, int R>
struct Kernels {
    static hipError_t apass(const Geom& g, const State& s, int K1, hipStream_t st) {
        const size_t lds = pass_lds_bytes(PP, R, g.L, 0);
        set_max_lds((const void*)k_apass<PP, R>, (int)lds);
        hipLaunchKernelGGL((k_apass<PP, R>), dim3(g.npg * g.nqc), dim3(kThreads), lds, st, g, s, (const float*)s.E, K1);
        return hipGetLastError();
    }
    static hipError_t bpass(const Geom& g, const State& s, int mode, const RunInit& ri, hipStream_t st) {
        const size_t lds = pass_lds_bytes(PP, R, g.L, 1);
        set_max_lds((const void*)k_bpass<PP, R>, (int)lds);
        hipLaunchKernelGGL((k_bpass<PP, R>), dim3(g.npg * g.nqc), dim3(kThreads), lds, st, g, s, (const float*)s.W, mode,
                           ri);
        return hipGetLastError();
    }
    static hipError_t close(const Geom& g, const State& s, hipStream_t st) {
        const size_t lds = pass_lds_bytes(PP, R, g.L, 2);
        set_max_lds((const void*)k_close<PP, R>, (int)lds);
        hipLaunchKernelGGL((k_close<PP, R>), dim3(g.npg * g.nqc), dim3(kThreads), lds, st, g, s, (const float*)s.E);
        return hipGetLastError();
    }
    static hipError_t reduce_b(const Geom& g, const State& s, int need_w, hipStream_t st) {
        constexpr int ROWS = kThreads / (PP * R);
        hipLaunchKernelGGL((k_reduce_b<PP, R>), dim3((g.L + ROWS - 1) / ROWS, g.nqc), dim3(kThreads), 0, st, g, s,
                           need_w);
        return hipGetLastError();
    }
    static hipError_t reduce_a(const Geom& g, const State& s, int t, hipStream_t st) {
        constexpr int ROWS = kThreads / (PP * R);
        hipLaunchKernelGGL((k_reduce_a<PP, R>), dim3((g.L + ROWS - 1) / ROWS, g.nqc), dim3(kThreads), 0, st, g, s, t);
        return hipGetLastError();
    }
};

template <int PP>
struct PKernels {
    static hipError_t eta(const Geom& g, const State& s, const RunInit& ri, hipStream_t st) {
        hipLaunchKernelGGL((k_eta<PP>), dim3(g.M), dim3(kThreads), 0, st, g, s, ri);
        return hipGetLastError();
    }
    static hipError_t final_(const Geom& g, const State& s, float* B_out, float* E_out, int cosine, hipStream_t st) {
        const size_t n = (size_t)g.N * PP;
        const int bx = (int)std::min<size_t>((n + kThreads - 1) / kThreads, 4096);
        if (B_out) hipLaunchKernelGGL((k_final_B<PP>), dim3(bx, g.M), dim3(kThreads), 0, st, g, s, B_out);
        hipLaunchKernelGGL((k_final_E<PP>), dim3(g.M), dim3(kThreads), 0, st, g, s, E_out, cosine);
        return hipGetLastError();
    }
};

constexpr int rmax_for(int PP) { return PP > 5 ? (PP > 8 ? 4 : 8) : (PP == 5 ? 12 : (PP == 4 ? 16 : 20)); }

// Dispatch (p, R) -> instantiation.  R is 1, 4 or rmax_for(p).

#define EDAA_CASE_P(PPV)                                                                    \
    case PPV:                                                                               \
        if (R == 1) return Op<PPV, 1>::run(args...);                                        \
        if (R == 4) return Op<PPV, 4>::run(args...);                                        \
        if (R == rmax_for(PPV) && rmax_for(PPV) != 4) return Op<PPV, rmax_for(PPV)>::run(args...); \
        break;

#define EDAA_DISPATCH_BODY                                                                  \
    switch (p) {                                                                            \
        EDAA_CASE_P(1) EDAA_CASE_P(2) EDAA_CASE_P(3) EDAA_CASE_P(4) EDAA_CASE_P(5)          \
        EDAA_CASE_P(6) EDAA_CASE_P(7) EDAA_CASE_P(8) EDAA_CASE_P(9) EDAA_CASE_P(10)         \
        EDAA_CASE_P(11) EDAA_CASE_P(12) EDAA_CASE_P(13) EDAA_CASE_P(14) EDAA_CASE_P(15)     \
        EDAA_CASE_P(16)                                                                     \
        default: break;                                                                     \
    }                                                                                       \
    return hipErrorInvalidValue;

template <int PP, int R> struct ApassOp { static hipError_t run(const Geom& g, const State& s, int K1, hipStream_t st) { return Kernels<PP, R>::apass(g, s, K1, st); } };
template <int PP, int R> struct BpassOp { static hipError_t run(const Geom& g, const State& s, int mode, const RunInit& ri, hipStream_t st) { return Kernels<PP, R>::bpass(g, s, mode, ri, st); } };
template <int PP, int R> struct CloseOp { static hipError_t run(const Geom& g, const State& s, hipStream_t st) { return Kernels<PP, R>::close(g, s, st); } };
template <int PP, int R> struct RedBOp { static hipError_t run(const Geom& g, const State& s, int need_w, hipStream_t st) { return Kernels<PP, R>::reduce_b(g, s, need_w, st); } };
template <int PP, int R> struct RedAOp { static hipError_t run(const Geom& g, const State& s, int t, hipStream_t st) { return Kernels<PP, R>::reduce_a(g, s, t, st); } };

template <template <int, int> class Op, typename... Args>
hipError_t run_pr(int p, int R, Args... args) { EDAA_DISPATCH_BODY }

template <template <int> class Op, typename... Args>
hipError_t run_p(int p, Args... args) {
    switch (p) {
#define EDAA_CASE_PONLY(PPV) case PPV: return Op<PPV>::run(args...);
        EDAA_CASE_PONLY(1) EDAA_CASE_PONLY(2) EDAA_CASE_PONLY(3) EDAA_CASE_PONLY(4)
        EDAA_CASE_PONLY(5) EDAA_CASE_PONLY(6) EDAA_CASE_PONLY(7) EDAA_CASE_PONLY(8)
        EDAA_CASE_PONLY(9) EDAA_CASE_PONLY(10) EDAA_CASE_PONLY(11) EDAA_CASE_PONLY(12)
        EDAA_CASE_PONLY(13) EDAA_CASE_PONLY(14) EDAA_CASE_PONLY(15) EDAA_CASE_PONLY(16)
#undef EDAA_CASE_PONLY
        default: break;
    }
    return hipErrorInvalidValue;
}

template <int PP> struct EtaOp { static hipError_t run(const Geom& g, const State& s, const RunInit& ri, hipStream_t st) { return PKernels<PP>::eta(g, s, ri, st); } };
template <int PP> struct FinalOp { static hipError_t run(const Geom& g, const State& s, float* Bo, float* Eo, int cos, hipStream_t st) { return PKernels<PP>::final_(g, s, Bo, Eo, cos, st); } };

}  // namespace

int runs_per_chunk(int p, int M) {
    if (M <= 1) return 1;
    if (M <= 4) return 4;
    return rmax_for(p);
}

Geom make_geom(int L, int N, int M, int p) {
    Geom g;
    g.L = L; g.N = N; g.M = M; g.p = p;
    g.R = runs_per_chunk(p, M);
    g.QC = g.R * p;
    g.nqc = (M + g.R - 1) / g.R;
    g.Qp = g.nqc * g.QC;
    g.ntiles = (N + kTile - 1) / kTile;
    int npg = kTargetWorkgroups / g.nqc;
    if (npg >= 8) npg &= ~7;
    npg = std::max(1, std::min(npg, g.ntiles));
    g.npg = npg;
    return g;
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

hipError_t launch_bpass(const Geom& g, const State& s, int mode, const RunInit& ri, hipStream_t st) {
    return run_pr<BpassOp>(g.p, g.R, g, s, mode, ri, st);
}
hipError_t launch_reduce_b(const Geom& g, const State& s, int need_w, hipStream_t st) {
    return run_pr<RedBOp>(g.p, g.R, g, s, need_w, st);
}
hipError_t launch_apass(const Geom& g, const State& s, int K1, int t, hipStream_t st) {
    (void)t;
    return run_pr<ApassOp>(g.p, g.R, g, s, K1, st);
}
hipError_t launch_reduce_a(const Geom& g, const State& s, int t, hipStream_t st) {
    return run_pr<RedAOp>(g.p, g.R, g, s, t, st);
}
hipError_t launch_close(const Geom& g, const State& s, hipStream_t st) {
    return run_pr<CloseOp>(g.p, g.R, g, s, st);
}
hipError_t launch_reduce_close(const Geom& g, const State& s, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_close, dim3((g.M + 255) / 256), dim3(256), 0, st, g, s);
    return hipGetLastError();
}
hipError_t launch_eta(const Geom& g, const State& s, const RunInit& ri, hipStream_t st) {
    return run_p<EtaOp>(g.p, g, s, ri, st);
}
hipError_t launch_finalize(const Geom& g, const State& s, float* B_out, float* E_out, int coherence_mode,
                           hipStream_t st) {
    return run_p<FinalOp>(g.p, g, s, B_out, E_out, coherence_mode == 0 ? 1 : 0, st);
}
hipError_t launch_normalize(const float* Xin, void* Xout, int L, int N, int out_bf16, int* n_zero_dev,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_normalize, dim3((N + kThreads - 1) / kThreads), dim3(kThreads), 0, st, Xin, Xout, L, N,
                       out_bf16, n_zero_dev);
    return hipGetLastError();
}

}  // namespace edaa
