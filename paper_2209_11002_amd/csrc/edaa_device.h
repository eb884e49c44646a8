// Device code of the EDAA pass kernels (gfx950, wave64), shared by the
// per-p instantiation units (edaa_inst.hip, compiled once per p) and the
// common unit (edaa_kernels.hip).
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
// Every pass streams X once in tiles of 64 pixels x L bands staged in LDS.  A
// tile serves both contractions of the pass:
//   * the per-pixel projection S = U^T X_tile (U = E or W, L x QC), and
//   * the accumulation V += X_tile Wt over the tile's 64 pixels (Wt = the
//     tile's new abundances or B weights, 64 x QC), which is a dense GEMM run
//     on the matrix cores (v_mfma_f32_16x16x4f32, float32 in and out).
// Runs of an ensemble are stacked along the endmember axis, R runs per
// workgroup column (a "chunk" of QC = R p columns), so one X tile serves every
// run of the chunk.  Both contractions run on 16-column MFMA blocks for every
// R (with R = 1 the chunk is one run's p columns, padded to 16).
// Cross-workgroup sums go through per-workgroup partials reduced in a fixed
// order (deterministic); the column softmax over N uses per-tile shifts and an
// online (max, sum) merge.
#pragma once

#include <math.h>

#include <type_traits>

#include "edaa_internal.h"
namespace edaa {
namespace {

// Waves per workgroup of the B-step pass (the A-pass and the closing pass
// use kThreads / 64 = 4).  With 8, each SIMD runs two waves of the
// workgroup, so one wave's LDS waits overlap the other's matrix
// instructions, and each wave issues half as many direct-to-LDS loads
// (their issue, about 55 clocks each, stalls the issuing wave); both waves
// share the one LDS allocation.
constexpr int kBpassWaves = 8;
// Waves per workgroup of the A-step pass: eight up to p = 9; above, the
// per-pixel A-steps (p x p products on p-vectors in registers) need more
// than the 256 registers a wave has at two waves per SIMD.
constexpr int apass_waves(int p) { return p <= 9 ? 8 : 4; }
// The A-pass on the bf16 matrix cores (bf16 X) takes the same wave counts.
// (Eight waves at p = 10..12, with the A-steps of a (run, pixel) over 2 or 4
// lanes reading their Gram rows from LDS, measured no faster: the A-steps
// there are bound by vector-ALU throughput, not latency.)
constexpr int xa_waves(int p) { return apass_waves(p); }
// Chunks whose float32-X A-pass runs on the bf16 matrix cores (k_apass_xs):
// up to p = 6 and three column blocks; the others need more than the 256
// registers a wave has at eight waves per workgroup (the float32 tile staged
// in registers takes 32) and keep the float64/float32 A-pass.
constexpr bool xas_chunk(int p, int R) { return p <= 6 && (p * R + 15) / 16 <= 3; }
constexpr int kXS = 68;   // LDS pitch (floats) of an X tile row of 64 pixels

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

// D(16x16) += A(16x4) B(4x16).  Lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; D[4 (l / 16) + v][l % 16] is element v of its float4.
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// The same shape in float64 (v_mfma_f64_16x16x4f64): same A and B lane
// layout, but element v of lane l's double4 is D[4 v + l / 16][l % 16].
__device__ __forceinline__ d4 mfma16d(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// The bf16 shape D(16x16) += A(16x32) B(32x16) (v_mfma_f32_16x16x32_bf16,
// float32 accumulation).  Lane l holds eight k of row l % 16 of A and the same
// eight k of column l % 16 of B, as 8 bf16 in 16 bytes (k = 8 (l / 16) + j
// for element j; the sum over k does not depend on that assignment as long as
// both operands use it); D as for mfma16.
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ f4 mfma16_bf16(u32x4 a, u32x4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                    0, 0, 0);
}

// x = hi + mid + lo with three bf16 terms (round to nearest at each step).
// Three 8-bit significands hold float32's 24, so the sum is exact for every
// x whose last term is a normal bf16 (|x| above about 1e-30), and a product
// of an exact bf16 value with each term is exact in float32.
__device__ __forceinline__ void split_bf16x3(const float (&x)[8], u32x4& hi, u32x4& mid, u32x4& lo) {
    bf16x8 h, m, l;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const __bf16 a = (__bf16)x[j];
        const float r = x[j] - (float)a;
        const __bf16 b = (__bf16)r;
        h[j] = a;
        m[j] = b;
        l[j] = (__bf16)(r - (float)b);
    }
    hi = __builtin_bit_cast(u32x4, h);
    mid = __builtin_bit_cast(u32x4, m);
    lo = __builtin_bit_cast(u32x4, l);
}

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

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

// A DPP lane permutation within rows of 16 lanes (all rows and banks
// enabled); the B-step softmax uses the quad permutes 0xB1 (lane ^ 1) and
// 0x4E (lane ^ 2), and the half-row mirror 0x141 (lane i <-> 7 - i within
// 8 lanes).
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Workgroup barrier for LDS traffic: waits for this wave's LDS operations
// only.  __syncthreads() would also wait for every outstanding global load,
// store and direct-to-LDS load (its release fence), which would stall the
// prefetch of the next tile at every barrier; the pass kernels wait for
// those explicitly where their data is used.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// e^x and ln x from the hardware base-2 instructions (v_exp_f32, v_log_f32).
__device__ __forceinline__ float fast_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ __forceinline__ float fast_log(float x) { return __builtin_amdgcn_logf(x) * 0.6931471805599453f; }

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
// the 8 XCDs (block b runs on XCD b % 8).  XCD x takes a contiguous range of
// the (pixel group, chunk) pairs in pixel-group-major order, so the chunks of
// a pixel group run on one XCD (at most one pixel group per XCD boundary is
// split over two) and share the X tiles in that XCD's L2, whatever the
// number of pixel groups.  A single chunk keeps pg = b.
__device__ __forceinline__ void wg_coords(const Geom& g, int b, int& pg, int& c) {
    if (g.nqc == 1) {
        pg = b;
        c = 0;
        return;
    }
    const int total = g.npg * g.nqc, x = b & 7;
    int off = 0;                                   // pairs of the XCDs before x
    for (int y = 0; y < x; ++y) off += (total - y + 7) >> 3;
    const int i = off + (b >> 3);
    pg = i / g.nqc;
    c = i - pg * g.nqc;
}

// X tile staging.  X here is the library's padded copy, [L][ldx] with
// ldx = ntiles * 64 and zero pixels past N, so every tile is whole and
// aligned.  Three ways to put X[:, tile*64 : +64] into rows [0, L) of an LDS
// tile (pitch kXS):
//  - dma_tile (float32 X): direct global->LDS loads, one 64-pixel row per
//    instruction, issued one tile ahead (measured faster than the register
//    staging below for float32);
//  - XRegs (bf16 X): register staging; wave w loads the row groups
//    4w + 16i .. +3, each lane 4 consecutive pixels of one row (8 B) per
//    instruction, one tile ahead, and store() widens them to float and
//    writes 16 B per lane to LDS once the loads have landed;
//  - load_tile_sync: synchronous loads through registers (bf16 kernels
//    without room for the staging registers, and the closing pass).
constexpr int kRegXGroups = 16;     // row groups of 4 rows per wave at 4 waves: L <= 4 * 4 * 16 = 256

// ON = false compiles to nothing (kernels without room for the registers).
template <bool ON, int NW = 4>
struct XRegs {
    static constexpr int NG = kRegXGroups * 4 / NW;   // row groups per wave
    uint2 v[NG];                                 // 4 bf16 per lane and row group

    __device__ __forceinline__ void issue(const void* X, size_t ldx, int L, int tile) {
        const int lane = threadIdx.x & 63, w = uniform_int(threadIdx.x >> 6);
        const int rsub = lane >> 4, col = 4 * (lane & 15);
#pragma unroll
        for (int i = 0; i < NG; ++i) {
            const int row = 4 * NW * i + 4 * w + rsub;
            if (4 * NW * i + 4 * w < L) {                  // uniform per wave
                const size_t off = (size_t)min(row, L - 1) * ldx + (size_t)tile * kTile + col;
                v[i] = *(const uint2*)((const uint16_t*)X + off);
            }
        }
    }
    __device__ __forceinline__ void store(float* Xs, int L) const {
        const int lane = threadIdx.x & 63, w = uniform_int(threadIdx.x >> 6);
        const int rsub = lane >> 4, col = 4 * (lane & 15);
#pragma unroll
        for (int i = 0; i < NG; ++i) {
            const int row = 4 * NW * i + 4 * w + rsub;
            if (4 * NW * i + 4 * w < L && row < L)
                *(f4*)(Xs + row * kXS + col) =
                    f4{__uint_as_float(v[i].x << 16), __uint_as_float(v[i].x & 0xffff0000u),
                       __uint_as_float(v[i].y << 16), __uint_as_float(v[i].y & 0xffff0000u)};
        }
    }
};
template <int NW>
struct XRegs<false, NW> {
    __device__ __forceinline__ void issue(const void*, size_t, int, int) {}
    __device__ __forceinline__ void store(float*, int) const {}
};

// Rows l = wd, wd + NWD, ... are loaded by wave wd of a group of NWD waves.
template <int NWD = 4>
__device__ __forceinline__ void dma_tile(const float* X, size_t ldx, int L, int tile, float* Xs, int wd) {
    const int lane = threadIdx.x & 63;
    const float* src = X + (size_t)tile * kTile + lane;
    for (int l = wd; l < L; l += NWD) __builtin_amdgcn_global_load_lds(src + (size_t)l * ldx, Xs + l * kXS, 4, 0, 0);
}

__device__ __forceinline__ void load_tile_sync(const void* X, int x_bf16, int L, size_t ldx, int tile, float* Xs) {
    const int i = threadIdx.x & 63, r0 = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const size_t pc = (size_t)tile * kTile + i;
    constexpr int B = 16;
    for (int l0 = r0; l0 < L; l0 += nw * B) {
        float v[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const size_t off = (size_t)min(l0 + nw * b, L - 1) * ldx + pc;
            v[b] = x_bf16 ? bf16_to_f32(((const uint16_t*)X)[off]) : ((const float*)X)[off];
        }
#pragma unroll
        for (int b = 0; b < B; ++b)
            if (l0 + nw * b < L) Xs[(l0 + nw * b) * kXS + i] = v[b];
    }
}

// Whether a pass kernel has room for the staging registers (compile time);
// at run time L must also fit the row groups.
template <int PP, int R, bool APASS>
constexpr bool kRegX = PP * R <= 48 && (!APASS || PP <= 12);
constexpr int kRegXMaxL = 4 * 4 * kRegXGroups;

// K1 entropic steps of eq. update_A for one pixel: a <- softmax(log a -
// eta1 (G a - P)), P = E^T x.  The logarithm is carried between steps.
template <int PP, typename GT>
__device__ __forceinline__ void a_steps(float (&a)[PP], const float (&P)[PP], const GT* G, float eta1, int K1) {
    float la[PP];
#pragma unroll
    for (int j = 0; j < PP; ++j) la[j] = fast_log(a[j]);
    for (int k = 0; k < K1; ++k) {
        float v[PP];
        float mx = -INFINITY;
#pragma unroll
        for (int j = 0; j < PP; ++j) {
            float gj = -P[j];
#pragma unroll
            for (int kk = 0; kk < PP; ++kk) gj = fmaf((float)G[j * PP + kk], a[kk], gj);
            v[j] = fmaf(-eta1, gj, la[j]);
            mx = fmaxf(mx, v[j]);
        }
        float ssum = 0.f;
#pragma unroll
        for (int j = 0; j < PP; ++j) {
            v[j] -= mx;
            a[j] = fast_exp(v[j]);
            ssum += a[j];
        }
        const float inv = 1.f / ssum, lsum = fast_log(ssum);
#pragma unroll
        for (int j = 0; j < PP; ++j) {
            a[j] *= inv;
            la[j] = v[j] - lsum;
        }
    }
}

// Sum, maximum and broadcast over the S consecutive lanes (S = 2 or 4) that
// share one pixel, with quad DPP permutes.  The XOR butterflies leave every
// lane of the group with the same value (each stage adds the same two
// operands in either lane).
template <int S>
__device__ __forceinline__ float group_sum(float v) {
    v += dpp<0xB1>(v);                              // lane ^ 1
    if (S == 4) v += dpp<0x4E>(v);                  // lane ^ 2
    return v;
}
template <int S>
__device__ __forceinline__ float group_max(float v) {
    v = fmaxf(v, dpp<0xB1>(v));
    if (S == 4) v = fmaxf(v, dpp<0x4E>(v));
    return v;
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int S>
__device__ __forceinline__ double group_sum(double v) {
    v += dpp_d<0xB1>(v);
    if (S == 4) v += dpp_d<0x4E>(v);
    return v;
}
// Value of sub-lane K of this lane's group of S.
template <int S, int K>
__device__ __forceinline__ float group_bcast(float v) {
    constexpr int c = (S == 4) ? (K | K << 2 | K << 4 | K << 6) : (K | K << 2 | (2 + K) << 4 | (2 + K) << 6);
    return dpp<c>(v);
}

// a[j] = ao[j / S] of sub-lane j % S, for the sub-lanes K, K + 1, ... < S.
template <int PP, int S, int K>
__device__ __forceinline__ void gather_rows(float (&a)[PP], const float (&ao)[(PP + S - 1) / S]) {
    if constexpr (K < S) {
#pragma unroll
        for (int jj = 0; jj < (PP + S - 1) / S; ++jj)
            if (S * jj + K < PP) a[S * jj + K] = group_bcast<S, K>(ao[jj]);
        gather_rows<PP, S, K + 1>(a, ao);
    }
}

// K1 entropic steps of eq. update_A for one pixel whose p rows are spread
// over S consecutive lanes (S = 2 or 4): sub-lane `sub` owns rows
// j = sub + S jj.  Every lane keeps the whole abundance vector `a` (for G a)
// and, for its own rows, the entries `ao`, their logarithms and the rows of
// G (`Gr`) and of P = E^T x (`Po`).  The softmax maximum and sum are
// combined over the S lanes; after each step every entry is broadcast from
// its owner.
template <int PP, int S>
__device__ __forceinline__ void a_steps_split(float (&a)[PP], float (&ao)[(PP + S - 1) / S],
                                              const float (&Po)[(PP + S - 1) / S],
                                              const float (&Gr)[(PP + S - 1) / S][PP], float eta1, int K1, int sub) {
    static_assert(S == 2 || S == 4, "two or four lanes per pixel");
    constexpr int JW = (PP + S - 1) / S;
    float la[JW];
#pragma unroll
    for (int jj = 0; jj < JW; ++jj) la[jj] = fast_log(ao[jj]);
    for (int k = 0; k < K1; ++k) {
        float v[JW];
        float mx = -INFINITY;
#pragma unroll
        for (int jj = 0; jj < JW; ++jj) {
            float gj = -Po[jj];
#pragma unroll
            for (int kk = 0; kk < PP; ++kk) gj = fmaf(Gr[jj][kk], a[kk], gj);
            v[jj] = fmaf(-eta1, gj, la[jj]);
            if (sub + S * jj < PP) mx = fmaxf(mx, v[jj]);
        }
        mx = group_max<S>(mx);
        float ssum = 0.f;
#pragma unroll
        for (int jj = 0; jj < JW; ++jj) {
            v[jj] -= mx;
            ao[jj] = (sub + S * jj < PP) ? fast_exp(v[jj]) : 0.f;
            ssum += ao[jj];
        }
        ssum = group_sum<S>(ssum);
        const float inv = 1.f / ssum, lsum = fast_log(ssum);
#pragma unroll
        for (int jj = 0; jj < JW; ++jj) {
            ao[jj] *= inv;
            la[jj] = v[jj] - lsum;
        }
        gather_rows<PP, S, 0>(a, ao);
    }
}


template <int PP, int R>
struct Shape {
    static constexpr int QC = PP * R;                   // columns per chunk
    static constexpr int QCP = (QC + 15) & ~15;         // padded to MFMA blocks of 16
    static constexpr int NCB = QCP / 16;                // column blocks
    static constexpr int WTS = QCP + 1;                 // LDS pitch of the per-pixel weight rows
    // accumulation row blocks of 16 bands per wave at four waves (the
    // accumulators are NRBW x NCB float64 blocks per wave; see
    // acc_row_blocks); a kernel with NW waves takes 4/NW of it
    static constexpr int NRBW = acc_row_blocks(PP, R);
    static constexpr int NGB = 2 * NCB - 1;             // Gram blocks (qb, qb) and (qb, qb+1)
};

// LDS layout of a pass kernel, in floats.  LP = L rounded up to 16.
struct PassLds {
    int xs, wt, f, fg, ec, gs, gf, xx, pd, xs2, total;
};
// dbuf: a second X tile buffer, so that the next tile loads while the
// current one is processed.
// ecs: LDS pitch of the staged projection operand (QCP + 4 avoids bank
// conflicts in the projections; QCP + 1 where LDS is short).
// gf: room for a float copy of the Gram matrices (A-steps).
__host__ __device__ inline PassLds pass_lds(int PP, int R, int L, int dbuf, int ecs, int gf) {
    const int QC = PP * R, QCP = (QC + 15) & ~15, WTS = QCP + 1, ECS = ecs;
    const int LP = (L + 15) & ~15;
    PassLds o;
    o.xs = 0;
    o.wt = o.xs + LP * kXS;                    // [64][WTS] or [QCP][kXS] weights / projection results
    o.f = o.wt + (kTile * WTS > QCP * kXS ? kTile * WTS : QCP * kXS);   // [QCP] rescale factors
    o.fg = o.f + QCP;                          // [QCP] factors of the tile's weights
    o.ec = o.fg + QCP;                         // [LP][ECS] projection operand chunk (E or W)
    o.gs = o.ec + LP * ECS;                    // [R][PP][PP] Gram matrices (double, 2 floats each)
    o.gs = (o.gs + 1) & ~1;
    o.gf = o.gs + 2 * R * PP * PP;             // [R][PP][PP] the same Gram matrices in float (A-steps)
    o.xx = (o.gf + (gf ? R * PP * PP : 0) + 1) & ~1;   // [64] squared pixel norms (double, 2 floats each)
    o.pd = o.xx + 2 * kTile;                   // [64][WTS] low part of the A-pass projection
    o.xs2 = o.pd + kTile * WTS;
    o.total = o.xs2 + (dbuf ? LP * kXS : 0);
    return o;
}

// LDS layout (bytes) of the B-pass on the bf16 matrix cores (bpass_xb_body),
// with LP32 = L rounded up to 32 (the k depth of one MFMA):
//   xn   [LP32][kXNP] bf16   X tile, pixels contiguous (rows >= L zero)
//   xo   [LP32/8][64][8] bf16  X tile, 8 consecutive bands of a pixel contiguous
//   wsp  [LP32/32][NCB][3][64] 16-byte MFMA operands of W (three bf16 terms)
//   wb   [2][NCB][3][64]       16-byte MFMA operands of the tile's weights
//   sq   [QCP][kXS] float      projection W^T x (sq2: second band half, NCB = 1)
//   f, fg [QCP] float          rescale factors
constexpr int kXNP = 72;   // bf16 per xn row: 64 pixels + 8, so 16 rows start on 16 distinct bank groups
struct XbLds {
    int xn, xo, wsp, wb, sq, sq2, f, fg, total;
};
__host__ __device__ inline XbLds xb_lds(int PP, int R, int L) {
    const int QCP = (PP * R + 15) & ~15, NCB = QCP / 16, LP32 = (L + 31) & ~31;
    XbLds o;
    o.xn = 0;
    o.xo = o.xn + LP32 * kXNP * 2;
    o.wsp = o.xo + LP32 * 64 * 2;
    o.wb = o.wsp + (LP32 / 32) * NCB * 3 * 1024;
    o.sq = o.wb + 2 * NCB * 3 * 1024;
    o.sq2 = o.sq + QCP * kXS * 4;
    o.f = o.sq2 + (NCB == 1 ? 16 * kXS * 4 : 0);
    o.fg = o.f + QCP * 4;
    o.total = o.fg + QCP * 4;
    return o;
}
// Bands the bf16 matrix-core passes stage: eight blocks of 32.
constexpr int kXbMaxL = 32 * 8;

// Bank swizzles of the bf16 passes' 16-byte LDS operands (64 banks of 4
// bytes: 16 slots of 16 bytes per bank cycle).  xo: pixel i of an 8-band row
// sits in slot i with its two low bits XORed with bits 4-5, so the writes of
// 16 lanes (pixels 4m + e, m = 0..15) hit 16 distinct slots while the
// projection's reads (16 consecutive pixels) stay a permutation of 16 slots.
// Weight operands: lane l = 16 kg + m of pixel block pb sits in slot 16 kg +
// ((m + 2 kg + 8 pb) & 15), so the softmax's writes (8 lanes of a column: kg
// and pb vary, m fixed) spread over 16 slots.
__device__ __forceinline__ int xo_slot(int px) { return (px & ~3) | ((px ^ (px >> 4)) & 3); }
__device__ __forceinline__ int wb_slot(int kg, int m, int pb) { return 16 * kg + ((m + 2 * kg + 8 * pb) & 15); }

// LDS layout (bytes) of the A-pass on the bf16 matrix cores (apass_xb_body):
//   xn, xo  the X tile as for the B-pass
//   esp  [LP32/32][NCB][3][64] 16-byte MFMA operands of E (three bf16 terms)
//   wt   [64][WTS] float      projection P (high part), then the new abundances
//   plo  [64][WTS] float      low part of P; once the A-steps have read it, the
//                             [2][NCB][3][64] MFMA operands of the abundances
//   gs   [R][PP][PP] double   Gram matrices (gf: [R][PP][PP] float copy)
//   xx   [64] double          squared pixel norms
struct XaLds {
    int xn, xo, esp, wt, plo, gs, gf, xx, total;
};
__host__ __device__ inline XaLds xa_lds(int PP, int R, int L, int gf) {
    const int QCP = (PP * R + 15) & ~15, NCB = QCP / 16, WTS = QCP + 1, LP32 = (L + 31) & ~31;
    const int wt_bytes = kTile * WTS * 4, op_bytes = 2 * NCB * 3 * 1024;
    XaLds o;
    o.xn = 0;
    o.xo = o.xn + LP32 * kXNP * 2;
    o.esp = o.xo + LP32 * 64 * 2;
    o.wt = o.esp + (LP32 / 32) * NCB * 3 * 1024;
    o.plo = o.wt + wt_bytes;
    o.gs = o.plo + (wt_bytes > op_bytes ? wt_bytes : op_bytes);
    o.gf = o.gs + R * PP * PP * 8;
    o.xx = (o.gf + (gf ? R * PP * PP * 4 : 0) + 7) & ~7;
    o.total = o.xx + kTile * 8;
    return o;
}

// LDS layout (bytes) of the B-pass for float32 X on the bf16 matrix cores
// (bpass_xs_body), LP32 = L rounded up to 32:
//   xf   [LP32][kXS] float       X tile, pixels contiguous (rows >= L zero)
//   wsp  [LP32/32][NCB][3][64]   16-byte MFMA operands of W (three bf16 terms),
//                                bands in the order of xs_band
//   wb   [2][NCB][3][64]         16-byte MFMA operands of the tile's weights
//   sq   [QCP][kXS] float        projection W^T x (the k blocks of waves 0-3)
//   sq2  [QCP][kXS] float        the k blocks of waves 4-7 (ksplit only)
//   f, fg [QCP] float            rescale factors
// ksplit: the two wave groups take alternate k blocks of every column block
// (each X operand is split once); without it (more than three column blocks,
// or no room for sq2) they take halves of the column blocks.
struct XsLds {
    int xf, wsp, wb, sq, sq2, f, fg, total, ksplit;
};
__host__ __device__ inline XsLds xs_lds(int PP, int R, int L) {
    const int QCP = (PP * R + 15) & ~15, NCB = QCP / 16, LP32 = (L + 31) & ~31;
    XsLds o;
    o.xf = 0;
    o.wsp = o.xf + LP32 * kXS * 4;
    o.wb = o.wsp + (LP32 / 32) * NCB * 3 * 1024;
    o.sq = o.wb + 2 * NCB * 3 * 1024;
    o.sq2 = o.sq + QCP * kXS * 4;
    o.ksplit = NCB <= 3 && o.sq2 + QCP * kXS * 4 + 2 * QCP * 4 <= 160 * 1024;
    if (NCB == 1) o.ksplit = 1;       // one column block: the second group has no other share
    o.f = o.sq2 + (o.ksplit ? QCP * kXS * 4 : 0);
    o.fg = o.f + QCP * 4;
    o.total = o.fg + QCP * 4;
    return o;
}

// Band of element j of the 8 a lane of k group kg holds in the float32-X
// projection (within a block of 32): 4 kg + (j & 3) + 16 (j >> 2), so that
// the eight single-float reads of the 64 lanes (rows 4 kg + c at pitch kXS,
// 16 consecutive pixels) fall on 64 distinct banks.  W's operands use the
// same order.
__device__ __forceinline__ int xs_band(int kg, int j) { return 4 * kg + (j & 3) + 16 * (j >> 2); }

// Two float32 values as three packed bf16 terms each (element 0 in the low
// half): hi = rn(x), mid = rn(x - hi), lo = rn(x - hi - mid), with exact
// differences, so hi + mid + lo == x for |x| above about 1e-30.
__device__ __forceinline__ unsigned pack_bf16(float a, float b) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(unsigned, __builtin_convertvector(f2{a, b}, bf16x2));
}
__device__ __forceinline__ void split2_bf16x3(float x0, float x1, unsigned& h, unsigned& m, unsigned& l) {
    h = pack_bf16(x0, x1);
    const float r0 = x0 - __builtin_bit_cast(float, h << 16);
    const float r1 = x1 - __builtin_bit_cast(float, h & 0xffff0000u);
    m = pack_bf16(r0, r1);
    const float s0 = r0 - __builtin_bit_cast(float, m << 16);
    const float s1 = r1 - __builtin_bit_cast(float, m & 0xffff0000u);
    l = pack_bf16(s0, s1);
}
__device__ __forceinline__ void split8_bf16x3(const float (&x)[8], u32x4 (&t)[3]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        unsigned h, m, l;
        split2_bf16x3(x[2 * i], x[2 * i + 1], h, m, l);
        t[0][i] = h;
        t[1][i] = m;
        t[2][i] = l;
    }
}

// Scheduling pattern for a block of NMFMA matrix instructions and the LDS
// reads of the next block's operands: the reads go, up to four at a time,
// between the first four MFMAs, so they complete while the later MFMAs of
// the block run instead of stalling the next block.
template <int NMFMA>
__device__ __forceinline__ void interleave_loads() {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);   // up to four LDS reads
    }
    if (NMFMA > 4) __builtin_amdgcn_sched_group_barrier(0x008, NMFMA - 4, 0);
}

// V += X_tile Wt on the matrix cores: each tile's 64-pixel sums are formed
// in float32 by the MFMAs and folded into float64 running sums, so that the
// partial of a workgroup carries no error that grows with its tile count
// (W = E A A^T - X A^T cancels and would amplify it).  Wave w owns the row blocks
// rb = w + NW j (16 bands each) and every column block; with SCALE the
// running accumulation of column q is first multiplied by F[q].  The B
// operands (Wt, 64 x QCP) are loaded once per tile and reused for every row
// block; the optional Gram accumulation Wt^T Wt reuses them as well.
// QMAJOR: the weights are stored column-major, Wt[q * kXS + pixel].
// With SCALE the running sums of column q are first multiplied by F[q] and
// the tile's sums by G[q].
template <int NCB, int NRBW, int WTS, bool SCALE, int NGBW, bool QMAJOR = false, int NW = 4>
__device__ __forceinline__ void mfma_accumulate(d4 (&acc)[NRBW][NCB], d4 (&gram)[NGBW], bool do_gram,
                                                const float* Xs, const float* Wt, const float* F, const float* G,
                                                int nrb, int w, int lane) {
    const int m = lane & 15, kk = lane >> 4;
    float bop[16][NCB];
#pragma unroll
    for (int k = 0; k < 16; ++k)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
            bop[k][cb] = QMAJOR ? Wt[(16 * cb + m) * kXS + 4 * k + kk] : Wt[(4 * k + kk) * WTS + 16 * cb + m];
    // the X operands of the next row block are read while the MFMAs of the
    // current one run (rows past the last block re-read the last one)
    float xa[16];
    {
        const float* xr = Xs + (16 * min(w, nrb - 1) + m) * kXS + kk;
#pragma unroll
        for (int k = 0; k < 16; ++k) xa[k] = xr[4 * k];
    }
    float fs[NCB], gs[NCB];
    if (SCALE) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            fs[cb] = F[16 * cb + m];
            gs[cb] = G[16 * cb + m];
        }
    }
#pragma unroll
    for (int j = 0; j < NRBW; ++j) {
        const int rb = w + NW * j;
        if (rb < nrb) {
            f4 t[NCB], t2[NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) t[cb] = t2[cb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 16; ++k) {
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    // a single column block alternates two chains (independent MFMAs)
                    if (NCB == 1 && (k & 1))
                        t2[cb] = mfma16(xa[k], bop[k][cb], t2[cb]);
                    else
                        t[cb] = mfma16(xa[k], bop[k][cb], t[cb]);
                }
            }
            if (NCB == 1) {
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) t[cb] += t2[cb];
            }
            float xn[16];
            if (j + 1 < NRBW) {
                const float* xr = Xs + (16 * min(rb + NW, nrb - 1) + m) * kXS + kk;
#pragma unroll
                for (int k = 0; k < 16; ++k) xn[k] = xr[4 * k];
                interleave_loads<16 * NCB>();
            }
            if (j + 1 < NRBW) {
#pragma unroll
                for (int k = 0; k < 16; ++k) xa[k] = xn[k];
            }
            // fold the tile's sums into the float64 running sums (rescaled
            // first with SCALE)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    acc[j][cb][v] = SCALE ? fma(acc[j][cb][v], (double)fs[cb], (double)t[cb][v] * (double)gs[cb])
                                          : acc[j][cb][v] + (double)t[cb][v];
        }
    }
    if (do_gram) {
#pragma unroll
        for (int gi = 0; gi < NGBW; ++gi) {
            const int gb = w + NW * gi;                // (qb, qb) for even gb, (qb, qb+1) for odd
            if (gb < 2 * NCB - 1) {
                const int q1 = gb >> 1, q2 = q1 + (gb & 1);
                f4 tg = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    float a = 0.f, b = 0.f;
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) {
                        if (cb == q1) a = bop[k][cb];
                        if (cb == q2) b = bop[k][cb];
                    }
                    tg = mfma16(a, b, tg);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) gram[gi][v] += (double)tg[v];
            }
        }
    }
}

// Write the accumulated V (rows < L, columns < QC) of this workgroup.
template <int NCB, int NRBW, int QC, int NW = 4>
__device__ __forceinline__ void store_acc(const d4 (&acc)[NRBW][NCB], float* Vp, int L, int nrb, int w, int lane) {
    const int m = lane & 15, kk = lane >> 4;
#pragma unroll
    for (int j = 0; j < NRBW; ++j) {
        const int rb = w + NW * j;
        if (rb < nrb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const int q = 16 * cb + m;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int l = 16 * rb + 4 * kk + v;
                    if (l < L && q < QC) Vp[(size_t)l * QC + q] = (float)acc[j][cb][v];
                }
            }
    }
}

// Projection of the tile by a chunk operand staged in LDS (R > 1): wave w
// computes the 16 pixels 16w..16w+15 for the NCB column blocks from CB0
// (16 columns each), S[q][i] =
// sum_l Ec[l][q] Xs[l][i]; results go to Sc[i][q] (or Sc[q][i] with QMAJOR).  Also returns, for the
// same pixels, the partial sums of x^2 over the bands this lane touched.
// LP (a multiple of 16) rows of both operands are read; rows L..LP-1 of
// both are zero.  Within a block of 16 bands, MFMA step u takes the bands
// u, u + 4, u + 8, u + 12 (lane group kk gets u + 4 kk): the four rows a
// wave reads are then 4 rows apart, which with the pitches kXS = 68 and
// ECS = QCP + 4 puts the 64 lanes on 64 distinct LDS banks.
// BS: stride between the 16-band blocks this wave takes, from block kb0
// (BS = 32: two wave groups take alternate blocks).  DUAL: the blocks
// alternate between two accumulators, summed at the end, so that consecutive
// MFMAs do not depend on each other (used with a single column block, where
// one chain would leave the matrix pipe waiting on each result).
template <int NCB, int WTS, bool QMAJOR = false, int CB0 = 0, int BS = 16, bool DUAL = false>
__device__ __forceinline__ float mfma_project(const float* Ec, int ECS, const float* Xs, float* Sc, int LP, int w,
                                              int lane, int kb0 = 0) {
    const int m = lane & 15, kk = lane >> 4;
    f4 s[NCB], s2[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) s[cb] = s2[cb] = f4{0.f, 0.f, 0.f, 0.f};
    float xx = 0.f;
    const float* xb = Xs + 4 * kk * kXS + 16 * w + m;
    const float* eb = Ec + 4 * kk * ECS + 16 * CB0 + m;
    // Software pipeline over blocks of 16 bands with two operand sets: the
    // operands of the next block are read between the first MFMAs of the
    // current one, so they arrive while the rest of its MFMAs run.
    float b0[4], e0[4][NCB], b1[4], e1[4][NCB];
    auto load = [&](float (&b)[4], float (&e)[4][NCB], int k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            b[u] = xb[(k0 + u) * kXS];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) e[u][cb] = eb[(k0 + u) * ECS + 16 * cb];
        }
    };
    auto mma = [&](const float (&b)[4], const float (&e)[4][NCB], f4 (&acc)[NCB]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            xx = fmaf(b[u], b[u], xx);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[cb] = mfma16(e[u][cb], b[u], acc[cb]);
        }
    };
    // One block per trip, no branch in the body: a branch (or a body that
    // alternates two accumulation orders) made the compiler copy the
    // accumulators out of and back into AGPRs on every trip, which drains
    // the MFMA pipeline.  Only the operands are copied between sets.
    if (kb0 < LP) {
        load(b0, e0, kb0);
        int k0 = kb0;
        for (; k0 + BS < LP; k0 += 2 * BS) {
            load(b1, e1, k0 + BS);
            __builtin_amdgcn_sched_barrier(0);
            mma(b0, e0, s);
            __builtin_amdgcn_sched_barrier(0);
            load(b0, e0, (k0 + 2 * BS < LP) ? k0 + 2 * BS : k0);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (DUAL)
                mma(b1, e1, s2);
            else
                mma(b1, e1, s);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (k0 < LP) mma(b0, e0, s);
    }
    if constexpr (DUAL) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) s[cb] += s2[cb];
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if (QMAJOR)
                Sc[(16 * (CB0 + cb) + 4 * kk + v) * kXS + 16 * w + m] = s[cb][v];
            else
                Sc[(16 * w + m) * WTS + 16 * (CB0 + cb) + 4 * kk + v] = s[cb][v];
        }
    return xx;
}

// The A-pass projection in float64: P = E^T x feeds the objective
// ||x - E a||^2 = ||x||^2 - 2 a.P + a.G a, whose terms are of order ||x||^2
// while the result is of the order of the residual, so P and ||x||^2 are
// accumulated in float64 (products of float32 values are exact in float64).
// P is kept as a float pair, hi = fl(P) (used by the A-steps) and
// lo = fl(P - hi), which carries it to about 48 bits; returns the partial
// ||x||^2 of this lane's bands.
// DUAL as for mfma_project: alternate blocks accumulate into two chains.
template <int NCB, int WTS, int CB0 = 0, bool DUAL = false>
__device__ __forceinline__ double mfma_project_f64(const float* Ec, int ECS, const float* Xs, float* Sc, float* Plo,
                                                   int LP, int w, int lane) {
    const int m = lane & 15, kk = lane >> 4;
    d4 s[NCB], s2[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) s[cb] = s2[cb] = d4{0.0, 0.0, 0.0, 0.0};
    double xx = 0.0;
    const float* xb = Xs + 4 * kk * kXS + 16 * w + m;
    const float* eb = Ec + 4 * kk * ECS + 16 * CB0 + m;
    // same software pipeline as mfma_project
    float b0[4], e0[4][NCB], b1[4], e1[4][NCB];
    auto load = [&](float (&b)[4], float (&e)[4][NCB], int k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            b[u] = xb[(k0 + u) * kXS];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) e[u][cb] = eb[(k0 + u) * ECS + 16 * cb];
        }
    };
    auto mma = [&](const float (&b)[4], const float (&e)[4][NCB], d4 (&acc)[NCB]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double bd = (double)b[u];
            xx = fma(bd, bd, xx);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[cb] = mfma16d((double)e[u][cb], bd, acc[cb]);
        }
    };
    // One block per trip, no branch in the body: a branch (or a body that
    // alternates two accumulation orders) made the compiler copy the
    // accumulators out of and back into AGPRs on every trip, which drains
    // the MFMA pipeline.  Only the operands are copied between sets.
    load(b0, e0, 0);
    int k0 = 0;
    for (; k0 + 16 < LP; k0 += 32) {
        load(b1, e1, k0 + 16);
        __builtin_amdgcn_sched_barrier(0);
        mma(b0, e0, s);
        __builtin_amdgcn_sched_barrier(0);
        load(b0, e0, (k0 + 32 < LP) ? k0 + 32 : k0);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (DUAL)
            mma(b1, e1, s2);
        else
            mma(b1, e1, s);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (k0 < LP) mma(b0, e0, s);
    if constexpr (DUAL) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) s[cb] += s2[cb];
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float hi = (float)s[cb][v];
            Sc[(16 * w + m) * WTS + 16 * (CB0 + cb) + 4 * v + kk] = hi;
            Plo[(16 * w + m) * WTS + 16 * (CB0 + cb) + 4 * v + kk] = (float)(s[cb][v] - (double)hi);
        }
    return xx;
}

// Stage U[:, chunk] (rows < L, QCP columns) in LDS with rows L..LP-1 zero.
template <int QC, int QCP>
__device__ __forceinline__ void stage_chunk(const float* __restrict__ U, int Qp, int col0, int L, int LP, float* Ec,
                                            int ECS) {
    for (int e = threadIdx.x; e < LP * QCP; e += blockDim.x) {
        const int l = e / QCP, q = e % QCP;
        Ec[l * ECS + q] = (l < L && q < QC) ? U[(size_t)l * Qp + col0 + q] : 0.f;
    }
}

// --------------------------------------------------------------------------
// A-pass: per tile, the objective at the incoming (A, E) for the trace,
// P = E^T x, K1 A-steps, write A, accumulate X A^T and A A^T partials.
// --------------------------------------------------------------------------
template <int PP, int R>
__device__ __forceinline__ void apass_body(const Geom& g, const State& s, int bid, const float* __restrict__ E, int K1) {
    using S = Shape<PP, R>;
    constexpr int NW = apass_waves(PP), NT = 64 * NW;
    constexpr int QC = S::QC, QCP = S::QCP, NCB = S::NCB, WTS = S::WTS;
    constexpr int RW = (R + NW - 1) / NW;          // runs per wave in the A-step phase (r = w + NW k < R)
    // With fewer runs than waves the A-steps of a (run, pixel) are spread
    // over SPL = min(NW / R, 4) consecutive lanes, so that (up to) four
    // waves per run take part: thread t < 64 R SPL handles run t / (64 SPL),
    // pixel (t / SPL) % 64 and the rows j = t % SPL + SPL jj of that pixel
    // (a_steps_split; quad permutes exchange the values).  This is done for
    // single runs and for the four-wave kernels; the eight-wave kernels with
    // 2 or 4 runs per chunk keep one lane per pixel (their float rows of G
    // would not fit the registers left at two waves per SIMD).
    constexpr int SPL = (R < NW && (R == 1 || NW == 4)) ? (NW / R < 4 ? NW / R : 4) : 1;
    constexpr bool SPLIT = SPL > 1;
    constexpr int JW = (PP + SPL - 1) / SPL;
    static_assert(!SPLIT || NW % R == 0, "runs per chunk must divide the waves");
    constexpr int NRBW = S::NRBW * 4 / NW;          // accumulation row blocks per wave
    constexpr int NGBW = (S::NGB + NW - 1) / NW;    // Gram blocks per wave
    // projection: waves w and w + 4 share the pixel block w & 3 (eight
    // waves), waves 0-3 taking the first NC0 column blocks
    constexpr int NC0 = (NW == 8) ? (NCB + 1) / 2 : NCB, NC1 = NCB - NC0;
    static_assert(NW == 4 || NW == 8, "four or eight waves");
    const int ECS = g.ecs;
    extern __shared__ float smem[];
    const PassLds lo = pass_lds(PP, R, g.L, g.dbuf, g.ecs, g.gf);
    float* Wt = smem + lo.wt;
    float* Ec = smem + lo.ec;
    double* Gd = (double*)(smem + lo.gs);
    float* Gf = smem + lo.gf;                  // used when g.gf
    const int xo[2] = {lo.xs, g.dbuf ? lo.xs2 : lo.xs};
    double* XX = (double*)(smem + lo.xx);
    float* Plo = smem + lo.pd;

    int pg, c;
    wg_coords(g, bid, pg, c);
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = uniform_int(tid >> 6);
    const int L = g.L, N = g.N, LP = (L + 15) & ~15, nrb = LP / 16;
    const int col0 = c * QC;
    float* __restrict__ A = s.A;

    // Gram matrices of this chunk's runs, in float64 from the float32 E the
    // projection uses (so that the objective formed from P and G below is
    // consistent with that E).
    stage_chunk<QC, QCP>(E, g.Qp, col0, L, LP, Ec, ECS);
    __syncthreads();
    // each entry by 8 consecutive lanes (bands l = sub, sub + 8, ...),
    // combined by a fixed butterfly
    for (int e0 = tid / 8; e0 < R * PP * PP; e0 += NT / 8) {
        const int sub = tid % 8;
        const int r = e0 / (PP * PP), jk = e0 % (PP * PP), j = jk / PP, k = jk % PP;
        const float* Ek = Ec + r * PP;
        double acc = 0.0;
        for (int l = sub; l < L; l += 8) acc = fma((double)Ek[l * ECS + j], (double)Ek[l * ECS + k], acc);
        acc += __shfl_xor(acc, 1);
        acc += __shfl_xor(acc, 2);
        acc += __shfl_xor(acc, 4);
        if (sub == 0) {
            Gd[e0] = acc;
            if (g.gf) Gf[e0] = (float)acc;
        }
    }
    __syncthreads();
    // zero the X rows beyond L and the weight padding (never written later)
    for (int e = tid; e < (LP - L) * kXS; e += NT) {
        smem[xo[0] + L * kXS + e] = 0.f;
        smem[xo[1] + L * kXS + e] = 0.f;
    }
    for (int e = tid; e < kTile * WTS; e += NT) Wt[e] = 0.f;

    d4 acc[NRBW][NCB], gram[NGBW];
#pragma unroll
    for (int j = 0; j < NRBW; ++j)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[j][cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < NGBW; ++j) gram[j] = d4{0.0, 0.0, 0.0, 0.0};
    double lacc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) lacc[r] = 0.0;
    // split A-steps: this thread's run, pixel and sub-lane, and its rows of
    // the run's Gram matrix in float (the steps; the objective reads the
    // float64 rows from LDS)
    const int sr = SPLIT ? tid / (64 * SPL) : 0, si = SPLIT ? (tid / SPL) % 64 : lane, ss = SPLIT ? tid % SPL : 0;
    const bool sact = !SPLIT || sr < R;            // uniform per wave
    float Gfr[JW][PP];
    if constexpr (SPLIT) {
#pragma unroll
        for (int jj = 0; jj < JW; ++jj)
#pragma unroll
            for (int kk = 0; kk < PP; ++kk) {
                const int j = ss + SPL * jj;
                Gfr[jj][kk] = (sact && j < PP) ? (float)Gd[min(sr, R - 1) * PP * PP + j * PP + kk] : 0.f;
            }
    }

    // Pipeline: the X tile and this thread's abundances (registers) of tile
    // t + npg are requested while tile t is processed.
    constexpr bool kRX = kRegX<PP, R, true>;
    const bool regx = kRX && L <= kRegXMaxL && s.x_bf16;      // float32 X: direct-to-LDS loads
    const bool dma = !regx && !s.x_bf16;
    XRegs<kRX, NW> xr;

    float an[RW][PP];
    float ano[JW];      // split: this thread's own rows
    auto load_a = [&](int tile) {
        if constexpr (SPLIT) {
            const size_t pixc = (size_t)min(tile * kTile + si, N - 1);
            const int m = min(c * R + min(sr, R - 1), g.M - 1);
#pragma unroll
            for (int j = 0; j < PP; ++j) an[0][j] = A[(size_t)(m * PP + j) * N + pixc];
#pragma unroll
            for (int jj = 0; jj < JW; ++jj) ano[jj] = A[(size_t)(m * PP + min(ss + SPL * jj, PP - 1)) * N + pixc];
        } else {
            const size_t pixc = (size_t)min(tile * kTile + lane, N - 1);
#pragma unroll
            for (int k = 0; k < RW; ++k) {
                const int m = c * R + min(w + NW * k, R - 1);
#pragma unroll
                for (int j = 0; j < PP; ++j) an[k][j] = A[(size_t)(min(m, g.M - 1) * PP + j) * N + pixc];
            }
        }
    };
    __syncthreads();
    if (pg < g.ntiles) {
        if (regx) {
            xr.issue(s.X, s.ldx, L, pg);
            xr.store(smem + xo[0], L);
        } else if (dma) {
            dma_tile<NW>((const float*)s.X, s.ldx, L, pg, smem + xo[0], w);
        }
        load_a(pg);
    }
    int it = 0;
    for (int tile = pg; tile < g.ntiles; tile += g.npg, ++it) {
        float* Xs = smem + ((it & 1) ? xo[1] : xo[0]);
        float* Xn = smem + ((it & 1) ? xo[0] : xo[1]);     // == Xs when single-buffered
        if (!dma && !regx) {
            lds_barrier();
            load_tile_sync(s.X, s.x_bf16, L, s.ldx, tile, Xs);
        }
        __builtin_amdgcn_s_waitcnt(0);
        lds_barrier();
        const int pix = tile * kTile + si;
        const bool pok = pix < N;
        float a[RW][PP];
        float ao[JW];
        if constexpr (SPLIT) {
            const bool ok = sact && c * R + sr < g.M && pok;
#pragma unroll
            for (int j = 0; j < PP; ++j) a[0][j] = ok ? an[0][j] : 0.f;
#pragma unroll
            for (int jj = 0; jj < JW; ++jj) ao[jj] = (ok && ss + SPL * jj < PP) ? ano[jj] : 0.f;
        } else {
#pragma unroll
            for (int k = 0; k < RW; ++k) {
                const int m = c * R + w + NW * k;
                const bool mok = m < g.M && w + NW * k < R;
#pragma unroll
                for (int j = 0; j < PP; ++j) a[k][j] = (mok && pok) ? an[k][j] : 0.f;
            }
        }
        const int nt = tile + g.npg;
        if (nt < g.ntiles) {
            load_a(nt);
            if (regx) xr.issue(s.X, s.ldx, L, nt);
            if (dma && g.dbuf) dma_tile<NW>((const float*)s.X, s.ldx, L, nt, Xn, w);
        }
        {
            // projection on the matrix cores: P for pixels 16w..16w+15
            // (16 (w - 4).. with eight waves, w >= 4)
            if (w < 4) {
                double xx = mfma_project_f64<NC0, WTS, 0, NCB == 1>(Ec, ECS, Xs, Wt, Plo, LP, w, lane);
                xx += __shfl_xor(xx, 16);       // the 4 band classes of the pixel
                xx += __shfl_xor(xx, 32);
                if (lane < 16) XX[16 * w + lane] = xx;
            } else if constexpr (NC1 > 0) {
                (void)mfma_project_f64<NC1, WTS, NC0>(Ec, ECS, Xs, Wt, Plo, LP, w - 4, lane);
            }
            lds_barrier();
            if constexpr (SPLIT) {
                // A-steps of run sr, pixel si, rows ss + SPL jj (see a_steps_split)
                const int m = c * R + sr;
                const bool ok = sact && m < g.M && pok;
                if (sact) {
                float Po[JW];
                double q = 0.0;
#pragma unroll
                for (int jj = 0; jj < JW; ++jj) {
                    const int j = ss + SPL * jj;
                    const int jc = min(j, PP - 1);
                    Po[jj] = j < PP ? Wt[si * WTS + sr * PP + jc] : 0.f;
                    // this thread's terms of ||x||^2 - 2 a.P + a.G a, in float64
                    const double* Gj = Gd + sr * PP * PP + jc * PP;
                    double ga = 0.0;
#pragma unroll
                    for (int kk = 0; kk < PP; ++kk) ga = fma(Gj[kk], (double)a[0][kk], ga);
                    const double pj = (double)Po[jj] + (double)(j < PP ? Plo[si * WTS + sr * PP + jc] : 0.f);
                    q = fma((double)ao[jj], ga - 2.0 * pj, q);
                }
                q = group_sum<SPL>(q);
                if (ok && ss == 0) lacc[0] += XX[si] + q;
                if (m < g.M) a_steps_split<PP, SPL>(a[0], ao, Po, Gfr, s.eta[2 * m], K1, ss);
#pragma unroll
                for (int jj = 0; jj < JW; ++jj) {
                    const int j = ss + SPL * jj;
                    if (j < PP) {
                        if (ok) A[(size_t)(m * PP + j) * N + pix] = ao[jj];
                        Wt[si * WTS + sr * PP + j] = ok ? ao[jj] : 0.f;
                    }
                }
                }
            } else {
            // A-steps: lane = pixel, runs r = w + NW k of the chunk
            const double xnorm = XX[lane];
#pragma unroll
            for (int k = 0; k < RW; ++k) {
                const int r = w + NW * k, m = c * R + r;
                if (r >= R) continue;                 // uniform per wave
                const bool mok = m < g.M;
                float P[PP];
#pragma unroll
                for (int j = 0; j < PP; ++j) P[j] = Wt[lane * WTS + r * PP + j];
                const double* Gr = Gd + r * PP * PP;
                if (mok && pok) {
                    // ||x - E a||^2 = ||x||^2 - 2 a.P + a.G a, in float64, with
                    // a.G a = 2 sum_j a_j (G_jj a_j / 2 + sum_{k > j} G_jk a_k)
                    // (G symmetric: half the products)
                    double quad = 0.0, lin = 0.0;
#pragma unroll
                    for (int j = 0; j < PP; ++j) {
                        const double aj = (double)a[k][j];
                        double sj = 0.5 * Gr[j * PP + j] * aj;
#pragma unroll
                        for (int kk = j + 1; kk < PP; ++kk) sj = fma(Gr[j * PP + kk], (double)a[k][kk], sj);
                        quad = fma(aj, sj, quad);
                        lin = fma(aj, (double)P[j] + (double)Plo[lane * WTS + r * PP + j], lin);
                    }
                    lacc[k] += xnorm + 2.0 * (quad - lin);
                }
                if (mok) {
                    if (g.gf)
                        a_steps<PP>(a[k], P, Gf + r * PP * PP, s.eta[2 * m], K1);
                    else
                        a_steps<PP>(a[k], P, Gr, s.eta[2 * m], K1);
                }
#pragma unroll
                for (int j = 0; j < PP; ++j) {
                    if (mok && pok) A[(size_t)(m * PP + j) * N + pix] = a[k][j];
                    Wt[lane * WTS + r * PP + j] = (mok && pok) ? a[k][j] : 0.f;
                }
            }
            }
        }
        lds_barrier();
        mfma_accumulate<NCB, NRBW, WTS, false, NGBW, false, NW>(acc, gram, true, Xs, Wt, nullptr, nullptr, nrb, w,
                                                                lane);
        if (nt < g.ntiles && (regx || dma)) {
            if (!g.dbuf) lds_barrier();           // single buffer: overwrite after every reader
            if (regx)
                xr.store(Xn, L);
            else if (!g.dbuf)
                dma_tile<NW>((const float*)s.X, s.ldx, L, nt, Xs, w);
        }
    }

    const size_t wgi = (size_t)pg * g.nqc + c;
    store_acc<NCB, NRBW, QC, NW>(acc, s.Vpart + wgi * (size_t)L * QC, L, nrb, w, lane);
    // A A^T of every run from the Gram blocks: entry (q1, q2) of block
    // (qb1, qb2) with q1 = 16 qb1 + 4 (lane/16) + v, q2 = 16 qb2 + lane%16.
    {
        const int m16 = lane & 15, kk = lane >> 4;
        float* AAp = s.AApart + wgi * (size_t)(R * PP * PP);
#pragma unroll
        for (int gi = 0; gi < NGBW; ++gi) {
            const int gb = w + NW * gi;
            if (gb < 2 * NCB - 1) {
                const int qb1 = gb >> 1, qb2 = qb1 + (gb & 1);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q1 = 16 * qb1 + 4 * kk + v, q2 = 16 * qb2 + m16;
                    if (q1 < QC && q2 < QC && q1 / PP == q2 / PP) {
                        const int r = q1 / PP, j = q1 % PP, k = q2 % PP;
                        AAp[r * PP * PP + j * PP + k] = (float)gram[gi][v];
                        if (qb1 != qb2) AAp[r * PP * PP + k * PP + j] = (float)gram[gi][v];
                    }
                }
            }
        }
    }
    if constexpr (SPLIT) {
        const double tot = wave_sum(lacc[0]);
        __syncthreads();
        if (lane == 0) XX[w] = tot;
        __syncthreads();
        if (tid < R) {                              // waves r SPL .. r SPL + SPL - 1 hold run r
            double t = 0.0;
            for (int w2 = tid * SPL; w2 < (tid + 1) * SPL; ++w2) t += XX[w2];
            if (c * R + tid < g.M) s.lpart[(size_t)pg * g.M + c * R + tid] = t;
        }
    } else {
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const int r = w + NW * k, m = c * R + r;
            if (r >= R) continue;
            const double tot = wave_sum(lacc[k]);
            if (lane == 0 && m < g.M) s.lpart[(size_t)pg * g.M + m] = tot;
        }
    }
}

template <int PP, int R>
__global__ __launch_bounds__(64 * apass_waves(PP), 1) void k_apass(Geom g, State s, const float* __restrict__ E, int K1) {
    apass_body<PP, R>(g, s, blockIdx.x, E, K1);
}
template <int PP, int R>
__global__ __launch_bounds__(64 * apass_waves(PP), 1) void k_apass_multi(const ImageJob* __restrict__ jobs, const int2* __restrict__ map,
                                                             int K1) {
    const int2 jl = map[blockIdx.x];
    const ImageJob& J = jobs[jl.x];
    apass_body<PP, R>(J.g, J.s, jl.y, J.s.E, K1);
}

// --------------------------------------------------------------------------
// B-pass: per tile, g = W^T x (STEP) and v = log b - eta2 g, or the start
// values (INIT: 0.1 u, or log B0); per-tile column max and online merge into
// the workgroup's running (max, sum); write the shifted weights and the
// tile's shift; accumulate X * weights^T.
//
// Softmax layout (NW waves): thread t owns column q = t / NW of the chunk
// and the 64 / NW pixels (t % NW) * 64 / NW .. of the tile, so a column's
// tile max and sum take two quad permutes (and a half-row mirror with eight
// waves), and the running (max, sum) stays in those lanes.  The projection
// results and the weights live column-major in LDS ([QCP][kXS]).  Bst rows
// are padded to whole tiles (pixels >= N hold zero weights), so the pixel
// segments are read and written as float4 without bounds checks.
// --------------------------------------------------------------------------
template <int PP, int R, bool STEP>
__device__ __forceinline__ void bpass_body(const Geom& g, const State& s, int bid, const float* __restrict__ W, int mode,
                                           const RunInit& ri) {
    using S = Shape<PP, R>;
    constexpr int NW = kBpassWaves, NT = 64 * NW;
    constexpr int QC = S::QC, QCP = S::QCP, NCB = S::NCB, WTS = S::WTS, NRBW = S::NRBW * 4 / NW;
    // softmax: NW lanes per column, SPX pixels each
    constexpr int SPX = kTile / NW, SV = SPX / 4;
    // projection: wave group 0 (waves 0-3) takes the first NC0 column
    // blocks, group 1 the other NC1, each for the pixel block w & 3
    constexpr int NC0 = (NW == 8) ? (NCB + 1) / 2 : NCB, NC1 = NCB - NC0;
    const int ECS = g.ecs;
    static_assert(NW == 4 || NW == 8, "four or eight waves");
    static_assert(QCP * NW <= NT, "NW threads per softmax column");
    extern __shared__ float smem[];
    const PassLds lo = pass_lds(PP, R, g.L, g.dbuf, g.ecs, g.gf);
    float* Wq = smem + lo.wt;                      // [QCP][kXS]
    float* Wq2 = smem + lo.pd;                     // [QCP][kXS] second projection half (one column block)
    float* F = smem + lo.f;
    float* FG = smem + lo.fg;
    float* Ec = smem + lo.ec;
    const int xo[2] = {lo.xs, g.dbuf ? lo.xs2 : lo.xs};

    int pg, c;
    wg_coords(g, bid, pg, c);
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = uniform_int(tid >> 6);
    const int L = g.L, N = g.N, LP = (L + 15) & ~15, nrb = LP / 16;
    const size_t Np = (size_t)g.ntiles * kTile;
    const int col0 = c * QC;

    for (int e = tid; e < (LP - L) * kXS; e += NT) {
        smem[xo[0] + L * kXS + e] = 0.f;
        smem[xo[1] + L * kXS + e] = 0.f;
    }
    for (int e = tid; e < QCP * kXS; e += NT) Wq[e] = 0.f;
    for (int e = tid; e < QCP; e += NT) F[e] = FG[e] = 0.f;
    if (STEP) stage_chunk<QC, QCP>(W, g.Qp, col0, L, LP, Ec, ECS);

    // this thread's softmax column and pixel segment
    const int sq = tid / NW, sub = tid % NW;
    const int sm = c * R + sq / PP, sj = sq % PP;
    const bool qin = sq < QC;                      // a column of the chunk
    const bool cok = qin && sm < g.M;              // ... of an existing run
    float* bcol = s.Bst + (size_t)(cok ? col0 + sq : 0) * Np + SPX * sub;
    float mrun = -INFINITY, lzc = 0.f, eta2 = 0.f;
    double srun = 0.0;                             // float64: it runs over every tile of the workgroup
    if (STEP && cok) {
        lzc = -s.colm[col0 + sq] - logf(s.cols[col0 + sq]);
        eta2 = s.eta[2 * sm + 1];
    }

    d4 acc[NRBW][NCB], gdummy[1];
#pragma unroll
    for (int jb = 0; jb < NRBW; ++jb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[jb][cb] = d4{0.0, 0.0, 0.0, 0.0};
    // single runs up to p = 4: X w^T on the vector ALU instead of 16-column
    // matrix blocks (p of 16 columns useful; measured faster at p = 3 and 4,
    // slower at p = 6).  Thread (row vl, pixel half vh) owns bands vl and
    // vl + 256 and sums its 32 pixels of the tile in float32, folded into
    // float64 per tile like the matrix-core sums.
    constexpr bool VACC = (R == 1 && PP <= 4);
    const int vl = tid & 255, vh = tid >> 8;
    double vacc[2][VACC ? PP : 1];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int j = 0; j < (VACC ? PP : 1); ++j) vacc[r][j] = 0.0;

    // Pipeline: the X tile and this thread's B segment and shift (registers)
    // of tile t + npg are requested while tile t is processed.
    constexpr bool kRX = kRegX<PP, R, false>;
    const bool regx = kRX && L <= kRegXMaxL && s.x_bf16;      // float32 X: direct-to-LDS loads
    const bool dma = !regx && !s.x_bf16;
    XRegs<kRX, NW> xr;

    f4 bn[SV];
    float tn = 0.f;
    auto load_b = [&](int tile) {
        if (STEP && cok) {
            const f4* src = (const f4*)(bcol + (size_t)tile * kTile);
#pragma unroll
            for (int u = 0; u < SV; ++u) bn[u] = src[u];
            tn = s.tshift[(size_t)tile * g.Qp + col0 + sq];
        }
    };
    __syncthreads();
    if (pg < g.ntiles) {
        if (regx) {
            xr.issue(s.X, s.ldx, L, pg);
            xr.store(smem + xo[0], L);
        } else if (dma) {
            dma_tile<NW>((const float*)s.X, s.ldx, L, pg, smem + xo[0], w);
        }
        load_b(pg);
    }
    int it = 0;
    for (int tile = pg; tile < g.ntiles; tile += g.npg, ++it) {
        float* Xs = smem + ((it & 1) ? xo[1] : xo[0]);
        float* Xn = smem + ((it & 1) ? xo[0] : xo[1]);     // == Xs when single-buffered
        if (!dma && !regx) {
            lds_barrier();
            load_tile_sync(s.X, s.x_bf16, L, s.ldx, tile, Xs);
        }
        __builtin_amdgcn_s_waitcnt(0);
        lds_barrier();
        f4 bv[SV];
#pragma unroll
        for (int u = 0; u < SV; ++u) bv[u] = bn[u];
        const float ts = tn;
        const int nt = tile + g.npg;
        if (nt < g.ntiles) {
            load_b(nt);
            if (regx) xr.issue(s.X, s.ldx, L, nt);
            if (dma && g.dbuf) dma_tile<NW>((const float*)s.X, s.ldx, L, nt, Xn, w);
        }

        if (STEP) {
            if constexpr (NCB == 1) {
                // one column block: waves w and w + 4 take alternate 16-band
                // blocks of pixel block w & 3, into Wq and Wq2 (summed below)
                (void)mfma_project<1, WTS, true, 0, 32, true>(Ec, ECS, Xs, (w < 4) ? Wq : Wq2, LP, w & 3, lane,
                                                              16 * (w >> 2));
            } else {
                if (w < 4)
                    (void)mfma_project<NC0, WTS, true>(Ec, ECS, Xs, Wq, LP, w, lane);
                else if constexpr (NC1 > 0)
                    (void)mfma_project<NC1, WTS, true, NC0>(Ec, ECS, Xs, Wq, LP, w - 4, lane);
            }
            lds_barrier();
        }

        if (qin) {
            const int pix0 = tile * kTile + SPX * sub;
            float* wrow = Wq + sq * kXS + SPX * sub;
            float v[SPX];
            if (STEP) {
                const float sh = ts + lzc;
#pragma unroll
                for (int u = 0; u < SV; ++u) {
                    f4 gv = *(const f4*)(wrow + 4 * u);
                    if constexpr (NCB == 1) gv += *(const f4*)(wrow - Wq + Wq2 + 4 * u);
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[4 * u + e] = fast_log(bv[u][e]) + sh - eta2 * gv[e];
                }
            } else if (mode == kModeInitRng) {
                const uint64_t seed = ri.seeds[cok ? sm : 0];
#pragma unroll
                for (int i = 0; i < SPX; ++i) v[i] = ri.init_scale * uniform_u(seed, pix0 + i, sj);
            } else {
#pragma unroll
                for (int i = 0; i < SPX; ++i) v[i] = fast_log(ri.B0[(size_t)min(pix0 + i, N - 1) * PP + sj]);
            }
            float mx = -INFINITY;
#pragma unroll
            for (int i = 0; i < SPX; ++i) {
                v[i] = (cok && pix0 + i < N) ? v[i] : -INFINITY;
                mx = fmaxf(mx, v[i]);
            }
            mx = fmaxf(mx, dpp<0xB1>(mx));             // the NW lanes of this column
            mx = fmaxf(mx, dpp<0x4E>(mx));
            if (NW == 8) mx = fmaxf(mx, dpp<0x141>(mx));
            // The tile's weights are stored relative to the tile's own max
            // (its largest weight is 1, so none underflows for being far
            // below a larger tile of this workgroup); the running sums are
            // relative to the running max: factors f (old sums) and fg
            // (this tile).
            const float mnew = fmaxf(mrun, mx);
            const float f = (mrun == -INFINITY) ? 0.f : fast_exp(mrun - mnew);
            const float fg = (mx == -INFINITY) ? 0.f : fast_exp(mx - mnew);
            float wv[SPX], sum = 0.f;
#pragma unroll
            for (int i = 0; i < SPX; ++i) {
                wv[i] = (v[i] == -INFINITY) ? 0.f : fast_exp(v[i] - mx);
                sum += wv[i];
            }
            sum += dpp<0xB1>(sum);
            sum += dpp<0x4E>(sum);
            if (NW == 8) sum += dpp<0x141>(sum);
            srun = fma(srun, (double)f, (double)sum * (double)fg);
            mrun = mnew;
#pragma unroll
            for (int u = 0; u < SV; ++u) {
                const f4 o = f4{wv[4 * u], wv[4 * u + 1], wv[4 * u + 2], wv[4 * u + 3]};
                *(f4*)(wrow + 4 * u) = o;
                if (cok) ((f4*)(bcol + (size_t)tile * kTile))[u] = o;
            }
            if (sub == 0) {
                F[sq] = f;
                FG[sq] = fg;
                if (cok) s.tshift[(size_t)tile * g.Qp + col0 + sq] = mx;
            }
        }
        lds_barrier();
        if constexpr (VACC) {
            float fq[PP], gq[PP];
#pragma unroll
            for (int j = 0; j < PP; ++j) {
                fq[j] = F[j];
                gq[j] = FG[j];
            }
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int l = vl + 256 * r;
                if (l < L) {
                    float t[PP];
#pragma unroll
                    for (int j = 0; j < PP; ++j) t[j] = 0.f;
                    const float* xr = Xs + l * kXS + 32 * vh;
                    const float* wr = Wq + 32 * vh;
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const f4 xv = *(const f4*)(xr + 4 * k);
#pragma unroll
                        for (int j = 0; j < PP; ++j) {
                            const f4 wv = *(const f4*)(wr + j * kXS + 4 * k);
                            t[j] = fmaf(xv[0], wv[0], t[j]);
                            t[j] = fmaf(xv[1], wv[1], t[j]);
                            t[j] = fmaf(xv[2], wv[2], t[j]);
                            t[j] = fmaf(xv[3], wv[3], t[j]);
                        }
                    }
#pragma unroll
                    for (int j = 0; j < PP; ++j)
                        vacc[r][j] = fma(vacc[r][j], (double)fq[j], (double)t[j] * (double)gq[j]);
                }
            }
        } else {
            mfma_accumulate<NCB, NRBW, WTS, true, 1, true, NW>(acc, gdummy, false, Xs, Wq, F, FG, nrb, w, lane);
        }
        if (nt < g.ntiles && (regx || dma)) {
            if (!g.dbuf) lds_barrier();           // single buffer: overwrite after every reader
            if (regx)
                xr.store(Xn, L);
            else if (!g.dbuf)
                dma_tile<NW>((const float*)s.X, s.ldx, L, nt, Xs, w);
        }
    }

    const size_t wgi = (size_t)pg * g.nqc + c;
    if constexpr (VACC) {
        // the two pixel halves of a band, added in a fixed order
        __syncthreads();                           // every wave is done with the X tiles
        double* hx = (double*)(smem + xo[0]);      // [L][PP]: L * PP * 8 <= L * kXS * 4 bytes
        float* Vp = s.Vpart + wgi * (size_t)L * QC;
        if (vh == 1)
#pragma unroll
            for (int r = 0; r < 2; ++r)
                if (vl + 256 * r < L)
#pragma unroll
                    for (int j = 0; j < PP; ++j) hx[(vl + 256 * r) * PP + j] = vacc[r][j];
        __syncthreads();
        if (vh == 0)
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int l = vl + 256 * r;
                if (l < L)
#pragma unroll
                    for (int j = 0; j < PP; ++j) Vp[(size_t)l * QC + j] = (float)(vacc[r][j] + hx[l * PP + j]);
            }
    } else {
        store_acc<NCB, NRBW, QC, NW>(acc, s.Vpart + wgi * (size_t)L * QC, L, nrb, w, lane);
    }
    if (qin && sub == 0) {
        s.mpart[(size_t)pg * g.Qp + col0 + sq] = cok ? mrun : -INFINITY;
        s.spart[(size_t)pg * g.Qp + col0 + sq] = cok ? (float)srun : 0.f;
    }
}

template <int PP, int R, bool STEP>
__global__ __launch_bounds__(64 * kBpassWaves, 1) void k_bpass(Geom g, State s, const float* __restrict__ W, int mode,
                                                       RunInit ri) {
    bpass_body<PP, R, STEP>(g, s, blockIdx.x, W, mode, ri);
}
template <int PP, int R, bool STEP>
__global__ __launch_bounds__(64 * kBpassWaves, 1) void k_bpass_multi(const ImageJob* __restrict__ jobs,
                                                             const int2* __restrict__ map, int mode) {
    const int2 jl = map[blockIdx.x];
    const ImageJob& J = jobs[jl.x];
    bpass_body<PP, R, STEP>(J.g, J.s, jl.y, J.s.W, mode, J.ri);
}

// --------------------------------------------------------------------------
// B-pass for bf16 X on the bf16 matrix cores: the same pass as bpass_body
// (same softmax, state, partials and results), with both contractions on
// v_mfma_f32_16x16x32_bf16.
//
// X stays bf16 in LDS, in two layouts (xb_lds): xn (pixels contiguous) is the
// A operand of the accumulation X * weights^T, whose k runs over pixels; xo
// (eight bands of a pixel contiguous) the B operand of the projection W^T x,
// whose k runs over bands.  The float32 operands, W and the tile's weights,
// are split into three bf16 terms (split_bf16x3): X is exact in bf16, so each
// product is exact in the float32 accumulation and the three MFMAs give the
// float32 product sums up to the order of the float32 additions.  Per 32
// bands (projection) or 32 pixels (accumulation) that is 3 MFMAs of 16
// clocks, against 8 float32 MFMAs of 32 clocks.
//
// X tiles are staged through registers one tile ahead (XbStage).
// Work split (8 waves): projection as bpass_body (one column block: waves w
// and w + 4 take alternate k blocks of pixel block w & 3; more: the two wave
// groups take halves of the column blocks); accumulation by row blocks of 16
// bands, rb = w + 8 j.
// --------------------------------------------------------------------------
// Register staging of a bf16 X tile into both LDS layouts of the bf16
// matrix-core passes: wave w stages the 32-band blocks w, w + NW, ... (L <=
// kXbMaxL); lane (kg, m) loads the 4 pixels 4 m.. of the bands 32 bi + 8 kg +
// j, j < 8, as eight 8-byte loads (issued one tile ahead), and store()
// writes them to xn as they are and, repacked with byte permutes, to xo.
template <int NW>
struct XbStage {
    static constexpr int NBW = kXbMaxL / 32 / NW;   // band blocks per wave
    uint2 v[NBW][8];

    __device__ __forceinline__ void issue(const void* X, size_t ldx, int L, int tile) {
        const int lane = threadIdx.x & 63, w = uniform_int(threadIdx.x >> 6), m = lane & 15, kg = lane >> 4;
        const uint16_t* src = (const uint16_t*)X + (size_t)tile * kTile + 4 * m;
#pragma unroll
        for (int i = 0; i < NBW; ++i) {
            const int bi = w + NW * i;
            if (32 * bi < L) {                         // uniform per wave
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int row = min(32 * bi + 8 * kg + j, L - 1);
                    v[i][j] = *(const uint2*)(src + (size_t)row * ldx);
                }
            }
        }
    }
    __device__ __forceinline__ void store(uint16_t* Xn, u32x4* Xo, int L) const {
        const int lane = threadIdx.x & 63, w = uniform_int(threadIdx.x >> 6), m = lane & 15, kg = lane >> 4;
#pragma unroll
        for (int i = 0; i < NBW; ++i) {
            const int bi = w + NW * i;
            if (32 * bi < L) {
                uint2 u[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int row = 32 * bi + 8 * kg + j;
                    u[j] = row < L ? v[i][j] : make_uint2(0u, 0u);
                    *(uint2*)(Xn + row * kXNP + 4 * m) = u[j];
                }
                // pixel 4 m + e: element j of its 16 bytes is band 32 bi + 8 kg + j
                u32x4* dst = Xo + (4 * bi + kg) * 64;
                constexpr unsigned LO = 0x05040100u, HI = 0x07060302u;
                dst[xo_slot(4 * m)] = u32x4{__builtin_amdgcn_perm(u[1].x, u[0].x, LO), __builtin_amdgcn_perm(u[3].x, u[2].x, LO),
                               __builtin_amdgcn_perm(u[5].x, u[4].x, LO), __builtin_amdgcn_perm(u[7].x, u[6].x, LO)};
                dst[xo_slot(4 * m + 1)] = u32x4{__builtin_amdgcn_perm(u[1].x, u[0].x, HI), __builtin_amdgcn_perm(u[3].x, u[2].x, HI),
                               __builtin_amdgcn_perm(u[5].x, u[4].x, HI), __builtin_amdgcn_perm(u[7].x, u[6].x, HI)};
                dst[xo_slot(4 * m + 2)] = u32x4{__builtin_amdgcn_perm(u[1].y, u[0].y, LO), __builtin_amdgcn_perm(u[3].y, u[2].y, LO),
                               __builtin_amdgcn_perm(u[5].y, u[4].y, LO), __builtin_amdgcn_perm(u[7].y, u[6].y, LO)};
                dst[xo_slot(4 * m + 3)] = u32x4{__builtin_amdgcn_perm(u[1].y, u[0].y, HI), __builtin_amdgcn_perm(u[3].y, u[2].y, HI),
                               __builtin_amdgcn_perm(u[5].y, u[4].y, HI), __builtin_amdgcn_perm(u[7].y, u[6].y, HI)};
            }
        }
    }
};

// Operands of one k block of a bf16 projection: the X operand and the three
// terms of NC column blocks of the float32 operand.
template <int NC>
struct XbOps {
    u32x4 b, e[NC][3];
    template <int CB0, int NCB>
    __device__ __forceinline__ void load(const u32x4* Xo, const u32x4* Esp, int kb, int pb, int lane) {
        b = Xo[(4 * kb + (lane >> 4)) * 64 + xo_slot(16 * pb + (lane & 15))];
        const u32x4* ep = Esp + (size_t)(kb * NCB + CB0) * 3 * 64 + lane;
#pragma unroll
        for (int cb = 0; cb < NC; ++cb)
#pragma unroll
            for (int sp = 0; sp < 3; ++sp) e[cb][sp] = ep[(3 * cb + sp) * 64];
    }
};

template <int NC, int CB0, int NCB, int KBS>
__device__ __forceinline__ void xb_project(const u32x4* Xo, const u32x4* Wsp, float* Sq, int nkb, int kb0, int pb,
                                           int lane) {
    const int m = lane & 15, kg = lane >> 4;
    f4 s[NC], s2[NC];
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) s[cb] = s2[cb] = f4{0.f, 0.f, 0.f, 0.f};
    auto mma = [&](const XbOps<NC>& o) {
#pragma unroll
        for (int cb = 0; cb < NC; ++cb) {
            // with one column block the middle term goes to a second chain
            s[cb] = mfma16_bf16(o.e[cb][0], o.b, s[cb]);
            if (NC == 1)
                s2[cb] = mfma16_bf16(o.e[cb][1], o.b, s2[cb]);
            else
                s[cb] = mfma16_bf16(o.e[cb][1], o.b, s[cb]);
            s[cb] = mfma16_bf16(o.e[cb][2], o.b, s[cb]);
        }
    };
    // software pipeline over k blocks with two operand sets (the next
    // block's LDS reads are in flight while the current block's MFMAs run);
    // no branch in the loop body
    if (kb0 < nkb) {
        XbOps<NC> o0, o1;
        o0.template load<CB0, NCB>(Xo, Wsp, kb0, pb, lane);
        int kb = kb0;
        for (; kb + KBS < nkb; kb += 2 * KBS) {
            o1.template load<CB0, NCB>(Xo, Wsp, kb + KBS, pb, lane);
            mma(o0);
            o0.template load<CB0, NCB>(Xo, Wsp, (kb + 2 * KBS < nkb) ? kb + 2 * KBS : kb, pb, lane);
            mma(o1);
        }
        if (kb < nkb) mma(o0);
    }
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) {
        if (NC == 1) s[cb] += s2[cb];
#pragma unroll
        for (int v = 0; v < 4; ++v) Sq[(16 * (CB0 + cb) + 4 * kg + v) * kXS + 16 * pb + m] = s[cb][v];
    }
}

// V += X_tile Wt on the bf16 matrix cores, folded into the float64 running
// sums like mfma_accumulate; with SCALE the running sums of column q are
// multiplied by F[q], the tile's by G[q].
template <int NCB, int NRBW, int NW, bool SCALE = true>
__device__ __forceinline__ void xb_accumulate(d4 (&acc)[NRBW][NCB], const uint16_t* Xn, const u32x4* Wb,
                                              const float* F, const float* G, int nrb, int w, int lane) {
    const int m = lane & 15, kg = lane >> 4;
    f4 t[NRBW][NCB];
#pragma unroll
    for (int j = 0; j < NRBW; ++j)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) t[j][cb] = f4{0.f, 0.f, 0.f, 0.f};
    // the operand reads of PK pixel blocks are issued before their first
    // MFMA (both blocks at once up to three column blocks: one LDS latency
    // per tile); rows past the last block re-read the last one
    constexpr int PK = NCB <= 3 ? 2 : 1;
#pragma unroll
    for (int p0 = 0; p0 < 2; p0 += PK) {
        u32x4 bop[PK][NCB][3], xa[NRBW][PK];
#pragma unroll
        for (int pk = 0; pk < PK; ++pk)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int sp = 0; sp < 3; ++sp)
                    bop[pk][cb][sp] = Wb[(((p0 + pk) * NCB + cb) * 3 + sp) * 64 + wb_slot(kg, m, p0 + pk)];
#pragma unroll
        for (int j = 0; j < NRBW; ++j)
#pragma unroll
            for (int pk = 0; pk < PK; ++pk)
                xa[j][pk] =
                    *(const u32x4*)(Xn + (16 * min(w + NW * j, nrb - 1) + m) * kXNP + 32 * (p0 + pk) + 8 * kg);
#pragma unroll
        for (int j = 0; j < NRBW; ++j) {
            if (w + NW * j < nrb) {
#pragma unroll
                for (int pk = 0; pk < PK; ++pk)
#pragma unroll
                    for (int sp = 0; sp < 3; ++sp)
#pragma unroll
                        for (int cb = 0; cb < NCB; ++cb)
                            t[j][cb] = mfma16_bf16(xa[j][pk], bop[pk][cb][sp], t[j][cb]);
            }
        }
    }
    float fs[NCB], gs[NCB];
    if (SCALE) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            fs[cb] = F[16 * cb + m];
            gs[cb] = G[16 * cb + m];
        }
    }
#pragma unroll
    for (int j = 0; j < NRBW; ++j)
        if (w + NW * j < nrb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    acc[j][cb][v] = SCALE ? fma(acc[j][cb][v], (double)fs[cb], (double)t[j][cb][v] * (double)gs[cb])
                                          : acc[j][cb][v] + (double)t[j][cb][v];
}

template <int PP, int R, bool STEP>
__device__ __forceinline__ void bpass_xb_body(const Geom& g, const State& s, int bid, const float* __restrict__ W,
                                              int mode, const RunInit& ri) {
    using S = Shape<PP, R>;
    constexpr int NW = 8, NT = 64 * NW;
    constexpr int QC = S::QC, QCP = S::QCP, NCB = S::NCB, NRBW = S::NRBW * 4 / NW;
    constexpr int SPX = kTile / NW, SV = SPX / 4;   // softmax: 8 lanes per column, 8 pixels each
    constexpr int NC0 = (NCB + 1) / 2, NC1 = NCB - NC0;
    static_assert(SPX == 8 && QCP * NW <= NT, "eight lanes of eight pixels per softmax column");
    extern __shared__ float smem[];
    char* const lds = (char*)smem;
    const XbLds lo = xb_lds(PP, R, g.L);
    uint16_t* Xn = (uint16_t*)(lds + lo.xn);
    u32x4* Xo = (u32x4*)(lds + lo.xo);
    u32x4* Wsp = (u32x4*)(lds + lo.wsp);
    u32x4* Wb = (u32x4*)(lds + lo.wb);
    float* Sq = (float*)(lds + lo.sq);
    float* Sq2 = (float*)(lds + lo.sq2);
    float* F = (float*)(lds + lo.f);
    float* FG = (float*)(lds + lo.fg);

    int pg, c;
    wg_coords(g, bid, pg, c);
    const int tid = threadIdx.x, lane = tid & 63, m = lane & 15, kg = lane >> 4;
    const int w = uniform_int(tid >> 6);
    const int L = g.L, N = g.N, nkb = (L + 31) >> 5, nrb = (L + 15) >> 4;
    const size_t Np = (size_t)g.ntiles * kTile;
    const int col0 = c * QC;

    for (int e = tid; e < QCP; e += NT) F[e] = FG[e] = 0.f;
    for (int e = tid; e < 2 * NCB * 3 * 64; e += NT) Wb[e] = u32x4{0u, 0u, 0u, 0u};
    if (STEP) {
        // W[:, chunk] as MFMA A operands: entry (kb, cb, lane) holds the rows
        // 32 kb + 8 (lane / 16) + j of column 16 cb + lane % 16, in three terms
        for (int e = tid; e < nkb * NCB * 64; e += NT) {
            const int ln = e & 63, kc = e >> 6;
            const int q = 16 * (kc % NCB) + (ln & 15), r0 = 32 * (kc / NCB) + 8 * (ln >> 4);
            float x[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) x[j] = (r0 + j < L && q < QC) ? W[(size_t)(r0 + j) * g.Qp + col0 + q] : 0.f;
            u32x4 h, md, lw;
            split_bf16x3(x, h, md, lw);
            Wsp[(kc * 3 + 0) * 64 + ln] = h;
            Wsp[(kc * 3 + 1) * 64 + ln] = md;
            Wsp[(kc * 3 + 2) * 64 + ln] = lw;
        }
    }

    const int sq = tid / NW, sub = tid % NW;
    const int sm = c * R + sq / PP, sj = sq % PP;
    const bool qin = sq < QC;
    const bool cok = qin && sm < g.M;
    float* bcol = s.Bst + (size_t)(cok ? col0 + sq : 0) * Np + SPX * sub;
    float mrun = -INFINITY, lzc = 0.f, eta2 = 0.f;
    double srun = 0.0;
    if (STEP && cok) {
        lzc = -s.colm[col0 + sq] - logf(s.cols[col0 + sq]);
        eta2 = s.eta[2 * sm + 1];
    }

    d4 acc[NRBW][NCB];
#pragma unroll
    for (int jb = 0; jb < NRBW; ++jb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[jb][cb] = d4{0.0, 0.0, 0.0, 0.0};

    XbStage<NW> xs;
    f4 bn[SV];
    float tn = 0.f;
    auto load_b = [&](int tile) {
        if (STEP && cok) {
            const f4* src = (const f4*)(bcol + (size_t)tile * kTile);
#pragma unroll
            for (int u = 0; u < SV; ++u) bn[u] = src[u];
            tn = s.tshift[(size_t)tile * g.Qp + col0 + sq];
        }
    };
    __syncthreads();
    if (pg < g.ntiles) {
        xs.issue(s.X, s.ldx, L, pg);
        xs.store(Xn, Xo, L);
        load_b(pg);
    }
    for (int tile = pg; tile < g.ntiles; tile += g.npg) {
        __builtin_amdgcn_s_waitcnt(0);
        lds_barrier();
        f4 bv[SV];
#pragma unroll
        for (int u = 0; u < SV; ++u) bv[u] = bn[u];
        const float ts = tn;
        const int nt = tile + g.npg;
        if (nt < g.ntiles) {
            load_b(nt);
            xs.issue(s.X, s.ldx, L, nt);
        }

        if (STEP) {
            if constexpr (NCB == 1)
                xb_project<1, 0, 1, 2>(Xo, Wsp, (w < 4) ? Sq : Sq2, nkb, w >> 2, w & 3, lane);
            else if (w < 4)
                xb_project<NC0, 0, NCB, 1>(Xo, Wsp, Sq, nkb, 0, w, lane);
            else if constexpr (NC1 > 0)
                xb_project<NC1, NC0, NCB, 1>(Xo, Wsp, Sq, nkb, 0, w - 4, lane);
            lds_barrier();
        }

        if (qin) {
            const int pix0 = tile * kTile + SPX * sub;
            float v[SPX];
            if (STEP) {
                const float sh = ts + lzc;
                const float* grow = Sq + sq * kXS + SPX * sub;
#pragma unroll
                for (int u = 0; u < SV; ++u) {
                    f4 gv = *(const f4*)(grow + 4 * u);
                    if constexpr (NCB == 1) gv += *(const f4*)(grow - Sq + Sq2 + 4 * u);
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[4 * u + e] = fast_log(bv[u][e]) + sh - eta2 * gv[e];
                }
            } else if (mode == kModeInitRng) {
                const uint64_t seed = ri.seeds[cok ? sm : 0];
#pragma unroll
                for (int i = 0; i < SPX; ++i) v[i] = ri.init_scale * uniform_u(seed, pix0 + i, sj);
            } else {
#pragma unroll
                for (int i = 0; i < SPX; ++i) v[i] = fast_log(ri.B0[(size_t)min(pix0 + i, N - 1) * PP + sj]);
            }
            float mx = -INFINITY;
#pragma unroll
            for (int i = 0; i < SPX; ++i) {
                v[i] = (cok && pix0 + i < N) ? v[i] : -INFINITY;
                mx = fmaxf(mx, v[i]);
            }
            mx = fmaxf(mx, dpp<0xB1>(mx));
            mx = fmaxf(mx, dpp<0x4E>(mx));
            mx = fmaxf(mx, dpp<0x141>(mx));
            const float mnew = fmaxf(mrun, mx);
            const float f = (mrun == -INFINITY) ? 0.f : fast_exp(mrun - mnew);
            const float fg = (mx == -INFINITY) ? 0.f : fast_exp(mx - mnew);
            float wv[SPX], sum = 0.f;
#pragma unroll
            for (int i = 0; i < SPX; ++i) {
                wv[i] = (v[i] == -INFINITY) ? 0.f : fast_exp(v[i] - mx);
                sum += wv[i];
            }
            sum += dpp<0xB1>(sum);
            sum += dpp<0x4E>(sum);
            sum += dpp<0x141>(sum);
            srun = fma(srun, (double)f, (double)sum * (double)fg);
            mrun = mnew;
            if (cok) {
#pragma unroll
                for (int u = 0; u < SV; ++u)
                    ((f4*)(bcol + (size_t)tile * kTile))[u] = f4{wv[4 * u], wv[4 * u + 1], wv[4 * u + 2], wv[4 * u + 3]};
            }
            // the accumulation's B operand: pixels 8 sub .. of column sq are
            // k = 8 (sub % 4) + j of pixel block sub / 4
            u32x4 h, md, lw;
            split_bf16x3(wv, h, md, lw);
            u32x4* dst = Wb + ((sub >> 2) * NCB + (sq >> 4)) * 3 * 64 + wb_slot(sub & 3, sq & 15, sub >> 2);
            dst[0] = h;
            dst[64] = md;
            dst[128] = lw;
            if (sub == 0) {
                F[sq] = f;
                FG[sq] = fg;
                if (cok) s.tshift[(size_t)tile * g.Qp + col0 + sq] = mx;
            }
        }
        lds_barrier();
        xb_accumulate<NCB, NRBW, NW>(acc, Xn, Wb, F, FG, nrb, w, lane);
        if (nt < g.ntiles) {
            lds_barrier();                         // every wave is done with this tile's X
            xs.store(Xn, Xo, L);
        }
    }

    const size_t wgi = (size_t)pg * g.nqc + c;
    store_acc<NCB, NRBW, QC, NW>(acc, s.Vpart + wgi * (size_t)L * QC, L, nrb, w, lane);
    if (qin && sub == 0) {
        s.mpart[(size_t)pg * g.Qp + col0 + sq] = cok ? mrun : -INFINITY;
        s.spart[(size_t)pg * g.Qp + col0 + sq] = cok ? (float)srun : 0.f;
    }
}

template <int PP, int R, bool STEP>
__global__ __launch_bounds__(64 * kBpassWaves, 1) void k_bpass_xb(Geom g, State s, const float* __restrict__ W,
                                                                  int mode, RunInit ri) {
    bpass_xb_body<PP, R, STEP>(g, s, blockIdx.x, W, mode, ri);
}

// --------------------------------------------------------------------------
// B-pass for float32 X on the bf16 matrix cores: the same pass as bpass_body
// (same softmax, state, partials and results).  Both float32 operands of each
// contraction are split exactly into three bf16 terms, x = xh + xm + xl and
// w = wh + wm + wl (split2_bf16x3), and the six products whose size is above
// about 2^-24 of x w (xh wh, xh wm, xm wh, xh wl, xl wh, xm wm) are summed on
// v_mfma_f32_16x16x32_bf16 with float32 accumulation; the three dropped ones
// are below 2^-23 of the product and unbiased, the size of a float32
// rounding (the "bf16x6" scheme of Henry, Tang and Heinecke, "Leveraging the
// bfloat16 artificial intelligence datatype for higher-precision
// computations", ARITH 2019).  Per 32 bands or pixels that is 6 MFMAs of 16
// clocks, against 8 float32 MFMAs of 32.
//
// The X tile is kept once in LDS as float32 (xf, pixels contiguous, staged
// through registers one tile ahead: XfStage); both contractions read their
// eight values per lane from it and split them in registers: the
// accumulation's A operand (eight consecutive pixels of a band) as two 16-byte
// reads, the projection's B operand (eight bands of a pixel, in the order of
// xs_band) as eight single reads.
// Work split (8 waves): projection: waves w and w + 4 take pixel block w & 3,
// with alternate k blocks of every column block (ksplit; sums in sq and sq2)
// or halves of the column blocks; accumulation by row blocks of 16 bands, rb
// = w + 8 j.
// --------------------------------------------------------------------------
// Register staging of a float32 X tile: round i, lane (r, q) of wave w loads
// pixels 4 q .. 4 q + 3 of band 4 (w + NW i) + r (16-byte loads, issued one
// tile ahead); store() writes them to xf.
template <int NW>
struct XfStage {
    static constexpr int NI = kXbMaxL / (4 * NW);   // rounds of 4 NW bands
    f4 v[NI];

    __device__ __forceinline__ void issue(const float* X, size_t ldx, int L, int tile) {
        const int lane = threadIdx.x & 63, w = uniform_int(threadIdx.x >> 6);
        const float* src = X + (size_t)tile * kTile + 4 * (lane & 15);
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int row = 4 * (w + NW * i) + (lane >> 4);
            if (4 * (w + NW * i) < L) v[i] = *(const f4*)(src + (size_t)min(row, L - 1) * ldx);
        }
    }
    __device__ __forceinline__ void store(float* Xf, int L) const {
        const int lane = threadIdx.x & 63, w = uniform_int(threadIdx.x >> 6);
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int row = 4 * (w + NW * i) + (lane >> 4);
            if (row < L) *(f4*)(Xf + row * kXS + 4 * (lane & 15)) = v[i];
        }
    }
};

// Operands of one k block of the float32-X projection: the eight float32 X
// values of the lane (split when used) and the three terms of NC column
// blocks of W.
template <int NC>
struct XsOps {
    float x[8];
    u32x4 e[NC][3];
    template <int CB0, int NCB>
    __device__ __forceinline__ void load(const float* Xf, const u32x4* Wsp, int kb, int pb, int lane) {
        const float* xb = Xf + (32 * kb + 4 * (lane >> 4)) * kXS + 16 * pb + (lane & 15);
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = xb[((j & 3) + 16 * (j >> 2)) * kXS];
        const u32x4* ep = Wsp + (size_t)(kb * NCB + CB0) * 3 * 64 + lane;
#pragma unroll
        for (int cb = 0; cb < NC; ++cb)
#pragma unroll
            for (int sp = 0; sp < 3; ++sp) e[cb][sp] = ep[(3 * cb + sp) * 64];
    }
};

// The six products of a split pair, smallest first: product u takes term
// x6a(u) of X and term x6b(u) of the other operand (0 hi, 1 mid, 2 lo).
constexpr int x6a(int u) { return u == 0 || u == 3 ? 1 : u == 1 ? 2 : 0; }
constexpr int x6b(int u) { return u == 0 || u == 4 ? 1 : u == 2 ? 2 : 0; }

template <int NC, int CB0, int NCB, int KBS>
__device__ __forceinline__ void xs_project(const float* Xf, const u32x4* Wsp, float* Sq, int nkb, int kb0, int pb,
                                           int lane) {
    const int m = lane & 15, kg = lane >> 4;
    f4 s[NC], s2[NC];
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) s[cb] = s2[cb] = f4{0.f, 0.f, 0.f, 0.f};
    auto mma = [&](const XsOps<NC>& o) {
        u32x4 xt[3];
        split8_bf16x3(o.x, xt);
#pragma unroll
        for (int u = 0; u < 6; ++u)
#pragma unroll
            for (int cb = 0; cb < NC; ++cb) {
                // with one column block alternate products go to a second chain
                if (NC == 1 && (u & 1))
                    s2[cb] = mfma16_bf16(o.e[cb][x6b(u)], xt[x6a(u)], s2[cb]);
                else
                    s[cb] = mfma16_bf16(o.e[cb][x6b(u)], xt[x6a(u)], s[cb]);
            }
    };
    if (kb0 < nkb) {
        XsOps<NC> o0, o1;
        o0.template load<CB0, NCB>(Xf, Wsp, kb0, pb, lane);
        int kb = kb0;
        for (; kb + KBS < nkb; kb += 2 * KBS) {
            o1.template load<CB0, NCB>(Xf, Wsp, kb + KBS, pb, lane);
            mma(o0);
            o0.template load<CB0, NCB>(Xf, Wsp, (kb + 2 * KBS < nkb) ? kb + 2 * KBS : kb, pb, lane);
            mma(o1);
        }
        if (kb < nkb) mma(o0);
    }
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) {
        if (NC == 1) s[cb] += s2[cb];
#pragma unroll
        for (int v = 0; v < 4; ++v) Sq[(16 * (CB0 + cb) + 4 * kg + v) * kXS + 16 * pb + m] = s[cb][v];
    }
}

// V += X_tile Wt on the bf16 matrix cores from the float32 X tile (xf) and the
// split weights, folded into the float64 running sums like xb_accumulate
// (SCALE as there).
template <int NCB, int NRBW, int NW, bool SCALE = true>
__device__ __forceinline__ void xs_accumulate(d4 (&acc)[NRBW][NCB], const float* Xf, const u32x4* Wb, const float* F,
                                              const float* G, int nrb, int w, int lane) {
    const int m = lane & 15, kg = lane >> 4;
    constexpr int JG = NRBW < 2 ? NRBW : 2, CG = NCB >= 4 ? 2 : NCB;
    static_assert(NRBW % JG == 0 && NCB % CG == 0, "row and column blocks in whole groups");
    f4 t[NRBW][NCB];
#pragma unroll
    for (int j = 0; j < NRBW; ++j)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) t[j][cb] = f4{0.f, 0.f, 0.f, 0.f};
    // Row blocks in groups of JG (the split X operands of a group are live
    // together: 20 registers per row block), column blocks in groups of CG.
    // A group's JN valid row blocks take both pixel halves in one branch-free
    // stretch of code, so the split of one half can be scheduled between the
    // other half's matrix products.
    auto group = [&](auto jn, int j0) {
        constexpr int JN = decltype(jn)::value;
#pragma unroll
        for (int pk = 0; pk < 2; ++pk) {
            u32x4 xa[JN][3];
            float xv[JN][8];
#pragma unroll
            for (int jj = 0; jj < JN; ++jj) {
                const float* xp = Xf + (16 * (w + NW * (j0 + jj)) + m) * kXS + 32 * pk + 8 * kg;
                const f4 a = *(const f4*)xp, b = *(const f4*)(xp + 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    xv[jj][e] = a[e];
                    xv[jj][4 + e] = b[e];
                }
            }
#pragma unroll
            for (int jj = 0; jj < JN; ++jj) split8_bf16x3(xv[jj], xa[jj]);
#pragma unroll
            for (int c0 = 0; c0 < NCB; c0 += CG) {
                u32x4 bop[CG][3];
#pragma unroll
                for (int cc = 0; cc < CG; ++cc)
#pragma unroll
                    for (int sp = 0; sp < 3; ++sp)
                        bop[cc][sp] = Wb[((pk * NCB + c0 + cc) * 3 + sp) * 64 + wb_slot(kg, m, pk)];
#pragma unroll
                for (int u = 0; u < 6; ++u)
#pragma unroll
                    for (int jj = 0; jj < JN; ++jj)
#pragma unroll
                        for (int cc = 0; cc < CG; ++cc)
                            t[j0 + jj][c0 + cc] = mfma16_bf16(xa[jj][x6a(u)], bop[cc][x6b(u)], t[j0 + jj][c0 + cc]);
            }
        }
    };
#pragma unroll
    for (int j0 = 0; j0 < NRBW; j0 += JG) {
        if (JG == 2 && w + NW * (j0 + 1) < nrb)
            group(std::integral_constant<int, JG>{}, j0);
        else if (w + NW * j0 < nrb)
            group(std::integral_constant<int, 1>{}, j0);
    }
    float fs[NCB], gs[NCB];
    if (SCALE) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            fs[cb] = F[16 * cb + m];
            gs[cb] = G[16 * cb + m];
        }
    }
#pragma unroll
    for (int j = 0; j < NRBW; ++j)
        if (w + NW * j < nrb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    acc[j][cb][v] = SCALE ? fma(acc[j][cb][v], (double)fs[cb], (double)t[j][cb][v] * (double)gs[cb])
                                          : acc[j][cb][v] + (double)t[j][cb][v];
}

template <int PP, int R, bool STEP>
__device__ __forceinline__ void bpass_xs_body(const Geom& g, const State& s, int bid, const float* __restrict__ W,
                                              int mode, const RunInit& ri) {
    using S = Shape<PP, R>;
    constexpr int NW = 8, NT = 64 * NW;
    constexpr int QC = S::QC, QCP = S::QCP, NCB = S::NCB, NRBW = S::NRBW * 4 / NW;
    constexpr int SPX = kTile / NW, SV = SPX / 4;   // softmax: 8 lanes per column, 8 pixels each
    constexpr int NC0 = (NCB + 1) / 2, NC1 = NCB - NC0;
    static_assert(SPX == 8 && QCP * NW <= NT, "eight lanes of eight pixels per softmax column");
    extern __shared__ float smem[];
    char* const lds = (char*)smem;
    const XsLds lo = xs_lds(PP, R, g.L);
    float* Xf = (float*)(lds + lo.xf);
    u32x4* Wsp = (u32x4*)(lds + lo.wsp);
    u32x4* Wb = (u32x4*)(lds + lo.wb);
    float* Sq = (float*)(lds + lo.sq);
    float* Sq2 = (float*)(lds + lo.sq2);
    float* F = (float*)(lds + lo.f);
    float* FG = (float*)(lds + lo.fg);
    const bool ksplit = NCB <= 3 && lo.ksplit;

    int pg, c;
    wg_coords(g, bid, pg, c);
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = uniform_int(tid >> 6);
    const int L = g.L, N = g.N, nkb = (L + 31) >> 5, nrb = (L + 15) >> 4;
    const size_t Np = (size_t)g.ntiles * kTile;
    const int col0 = c * QC;

    for (int e = tid; e < QCP; e += NT) F[e] = FG[e] = 0.f;
    for (int e = tid; e < 2 * NCB * 3 * 64; e += NT) Wb[e] = u32x4{0u, 0u, 0u, 0u};
    // X rows L .. 32 nkb - 1 (read by the last k block and row block) stay zero
    for (int e = tid; e < (32 * nkb - L) * kXS; e += NT) Xf[L * kXS + e] = 0.f;
    if (STEP) {
        // W[:, chunk] as MFMA A operands: entry (kb, cb, lane) holds the rows
        // 32 kb + xs_band(lane / 16, j) of column 16 cb + lane % 16
        for (int e = tid; e < nkb * NCB * 64; e += NT) {
            const int ln = e & 63, kc = e >> 6;
            const int q = 16 * (kc % NCB) + (ln & 15), r0 = 32 * (kc / NCB);
            float x[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int r = r0 + xs_band(ln >> 4, j);
                x[j] = (r < L && q < QC) ? W[(size_t)r * g.Qp + col0 + q] : 0.f;
            }
            u32x4 t[3];
            split8_bf16x3(x, t);
            Wsp[(kc * 3 + 0) * 64 + ln] = t[0];
            Wsp[(kc * 3 + 1) * 64 + ln] = t[1];
            Wsp[(kc * 3 + 2) * 64 + ln] = t[2];
        }
    }

    const int sq = tid / NW, sub = tid % NW;
    const int sm = c * R + sq / PP, sj = sq % PP;
    const bool qin = sq < QC;
    const bool cok = qin && sm < g.M;
    float* bcol = s.Bst + (size_t)(cok ? col0 + sq : 0) * Np + SPX * sub;
    // the softmax works with log weights in base 2 (v / ln 2), so that log and
    // exp are the hardware's log2 and exp2 with one multiply per column and
    // tile; mrun and the shifts written out are converted back
    constexpr float kLog2e = 1.4426950408889634f, kLn2 = 0.6931471805599453f;
    float mrun = -INFINITY, lzc = 0.f, eta2 = 0.f;
    double srun = 0.0;
    if (STEP && cok) {
        lzc = -s.colm[col0 + sq] - logf(s.cols[col0 + sq]);
        eta2 = s.eta[2 * sm + 1] * kLog2e;
    }

    d4 acc[NRBW][NCB];
#pragma unroll
    for (int jb = 0; jb < NRBW; ++jb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[jb][cb] = d4{0.0, 0.0, 0.0, 0.0};

    XfStage<NW> xs;
    f4 bn[SV];
    float tn = 0.f;
    auto load_b = [&](int tile) {
        if (STEP && cok) {
            const f4* src = (const f4*)(bcol + (size_t)tile * kTile);
#pragma unroll
            for (int u = 0; u < SV; ++u) bn[u] = src[u];
            tn = s.tshift[(size_t)tile * g.Qp + col0 + sq];
        }
    };
    __syncthreads();
    if (pg < g.ntiles) {
        xs.issue((const float*)s.X, s.ldx, L, pg);
        xs.store(Xf, L);
        load_b(pg);
    }
    for (int tile = pg; tile < g.ntiles; tile += g.npg) {
        __builtin_amdgcn_s_waitcnt(0);
        lds_barrier();
        f4 bv[SV];
#pragma unroll
        for (int u = 0; u < SV; ++u) bv[u] = bn[u];
        const float ts = tn;
        const int nt = tile + g.npg;
        if (nt < g.ntiles) {
            load_b(nt);
            xs.issue((const float*)s.X, s.ldx, L, nt);
        }

        if (STEP) {
            if (ksplit) {
                if constexpr (NCB <= 3)
                    xs_project<NCB, 0, NCB, 2>(Xf, Wsp, (w < 4) ? Sq : Sq2, nkb, w >> 2, w & 3, lane);
            } else if (w < 4) {
                xs_project<NC0, 0, NCB, 1>(Xf, Wsp, Sq, nkb, 0, w, lane);
            } else if constexpr (NC1 > 0) {
                xs_project<NC1, NC0, NCB, 1>(Xf, Wsp, Sq, nkb, 0, w - 4, lane);
            }
            lds_barrier();
        }

        if (qin) {
            const int pix0 = tile * kTile + SPX * sub;
            float v[SPX];
            if (STEP) {
                const float sh = (ts + lzc) * kLog2e;
                const float* grow = Sq + sq * kXS + SPX * sub;
#pragma unroll
                for (int u = 0; u < SV; ++u) {
                    f4 gv = *(const f4*)(grow + 4 * u);
                    if (ksplit) gv += *(const f4*)(grow - Sq + Sq2 + 4 * u);
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[4 * u + e] = __builtin_amdgcn_logf(bv[u][e]) + fmaf(-eta2, gv[e], sh);
                }
            } else if (mode == kModeInitRng) {
                const uint64_t seed = ri.seeds[cok ? sm : 0];
                const float sc = ri.init_scale * kLog2e;
#pragma unroll
                for (int i = 0; i < SPX; ++i) v[i] = sc * uniform_u(seed, pix0 + i, sj);
            } else {
#pragma unroll
                for (int i = 0; i < SPX; ++i) v[i] = __builtin_amdgcn_logf(ri.B0[(size_t)min(pix0 + i, N - 1) * PP + sj]);
            }
            // padding runs, and pixels past N in the last tile, take no weight
            if (!cok) {
#pragma unroll
                for (int i = 0; i < SPX; ++i) v[i] = -INFINITY;
            } else if (pix0 + SPX > N) {
#pragma unroll
                for (int i = 0; i < SPX; ++i)
                    if (pix0 + i >= N) v[i] = -INFINITY;
            }
            float mx = v[0];
#pragma unroll
            for (int i = 1; i < SPX; ++i) mx = fmaxf(mx, v[i]);
            mx = fmaxf(mx, dpp<0xB1>(mx));
            mx = fmaxf(mx, dpp<0x4E>(mx));
            mx = fmaxf(mx, dpp<0x141>(mx));
            const float mnew = fmaxf(mrun, mx);
            const float f = (mrun == -INFINITY) ? 0.f : __builtin_amdgcn_exp2f(mrun - mnew);
            const float fg = (mx == -INFINITY) ? 0.f : __builtin_amdgcn_exp2f(mx - mnew);
            const float mxs = (mx == -INFINITY) ? 0.f : mx;     // exp2(-inf - mxs) = 0
            float wv[SPX], sum = 0.f;
#pragma unroll
            for (int i = 0; i < SPX; ++i) {
                wv[i] = __builtin_amdgcn_exp2f(v[i] - mxs);
                sum += wv[i];
            }
            sum += dpp<0xB1>(sum);
            sum += dpp<0x4E>(sum);
            sum += dpp<0x141>(sum);
            srun = fma(srun, (double)f, (double)sum * (double)fg);
            mrun = mnew;
            if (cok) {
#pragma unroll
                for (int u = 0; u < SV; ++u)
                    ((f4*)(bcol + (size_t)tile * kTile))[u] = f4{wv[4 * u], wv[4 * u + 1], wv[4 * u + 2], wv[4 * u + 3]};
            }
            // the accumulation's B operand: pixels 8 sub .. of column sq are
            // k = 8 (sub % 4) + j of pixel block sub / 4
            u32x4 t[3];
            split8_bf16x3(wv, t);
            u32x4* dst = Wb + ((sub >> 2) * NCB + (sq >> 4)) * 3 * 64 + wb_slot(sub & 3, sq & 15, sub >> 2);
            dst[0] = t[0];
            dst[64] = t[1];
            dst[128] = t[2];
            if (sub == 0) {
                F[sq] = f;
                FG[sq] = fg;
                if (cok) s.tshift[(size_t)tile * g.Qp + col0 + sq] = mx * kLn2;
            }
        }
        lds_barrier();
        xs_accumulate<NCB, NRBW, NW>(acc, Xf, Wb, F, FG, nrb, w, lane);
        if (nt < g.ntiles) {
            lds_barrier();                         // every wave is done with this tile's X
            xs.store(Xf, L);
        }
    }

    const size_t wgi = (size_t)pg * g.nqc + c;
    store_acc<NCB, NRBW, QC, NW>(acc, s.Vpart + wgi * (size_t)L * QC, L, nrb, w, lane);
    if (qin && sub == 0) {
        s.mpart[(size_t)pg * g.Qp + col0 + sq] = cok ? mrun * kLn2 : -INFINITY;
        s.spart[(size_t)pg * g.Qp + col0 + sq] = cok ? (float)srun : 0.f;
    }
}

template <int PP, int R, bool STEP>
__global__ __launch_bounds__(64 * kBpassWaves, 1) void k_bpass_xs(Geom g, State s, const float* __restrict__ W,
                                                                  int mode, RunInit ri) {
    bpass_xs_body<PP, R, STEP>(g, s, blockIdx.x, W, mode, ri);
}

// --------------------------------------------------------------------------
// A-pass for bf16 X on the bf16 matrix cores: the same pass as apass_body
// (objective at the incoming state, K1 A-steps per pixel and run, X A^T and
// A A^T partials), with the X tile kept in bf16 (XbStage) and
//   * the projection P = E^T x on v_mfma_f32_16x16x32_bf16, E in three bf16
//     terms (exact, so each product is exact): each block of 32 bands is
//     summed in float32 by the matrix core and folded into float64, and P is
//     kept as a float pair (high, low) as in mfma_project_f64; the float32
//     rounding inside a block is unbiased and independent from pixel to pixel,
//     so it averages out of the objective's sum over pixels;
//   * X A^T on the bf16 matrix cores with the abundances in three bf16 terms
//     (xb_accumulate);
//   * A A^T on the float32 matrix cores from the float32 abundances, as in
//     apass_body (mfma_gram).
// --------------------------------------------------------------------------
template <int NC, int CB0, int NCB, int WTS>
__device__ __forceinline__ double xa_project(const u32x4* Xo, const u32x4* Esp, float* Phi, float* Plo, int nkb,
                                             int pb, int lane) {
    const int m = lane & 15, kg = lane >> 4;
    d4 s[NC];
    f4 tp[NC];
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) {
        s[cb] = d4{0.0, 0.0, 0.0, 0.0};
        tp[cb] = f4{0.f, 0.f, 0.f, 0.f};
    }
    double xx = 0.0;
    auto step = [&](const XbOps<NC>& o) {
        f4 t[NC];
#pragma unroll
        for (int cb = 0; cb < NC; ++cb) {
            t[cb] = mfma16_bf16(o.e[cb][0], o.b, f4{0.f, 0.f, 0.f, 0.f});
            t[cb] = mfma16_bf16(o.e[cb][1], o.b, t[cb]);
            t[cb] = mfma16_bf16(o.e[cb][2], o.b, t[cb]);
        }
        // while those run: this lane's 8 bands of ||x||^2 and the fold of
        // the previous block
        const bf16x8 bv = __builtin_bit_cast(bf16x8, o.b);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const double x = (double)(float)bv[j];
            xx = fma(x, x, xx);
        }
#pragma unroll
        for (int cb = 0; cb < NC; ++cb) {
#pragma unroll
            for (int v = 0; v < 4; ++v) s[cb][v] += (double)tp[cb][v];
            tp[cb] = t[cb];
        }
    };
    // software pipeline as in xb_project
    XbOps<NC> o0, o1;
    o0.template load<CB0, NCB>(Xo, Esp, 0, pb, lane);
    int kb = 0;
    for (; kb + 1 < nkb; kb += 2) {
        o1.template load<CB0, NCB>(Xo, Esp, kb + 1, pb, lane);
        step(o0);
        o0.template load<CB0, NCB>(Xo, Esp, (kb + 2 < nkb) ? kb + 2 : kb, pb, lane);
        step(o1);
    }
    if (kb < nkb) step(o0);
#pragma unroll
    for (int cb = 0; cb < NC; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double P = s[cb][v] + (double)tp[cb][v];
            const float hi = (float)P;
            const int idx = (16 * pb + m) * WTS + 16 * (CB0 + cb) + 4 * kg + v;
            Phi[idx] = hi;
            Plo[idx] = (float)(P - (double)hi);
        }
    return xx;
}

// The same projection from a float32 X tile (xf, read and split as in
// xs_project, E in the band order of xs_band): six products per block of 32
// bands, summed in float32 by the matrix core and folded into float64.
template <int NC, int CB0, int NCB, int WTS>
__device__ __forceinline__ double xs_pa_project(const float* Xf, const u32x4* Esp, float* Phi, float* Plo, int nkb,
                                                int pb, int lane) {
    const int m = lane & 15, kg = lane >> 4;
    d4 s[NC];
    f4 tp[NC];
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) {
        s[cb] = d4{0.0, 0.0, 0.0, 0.0};
        tp[cb] = f4{0.f, 0.f, 0.f, 0.f};
    }
    double xx = 0.0;
    auto step = [&](const XsOps<NC>& o) {
        u32x4 xt[3];
        split8_bf16x3(o.x, xt);
        f4 t[NC], t2[NC];
#pragma unroll
        for (int cb = 0; cb < NC; ++cb) t[cb] = t2[cb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int u = 0; u < 6; ++u)
#pragma unroll
            for (int cb = 0; cb < NC; ++cb) {
                // with one column block alternate products go to a second chain
                if (NC == 1 && (u & 1))
                    t2[cb] = mfma16_bf16(o.e[cb][x6b(u)], xt[x6a(u)], t2[cb]);
                else
                    t[cb] = mfma16_bf16(o.e[cb][x6b(u)], xt[x6a(u)], t[cb]);
            }
        // while those run: this lane's 8 bands of ||x||^2 and the fold of
        // the previous block
#pragma unroll
        for (int j = 0; j < 8; ++j) xx = fma((double)o.x[j], (double)o.x[j], xx);
#pragma unroll
        for (int cb = 0; cb < NC; ++cb) {
#pragma unroll
            for (int v = 0; v < 4; ++v) s[cb][v] += (double)tp[cb][v];
            tp[cb] = NC == 1 ? t[cb] + t2[cb] : t[cb];
        }
    };
    XsOps<NC> o0, o1;
    o0.template load<CB0, NCB>(Xf, Esp, 0, pb, lane);
    int kb = 0;
    for (; kb + 1 < nkb; kb += 2) {
        o1.template load<CB0, NCB>(Xf, Esp, kb + 1, pb, lane);
        step(o0);
        o0.template load<CB0, NCB>(Xf, Esp, (kb + 2 < nkb) ? kb + 2 : kb, pb, lane);
        step(o1);
    }
    if (kb < nkb) step(o0);
#pragma unroll
    for (int cb = 0; cb < NC; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double P = s[cb][v] + (double)tp[cb][v];
            const float hi = (float)P;
            const int idx = (16 * pb + m) * WTS + 16 * (CB0 + cb) + 4 * kg + v;
            Phi[idx] = hi;
            Plo[idx] = (float)(P - (double)hi);
        }
    return xx;
}

// A A^T blocks (qb, qb) and (qb, qb + 1) of the tile on the float32 matrix
// cores, from the abundances Wt [64][WTS], folded into float64 (the Gram part
// of mfma_accumulate).
template <int NCB, int NGBW, int WTS, int NW>
__device__ __forceinline__ void mfma_gram(d4 (&gram)[NGBW], const float* Wt, int w, int lane) {
    const int m = lane & 15, kk = lane >> 4;
#pragma unroll
    for (int gi = 0; gi < NGBW; ++gi) {
        const int gb = w + NW * gi;
        if (gb < 2 * NCB - 1) {
            const int q1 = gb >> 1, q2 = q1 + (gb & 1);
            f4 tg = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 16; ++k)
                tg = mfma16(Wt[(4 * k + kk) * WTS + 16 * q1 + m], Wt[(4 * k + kk) * WTS + 16 * q2 + m], tg);
#pragma unroll
            for (int v = 0; v < 4; ++v) gram[gi][v] += (double)tg[v];
        }
    }
}

template <int PP, int R, bool XF = false>
__device__ __forceinline__ void apass_xb_body(const Geom& g, const State& s, int bid, const float* __restrict__ E,
                                              int K1) {
    using S = Shape<PP, R>;
    constexpr int NW = xa_waves(PP), NT = 64 * NW;
    constexpr int QC = S::QC, QCP = S::QCP, NCB = S::NCB, WTS = S::WTS;
    constexpr int RW = (R + NW - 1) / NW;
    // A-step layout as in apass_body; without the float64 projection the
    // eight-wave kernels up to p = 4 also have the registers to spread 2 or 4
    // runs over lane pairs or quads
    constexpr int SPL = (R < NW && (R == 1 || NW == 4 || PP <= 4)) ? (NW / R < 4 ? NW / R : 4) : 1;
    constexpr bool SPLIT = SPL > 1;
    constexpr int JW = (PP + SPL - 1) / SPL;
    static_assert(!SPLIT || NW % R == 0, "runs per chunk must divide the waves");
    constexpr int NRBW = S::NRBW * 4 / NW;
    constexpr int NGBW = (S::NGB + NW - 1) / NW;
    constexpr int NC0 = (NW == 8) ? (NCB + 1) / 2 : NCB, NC1 = NCB - NC0;
    static_assert(!XF || NW == 8, "float32 X tiles are staged by eight waves");
    extern __shared__ float smem[];
    char* const lds = (char*)smem;
    const int L = g.L, N = g.N, nkb = (L + 31) >> 5, nrb = (L + 15) >> 4;
    const bool gfx = (size_t)xa_lds(PP, R, L, 1).total <= kMaxLdsBytes;   // room for the float Gram copy
    const XaLds lo = xa_lds(PP, R, L, gfx ? 1 : 0);
    uint16_t* Xn = (uint16_t*)(lds + lo.xn);
    u32x4* Xo = (u32x4*)(lds + lo.xo);
    float* Xf = (float*)(lds + lo.xn);          // float32 X: [LP32][kXS] over xn and xo
    u32x4* Esp = (u32x4*)(lds + lo.esp);
    float* Wt = (float*)(lds + lo.wt);
    float* Plo = (float*)(lds + lo.plo);
    u32x4* Wb = (u32x4*)(lds + lo.plo);
    double* Gd = (double*)(lds + lo.gs);
    float* Gf = (float*)(lds + lo.gf);
    double* XX = (double*)(lds + lo.xx);

    int pg, c;
    wg_coords(g, bid, pg, c);
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = uniform_int(tid >> 6);
    const int col0 = c * QC;
    float* __restrict__ A = s.A;

    // E[:, chunk] as MFMA A operands (three bf16 terms; float32 X: bands in
    // the order of xs_band), and the Gram matrices in float64 from the
    // float32 E
    for (int e = tid; e < nkb * NCB * 64; e += NT) {
        const int ln = e & 63, kc = e >> 6;
        const int q = 16 * (kc % NCB) + (ln & 15), r0 = 32 * (kc / NCB);
        float x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int r = r0 + (XF ? xs_band(ln >> 4, j) : 8 * (ln >> 4) + j);
            x[j] = (r < L && q < QC) ? E[(size_t)r * g.Qp + col0 + q] : 0.f;
        }
        u32x4 h, md, lw;
        split_bf16x3(x, h, md, lw);
        Esp[(kc * 3 + 0) * 64 + ln] = h;
        Esp[(kc * 3 + 1) * 64 + ln] = md;
        Esp[(kc * 3 + 2) * 64 + ln] = lw;
    }
    for (int e0 = tid / 8; e0 < R * PP * PP; e0 += NT / 8) {
        const int sub = tid % 8;
        const int r = e0 / (PP * PP), jk = e0 % (PP * PP), j = jk / PP, k = jk % PP;
        const float* Ek = E + col0 + r * PP;
        double acc = 0.0;
        for (int l = sub; l < L; l += 8) acc = fma((double)Ek[(size_t)l * g.Qp + j], (double)Ek[(size_t)l * g.Qp + k], acc);
        acc += __shfl_xor(acc, 1);
        acc += __shfl_xor(acc, 2);
        acc += __shfl_xor(acc, 4);
        if (sub == 0) {
            Gd[e0] = acc;
            if (gfx) Gf[e0] = (float)acc;
        }
    }
    // the weight padding columns (never written later); float32 X: the rows
    // L .. 32 nkb - 1 of the tile (never written later)
    for (int e = tid; e < kTile * WTS; e += NT) Wt[e] = 0.f;
    if (XF)
        for (int e = tid; e < (32 * nkb - L) * kXS; e += NT) Xf[L * kXS + e] = 0.f;
    __syncthreads();

    d4 acc[NRBW][NCB], gram[NGBW];
#pragma unroll
    for (int j = 0; j < NRBW; ++j)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[j][cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < NGBW; ++j) gram[j] = d4{0.0, 0.0, 0.0, 0.0};
    double lacc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) lacc[r] = 0.0;
    const int sr = SPLIT ? tid / (64 * SPL) : 0, si = SPLIT ? (tid / SPL) % 64 : lane, ss = SPLIT ? tid % SPL : 0;
    const bool sact = !SPLIT || sr < R;
    float Gfr[JW][PP];
    if constexpr (SPLIT) {
#pragma unroll
        for (int jj = 0; jj < JW; ++jj)
#pragma unroll
            for (int kk = 0; kk < PP; ++kk) {
                const int j = ss + SPL * jj;
                Gfr[jj][kk] = (sact && j < PP) ? (float)Gd[min(sr, R - 1) * PP * PP + j * PP + kk] : 0.f;
            }
    }

    std::conditional_t<XF, XfStage<NW>, XbStage<NW>> xs;
    auto stage_store = [&]() {
        if constexpr (XF)
            xs.store(Xf, L);
        else
            xs.store(Xn, Xo, L);
    };
    float an[RW][PP];
    float ano[JW];
    auto load_a = [&](int tile) {
        if constexpr (SPLIT) {
            const size_t pixc = (size_t)min(tile * kTile + si, N - 1);
            const int m = min(c * R + min(sr, R - 1), g.M - 1);
#pragma unroll
            for (int j = 0; j < PP; ++j) an[0][j] = A[(size_t)(m * PP + j) * N + pixc];
#pragma unroll
            for (int jj = 0; jj < JW; ++jj) ano[jj] = A[(size_t)(m * PP + min(ss + SPL * jj, PP - 1)) * N + pixc];
        } else {
            const size_t pixc = (size_t)min(tile * kTile + lane, N - 1);
#pragma unroll
            for (int k = 0; k < RW; ++k) {
                const int m = c * R + min(w + NW * k, R - 1);
#pragma unroll
                for (int j = 0; j < PP; ++j) an[k][j] = A[(size_t)(min(m, g.M - 1) * PP + j) * N + pixc];
            }
        }
    };
    if (pg < g.ntiles) {
        xs.issue((const std::conditional_t<XF, float, void>*)s.X, s.ldx, L, pg);
        stage_store();
        load_a(pg);
    }
    for (int tile = pg; tile < g.ntiles; tile += g.npg) {
        __builtin_amdgcn_s_waitcnt(0);
        lds_barrier();
        const int pix = tile * kTile + si;
        const bool pok = pix < N;
        float a[RW][PP];
        float ao[JW];
        if constexpr (SPLIT) {
            const bool ok = sact && c * R + sr < g.M && pok;
#pragma unroll
            for (int j = 0; j < PP; ++j) a[0][j] = ok ? an[0][j] : 0.f;
#pragma unroll
            for (int jj = 0; jj < JW; ++jj) ao[jj] = (ok && ss + SPL * jj < PP) ? ano[jj] : 0.f;
        } else {
#pragma unroll
            for (int k = 0; k < RW; ++k) {
                const int m = c * R + w + NW * k;
                const bool mok = m < g.M && w + NW * k < R;
#pragma unroll
                for (int j = 0; j < PP; ++j) a[k][j] = (mok && pok) ? an[k][j] : 0.f;
            }
        }
        const int nt = tile + g.npg;
        if (nt < g.ntiles) {
            load_a(nt);
            xs.issue((const std::conditional_t<XF, float, void>*)s.X, s.ldx, L, nt);
        }
        // projection: P for pixels 16w..16w+15 (16 (w - 4).. with eight
        // waves, w >= 4, which take the last NC1 column blocks)
        if (w < 4) {
            double xx = XF ? xs_pa_project<NC0, 0, NCB, WTS>(Xf, Esp, Wt, Plo, nkb, w, lane)
                           : xa_project<NC0, 0, NCB, WTS>(Xo, Esp, Wt, Plo, nkb, w, lane);
            xx += __shfl_xor(xx, 16);
            xx += __shfl_xor(xx, 32);
            if (lane < 16) XX[16 * w + lane] = xx;
        } else if constexpr (NC1 > 0) {
            if constexpr (XF)
                (void)xs_pa_project<NC1, NC0, NCB, WTS>(Xf, Esp, Wt, Plo, nkb, w - 4, lane);
            else
                (void)xa_project<NC1, NC0, NCB, WTS>(Xo, Esp, Wt, Plo, nkb, w - 4, lane);
        }
        lds_barrier();
        if constexpr (SPLIT) {
            const int m = c * R + sr;
            const bool ok = sact && m < g.M && pok;
            if (sact) {
                float Po[JW];
                double q = 0.0;
#pragma unroll
                for (int jj = 0; jj < JW; ++jj) {
                    const int j = ss + SPL * jj;
                    const int jc = min(j, PP - 1);
                    Po[jj] = j < PP ? Wt[si * WTS + sr * PP + jc] : 0.f;
                    const double* Gj = Gd + sr * PP * PP + jc * PP;
                    double ga = 0.0;
#pragma unroll
                    for (int kk = 0; kk < PP; ++kk) ga = fma(Gj[kk], (double)a[0][kk], ga);
                    const double pj = (double)Po[jj] + (double)(j < PP ? Plo[si * WTS + sr * PP + jc] : 0.f);
                    q = fma((double)ao[jj], ga - 2.0 * pj, q);
                }
                q = group_sum<SPL>(q);
                if (ok && ss == 0) lacc[0] += XX[si] + q;
                if (m < g.M) a_steps_split<PP, SPL>(a[0], ao, Po, Gfr, s.eta[2 * m], K1, ss);
#pragma unroll
                for (int jj = 0; jj < JW; ++jj) {
                    const int j = ss + SPL * jj;
                    if (j < PP) {
                        if (ok) A[(size_t)(m * PP + j) * N + pix] = ao[jj];
                        Wt[si * WTS + sr * PP + j] = ok ? ao[jj] : 0.f;
                    }
                }
            }
        } else {
            const double xnorm = XX[lane];
#pragma unroll
            for (int k = 0; k < RW; ++k) {
                const int r = w + NW * k, m = c * R + r;
                if (r >= R) continue;
                const bool mok = m < g.M;
                float P[PP];
#pragma unroll
                for (int j = 0; j < PP; ++j) P[j] = Wt[lane * WTS + r * PP + j];
                const double* Gr = Gd + r * PP * PP;
                if (mok && pok) {
                    // ||x||^2 - 2 a.P + a.G a with a.G a = 2 sum_j a_j (G_jj a_j / 2
                    // + sum_{k > j} G_jk a_k) (G symmetric: half the products)
                    double quad = 0.0, lin = 0.0;
#pragma unroll
                    for (int j = 0; j < PP; ++j) {
                        const double aj = (double)a[k][j];
                        double sj = 0.5 * Gr[j * PP + j] * aj;
#pragma unroll
                        for (int kk = j + 1; kk < PP; ++kk) sj = fma(Gr[j * PP + kk], (double)a[k][kk], sj);
                        quad = fma(aj, sj, quad);
                        lin = fma(aj, (double)P[j] + (double)Plo[lane * WTS + r * PP + j], lin);
                    }
                    lacc[k] += xnorm + 2.0 * (quad - lin);
                }
                if (mok) {
                    if (gfx)
                        a_steps<PP>(a[k], P, Gf + r * PP * PP, s.eta[2 * m], K1);
                    else
                        a_steps<PP>(a[k], P, Gr, s.eta[2 * m], K1);
                }
#pragma unroll
                for (int j = 0; j < PP; ++j) {
                    if (mok && pok) A[(size_t)(m * PP + j) * N + pix] = a[k][j];
                    Wt[lane * WTS + r * PP + j] = (mok && pok) ? a[k][j] : 0.f;
                }
            }
        }
        lds_barrier();
        // the new abundances as MFMA B operands (over the low parts of P,
        // which the A-steps have consumed): entry (pkb, cb, lane) holds
        // pixels 32 pkb + 8 (lane / 16) + j of column 16 cb + lane % 16
        for (int e = tid; e < 2 * NCB * 64; e += NT) {
            const int ln = e & 63, pc = e >> 6;
            const int q = 16 * (pc % NCB) + (ln & 15), p0 = 32 * (pc / NCB) + 8 * (ln >> 4);
            float x[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) x[j] = Wt[(p0 + j) * WTS + q];
            u32x4 h, md, lw;
            split_bf16x3(x, h, md, lw);
            const int sl = wb_slot(ln >> 4, ln & 15, pc / NCB);
            Wb[(pc * 3 + 0) * 64 + sl] = h;
            Wb[(pc * 3 + 1) * 64 + sl] = md;
            Wb[(pc * 3 + 2) * 64 + sl] = lw;
        }
        lds_barrier();
        if constexpr (XF)
            xs_accumulate<NCB, NRBW, NW, false>(acc, Xf, Wb, nullptr, nullptr, nrb, w, lane);
        else
            xb_accumulate<NCB, NRBW, NW, false>(acc, Xn, Wb, nullptr, nullptr, nrb, w, lane);
        mfma_gram<NCB, NGBW, WTS, NW>(gram, Wt, w, lane);
        if (nt < g.ntiles) {
            lds_barrier();                         // every wave is done with this tile's X and weights
            stage_store();
        }
    }

    const size_t wgi = (size_t)pg * g.nqc + c;
    store_acc<NCB, NRBW, QC, NW>(acc, s.Vpart + wgi * (size_t)L * QC, L, nrb, w, lane);
    {
        const int m16 = lane & 15, kk = lane >> 4;
        float* AAp = s.AApart + wgi * (size_t)(R * PP * PP);
#pragma unroll
        for (int gi = 0; gi < NGBW; ++gi) {
            const int gb = w + NW * gi;
            if (gb < 2 * NCB - 1) {
                const int qb1 = gb >> 1, qb2 = qb1 + (gb & 1);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q1 = 16 * qb1 + 4 * kk + v, q2 = 16 * qb2 + m16;
                    if (q1 < QC && q2 < QC && q1 / PP == q2 / PP) {
                        const int r = q1 / PP, j = q1 % PP, k = q2 % PP;
                        AAp[r * PP * PP + j * PP + k] = (float)gram[gi][v];
                        if (qb1 != qb2) AAp[r * PP * PP + k * PP + j] = (float)gram[gi][v];
                    }
                }
            }
        }
    }
    if constexpr (SPLIT) {
        const double tot = wave_sum(lacc[0]);
        __syncthreads();
        if (lane == 0) XX[w] = tot;
        __syncthreads();
        if (tid < R) {
            double t = 0.0;
            for (int w2 = tid * SPL; w2 < (tid + 1) * SPL; ++w2) t += XX[w2];
            if (c * R + tid < g.M) s.lpart[(size_t)pg * g.M + c * R + tid] = t;
        }
    } else {
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const int r = w + NW * k, m = c * R + r;
            if (r >= R) continue;
            const double tot = wave_sum(lacc[k]);
            if (lane == 0 && m < g.M) s.lpart[(size_t)pg * g.M + m] = tot;
        }
    }
}

template <int PP, int R>
__global__ __launch_bounds__(64 * xa_waves(PP), 1) void k_apass_xb(Geom g, State s, const float* __restrict__ E,
                                                                      int K1) {
    apass_xb_body<PP, R>(g, s, blockIdx.x, E, K1);
}

// The A-pass for float32 X on the bf16 matrix cores (eight-wave kernels, p <=
// 9): the X tile kept once in float32 (XfStage, same LDS bytes as the two bf16
// layouts), the projection and X A^T with both operands in three bf16 terms
// and six products (xs_pa_project, xs_accumulate).
template <int PP, int R>
__global__ __launch_bounds__(64 * xa_waves(PP), 1) void k_apass_xs(Geom g, State s, const float* __restrict__ E,
                                                                      int K1) {
    apass_xb_body<PP, R, true>(g, s, blockIdx.x, E, K1);
}

// --------------------------------------------------------------------------
// Closing pass: objective and l1 fit of every run at the final (A, E), from
// the per-band residual (the l1 fit needs it band by band).
// --------------------------------------------------------------------------
// Workgroups of NW waves (R == 1: 8, the band sums of a pixel split over the
// waves; R > 1: 4, R / 4 runs per wave).
template <int PP, int R, int NW>
__device__ __forceinline__ void close_body(const Geom& g, const State& s, int bid, const float* __restrict__ E) {
    constexpr int QC = PP * R;
    constexpr int RW = (R + 3) / 4;                   // runs per wave (R > 1): w RW + r < R
    static_assert(R == 1 || NW == 4, "stacked runs use four waves");
    extern __shared__ float smem[];
    float* Xs = smem;                                  // [L][kXS]
    float* Ls = Xs + g.L * kXS;                        // R == 1: [2][NW][kTile]

    int pg, c;
    wg_coords(g, bid, pg, c);
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = uniform_int(tid >> 6);
    const int L = g.L, N = g.N, col0 = c * QC;
    double lacc[RW], facc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) lacc[r] = facc[r] = 0.0;

    for (int tile = pg; tile < g.ntiles; tile += g.npg) {
        __syncthreads();
        load_tile_sync(s.X, s.x_bf16, L, s.ldx, tile, Xs);
        const int pix = tile * kTile + lane;
        const bool pok = pix < N;
        __syncthreads();
        if constexpr (R == 1) {
            const int m = c;
            float a[PP];
#pragma unroll
            for (int j = 0; j < PP; ++j) a[j] = pok ? s.A[(size_t)(m * PP + j) * N + pix] : 0.f;
            float ls = 0.f, fs = 0.f;
            const int Lq = (L + NW - 1) / NW, l0 = min(L, w * Lq), l1 = min(L, l0 + Lq);
            for (int l = l0; l < l1; ++l) {
                const float* El = E + (size_t)l * g.Qp + col0;
                float r = Xs[l * kXS + lane];
#pragma unroll
                for (int j = 0; j < PP; ++j) r = fmaf(-El[j], a[j], r);
                ls = fmaf(r, r, ls);
                fs += fabsf(r);
            }
            Ls[w * kTile + lane] = ls;
            Ls[(NW + w) * kTile + lane] = fs;
            __syncthreads();
            if (w == 0 && pok) {
                float lt = Ls[lane], ft = Ls[NW * kTile + lane];
#pragma unroll
                for (int k = 1; k < NW; ++k) {
                    lt += Ls[k * kTile + lane];
                    ft += Ls[(NW + k) * kTile + lane];
                }
                lacc[0] += (double)lt;
                facc[0] += (double)ft;
            }
        } else {
            float a[RW][PP], ls[RW], fs[RW];
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const int m = c * R + w * RW + r;
                const bool rok = pok && m < g.M && w * RW + r < R;
#pragma unroll
                for (int j = 0; j < PP; ++j) a[r][j] = rok ? s.A[(size_t)(m * PP + j) * N + pix] : 0.f;
                ls[r] = fs[r] = 0.f;
            }
            const float* Ew = E + col0 + w * RW * PP;
            for (int l = 0; l < L; ++l) {
                const float x = Xs[l * kXS + lane];
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
            if (lane == 0 && m < g.M && w * RW + r < R) {
                s.lpart[(size_t)pg * g.M + m] = lt;
                s.fpart[(size_t)pg * g.M + m] = ft;
            }
        }
    }
}

constexpr int close_waves(int R) { return R == 1 ? 8 : 4; }
template <int PP, int R>
__global__ __launch_bounds__(64 * close_waves(R)) void k_close(Geom g, State s, const float* __restrict__ E) {
    close_body<PP, R, close_waves(R)>(g, s, blockIdx.x, E);
}
template <int PP>
__global__ __launch_bounds__(512) void k_close_multi(const ImageJob* __restrict__ jobs, const int2* __restrict__ map) {
    const int2 jl = map[blockIdx.x];
    const ImageJob& J = jobs[jl.x];
    close_body<PP, 1, 8>(J.g, J.s, jl.y, J.s.E);
}


// --------------------------------------------------------------------------
// Reductions of the per-workgroup partials, in a fixed order.  Grid:
// (row blocks, chunks); a workgroup owns whole rows of its chunk.
// --------------------------------------------------------------------------
// The cross-workgroup sums, E and W = E (A A^T) - X A^T are formed in float64:
// E A A^T and X A^T are both of order N/p while W is of the order of the
// residual, so forming the difference in float32 would lose most digits.
//
// Every sum over the npg per-workgroup partials is split into fixed slices
// of the partial index (one slice per thread) whose results are combined in
// slice order, so the result does not depend on scheduling.

// Threads of the row reductions (reduce_a, reduce_b).  The same code runs
// as its own kernel (one row per workgroup) and inside the persistent ragged
// kernel (several rows per workgroup); both have 512 threads.
constexpr int kRedThreads = 512;

// Slices of the partial index for `no` outputs of npg partials each: as many
// as the workgroup holds, but no more than one per four partials (the slice
// results are combined serially).  Depends on (npg, no) only, so the order
// of every sum is fixed whatever the workgroup computes besides.
__device__ __forceinline__ int red_slices(int npg, int no) {
    return max(1, min(kRedThreads / no, (npg + 3) / 4));
}

// Rows of the partial arrays reduced together by one workgroup.
__device__ __forceinline__ int red_rows(int npg, int no) { return max(1, kRedThreads / (red_slices(npg, no) * no)); }

// For the rows r < nr packed in this workgroup: out[r * no + o] = sum over pg
// of src(r)[pg * stride + o] (src(r) = src + r * rstride), o < no.  Thread t
// takes row t / (S no), slice (t / no) % S and output t % no; slice sl walks
// the partials sl, sl + S, ... in order, and the slices are then added in
// slice order.  red: kRedThreads doubles of scratch.
__device__ __forceinline__ void sliced_sum(const float* __restrict__ src, size_t rstride, size_t stride, int npg,
                                           int no, int nr, double* red, double* out) {
    const int tid = threadIdx.x, S = red_slices(npg, no);
    const int r = tid / (S * no), sl = (tid / no) % S, o = tid % no;
    double acc = 0.0;
    if (r < nr) {
        const float* sr = src + (size_t)r * rstride;
        for (int pg0 = sl; pg0 < npg; pg0 += 4 * S) {     // loads first, sums in the plain order
            // (unconditional loads from clamped indexes, so that the four
            // are issued together)
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = sr[(size_t)min(pg0 + u * S, npg - 1) * stride + o];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (pg0 + u * S < npg) acc += (double)v[u];
        }
    }
    red[tid] = acc;
    __syncthreads();
    if (tid < nr * no) {
        const int rr = tid / no, oo = tid % no;
        double t = 0.0;
        for (int k = 0; k < S; ++k) t += red[(rr * S + k) * no + oo];
        out[tid] = t;
    }
    __syncthreads();
}

// A A^T of run m and its objective at the incoming state (trace[t]), summed
// over the npg workgroup partials.  Each output is summed by one wave: lane
// l takes the partials l, l + 64, ... in order and the lanes are combined by
// a fixed butterfly (lane 0's result), so the sums do not depend on
// scheduling.  The waves of this workgroup take the outputs o0 + w,
// o0 + w + ostride, ... (w = wave index).
template <int PP, int R>
__device__ __forceinline__ void reduce_aa_body(const Geom& g, const State& s, int m, int o0, int ostride, int t) {
    constexpr int P2 = PP * PP;
    const int lane = threadIdx.x & 63, w = uniform_int(threadIdx.x >> 6);
    for (int o = o0 + w; o <= P2; o += ostride) {
        double acc = 0.0;
        if (o < P2) {
            const float* src = s.AApart + (size_t)m * P2 + o;          // [npg][nqc R][p][p]
            const size_t st = (size_t)g.nqc * R * P2;
            for (int pg = lane; pg < g.npg; pg += 64) acc += (double)src[(size_t)pg * st];
        } else {
            for (int pg = lane; pg < g.npg; pg += 64) acc += s.lpart[(size_t)pg * g.M + m];
        }
        acc = wave_sum(acc);
        if (lane == 0) {
            if (o < P2)
                s.AAtd[(size_t)m * P2 + o] = acc;
            else
                s.trace[(size_t)m * (s.T + 1) + t] = 0.5 * acc;
        }
    }
}

template <int PP, int R>
__global__ __launch_bounds__(kThreads) void k_reduce_aa(Geom g, State s, int t) {
    reduce_aa_body<PP, R>(g, s, blockIdx.x, 4 * blockIdx.y, 4 * gridDim.y, t);
}

// Rows l0 .. l0 + nl - 1 of chunk c: X A^T[l][:] and W[l][:] = E[l][:] A A^T
// - X A^T[l][:].  scratch: kRedThreads + red_rows * QC doubles.
template <int PP, int R>
__device__ __forceinline__ void reduce_a_rows(const Geom& g, const State& s, int l0, int nl, int c, double* scratch) {
    constexpr int QC = PP * R;
    double* red = scratch;
    double* xa = scratch + kRedThreads;
    const int tid = threadIdx.x, col0 = c * QC, L = g.L;
    const int RP = red_rows(g.npg, QC);
    for (int lb = l0; lb < l0 + nl; lb += RP) {
        const int nr = min(RP, l0 + nl - lb);
        sliced_sum(s.Vpart + ((size_t)c * L + lb) * QC, QC, (size_t)g.nqc * L * QC, g.npg, QC, nr, red, xa);
        if (tid < nr * QC) {
            const int l = lb + tid / QC, q = tid % QC, m = c * R + q / PP, ml = q / PP, j = q % PP;
            double x = xa[tid], wv = 0.0;
            if (m < g.M) {
                wv = -x;
                const double* El = s.Ed + (size_t)l * g.Qp + col0 + ml * PP;
                const double* aat = s.AAtd + (size_t)m * PP * PP;
#pragma unroll
                for (int k = 0; k < PP; ++k) wv = fma(El[k], aat[k * PP + j], wv);
            } else {
                x = 0.0;
            }
            s.XAtd[(size_t)l * g.Qp + col0 + q] = x;
            s.W[(size_t)l * g.Qp + col0 + q] = (float)wv;
        }
        __syncthreads();
    }
}

template <int PP, int R>
__global__ __launch_bounds__(kRedThreads) void k_reduce_a(Geom g, State s, int t) {
    __shared__ double scratch[kRedThreads + PP * R];
    (void)t;
    reduce_a_rows<PP, R>(g, s, blockIdx.x, 1, blockIdx.y, scratch);
}
// Single-run images (R = 1, one chunk): the objective and A A^T of the run
// (aa_blocks(p) workgroups per image), then, in a second launch since W needs
// A A^T, the rows of X A^T and W (L workgroups per image).
template <int PP>
__global__ __launch_bounds__(kThreads) void k_reduce_aa_multi(const ImageJob* __restrict__ jobs,
                                                              const int2* __restrict__ map, int t) {
    const int2 jl = map[blockIdx.x];
    const ImageJob& J = jobs[jl.x];
    reduce_aa_body<PP, 1>(J.g, J.s, 0, 4 * jl.y, 4 * aa_blocks(PP), t);
}
template <int PP>
__global__ __launch_bounds__(kRedThreads) void k_reduce_a_multi(const ImageJob* __restrict__ jobs,
                                                             const int2* __restrict__ map, int t) {
    __shared__ double scratch[kRedThreads + PP];
    const int2 jl = map[blockIdx.x];
    const ImageJob& J = jobs[jl.x];
    (void)t;
    reduce_a_rows<PP, 1>(J.g, J.s, jl.y, 1, 0, scratch);
}

// Rows l0 .. l0 + nl - 1 of chunk c after a B-pass: column statistics (max,
// sum relative to the max) of the softmax over all N pixels, E[l][:] = X B_new
// and W for the next B-step.  Several rows are packed per pass over the
// partials (the column statistics are recomputed per row, in the same order).
// scratch: kRedThreads + 3 * kRedThreads doubles.
template <int PP, int R>
__device__ __forceinline__ void reduce_b_rows(const Geom& g, const State& s, int l0, int nl, int c, int need_w,
                                              double* scratch) {
    constexpr int QC = PP * R;
    double* red = scratch;
    float* Ms = (float*)(scratch + kRedThreads);          // [rows][QC]
    double* Ss = scratch + 2 * kRedThreads;               // [rows][QC]
    double* Ev = scratch + 3 * kRedThreads;               // [rows][QC]
    const int tid = threadIdx.x;
    const int col0 = c * QC, L = g.L;
    const int S = red_slices(g.npg, QC), RP = red_rows(g.npg, QC);
    const int r = tid / (S * QC), sl = (tid / QC) % S, o = tid % QC;
    // column maxima over the workgroup partials; the partials of a slice are
    // walked four at a time, loads first, the arithmetic in the same order
    // as a plain walk
    constexpr int U = 4;
    for (int lb = l0; lb < l0 + nl; lb += RP) {
        const int nr = min(RP, l0 + nl - lb);
        const bool act = r < nr;
        const int l = lb + r;
        float mx = -INFINITY;
        if (act)
            for (int pg0 = sl; pg0 < g.npg; pg0 += U * S) {
                float v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int pg = pg0 + u * S;
                    const float mv = s.mpart[(size_t)min(pg, g.npg - 1) * g.Qp + col0 + o];
                    v[u] = pg < g.npg ? mv : -INFINITY;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) mx = fmaxf(mx, v[u]);
            }
        red[tid] = (double)mx;
        __syncthreads();
        if (tid < nr * QC) {
            const int rr = tid / QC, oo = tid % QC;
            float t = -INFINITY;
            for (int k = 0; k < S; ++k) t = fmaxf(t, (float)red[(rr * S + k) * QC + oo]);
            Ms[tid] = t;
        }
        __syncthreads();
        // column sums and the row of X B (relative to the maxima)
        const float mq = act ? Ms[r * QC + o] : -INFINITY;
        double sa = 0.0, ea = 0.0;
        if (act && mq != -INFINITY)
            for (int pg0 = sl; pg0 < g.npg; pg0 += U * S) {
                float mp[U], sp[U], vp[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int pg = pg0 + u * S, pgc = min(pg, g.npg - 1);
                    const bool ok = pg < g.npg;
                    const float mv = s.mpart[(size_t)pgc * g.Qp + col0 + o], sv = s.spart[(size_t)pgc * g.Qp + col0 + o];
                    const float vv = s.Vpart[(((size_t)pgc * g.nqc + c) * L + l) * QC + o];
                    mp[u] = ok ? mv : -INFINITY;
                    sp[u] = ok ? sv : 0.f;
                    vp[u] = ok ? vv : 0.f;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (mp[u] == -INFINITY) continue;
                    const double f = (double)expf(mp[u] - mq);
                    sa += (double)sp[u] * f;
                    ea += (double)vp[u] * f;
                }
            }
        red[tid] = sa;
        __syncthreads();
        if (tid < nr * QC) {
            const int rr = tid / QC, oo = tid % QC;
            double t = 0.0;
            for (int k = 0; k < S; ++k) t += red[(rr * S + k) * QC + oo];
            Ss[tid] = t;
        }
        __syncthreads();
        red[tid] = ea;
        __syncthreads();
        if (tid < nr * QC) {
            const int rr = tid / QC, q = tid % QC, lr = lb + rr;
            double t = 0.0;
            for (int k = 0; k < S; ++k) t += red[(rr * S + k) * QC + q];
            const int m = c * R + q / PP;
            const double e = (m < g.M) ? t / Ss[tid] : 0.0;
            Ev[tid] = e;
            s.E[(size_t)lr * g.Qp + col0 + q] = (float)e;
            s.Ed[(size_t)lr * g.Qp + col0 + q] = e;
            if (lr == 0 && m < g.M) {
                s.colm[col0 + q] = Ms[tid];
                s.cols[col0 + q] = (float)Ss[tid];
            }
        }
        __syncthreads();
        if (need_w && tid < nr * QC) {
            const int rr = tid / QC, q = tid % QC, lr = lb + rr, m = c * R + q / PP, ml = q / PP, j = q % PP;
            double wv = 0.0;
            if (m < g.M) {
                wv = -s.XAtd[(size_t)lr * g.Qp + col0 + q];
                const double* aat = s.AAtd + (size_t)m * PP * PP;
#pragma unroll
                for (int k = 0; k < PP; ++k) wv = fma(Ev[rr * QC + ml * PP + k], aat[k * PP + j], wv);
            }
            s.W[(size_t)lr * g.Qp + col0 + q] = (float)wv;
        }
        __syncthreads();
    }
}

template <int PP, int R>
__global__ __launch_bounds__(kRedThreads) void k_reduce_b(Geom g, State s, int need_w) {
    __shared__ double scratch[4 * kRedThreads];
    reduce_b_rows<PP, R>(g, s, blockIdx.x, 1, blockIdx.y, need_w, scratch);
}

// The results of reduce_b_rows, bit for bit (every sum over the partials in
// the same order), for up to kRedRows rows per workgroup: each thread keeps
// the partials of its slice (at most kRedHeld of them) in registers, so the
// column statistics and the factors f = exp(m_pg - M) are formed once for
// all rows, and the rows' loads are issued together.
constexpr int kRedRows = 4, kRedHeld = 16;
template <int PP, int R, int KM>
__device__ __forceinline__ void reduce_b_rows_f(const Geom& g, const State& s, int l0, int nl, int c, int need_w,
                                                double* scratch) {
    constexpr int QC = PP * R, NLM = kRedRows;
    static_assert(KM <= kRedHeld, "partials held per thread");
    double* red = scratch;                                       // [NLM][kRedThreads]
    double* Ss = scratch + NLM * kRedThreads;                    // [QC]
    double* Ev = Ss + QC;                                        // [NLM][QC]
    float* Ms = (float*)(Ev + NLM * QC);                         // [QC]
    const int tid = threadIdx.x;
    const int col0 = c * QC, L = g.L, npg = g.npg;
    const int S = red_slices(npg, QC);
    const bool act = tid < S * QC;
    const int sl = tid / QC, o = tid % QC;
    nl = min(nl, L - l0);
    // this thread's partials pg = sl + k S: maxima, then factors and sums
    float f[KM], sp[KM];
    // (the loads are unconditional, from clamped indexes, so that they are
    // issued together; the values past the partials are then replaced)
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const int pg = sl + k * S;
        const size_t at = (size_t)min(pg, npg - 1) * g.Qp + col0 + o;
        const float mv = s.mpart[at], sv = s.spart[at];
        const bool ok = act && pg < npg;
        f[k] = ok ? mv : -INFINITY;
        sp[k] = ok ? sv : 0.f;
    }
    float mx = -INFINITY;
#pragma unroll
    for (int k = 0; k < KM; ++k) mx = fmaxf(mx, f[k]);
    red[tid] = (double)mx;
    __syncthreads();
    if (tid < QC) {
        float t = -INFINITY;
        for (int k = 0; k < S; ++k) t = fmaxf(t, (float)red[k * QC + tid]);
        Ms[tid] = t;
    }
    __syncthreads();
    const float mq = act ? Ms[o] : -INFINITY;
    double sa = 0.0;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        float fk = -1.f;                                         // -1: no weight
        if (mq != -INFINITY && f[k] != -INFINITY) {
            fk = expf(f[k] - mq);
            sa += (double)sp[k] * (double)fk;
        }
        f[k] = fk;
    }
    // the rows' partials of X B, all loads issued before the first sum
    float vv[NLM][KM];
    const float* vp = s.Vpart + ((size_t)c * L + l0) * QC + o;
    const size_t vstride = (size_t)g.nqc * L * QC;
#pragma unroll
    for (int r = 0; r < NLM; ++r)
#pragma unroll
        for (int k = 0; k < KM; ++k)
            vv[r][k] = vp[(size_t)min(sl + k * S, npg - 1) * vstride + (size_t)min(r, nl - 1) * QC];
    red[tid] = sa;
    __syncthreads();
    if (tid < QC) {
        double t = 0.0;
        for (int k = 0; k < S; ++k) t += red[k * QC + tid];
        Ss[tid] = t;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NLM; ++r) {
        double ea = 0.0;
#pragma unroll
        for (int k = 0; k < KM; ++k)
            if (f[k] >= 0.f) ea += (double)vv[r][k] * (double)f[k];
        red[r * kRedThreads + tid] = ea;
    }
    __syncthreads();
    for (int e = tid; e < nl * QC; e += kRedThreads) {
        const int r = e / QC, q = e % QC, l = l0 + r, m = c * R + q / PP;
        double t = 0.0;
        for (int k = 0; k < S; ++k) t += red[r * kRedThreads + k * QC + q];
        const double ev = (m < g.M) ? t / Ss[q] : 0.0;
        Ev[e] = ev;
        s.E[(size_t)l * g.Qp + col0 + q] = (float)ev;
        s.Ed[(size_t)l * g.Qp + col0 + q] = ev;
        if (l == 0 && m < g.M) {
            s.colm[col0 + q] = Ms[q];
            s.cols[col0 + q] = (float)Ss[q];
        }
    }
    __syncthreads();
    if (need_w)
        for (int e = tid; e < nl * QC; e += kRedThreads) {
            const int r = e / QC, q = e % QC, l = l0 + r, m = c * R + q / PP, ml = q / PP, j = q % PP;
            double wv = 0.0;
            if (m < g.M) {
                wv = -s.XAtd[(size_t)l * g.Qp + col0 + q];
                const double* aat = s.AAtd + (size_t)m * PP * PP;
#pragma unroll
                for (int k = 0; k < PP; ++k) wv = fma(Ev[r * QC + ml * PP + k], aat[k * PP + j], wv);
            }
            s.W[(size_t)l * g.Qp + col0 + q] = (float)wv;
        }
}

// KM: partials held per thread, at least ceil(npg / red_slices(npg, QC))
template <int PP, int R, int KM>
__global__ __launch_bounds__(kRedThreads) void k_reduce_b_f(Geom g, State s, int need_w, int nl) {
    __shared__ double scratch[kRedRows * kRedThreads + (2 * kRedRows + 2) * 64];
    reduce_b_rows_f<PP, R, KM>(g, s, blockIdx.x * nl, nl, blockIdx.y, need_w, scratch);
}
template <int PP>
__global__ __launch_bounds__(kRedThreads) void k_reduce_b_multi(const ImageJob* __restrict__ jobs,
                                                             const int2* __restrict__ map, int need_w) {
    __shared__ double scratch[4 * kRedThreads];
    const int2 jl = map[blockIdx.x];
    const ImageJob& J = jobs[jl.x];
    reduce_b_rows<PP, 1>(J.g, J.s, jl.y, 1, 0, need_w, scratch);
}

__device__ __forceinline__ void reduce_close_body(const Geom& g, const State& s, int first, int stride) {
    for (int m = first; m < g.M; m += stride) {
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
__device__ __forceinline__ void eta_body(const Geom& g, const State& s, int bx, const RunInit& ri, double* Gd) {
    const int m = bx, tid = threadIdx.x;
    const int c = m / g.R, col0 = c * g.QC + (m % g.R) * PP;
    for (int e = tid; e < PP * PP; e += blockDim.x) {
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

template <int PP>
__global__ __launch_bounds__(kThreads) void k_eta(Geom g, State s, RunInit ri) {
    __shared__ double Gd[PP * PP];
    eta_body<PP>(g, s, blockIdx.x, ri, Gd);
}

// --------------------------------------------------------------------------
// Outputs: normalised B in [M][N][p], E in [M][L][p], coherence per run.
// --------------------------------------------------------------------------
template <int PP>
__device__ __forceinline__ void final_B_body(const Geom& g, const State& s, int bx, int by, int nbx, float* B_out) {
    const int m = by;
    const size_t n = (size_t)g.N * PP;
    const int c = m / g.R, base = c * g.QC + (m % g.R) * PP;
    for (size_t e = (size_t)bx * blockDim.x + threadIdx.x; e < n; e += (size_t)nbx * blockDim.x) {
        const int pix = (int)(e / PP), j = (int)(e % PP);
        const int qp = base + j, tile = pix / kTile;
        const float b = s.Bst[(size_t)(m * PP + j) * ((size_t)g.ntiles * kTile) + pix];
        B_out[(size_t)m * n + e] = b * expf(s.tshift[(size_t)tile * g.Qp + qp] - s.colm[qp] - logf(s.cols[qp]));
    }
}

template <int PP>
__global__ __launch_bounds__(kThreads) void k_final_B(Geom g, State s, float* B_out) {
    final_B_body<PP>(g, s, blockIdx.x, blockIdx.y, gridDim.x, B_out);
}

template <int PP>
__device__ __forceinline__ void final_E_body(const Geom& g, const State& s, int bx, float* E_out, int cosine,
                                             double* Gd) {
    const int m = bx, tid = threadIdx.x;
    const int c = m / g.R, base = c * g.QC + (m % g.R) * PP;
    if (E_out)
        for (int e = tid; e < g.L * PP; e += blockDim.x) {
            const int l = e / PP, j = e % PP;
            E_out[(size_t)m * g.L * PP + e] = s.E[(size_t)l * g.Qp + base + j];
        }
    for (int e = tid; e < PP * PP; e += blockDim.x) {
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

template <int PP>
__global__ __launch_bounds__(kThreads) void k_final_E(Geom g, State s, float* E_out, int cosine) {
    __shared__ double Gd[PP * PP];
    final_E_body<PP>(g, s, blockIdx.x, E_out, cosine, Gd);
}

// Multi-image helpers (single-run images of one p).

// Start state of one single-run image: E, W, X A^T and E (float64) zero, A =
// 1/p.  Workgroup `first` of `nblk` strides over the elements.
template <int PP>
__device__ __forceinline__ void prep_body(const Geom& g, const State& s, int first, int nblk) {
    const size_t i0 = (size_t)first * blockDim.x + threadIdx.x, st = (size_t)nblk * blockDim.x;
    const size_t nf = (size_t)(g.L + kPadRows) * g.Qp, nd = (size_t)g.L * g.Qp;
    for (size_t i = i0; i < nf; i += st) {
        s.E[i] = 0.f;
        s.W[i] = 0.f;
    }
    for (size_t i = i0; i < nd; i += st) {
        s.XAtd[i] = 0.0;
        s.Ed[i] = 0.0;
    }
    const size_t na = (size_t)PP * g.N;
    for (size_t i = i0; i < na; i += st) s.A[i] = 1.f / (float)PP;
}

template <int PP>
__global__ __launch_bounds__(kThreads) void k_prep_multi(const ImageJob* __restrict__ jobs,
                                                         const int2* __restrict__ map) {
    const int2 jl = map[blockIdx.x];
    const ImageJob& J = jobs[jl.x];
    prep_body<PP>(J.g, J.s, jl.y, kElemBlocks);
}

template <int PP>
__global__ __launch_bounds__(kThreads) void k_eta_multi(const ImageJob* __restrict__ jobs, const int2* __restrict__ map) {
    __shared__ double Gd[PP * PP];
    const ImageJob& J = jobs[map[blockIdx.x].x];
    eta_body<PP>(J.g, J.s, 0, J.ri, Gd);
}

__global__ __launch_bounds__(kThreads) void k_reduce_close_multi(const ImageJob* __restrict__ jobs,
                                                                 const int2* __restrict__ map) {
    const ImageJob& J = jobs[map[blockIdx.x].x];
    reduce_close_body(J.g, J.s, threadIdx.x, kThreads);
}

template <int PP>
__global__ __launch_bounds__(kThreads) void k_final_multi(const ImageJob* __restrict__ jobs,
                                                          const int2* __restrict__ map, int cosine) {
    __shared__ double Gd[PP * PP];
    const int2 jl = map[blockIdx.x];
    const ImageJob& J = jobs[jl.x];
    final_B_body<PP>(J.g, J.s, jl.y, 0, kElemBlocks, J.B_out);
    if (jl.y == 0) final_E_body<PP>(J.g, J.s, 0, J.E_out, cosine, Gd);
}

}  // namespace
}  // namespace edaa
