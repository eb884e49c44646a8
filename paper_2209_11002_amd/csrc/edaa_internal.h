// Internal declarations shared by the kernel and host translation units of the
// EDAA library.  Not part of the public C ABI (include/edaa.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace edaa {

// The pass kernels work on tiles of 64 consecutive pixels.  kThreads is the
// workgroup size of the kernels with 4 wave64s (reductions, the closing
// pass, the A-pass above p = 9); the B-pass and the A-pass up to p = 9 use
// 8 wave64s.
constexpr int kTile = 64;
constexpr int kThreads = 256;
constexpr int kMaxL = 448;
constexpr int kMaxP = 16;
constexpr int kTargetWorkgroups = 256;   // default pass grid: one workgroup per CU (256 CUs)
constexpr int kPadRows = 17;             // zero rows after the L rows of E and W

enum PassMode { kModeStep = 0, kModeInitRng = 1, kModeInitB0 = 2 };

// Accumulation row blocks (16 bands each) per wave at four waves for a chunk
// of R runs of p endmembers.  A wave keeps NRBW x NCB float64 accumulator
// blocks (NCB = column blocks of 16), so chunks of up to two column blocks
// hold eight row blocks and wider chunks four: the pass kernels of a chunk
// cover at most max_bands(p, R) bands.
__host__ __device__ constexpr int acc_row_blocks(int p, int R) { return (p * R + 15) / 16 <= 2 ? 8 : 4; }
__host__ __device__ constexpr int max_bands(int p, int R) { return 4 * 16 * acc_row_blocks(p, R); }

// Runs per chunk with compiled pass kernels, largest first (the list ends
// with 1).  The largest fills at most 64 columns.
__host__ __device__ constexpr int runs_max(int p) {
    return p > 8 ? 4 : p > 5 ? 8 : p == 5 ? 12 : p == 4 ? 16 : 20;
}
__host__ __device__ constexpr int run_choices(int p, int* out) {
    int n = 0;
    if (p > 8) {
        out[n++] = 4;
        out[n++] = 2;
    } else {
        out[n++] = runs_max(p);
        if (runs_max(p) > 8) out[n++] = 8;
        out[n++] = 4;
    }
    out[n++] = 1;
    return n;
}
__host__ __device__ constexpr bool has_runs(int p, int R) {
    int c[4] = {0, 0, 0, 0};
    const int n = run_choices(p, c);
    for (int i = 0; i < n; ++i)
        if (c[i] == R) return true;
    return false;
}

// Workgroups (of four waves) of the A A^T reduction per run: output o of a
// run (o < p^2: an entry of A A^T; o = p^2: the objective) goes to wave o % 4
// of workgroup o / 4.
__host__ __device__ constexpr int aa_blocks(int p) { return (p * p + 1 + 3) / 4; }

// Geometry of one batched problem: M runs of p endmembers on an L x N image,
// the runs grouped in chunks of R (one workgroup column per chunk).
struct Geom {
    int L, N, M, p;
    int R;        // runs per chunk (1: single-run kernels)
    int QC;       // columns per chunk = R * p
    int nqc;      // number of chunks = ceil(M / R)
    int Qp;       // padded column count = nqc * QC
    int ntiles;   // ceil(N / 64)
    int npg;      // pixel groups (workgroups per chunk)
    int dbuf;     // pass kernels double-buffer the X tile in LDS
    int ecs;      // LDS pitch (floats) of the staged projection operand
    int gf;       // the A-pass keeps a float copy of the Gram matrices in LDS
};

// Device-side state of a batched problem.  Column q = m * p + j (run m,
// endmember j) in the unpadded [Q][N] arrays; padded column c * QC + qq in the
// [L][Qp] arrays.
struct State {
    const void* X;      // [L][ldx] padded copy of the caller's X (float32 or bf16 bits), pixels >= N zero
    size_t ldx;         // ntiles * 64
    int x_bf16;
    int x_mfma;         // passes on the bf16 matrix cores: bit 0 the B-pass (k_bpass_xb for bf16 X,
                        // k_bpass_xs for float32 X), bit 1 the A-pass (k_apass_xb, k_apass_xs)
    float* A;           // [Q][N] abundances (the caller's A_all)
    float* Bst;         // [Q][ntiles * 64] unnormalised pixel weights (pixels >= N: zero)
    float* tshift;      // [ntiles][Qp] shift used when a tile of Bst was written
    float* colm;        // [Qp] column maximum of the last B-pass
    float* cols;        // [Qp] column sum (relative to colm) of the last B-pass
    float* E;           // [L + kPadRows][Qp]  endmembers X B (float32 copy read by the
                        // passes; rows >= L are zero)
    double* Ed;         // [L][Qp]  the same in float64
    float* W;           // [L + kPadRows][Qp]  E (A A^T) - X A^T (rows >= L zero)
    double* XAtd;       // [L][Qp]  X A^T
    double* AAtd;       // [M][p][p] A A^T
    float* eta;         // [M][2] step sizes used by the kernels
    double* etad;       // [M][2] the same in float64 (reported)
    double* trace;      // [M][T+1]
    double* fit;        // [M]
    double* mu;         // [M]
    float* Vpart;       // [npg][nqc][L][QC]
    float* mpart;       // [npg][Qp]
    float* spart;       // [npg][Qp]
    float* AApart;      // [npg][nqc][R][p][p]
    double* lpart;      // [npg][M]
    double* fpart;      // [npg][M]
    int T;              // trace stride is T+1
};

struct RunInit {
    const uint64_t* seeds;   // device [M]
    const double* gammas;    // device [M]
    float init_scale;
    const float* B0;         // device [N][p] or null (single run only)
    const float* A0;         // device [p][N] or null
    double eta1, eta2;       // > 0: overrides
};

// One image of a ragged batch (single run, R = 1): its geometry, state,
// start values and outputs.  Multi-image launches read a table of these in
// device memory and a map from workgroup to (image, workgroup within the
// image), so one launch serves every image of a group of equal p.
struct ImageJob {
    Geom g;
    State s;
    RunInit ri;
    float* B_out;       // device [N][p]
    float* E_out;       // device [L][p] or null
};

// Multi-image launch maps; per image: kMapPass: npg workgroups; kMapRows:
// L (one per band); kMapOne: 1; kMapElem: kElemBlocks; kMapAA: aa_blocks(p).
enum MultiMap { kMapPass = 0, kMapRows = 1, kMapOne = 2, kMapElem = 3, kMapAA = 4, kMapKinds = 5 };
constexpr int kElemBlocks = 32;
enum MultiKernel {
    kMultiPrep = 0,        // zero E, W, X A^T, E (f64); A = 1/p            (kMapElem)
    kMultiBpassInit,       // B-pass from the seeded start values         (kMapPass)
    kMultiBpassStep,       // B-step pass                                 (kMapPass)
    kMultiRedB,            // column statistics, E, W (arg: need_w)       (kMapRows)
    kMultiEta,             // step sizes                                  (kMapOne)
    kMultiApass,           // A-pass (arg: K1)                            (kMapPass)
    kMultiRedAA,           // A A^T and the objective (arg: t)            (kMapAA)
    kMultiRedA,            // X A^T and W (arg: t)                        (kMapRows)
    kMultiClose,           // closing pass                                (kMapPass)
    kMultiCloseReduce,     // final objective and l1 fit                  (kMapOne)
    kMultiFinal,           // B and E outputs, coherence (arg: cosine)    (kMapElem)
};
// Persistent ragged execution (edaa_persist.hip).  Sub-stage kinds of an
// image's sequence; the items of each kind per image are: the passes npg
// (one per pixel group), the row reductions ceil(L / kPersistRows), the
// A A^T reduction ceil((p^2 + 1) / 8), the outputs kPersistFinal, the rest 1.
enum PersistKind {
    kPkBpassInit = 0,  // B-pass from the seeded start values
    kPkBpassStep,      // B-step pass
    kPkApass,          // A-pass
    kPkRowsB,          // column statistics, E, W (arg: need_w)
    kPkAA,             // A A^T and the objective at the incoming state
    kPkRowsA,          // X A^T and W
    kPkEta,            // step sizes
    kPkClose,          // closing pass
    kPkCloseRed,       // final objective and l1 fit
    kPkFinal,          // B and E outputs, coherence
    kPkKinds
};
constexpr int kPersistRows = 8;     // band rows per reduction item
constexpr int kPersistFinal = 8;    // items of the output stage per image
constexpr int kPersistMaxP = 9;     // the persistent kernel holds p <= 9 (eight-wave A-pass)
constexpr int kDefaultTilesPerItem = 8;

// The schedule of a persistent launch: three segments (prologue, the outer
// iteration repeated T times, epilogue) of sub-stages; tickets run through
// the segments in order, sub-stage by sub-stage, image by image.
struct PersistPlan {
    const ImageJob* jobs;       // [n_images] device
    int n_images, T, K1, cosine;
    long long seg_len[3];       // tickets of each segment (one iteration for segment 1)
    int nsub[3];                // sub-stages of each segment
    int sub_stride;
    const int* seg_kind;        // [3][sub_stride] PersistKind
    const int* seg_arg;         // [3][sub_stride]
    const long long* seg_base;  // [3][sub_stride] first ticket of each sub-stage within its segment
    const int* cnt;             // [kPkKinds][n_images] items per image
    const long long* pre;       // [kPkKinds][n_images + 1] prefix sums of cnt over images
    const long long* need0;     // [3][n_images] items of an image before each segment (iteration 0)
    const long long* iter;      // [n_images] items of an image per outer iteration
    unsigned long long* ticket; // device counters, zeroed by the launcher's first kernel
    unsigned long long* done;   // [n_images]
    int* status;                // set to 1 if a wait exceeded its bound
};
hipError_t launch_ragged_persistent(const PersistPlan& P, size_t lds_bytes, int n_workgroups, hipStream_t st);

// Launchers of the kernels compiled for one p (edaa_inst.hip, built once per
// p).  The pass launchers take the chunk size from g.R, which must be one of
// run_choices(p); they return hipErrorInvalidValue otherwise.
struct PassOps {
    hipError_t (*apass)(const Geom& g, const State& s, int K1, hipStream_t st);
    hipError_t (*bpass)(const Geom& g, const State& s, int mode, const RunInit& ri, hipStream_t st);
    hipError_t (*close)(const Geom& g, const State& s, hipStream_t st);
    hipError_t (*reduce_b)(const Geom& g, const State& s, int need_w, hipStream_t st);
    hipError_t (*reduce_a)(const Geom& g, const State& s, int t, hipStream_t st);
    hipError_t (*reduce_aa)(const Geom& g, const State& s, int t, hipStream_t st);
    hipError_t (*eta)(const Geom& g, const State& s, const RunInit& ri, hipStream_t st);
    hipError_t (*finalize)(const Geom& g, const State& s, float* B_out, float* E_out, int cosine, hipStream_t st);
    hipError_t (*multi)(int kernel, const ImageJob* jobs, const int2* map, int nblocks, size_t lds_bytes, int arg,
                        hipStream_t st);
};
// The table for p (1 <= p <= kMaxP), or null.
const PassOps* pass_ops(int p);

// Enqueue one multi-image kernel for the images of one p (all R = 1).
hipError_t launch_multi(int kernel, int p, const ImageJob* jobs, const int2* map, int nblocks, size_t lds_bytes,
                        int arg, hipStream_t st);

// Launchers (edaa_kernels.hip).  All enqueue on `st` and return the HIP error
// of the last launch.
hipError_t launch_pad_x(const void* X, void* Xp, int L, int N, size_t ldx, int bf16, hipStream_t st);
hipError_t launch_fill(float* dst, size_t n, float value, hipStream_t st);
hipError_t launch_init_A(const Geom& g, const State& s, const float* A0, hipStream_t st);
hipError_t launch_bpass(const Geom& g, const State& s, int mode, const RunInit& ri, hipStream_t st);
hipError_t launch_reduce_b(const Geom& g, const State& s, int need_w, hipStream_t st);
hipError_t launch_eta(const Geom& g, const State& s, const RunInit& ri, hipStream_t st);
hipError_t launch_apass(const Geom& g, const State& s, int K1, int t, hipStream_t st);
hipError_t launch_reduce_a(const Geom& g, const State& s, int t, hipStream_t st);
hipError_t launch_reduce_aa(const Geom& g, const State& s, int t, hipStream_t st);
hipError_t launch_set_e(const float* E_given, const Geom& g, const State& s, hipStream_t st);
hipError_t launch_close(const Geom& g, const State& s, hipStream_t st);
hipError_t launch_set_run(uint64_t* seeds, double* gammas, uint64_t seed, double gamma, hipStream_t st);
hipError_t launch_reduce_close(const Geom& g, const State& s, hipStream_t st);
hipError_t launch_finalize(const Geom& g, const State& s, float* B_out, float* E_out,
                           int coherence_mode, hipStream_t st);
hipError_t launch_normalize(const float* Xin, void* Xout, int L, int N, int out_bf16,
                            int* n_zero_dev, hipStream_t st);

// Autograd / mirror-step kernels (edaa_grad.hip).
struct GradWork {
    float* E;        // [L][p]  X B rounded to float32
    double* Ed;      // [L][p]  X B
    double* Wd;      // [L][p]  (X B A - X) A^T
    double* Vpart;   // [nblk][L][p]
    double* lpart;   // [nblk]
    float* cm;       // [nblk][p] column max partials (mirror B)
    float* cs;       // [nblk][p] column sum partials (mirror B)
    float* colstat;  // [2][p]
    int nblk;
};
hipError_t launch_loss_fwd(const float* X, const float* A, const float* B, int L, int N, int p,
                           const GradWork& w, float* loss_dev, hipStream_t st);
hipError_t launch_loss_bwd(const float* X, const float* A, const float* B, int L, int N, int p,
                           const float* grad_out, const GradWork& w, float* gA, float* gB,
                           hipStream_t st);
hipError_t launch_mirror_A(float* A, const float* gA, int p, int N, float eta, hipStream_t st);
hipError_t launch_mirror_B(float* B, const float* gB, int N, int p, float eta, const GradWork& w,
                           hipStream_t st);

// Raise a kernel's dynamic LDS limit (needed above 64 KiB); idempotent.
inline void set_max_lds(const void* fn, int bytes) {
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// Number of workgroups used by the autograd kernels for an N-pixel image.
int grad_blocks(int N);

// Dynamic LDS bytes of a pass kernel (kind 0: A-pass, 1: B-pass, 2: closing).
size_t pass_lds_bytes(int PP, int R, int L, int kind);
// Dynamic LDS bytes the launchers give a pass kernel for geometry g (with its
// double-buffer and operand-pitch choices); kind as above.
size_t launch_lds_bytes(const Geom& g, int kind);
constexpr size_t kMaxLdsBytes = 160 * 1024;

// Geometry helpers (edaa_kernels.hip).
// Whether chunks of R runs have compiled kernels that fit L bands (LDS of all
// three pass kernels and the accumulators' band capacity).
bool runs_fit(int p, int R, int L);
// Whether the B-pass (xb_fits) or the A-pass (xa_fits) of a chunk of R runs
// can keep bf16 X tiles in bf16 and run on the bf16 matrix cores (L and LDS
// limits).
bool xb_fits(int p, int R, int L);
bool xa_fits(int p, int R, int L);
// Whether the float32-X B-pass (k_bpass_xs) or A-pass (k_apass_xs, xas_chunk)
// on the bf16 matrix cores fits.
bool xs_fits(int p, int R, int L);
bool xas_fits(int p, int R, int L);
// Default runs per chunk for M runs (1 when M = 1 or when nothing else fits).
int runs_per_chunk(int p, int M, int L);
// Geometry with R runs per chunk and npg pixel groups (0: defaults).
Geom make_geom(int L, int N, int M, int p, int R = 0, int npg = 0);
// Whether the pass kernels can run geometry g.
bool geom_valid(const Geom& g);

}  // namespace edaa
