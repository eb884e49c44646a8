// Launchers of the pass kernels for one number of endmembers p.  This unit is
// compiled once per p with -DEDAA_INST_P=<p> (1 <= p <= kMaxP), so the
// instantiations of the different p build in parallel; each exports the function
// edaa::ops_p<p>() that returns the table pass_ops(p) hands out.
#include "edaa_device.h"

#include <algorithm>
#include <cstdlib>

#ifndef EDAA_INST_P
#error "compile with -DEDAA_INST_P=<p>"
#endif

namespace edaa {
namespace {

constexpr int PP = EDAA_INST_P;
static_assert(PP >= 1 && PP <= kMaxP, "EDAA_INST_P out of range");

template <int R>
struct Kernels {
    static hipError_t apass(const Geom& g, const State& s, int K1, hipStream_t st) {
        if constexpr (xas_chunk(PP, R)) {   // xas_fits: the float32-X A-pass
            if ((s.x_mfma & 2) && !s.x_bf16) {
                const bool gf = (size_t)xa_lds(PP, R, g.L, 1).total <= kMaxLdsBytes;
                const size_t lds = xa_lds(PP, R, g.L, gf ? 1 : 0).total;
                set_max_lds((const void*)k_apass_xs<PP, R>, (int)lds);
                hipLaunchKernelGGL((k_apass_xs<PP, R>), dim3(g.npg * g.nqc), dim3(64 * xa_waves(PP)), lds, st, g,
                                   s, (const float*)s.E, K1);
                return hipGetLastError();
            }
        }
        if constexpr (PP <= 12) {          // xa_fits: the bf16 A-pass up to p = 12
            if (s.x_mfma & 2) {
                const bool gf = (size_t)xa_lds(PP, R, g.L, 1).total <= kMaxLdsBytes;
                const size_t lds = xa_lds(PP, R, g.L, gf ? 1 : 0).total;
                set_max_lds((const void*)k_apass_xb<PP, R>, (int)lds);
                hipLaunchKernelGGL((k_apass_xb<PP, R>), dim3(g.npg * g.nqc), dim3(64 * xa_waves(PP)), lds, st, g,
                                   s, (const float*)s.E, K1);
                return hipGetLastError();
            }
        }
        const size_t lds = (size_t)pass_lds(PP, R, g.L, g.dbuf, g.ecs, g.gf).total * sizeof(float);
        set_max_lds((const void*)k_apass<PP, R>, (int)lds);
        hipLaunchKernelGGL((k_apass<PP, R>), dim3(g.npg * g.nqc), dim3(64 * apass_waves(PP)), lds, st, g, s,
                           (const float*)s.E, K1);
        return hipGetLastError();
    }
    static hipError_t bpass(const Geom& g, const State& s, int mode, const RunInit& ri, hipStream_t st) {
        if ((s.x_mfma & 1) && !s.x_bf16) {       // float32 X, three-term bf16 products
            const size_t lds = xs_lds(PP, R, g.L).total;
            if (mode == kModeStep) {
                set_max_lds((const void*)k_bpass_xs<PP, R, true>, (int)lds);
                hipLaunchKernelGGL((k_bpass_xs<PP, R, true>), dim3(g.npg * g.nqc), dim3(64 * kBpassWaves), lds, st, g,
                                   s, (const float*)s.W, mode, ri);
            } else {
                set_max_lds((const void*)k_bpass_xs<PP, R, false>, (int)lds);
                hipLaunchKernelGGL((k_bpass_xs<PP, R, false>), dim3(g.npg * g.nqc), dim3(64 * kBpassWaves), lds, st,
                                   g, s, (const float*)s.W, mode, ri);
            }
            return hipGetLastError();
        }
        if (s.x_mfma & 1) {
            const size_t lds = xb_lds(PP, R, g.L).total;
            if (mode == kModeStep) {
                set_max_lds((const void*)k_bpass_xb<PP, R, true>, (int)lds);
                hipLaunchKernelGGL((k_bpass_xb<PP, R, true>), dim3(g.npg * g.nqc), dim3(64 * kBpassWaves), lds, st, g,
                                   s, (const float*)s.W, mode, ri);
            } else {
                set_max_lds((const void*)k_bpass_xb<PP, R, false>, (int)lds);
                hipLaunchKernelGGL((k_bpass_xb<PP, R, false>), dim3(g.npg * g.nqc), dim3(64 * kBpassWaves), lds, st,
                                   g, s, (const float*)s.W, mode, ri);
            }
            return hipGetLastError();
        }
        const size_t lds = (size_t)pass_lds(PP, R, g.L, g.dbuf, g.ecs, g.gf).total * sizeof(float);
        if (mode == kModeStep) {
            set_max_lds((const void*)k_bpass<PP, R, true>, (int)lds);
            hipLaunchKernelGGL((k_bpass<PP, R, true>), dim3(g.npg * g.nqc), dim3(64 * kBpassWaves), lds, st, g, s,
                               (const float*)s.W, mode, ri);
        } else {
            set_max_lds((const void*)k_bpass<PP, R, false>, (int)lds);
            hipLaunchKernelGGL((k_bpass<PP, R, false>), dim3(g.npg * g.nqc), dim3(64 * kBpassWaves), lds, st, g, s,
                               (const float*)s.W, mode, ri);
        }
        return hipGetLastError();
    }
    static hipError_t close(const Geom& g, const State& s, hipStream_t st) {
        const size_t lds = pass_lds_bytes(PP, R, g.L, 2);
        set_max_lds((const void*)k_close<PP, R>, (int)lds);
        hipLaunchKernelGGL((k_close<PP, R>), dim3(g.npg * g.nqc), dim3(64 * close_waves(R)), lds, st, g, s,
                           (const float*)s.E);
        return hipGetLastError();
    }
    static hipError_t reduce_b(const Geom& g, const State& s, int need_w, hipStream_t st) {
        // several rows per workgroup (about one workgroup per CU) when there
        // are rows enough and each thread can hold the partials of its slice
        // (red_slices); otherwise one row per workgroup
        // EDAA_REDUCE_ROWS (1 .. kRedRows) overrides the rows per workgroup
        const int QC = PP * R, S = std::max(1, std::min(kRedThreads / QC, (g.npg + 3) / 4));
        const char* env = std::getenv("EDAA_REDUCE_ROWS");
        const int want = env ? std::atoi(env) : 0;
        const int nl = want > 0 ? std::min(kRedRows, want) : std::min(kRedRows, std::max(1, g.L * g.nqc / 256));
        const int held = (g.npg + S - 1) / S;   // partials per thread
        const dim3 grid((g.L + nl - 1) / nl, g.nqc);
        if (nl > 1 && held <= 4) {
            hipLaunchKernelGGL((k_reduce_b_f<PP, R, 4>), grid, dim3(kRedThreads), 0, st, g, s, need_w, nl);
        } else if (nl > 1 && held <= 8) {
            hipLaunchKernelGGL((k_reduce_b_f<PP, R, 8>), grid, dim3(kRedThreads), 0, st, g, s, need_w, nl);
        } else if (nl > 1 && held <= kRedHeld) {
            hipLaunchKernelGGL((k_reduce_b_f<PP, R, kRedHeld>), grid, dim3(kRedThreads), 0, st, g, s, need_w, nl);
        } else {
            hipLaunchKernelGGL((k_reduce_b<PP, R>), dim3(g.L, g.nqc), dim3(kRedThreads), 0, st, g, s, need_w);
        }
        return hipGetLastError();
    }
    static hipError_t reduce_aa(const Geom& g, const State& s, int t, hipStream_t st) {
        hipLaunchKernelGGL((k_reduce_aa<PP, R>), dim3(g.M, aa_blocks(PP)), dim3(kThreads), 0, st, g, s, t);
        return hipGetLastError();
    }
    static hipError_t reduce_a(const Geom& g, const State& s, int t, hipStream_t st) {
        hipError_t e = reduce_aa(g, s, t, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_reduce_a<PP, R>), dim3(g.L, g.nqc), dim3(kRedThreads), 0, st, g, s, t);
        return hipGetLastError();
    }
};

// g.R -> the instantiation for that chunk size (run_choices(PP) only).
template <typename F>
hipError_t with_runs(int R, F&& f) {
    switch (R) {
#define EDAA_R_CASE(RV)                                                  \
    case RV:                                                             \
        if constexpr (has_runs(PP, RV)) return f(Kernels<RV>());        \
        break;
        EDAA_R_CASE(1) EDAA_R_CASE(2) EDAA_R_CASE(4) EDAA_R_CASE(8) EDAA_R_CASE(12) EDAA_R_CASE(16)
        EDAA_R_CASE(20)
#undef EDAA_R_CASE
        default: break;
    }
    return hipErrorInvalidValue;
}

hipError_t op_apass(const Geom& g, const State& s, int K1, hipStream_t st) {
    return with_runs(g.R, [&](auto k) { return decltype(k)::apass(g, s, K1, st); });
}
hipError_t op_bpass(const Geom& g, const State& s, int mode, const RunInit& ri, hipStream_t st) {
    return with_runs(g.R, [&](auto k) { return decltype(k)::bpass(g, s, mode, ri, st); });
}
hipError_t op_close(const Geom& g, const State& s, hipStream_t st) {
    return with_runs(g.R, [&](auto k) { return decltype(k)::close(g, s, st); });
}
hipError_t op_reduce_b(const Geom& g, const State& s, int need_w, hipStream_t st) {
    return with_runs(g.R, [&](auto k) { return decltype(k)::reduce_b(g, s, need_w, st); });
}
hipError_t op_reduce_a(const Geom& g, const State& s, int t, hipStream_t st) {
    return with_runs(g.R, [&](auto k) { return decltype(k)::reduce_a(g, s, t, st); });
}
hipError_t op_reduce_aa(const Geom& g, const State& s, int t, hipStream_t st) {
    return with_runs(g.R, [&](auto k) { return decltype(k)::reduce_aa(g, s, t, st); });
}

hipError_t op_eta(const Geom& g, const State& s, const RunInit& ri, hipStream_t st) {
    hipLaunchKernelGGL((k_eta<PP>), dim3(g.M), dim3(kThreads), 0, st, g, s, ri);
    return hipGetLastError();
}

hipError_t op_finalize(const Geom& g, const State& s, float* B_out, float* E_out, int cosine, hipStream_t st) {
    const size_t n = (size_t)g.N * PP;
    const int bx = (int)std::min<size_t>((n + kThreads - 1) / kThreads, 4096);
    if (B_out) hipLaunchKernelGGL((k_final_B<PP>), dim3(bx, g.M), dim3(kThreads), 0, st, g, s, B_out);
    hipLaunchKernelGGL((k_final_E<PP>), dim3(g.M), dim3(kThreads), 0, st, g, s, E_out, cosine);
    return hipGetLastError();
}

hipError_t op_multi(int kernel, const ImageJob* jobs, const int2* map, int nb, size_t lds, int arg, hipStream_t st) {
    const dim3 grid(nb), block(kThreads), rblock(kRedThreads), bblock(64 * kBpassWaves), ablock(64 * apass_waves(PP));
    switch (kernel) {
        case kMultiPrep:
            hipLaunchKernelGGL((k_prep_multi<PP>), grid, block, 0, st, jobs, map);
            break;
        case kMultiBpassInit:
            set_max_lds((const void*)k_bpass_multi<PP, 1, false>, (int)lds);
            hipLaunchKernelGGL((k_bpass_multi<PP, 1, false>), grid, bblock, lds, st, jobs, map, (int)kModeInitRng);
            break;
        case kMultiBpassStep:
            set_max_lds((const void*)k_bpass_multi<PP, 1, true>, (int)lds);
            hipLaunchKernelGGL((k_bpass_multi<PP, 1, true>), grid, bblock, lds, st, jobs, map, (int)kModeStep);
            break;
        case kMultiRedB:
            hipLaunchKernelGGL((k_reduce_b_multi<PP>), grid, rblock, 0, st, jobs, map, arg);
            break;
        case kMultiEta:
            hipLaunchKernelGGL((k_eta_multi<PP>), grid, block, 0, st, jobs, map);
            break;
        case kMultiApass:
            set_max_lds((const void*)k_apass_multi<PP, 1>, (int)lds);
            hipLaunchKernelGGL((k_apass_multi<PP, 1>), grid, ablock, lds, st, jobs, map, arg);
            break;
        case kMultiRedAA:
            hipLaunchKernelGGL((k_reduce_aa_multi<PP>), grid, block, 0, st, jobs, map, arg);
            break;
        case kMultiRedA:
            hipLaunchKernelGGL((k_reduce_a_multi<PP>), grid, rblock, 0, st, jobs, map, arg);
            break;
        case kMultiClose:
            set_max_lds((const void*)k_close_multi<PP>, (int)lds);
            hipLaunchKernelGGL((k_close_multi<PP>), grid, bblock, lds, st, jobs, map);
            break;
        case kMultiCloseReduce:
            hipLaunchKernelGGL(k_reduce_close_multi, grid, block, 0, st, jobs, map);
            break;
        case kMultiFinal:
            hipLaunchKernelGGL((k_final_multi<PP>), grid, block, 0, st, jobs, map, arg);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

#define EDAA_OPS_NAME2(P) ops_p##P
#define EDAA_OPS_NAME(P) EDAA_OPS_NAME2(P)
const PassOps* EDAA_OPS_NAME(EDAA_INST_P)();
const PassOps* EDAA_OPS_NAME(EDAA_INST_P)() {
    static const PassOps table = {op_apass,     op_bpass, op_close,    op_reduce_b, op_reduce_a,
                                  op_reduce_aa, op_eta,   op_finalize, op_multi};
    return &table;
}

}  // namespace edaa
