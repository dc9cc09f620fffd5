// Whole-graph sweep with the level held in LDS, for graphs whose widest level
// fits on chip (narrow CoS graphs: low diagram orders, paper Sec. III notes
// that small levels leave most of a window idle and suggests processing
// several small levels in one block).
//
// One workgroup of 16 wavefronts evaluates every level for a tile of 64*K
// samples (K per lane); see fused_tile.  HBM traffic is x, the edge records and
// the output only.  Arithmetic is identical to the streamed kernels (same
// factor, same segment order, same rescale, and a final-node reduction in the
// same quarters of 64 edges combined in the same order), so both give
// bit-identical results.
#include <algorithm>
#include <atomic>

#include "fused_plan.h"
#include "mc_device.h"
#include "sweep_device.h"

namespace cosdag {
namespace {

template <typename T, int K, int RMAX, bool RESCALE, int KIND>
__global__ __launch_bounds__(kFusedThreads) void fused_sweep_kernel(FusedGraph G, uint32_t off_red, uint32_t off_part) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    fused_tile<T, K, RMAX, RESCALE, KIND>(G, static_cast<int64_t>(blockIdx.x) * (kWave * K), reinterpret_cast<T *>(lds),
                                    reinterpret_cast<uint32_t *>(lds + off_red),
                                    reinterpret_cast<double *>(lds + off_part), wave, lane);
}

// A whole Monte Carlo run (steps a.step0 .. a.step0 + a.n_steps - 1) of the
// walkers of one tile in one launch: each step, the tile's threads write their
// walkers' proposals to a.xp, the group sweeps them (G.x = a.xp, G.out = a.vp),
// and the same threads take the Metropolis decisions.  The per-walker
// arithmetic is that of the step-by-step kernels and of the fused sweep, so
// the chain is bit-identical to the launch-per-step run; only the launches go.
// Every thread runs every step (the barriers inside fused_tile are reached by
// the whole group); threads beyond the tile's walkers only take part in the
// sweep.
template <typename T, int K, int RMAX, bool RESCALE>
__global__ __launch_bounds__(kFusedThreads) void mc_fused_kernel(FusedGraph G, uint32_t off_red, uint32_t off_part,
                                                                 McArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t tbase = static_cast<int64_t>(blockIdx.x) * (kWave * K);
    const int64_t c = tbase + threadIdx.x;
    const bool mine = threadIdx.x < kWave * K && c < a.C;
    for (int64_t t = a.step0; t < a.step0 + a.n_steps; ++t) {
        if (mine)
            mc_propose(a.x, a.xp, a.C, c, t, a.seed, a.sigma);
        __syncthreads();  // the tile's proposals are written
        fused_tile<T, K, RMAX, RESCALE, FK_RATIONAL>(G, tbase, reinterpret_cast<T *>(lds),
                                                     reinterpret_cast<uint32_t *>(lds + off_red),
                                                     reinterpret_cast<double *>(lds + off_part), wave, lane);
        // fused_tile ends with a group barrier: the tile's values V(x') are written
        if (mine)
            mc_accept(a.x, a.v, a.xp, a.vp, a.C, c, t, a.seed, a.accepted, a.acc);
    }
}

template <typename Kern>
hipError_t allow_full_lds(Kern kern, std::atomic<bool> &attr_set) {
    if (!attr_set.load(std::memory_order_acquire)) {
        const hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   static_cast<int>(kLdsBytes));
        if (err != hipSuccess)
            return err;
        attr_set.store(true, std::memory_order_release);  // per instantiation; setting it twice is harmless
    }
    return hipSuccess;
}

// mc: NULL for a sweep of x into out; else a whole walker run (rational factors).
template <typename T, int K, int RMAX, bool RESCALE, int KIND>
hipError_t launch_fused_t(const Graph &g, const double *x, int64_t S, double *out, int32_t *out_exp, hipStream_t s,
                          const McArgs *mc, const float *t32, int64_t ld32) {
    if constexpr (!acc_fits(sizeof(T), K, RMAX)) {
        return hipErrorInvalidValue;  // never selected by fused_k
    } else {
        const FusedLayout f = fused_layout(g, sizeof(T), RESCALE, K);
        const dim3 grid(static_cast<unsigned>((S + kWave * K - 1) / (kWave * K)));
        if (mc) {
            if constexpr (KIND != FK_RATIONAL) {
                return hipErrorInvalidValue;
            } else {
                auto kern = mc_fused_kernel<T, K, RMAX, RESCALE>;
                static std::atomic<bool> attr_set{false};
                hipError_t err = allow_full_lds(kern, attr_set);
                if (err != hipSuccess)
                    return err;
                const FusedGraph G{g.d_row_ptr, g.d_edges, g.d_edges32, g.d_edgesL, g.d_levels, g.L,
                                   mc->xp, mc->C, mc->vp, nullptr};
                TimedLaunch tl(KK_FUSED, s);
                hipLaunchKernelGGL(kern, grid, dim3(kFusedThreads), f.total, s, G, static_cast<uint32_t>(f.off_red),
                                   static_cast<uint32_t>(f.off_part), *mc);
                return hipGetLastError();
            }
        }
        auto kern = fused_sweep_kernel<T, K, RMAX, RESCALE, KIND>;
        static std::atomic<bool> attr_set{false};
        hipError_t err = allow_full_lds(kern, attr_set);
        if (err != hipSuccess)
            return err;
        const FusedGraph G{g.d_row_ptr, g.d_edges, g.d_edges32, g.d_edgesL, g.d_levels, g.L, x, S, out, out_exp,
                           t32, ld32};
        TimedLaunch tl(KK_FUSED, s);
        hipLaunchKernelGGL(kern, grid, dim3(kFusedThreads), f.total, s, G, static_cast<uint32_t>(f.off_red),
                           static_cast<uint32_t>(f.off_part));
        return hipGetLastError();
    }
}

template <typename T, int K, bool RESCALE, int KIND>
hipError_t dispatch_rows(const Graph &g, const double *x, int64_t S, double *out, int32_t *out_exp, hipStream_t s,
                         const McArgs *mc, const float *t32, int64_t ld32) {
    switch (rows_variant((g.max_width + kFusedWaves - 1) / kFusedWaves)) {
    case 2:
        return launch_fused_t<T, K, 2, RESCALE, KIND>(g, x, S, out, out_exp, s, mc, t32, ld32);
    case 4:
        return launch_fused_t<T, K, 4, RESCALE, KIND>(g, x, S, out, out_exp, s, mc, t32, ld32);
    case 8:
        return launch_fused_t<T, K, 8, RESCALE, KIND>(g, x, S, out, out_exp, s, mc, t32, ld32);
    case 16:
        return launch_fused_t<T, K, 16, RESCALE, KIND>(g, x, S, out, out_exp, s, mc, t32, ld32);
    case 24:
        return launch_fused_t<T, K, 24, RESCALE, KIND>(g, x, S, out, out_exp, s, mc, t32, ld32);
    case kMaxRows:
        return launch_fused_t<T, K, kMaxRows, RESCALE, KIND>(g, x, S, out, out_exp, s, mc, t32, ld32);
    }
    return hipErrorInvalidValue;
}

template <typename T, bool RESCALE, int KIND>
hipError_t dispatch_k(const Graph &g, int K, const double *x, int64_t S, double *out, int32_t *out_exp,
                      hipStream_t s, const McArgs *mc, const float *t32, int64_t ld32) {
    if (K == 4)
        return dispatch_rows<T, 4, RESCALE, KIND>(g, x, S, out, out_exp, s, mc, t32, ld32);
    if (K == 2)
        return dispatch_rows<T, 2, RESCALE, KIND>(g, x, S, out, out_exp, s, mc, t32, ld32);
    return dispatch_rows<T, 1, RESCALE, KIND>(g, x, S, out, out_exp, s, mc, t32, ld32);
}

template <typename T, bool RESCALE>
hipError_t dispatch_kind(const Graph &g, int K, const double *x, int64_t S, double *out, int32_t *out_exp,
                         hipStream_t s, const McArgs *mc, const float *t32, int64_t ld32) {
    if (g.kind == FK_LOOKUP) {
        if constexpr (sizeof(T) == sizeof(float)) {
            if (t32)
                return dispatch_k<T, RESCALE, FK_LOOKUP_T32>(g, K, x, S, out, out_exp, s, mc, t32, ld32);
        }
        return dispatch_k<T, RESCALE, FK_LOOKUP>(g, K, x, S, out, out_exp, s, mc, t32, ld32);
    }
    return dispatch_k<T, RESCALE, FK_RATIONAL>(g, K, x, S, out, out_exp, s, mc, t32, ld32);
}

}  // namespace

bool fused_fits(const Graph &g, cos_precision p) { return fused_k(g, p) > 0; }

hipError_t launch_fused(const Graph &g, cos_precision p, const double *x, int64_t S, double *out, int32_t *out_exp,
                        hipStream_t s, const McArgs *mc, const float *t32, int64_t ld32) {
    int K = fused_k(g, p);
    if (K == 0)
        return hipErrorInvalidValue;
    // the walker kernel keeps its state and loop in registers: K = 4 would
    // spill (results do not depend on K)
    if (mc)
        K = std::min(K, 2);
    switch (p) {
    case COS_FP64:
        return dispatch_kind<double, false>(g, K, x, S, out, out_exp, s, mc, t32, ld32);
    case COS_FP32_RESCALED:
        return dispatch_kind<float, true>(g, K, x, S, out, out_exp, s, mc, t32, ld32);
    case COS_FP32:
        return dispatch_kind<float, false>(g, K, x, S, out, out_exp, s, mc, t32, ld32);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace cosdag
