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
#include <atomic>

#include "fused_plan.h"
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

template <typename T, int K, int RMAX, bool RESCALE, int KIND>
hipError_t launch_fused_t(const Graph &g, const double *x, int64_t S, double *out, int32_t *out_exp, hipStream_t s) {
    if constexpr (!acc_fits(sizeof(T), K, RMAX)) {
        return hipErrorInvalidValue;  // never selected by fused_k
    } else {
        auto kern = fused_sweep_kernel<T, K, RMAX, RESCALE, KIND>;
        static std::atomic<bool> attr_set{false};  // per instantiation; setting it twice is harmless
        if (!attr_set.load(std::memory_order_acquire)) {
            hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 static_cast<int>(kLdsBytes));
            if (err != hipSuccess)
                return err;
            attr_set.store(true, std::memory_order_release);
        }
        const FusedLayout f = fused_layout(g, sizeof(T), RESCALE, K);
        const FusedGraph G{g.d_row_ptr, g.d_edges, g.d_edges32, g.d_edgesL, g.d_levels, g.L, x, S, out, out_exp};
        const dim3 grid(static_cast<unsigned>((S + kWave * K - 1) / (kWave * K)));
        TimedLaunch tl(KK_FUSED, s);
        hipLaunchKernelGGL(kern, grid, dim3(kFusedThreads), f.total, s, G, static_cast<uint32_t>(f.off_red),
                           static_cast<uint32_t>(f.off_part));
        return hipGetLastError();
    }
}

template <typename T, int K, bool RESCALE, int KIND>
hipError_t dispatch_rows(const Graph &g, const double *x, int64_t S, double *out, int32_t *out_exp, hipStream_t s) {
    switch (rows_variant((g.max_width + kFusedWaves - 1) / kFusedWaves)) {
    case 2:
        return launch_fused_t<T, K, 2, RESCALE, KIND>(g, x, S, out, out_exp, s);
    case 4:
        return launch_fused_t<T, K, 4, RESCALE, KIND>(g, x, S, out, out_exp, s);
    case 8:
        return launch_fused_t<T, K, 8, RESCALE, KIND>(g, x, S, out, out_exp, s);
    case 16:
        return launch_fused_t<T, K, 16, RESCALE, KIND>(g, x, S, out, out_exp, s);
    case 24:
        return launch_fused_t<T, K, 24, RESCALE, KIND>(g, x, S, out, out_exp, s);
    case kMaxRows:
        return launch_fused_t<T, K, kMaxRows, RESCALE, KIND>(g, x, S, out, out_exp, s);
    }
    return hipErrorInvalidValue;
}

template <typename T, bool RESCALE, int KIND>
hipError_t dispatch_k(const Graph &g, int K, const double *x, int64_t S, double *out, int32_t *out_exp,
                      hipStream_t s) {
    if (K == 4)
        return dispatch_rows<T, 4, RESCALE, KIND>(g, x, S, out, out_exp, s);
    if (K == 2)
        return dispatch_rows<T, 2, RESCALE, KIND>(g, x, S, out, out_exp, s);
    return dispatch_rows<T, 1, RESCALE, KIND>(g, x, S, out, out_exp, s);
}

template <typename T, bool RESCALE>
hipError_t dispatch_kind(const Graph &g, int K, const double *x, int64_t S, double *out, int32_t *out_exp,
                         hipStream_t s) {
    if (g.kind == FK_LOOKUP)
        return dispatch_k<T, RESCALE, FK_LOOKUP>(g, K, x, S, out, out_exp, s);
    return dispatch_k<T, RESCALE, FK_RATIONAL>(g, K, x, S, out, out_exp, s);
}

}  // namespace

bool fused_fits(const Graph &g, cos_precision p) { return fused_k(g, p) > 0; }

hipError_t launch_fused(const Graph &g, cos_precision p, const double *x, int64_t S, double *out, int32_t *out_exp,
                        hipStream_t s) {
    const int K = fused_k(g, p);
    if (K == 0)
        return hipErrorInvalidValue;
    switch (p) {
    case COS_FP64:
        return dispatch_kind<double, false>(g, K, x, S, out, out_exp, s);
    case COS_FP32_RESCALED:
        return dispatch_kind<float, true>(g, K, x, S, out, out_exp, s);
    case COS_FP32:
        return dispatch_kind<float, false>(g, K, x, S, out, out_exp, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace cosdag
