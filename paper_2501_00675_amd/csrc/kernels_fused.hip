// Whole-graph sweep with the level held in LDS, for graphs whose widest level
// fits on chip (narrow CoS graphs: low diagram orders, paper Sec. III notes
// that small levels leave most of a window idle and suggests processing
// several small levels in one block).
//
// One workgroup of 16 wavefronts evaluates every level for a tile of 64*K
// samples (K per lane).  The values of the current level sit in LDS as
// [node][64K]; wave w owns rows [w*RMAX, (w+1)*RMAX), computes them into
// registers, the group synchronises, and the rows overwrite the previous level
// in place.  The per-sample maximum of the rescaled binary32 path is reduced
// across the 16 waves in LDS, so no global atomics are needed.  HBM traffic is
// x, the edge records and the output only.
//
// Arithmetic is identical to the streamed kernels (same factor, same segment
// order, same rescale, and a final-node reduction in the same quarters of 64
// edges combined in the same order), so both give bit-identical results.
#include <atomic>

#include "kernels_common.h"

namespace cosdag {
namespace {

constexpr int kFusedWaves = 16;
constexpr int kFusedThreads = kFusedWaves * kWave;
constexpr size_t kLdsBytes = 160 * 1024;  // LDS per CU on gfx950
constexpr int kQuarter = kFinalChunk / 4;
constexpr int kChunk = kEdgePad;          // records fetched per step (the edge array is padded)
constexpr int kMaxRows = 40;              // rows per wave supported (widest level 640)

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

struct FusedLayout {
    size_t off_red = 0, off_part = 0, total = 0;
    int32_t n_quarters = 0;
};

FusedLayout fused_layout(const Graph &g, size_t elem, bool rescale, int K) {
    FusedLayout f;
    const int64_t tile = static_cast<int64_t>(kWave) * K;
    f.n_quarters = static_cast<int32_t>((g.levels.back().n_edges + kQuarter - 1) / kQuarter);
    size_t off = static_cast<size_t>(round_up(g.max_width * tile * static_cast<int64_t>(elem), 16));
    f.off_red = off;
    if (rescale)
        off += kFusedWaves * tile * sizeof(uint32_t);
    f.off_part = off;
    off += static_cast<size_t>(f.n_quarters) * tile * sizeof(double);
    f.total = std::max<size_t>(off, 16);
    return f;
}

// Rows-per-wave variants; a (K, RMAX) pair is built only when its register
// accumulators (K * RMAX values per lane) take at most 48 dwords, which keeps
// every variant free of register spills at 1024 threads per group.
constexpr int kRowVariants[] = {2, 4, 8, 16, 24, kMaxRows};
constexpr bool acc_fits(size_t elem, int K, int rmax) { return K * rmax * static_cast<int>(elem / 4) <= 48; }

int rows_variant(int64_t rows) {
    for (int r : kRowVariants)
        if (rows <= r)
            return r;
    return 0;
}

// Largest samples-per-lane K in {4, 2, 1} whose accumulators fit in registers
// and whose layout fits in LDS (0: the graph does not fit the fused plan).
int fused_k(const Graph &g, cos_precision p) {
    const int rmax = rows_variant((g.max_width + kFusedWaves - 1) / kFusedWaves);
    if (rmax == 0)
        return 0;
    const size_t elem = p == COS_FP64 ? sizeof(double) : sizeof(float);
    for (int K : {4, 2, 1})
        if (acc_fits(elem, K, rmax) && fused_layout(g, elem, p == COS_FP32_RESCALED, K).total <= kLdsBytes)
            return K;
    return 0;
}

template <typename T, int K, int RMAX, bool RESCALE>
__global__ __launch_bounds__(kFusedThreads) void fused_sweep_kernel(
    const int32_t *__restrict__ row_ptr, const EdgeRec *__restrict__ edges, const LevelDev *__restrict__ levels,
    int32_t L, const double *__restrict__ x, int64_t S, uint32_t off_red, uint32_t off_part,
    double *__restrict__ out, int32_t *__restrict__ out_exp) {
    constexpr int kTile = kWave * K;
    extern __shared__ __align__(16) unsigned char lds[];
    T *vals = reinterpret_cast<T *>(lds);
    uint32_t *red = reinterpret_cast<uint32_t *>(lds + off_red);
    double *part = reinterpret_cast<double *>(lds + off_part);

    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t tbase = static_cast<int64_t>(blockIdx.x) * kTile;
    double x0[K], x1[K], x2[K], q[K];
    int esh[K], E[K];  // e_{l-1} and sum of e_1 .. e_{L-2} for this lane's samples
#pragma unroll
    for (int m = 0; m < K; ++m) {
        const int64_t s = tbase + lane + kWave * m;
        const bool in = s < S;
        x0[m] = in ? x[s] : 0.0;
        x1[m] = in ? x[S + s] : 0.0;
        x2[m] = in ? x[2 * S + s] : 0.0;
        q[m] = __builtin_fma(x2[m], x2[m], __builtin_fma(x1[m], x1[m], x0[m] * x0[m]));
        esh[m] = 0;
        E[m] = 0;
    }

    for (int l = 1; l < L; ++l) {
        const LevelDev lv = levels[l - 1];
        const int32_t *rp = row_ptr + lv.rp_begin;
        const int jb = min(wave * RMAX, lv.w_dst);
        const int nb = min(jb + RMAX, lv.w_dst) - jb;
        // lane i (i <= nb) holds the start of row jb + i: one load per wave and level
        const int rpl = lane <= nb ? rp[jb + lane] : 0;
        T acc[RMAX][K];
        uint32_t lmax[K];
#pragma unroll
        for (int m = 0; m < K; ++m)
            lmax[m] = 0u;
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
#pragma unroll
            for (int m = 0; m < K; ++m)
                acc[r][m] = T(0);
            if (r < nb) {
                const int e1 = __builtin_amdgcn_readlane(rpl, r + 1);
                for (int e = __builtin_amdgcn_readlane(rpl, r); e < e1; e += kChunk) {
                    const int n = min(kChunk, e1 - e);
                    EdgeRec rr[kChunk];
#pragma unroll
                    for (int u = 0; u < kChunk; ++u)
                        rr[u] = edges[e + u];
                    // records past the row name rows < widest level: the
                    // unused LDS reads stay in bounds
                    T v[kChunk][K];
#pragma unroll
                    for (int u = 0; u < kChunk; ++u)
#pragma unroll
                        for (int m = 0; m < K; ++m)
                            v[u][m] = (l == 1) ? T(1) : vals[rr[u].src * kTile + lane + kWave * m];
#pragma unroll
                    for (int u = 0; u < kChunk; ++u)
                        if (u < n)
#pragma unroll
                            for (int m = 0; m < K; ++m)
                                acc[r][m] = fma_t(edge_factor<T>(rr[u], x0[m], x1[m], x2[m], q[m]), v[u][m], acc[r][m]);
                }
                if constexpr (RESCALE) {
#pragma unroll
                    for (int m = 0; m < K; ++m) {
                        acc[r][m] = scale_pow2(acc[r][m], esh[m]);
                        lmax[m] = max(lmax[m], abs_bits(acc[r][m]));
                    }
                }
            }
        }
        __syncthreads();  // every wave has finished reading level l-1
#pragma unroll
        for (int r = 0; r < RMAX; ++r)
            if (r < nb)
#pragma unroll
                for (int m = 0; m < K; ++m)
                    vals[(jb + r) * kTile + lane + kWave * m] = acc[r][m];
        if constexpr (RESCALE)
#pragma unroll
            for (int m = 0; m < K; ++m)
                red[wave * kTile + lane + kWave * m] = lmax[m];
        __syncthreads();  // level l complete
        if constexpr (RESCALE) {
            if (l <= L - 2) {
#pragma unroll
                for (int m = 0; m < K; ++m) {
                    uint32_t mx = 0u;
#pragma unroll
                    for (int w = 0; w < kFusedWaves; ++w)
                        mx = max(mx, red[w * kTile + lane + kWave * m]);
                    esh[m] = ilogb_bits(mx);
                    E[m] += esh[m];
                }
            }
        }
    }

    // final node: quarter p holds edges [64p, 64p + 64) of the last level
    const LevelDev lf = levels[L - 1];
    const int nq = (lf.n_edges + kQuarter - 1) / kQuarter;
    for (int p = wave; p < nq; p += kFusedWaves) {
        double acc[K];
#pragma unroll
        for (int m = 0; m < K; ++m)
            acc[m] = 0.0;
        const int e_lo = p * kQuarter;
        const int e_hi = min(e_lo + kQuarter, lf.n_edges);
        for (int e = e_lo; e < e_hi; e += kChunk) {
            const int n = min(kChunk, e_hi - e);
            EdgeRec rr[kChunk];
#pragma unroll
            for (int u = 0; u < kChunk; ++u)
                rr[u] = edges[lf.e_begin + e + u];
            double v[kChunk][K];
#pragma unroll
            for (int u = 0; u < kChunk; ++u)
#pragma unroll
                for (int m = 0; m < K; ++m)
                    v[u][m] = (L == 1) ? 1.0 : static_cast<double>(vals[rr[u].src * kTile + lane + kWave * m]);
#pragma unroll
            for (int u = 0; u < kChunk; ++u)
                if (u < n)
#pragma unroll
                    for (int m = 0; m < K; ++m)
                        acc[m] = __builtin_fma(edge_factor64(rr[u], x0[m], x1[m], x2[m], q[m]), v[u][m], acc[m]);
        }
#pragma unroll
        for (int m = 0; m < K; ++m)
            part[p * kTile + lane + kWave * m] = acc[m];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const int64_t s = tbase + lane + kWave * m;
            if (s >= S)
                continue;
            double tot = 0.0;
            const int nc = (nq + 3) / 4;
            for (int c = 0; c < nc; ++c) {
                double cs = part[(4 * c) * kTile + lane + kWave * m];
#pragma unroll
                for (int i = 1; i < 4; ++i)
                    cs += (4 * c + i < nq) ? part[(4 * c + i) * kTile + lane + kWave * m] : 0.0;
                tot += cs;
            }
            if (out_exp) {
                out[s] = tot;
                out_exp[s] = E[m];
            } else {
                out[s] = ldexp(tot, E[m]);
            }
        }
    }
}

template <typename T, int K, int RMAX, bool RESCALE>
hipError_t launch_fused_t(const Graph &g, const FusedLayout &f, const double *x, int64_t S, double *out,
                          int32_t *out_exp, hipStream_t s) {
    auto kern = fused_sweep_kernel<T, K, RMAX, RESCALE>;
    static std::atomic<bool> attr_set{false};  // per instantiation; setting it twice is harmless
    if (!attr_set.load(std::memory_order_acquire)) {
        hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsBytes));
        if (err != hipSuccess)
            return err;
        attr_set.store(true, std::memory_order_release);
    }
    const dim3 grid(static_cast<unsigned>((S + kWave * K - 1) / (kWave * K)));
    TimedLaunch tl(KK_FUSED, s);
    hipLaunchKernelGGL(kern, grid, dim3(kFusedThreads), f.total, s, g.d_row_ptr, g.d_edges, g.d_levels, g.L, x, S,
                       static_cast<uint32_t>(f.off_red), static_cast<uint32_t>(f.off_part), out, out_exp);
    return hipGetLastError();
}

template <typename T, int K, int RMAX, bool RESCALE>
hipError_t launch_if_fits(const Graph &g, const double *x, int64_t S, double *out, int32_t *out_exp, hipStream_t s) {
    if constexpr (acc_fits(sizeof(T), K, RMAX))
        return launch_fused_t<T, K, RMAX, RESCALE>(g, fused_layout(g, sizeof(T), RESCALE, K), x, S, out, out_exp, s);
    else
        return hipErrorInvalidValue;  // never selected by fused_k
}

template <typename T, int K, bool RESCALE>
hipError_t dispatch_rows(const Graph &g, const double *x, int64_t S, double *out, int32_t *out_exp, hipStream_t s) {
    switch (rows_variant((g.max_width + kFusedWaves - 1) / kFusedWaves)) {
    case 2:
        return launch_if_fits<T, K, 2, RESCALE>(g, x, S, out, out_exp, s);
    case 4:
        return launch_if_fits<T, K, 4, RESCALE>(g, x, S, out, out_exp, s);
    case 8:
        return launch_if_fits<T, K, 8, RESCALE>(g, x, S, out, out_exp, s);
    case 16:
        return launch_if_fits<T, K, 16, RESCALE>(g, x, S, out, out_exp, s);
    case 24:
        return launch_if_fits<T, K, 24, RESCALE>(g, x, S, out, out_exp, s);
    case kMaxRows:
        return launch_if_fits<T, K, kMaxRows, RESCALE>(g, x, S, out, out_exp, s);
    }
    return hipErrorInvalidValue;
}

template <typename T, bool RESCALE>
hipError_t dispatch_k(const Graph &g, int K, const double *x, int64_t S, double *out, int32_t *out_exp,
                      hipStream_t s) {
    if (K == 4)
        return dispatch_rows<T, 4, RESCALE>(g, x, S, out, out_exp, s);
    if (K == 2)
        return dispatch_rows<T, 2, RESCALE>(g, x, S, out, out_exp, s);
    return dispatch_rows<T, 1, RESCALE>(g, x, S, out, out_exp, s);
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
        return dispatch_k<double, false>(g, K, x, S, out, out_exp, s);
    case COS_FP32_RESCALED:
        return dispatch_k<float, true>(g, K, x, S, out, out_exp, s);
    case COS_FP32:
        return dispatch_k<float, false>(g, K, x, S, out, out_exp, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace cosdag
