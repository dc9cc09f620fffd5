// Level-sweep kernels for gfx950.
//
// One launch per interior edge level l = 1..L-1 computes, for every node j of
// level l and every sample s,
//     v_l[j][s] = sum_{e into j} w_e(x_s) * v_{l-1}[src_e][s]
// (paper Sec. II.B), the edge factor w_e(x) = a_e / (1 + b_e |x - k_e|^2)
// being evaluated inside the same loop.  Stream order between the launches is
// the level barrier: a level is complete before the next one reads it
// (Sec. II.C, "Windowing").
//
// Mapping (MI355X-first, not the paper's thread-per-edge window): node values
// live as rows [node][sample] of S_pad contiguous values, the 64 lanes of a
// wavefront run along samples and every lane of a wave works on the same
// destination node and the same edge.  Edge records are therefore wave-uniform
// and come through scalar loads; each source-row read is one contiguous,
// coalesced 64-lane access; uneven in-degrees cause no divergence (the
// concern of Sec. II.C, "Graph flattening") because a whole wave follows one
// segment.  Edges of a destination are contiguous (CSR over destinations), so
// each output value is produced by exactly one lane with a fixed summation
// order: no atomics on values and bit-identical results run to run.
//
// The final node, whose in-degree is the whole of level L-1, is reduced in
// binary64 by a two-pass split reduction with a fixed combination order.
#include "cos_internal.h"

namespace cosdag {
namespace {

template <typename T>
struct EdgeOf;
template <>
struct EdgeOf<double> {
    using type = EdgeF64;
};
template <>
struct EdgeOf<float> {
    using type = EdgeF32;
};

// ilogb of a non-negative binary32 given by its bit pattern; 0, inf and NaN
// give 0 (no rescale).
__device__ __forceinline__ int ilogb_bits(uint32_t u) {
    if (u == 0u || u >= 0x7f800000u)
        return 0;
    const uint32_t ex = u >> 23;
    if (ex)
        return static_cast<int>(ex) - 127;
    return (31 - __clz(u)) - 149;  // subnormal
}

__device__ __forceinline__ double edge_factor(const EdgeF64 &e, double x0, double x1, double x2) {
    const double d0 = x0 - e.k0, d1 = x1 - e.k1, d2 = x2 - e.k2;
    const double r2 = __builtin_fma(d2, d2, __builtin_fma(d1, d1, d0 * d0));
    return e.a / __builtin_fma(e.b, r2, 1.0);
}

__device__ __forceinline__ float edge_factor(const EdgeF32 &e, float x0, float x1, float x2) {
    const float d0 = x0 - e.k0, d1 = x1 - e.k1, d2 = x2 - e.k2;
    const float r2 = __builtin_fmaf(d2, d2, __builtin_fmaf(d1, d1, d0 * d0));
    // v_rcp_f32 (1 ulp): the denominator is >= 1, far from the rcp's edge cases
    return e.a * __builtin_amdgcn_rcpf(__builtin_fmaf(e.b, r2, 1.0f));
}

__device__ __forceinline__ uint32_t abs_bits(float v) { return __float_as_uint(v) & 0x7fffffffu; }

// Interior level.  Workgroup = 4 waves; the group owns 4*ROWS consecutive
// destination rows (wave w takes rows w, w+4, ...) for one tile of 64*K
// samples; lane i of a wave handles samples tile*64K + i + 64m, m < K, so every
// load and store instruction covers 64 consecutive values of one row.
//
// FROM_ROOT: level 1, whose only source is the root (value 1).
// RESCALE:   binary32 with per-(level, sample) power-of-two scaling: the
//            accumulated sum is multiplied by 2^-e_{l-1}[s], e_{l-1}[s] being
//            ilogb of the largest |value| of level l-1 for sample s (exact
//            scaling); the largest |value| of this level is folded into
//            cur_max[s] with an integer max over bit patterns (order-free).
template <typename T, int K, int ROWS, bool FROM_ROOT, bool RESCALE>
__global__ __launch_bounds__(kBlock) void level_gather_kernel(
    const int32_t *__restrict__ row_ptr, const typename EdgeOf<T>::type *__restrict__ edges,
    int32_t w_dst, int32_t n_row_groups, const T *__restrict__ prev, T *__restrict__ cur, int64_t ld,
    const double *__restrict__ x, int64_t S, const uint32_t *__restrict__ prev_max,
    uint32_t *__restrict__ cur_max) {
    using Edge = typename EdgeOf<T>::type;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = blockIdx.x / n_row_groups;
    const int rg = blockIdx.x - tile * n_row_groups;
    const int64_t s0 = static_cast<int64_t>(tile) * (kWave * K) + lane;

    T x0[K], x1[K], x2[K];
    int esh[K];
    uint32_t lmax[K];
#pragma unroll
    for (int m = 0; m < K; ++m) {
        const int64_t s = s0 + kWave * m;
        const bool in = s < S;
        x0[m] = in ? static_cast<T>(x[s]) : T(0);
        x1[m] = in ? static_cast<T>(x[S + s]) : T(0);
        x2[m] = in ? static_cast<T>(x[2 * S + s]) : T(0);
        esh[m] = (RESCALE && prev_max) ? ilogb_bits(prev_max[s]) : 0;
        lmax[m] = 0u;
    }

    const int row0 = rg * (4 * ROWS);
#pragma unroll 1
    for (int r = 0; r < ROWS; ++r) {
        const int j = row0 + r * 4 + wave;
        if (j >= w_dst)
            break;
        const int e0 = row_ptr[j], e1 = row_ptr[j + 1];
        T acc[K];
#pragma unroll
        for (int m = 0; m < K; ++m)
            acc[m] = T(0);
#pragma unroll 2
        for (int e = e0; e < e1; ++e) {
            const Edge ed = edges[e];
            const T *srow = prev + static_cast<int64_t>(ed.src) * ld + s0;
#pragma unroll
            for (int m = 0; m < K; ++m) {
                const T v = FROM_ROOT ? T(1) : srow[kWave * m];
                acc[m] = fma(edge_factor(ed, x0[m], x1[m], x2[m]), v, acc[m]);
            }
        }
        T *crow = cur + static_cast<int64_t>(j) * ld + s0;
#pragma unroll
        for (int m = 0; m < K; ++m) {
            T z = acc[m];
            if constexpr (RESCALE) {
                z = ldexpf(z, -esh[m]);
                lmax[m] = max(lmax[m], abs_bits(z));
            }
            crow[kWave * m] = z;
        }
    }

    if constexpr (RESCALE) {
        if (cur_max) {
            __shared__ uint32_t red[4][kWave * K];
#pragma unroll
            for (int m = 0; m < K; ++m)
                red[wave][lane + kWave * m] = lmax[m];
            __syncthreads();
            for (int i = threadIdx.x; i < kWave * K; i += kBlock) {
                const uint32_t v = max(max(red[0][i], red[1][i]), max(red[2][i], red[3][i]));
                if (v)
                    atomicMax(cur_max + static_cast<int64_t>(tile) * (kWave * K) + i, v);
            }
        }
    }
}

// Final node, pass 1: block (chunk c, sample tile t) sums the edges of chunk c
// in binary64; wave w takes the w-th quarter of the chunk; the four wave sums
// are added in a fixed order and written to partial[c][s].
template <typename TV, int K, bool FROM_ROOT>
__global__ __launch_bounds__(kBlock) void final_partial_kernel(
    const EdgeF64 *__restrict__ edges, int32_t n_edges, int32_t chunk, int32_t n_chunks,
    const TV *__restrict__ prev, int64_t ld, const double *__restrict__ x, int64_t S,
    double *__restrict__ partial) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = blockIdx.x / n_chunks;
    const int c = blockIdx.x - tile * n_chunks;
    const int64_t s0 = static_cast<int64_t>(tile) * (kWave * K) + lane;
    double x0[K], x1[K], x2[K], acc[K];
#pragma unroll
    for (int m = 0; m < K; ++m) {
        const int64_t s = s0 + kWave * m;
        const bool in = s < S;
        x0[m] = in ? x[s] : 0.0;
        x1[m] = in ? x[S + s] : 0.0;
        x2[m] = in ? x[2 * S + s] : 0.0;
        acc[m] = 0.0;
    }
    const int q = (chunk + 3) / 4;
    const int c_end = min((c + 1) * chunk, n_edges);
    const int e_lo = min(c * chunk + wave * q, c_end);
    const int e_hi = min(e_lo + q, c_end);
#pragma unroll 2
    for (int e = e_lo; e < e_hi; ++e) {
        const EdgeF64 ed = edges[e];
        const TV *srow = prev + static_cast<int64_t>(ed.src) * ld + s0;
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const double v = FROM_ROOT ? 1.0 : static_cast<double>(srow[kWave * m]);
            acc[m] = __builtin_fma(edge_factor(ed, x0[m], x1[m], x2[m]), v, acc[m]);
        }
    }
    __shared__ double red[4][kWave * K];
#pragma unroll
    for (int m = 0; m < K; ++m)
        red[wave][lane + kWave * m] = acc[m];
    __syncthreads();
    const int64_t S_pad = ld;
    for (int i = threadIdx.x; i < kWave * K; i += kBlock)
        partial[static_cast<int64_t>(c) * S_pad + static_cast<int64_t>(tile) * (kWave * K) + i] =
            ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
}

// Final node, pass 2: out[s] = sum over chunks in ascending order, then the
// binary32 path's accumulated exponent E[s] = sum_{l=1}^{L-2} e_l[s] is applied
// (or returned separately).
__global__ __launch_bounds__(kBlock) void final_combine_kernel(
    const double *__restrict__ partial, int32_t n_chunks, int64_t S_pad, int64_t S,
    const uint32_t *__restrict__ maxbits, int32_t L, double *__restrict__ out, int32_t *__restrict__ out_exp) {
    const int64_t s = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (s >= S)
        return;
    double v = 0.0;
    for (int c = 0; c < n_chunks; ++c)
        v += partial[static_cast<int64_t>(c) * S_pad + s];
    int E = 0;
    if (maxbits)
        for (int l = 1; l <= L - 2; ++l)
            E += ilogb_bits(maxbits[static_cast<int64_t>(l) * S_pad + s]);
    if (out_exp) {
        out[s] = v;
        out_exp[s] = E;
    } else {
        out[s] = ldexp(v, E);
    }
}

__global__ __launch_bounds__(kBlock) void fill_u32_kernel(uint32_t *__restrict__ p, uint32_t v, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock)
        p[i] = v;
}

constexpr int kRows = 4;      // rows per wave in the interior-level kernel
constexpr int kK = 2;         // samples per lane
constexpr int kFinalChunk = 256;

template <typename T, bool RESCALE>
hipError_t launch_level_t(const Graph &g, int l, const void *prev, void *cur, int64_t ld, const double *x,
                          int64_t S, const uint32_t *prev_max, uint32_t *cur_max, hipStream_t s) {
    const LevelDesc &d = g.levels[l - 1];
    const int32_t rows_per_group = 4 * kRows;
    const int32_t n_rg = static_cast<int32_t>((d.w_dst + rows_per_group - 1) / rows_per_group);
    const int64_t n_tiles = ld / (kWave * kK);
    const int64_t grid = n_tiles * n_rg;
    if (grid <= 0)
        return hipSuccess;
    if (grid > INT32_MAX)
        return hipErrorInvalidConfiguration;
    const int32_t *rp = g.d_row_ptr + d.rp_begin;
    const auto *edges = [&]() {
        if constexpr (sizeof(T) == 8)
            return g.d_e64;
        else
            return g.d_e32;
    }();
    TimedLaunch tl(KK_LEVEL, s);
    if (prev == nullptr)
        hipLaunchKernelGGL((level_gather_kernel<T, kK, kRows, true, RESCALE>), dim3(grid), dim3(kBlock), 0, s, rp,
                           edges, static_cast<int32_t>(d.w_dst), n_rg, nullptr, static_cast<T *>(cur), ld, x, S,
                           prev_max, cur_max);
    else
        hipLaunchKernelGGL((level_gather_kernel<T, kK, kRows, false, RESCALE>), dim3(grid), dim3(kBlock), 0, s, rp,
                           edges, static_cast<int32_t>(d.w_dst), n_rg, static_cast<const T *>(prev),
                           static_cast<T *>(cur), ld, x, S, prev_max, cur_max);
    return hipGetLastError();
}

}  // namespace

int32_t final_chunk_count(int64_t final_in_degree) {
    return static_cast<int32_t>(std::max<int64_t>(1, (final_in_degree + kFinalChunk - 1) / kFinalChunk));
}

hipError_t launch_level(const Graph &g, int l, cos_precision p, const void *prev, void *cur, int64_t ld,
                        const double *x, int64_t S, const uint32_t *prev_max, uint32_t *cur_max, hipStream_t s) {
    switch (p) {
    case COS_FP64:
        return launch_level_t<double, false>(g, l, prev, cur, ld, x, S, nullptr, nullptr, s);
    case COS_FP32_RESCALED:
        return launch_level_t<float, true>(g, l, prev, cur, ld, x, S, prev_max, cur_max, s);
    case COS_FP32:
        return launch_level_t<float, false>(g, l, prev, cur, ld, x, S, nullptr, nullptr, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_final(const Graph &g, cos_precision p, const void *prev, int64_t ld, const double *x, int64_t S,
                        const uint32_t *maxbits, double *partial, int32_t chunks, double *out, int32_t *out_exp,
                        hipStream_t s) {
    const LevelDesc &d = g.levels[g.L - 1];
    const int64_t n_tiles = ld / (kWave * kK);
    const EdgeF64 *edges = g.d_e64 + d.e_begin;
    const int32_t ne = static_cast<int32_t>(d.n_edges);
    {
        TimedLaunch tl(KK_FINAL_PARTIAL, s);
        const dim3 grid(static_cast<unsigned>(n_tiles * chunks));
        if (prev == nullptr)
            hipLaunchKernelGGL((final_partial_kernel<double, kK, true>), grid, dim3(kBlock), 0, s, edges, ne,
                               kFinalChunk, chunks, static_cast<const double *>(nullptr), ld, x, S, partial);
        else if (p == COS_FP64)
            hipLaunchKernelGGL((final_partial_kernel<double, kK, false>), grid, dim3(kBlock), 0, s, edges, ne,
                               kFinalChunk, chunks, static_cast<const double *>(prev), ld, x, S, partial);
        else
            hipLaunchKernelGGL((final_partial_kernel<float, kK, false>), grid, dim3(kBlock), 0, s, edges, ne,
                               kFinalChunk, chunks, static_cast<const float *>(prev), ld, x, S, partial);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess)
            return err;
    }
    TimedLaunch tl(KK_FINAL_COMBINE, s);
    const dim3 grid(static_cast<unsigned>((S + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(final_combine_kernel, grid, dim3(kBlock), 0, s, partial, chunks, ld, S,
                       p == COS_FP32_RESCALED ? maxbits : nullptr, g.L, out, out_exp);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0)
        return hipSuccess;
    TimedLaunch tl(KK_FILL, s);
    const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace cosdag
