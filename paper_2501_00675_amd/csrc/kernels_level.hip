// Level-sweep kernels for gfx950: one launch per interior level (streamed
// through HBM) and the final-node split reduction.
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
#include "sweep_device.h"

namespace cosdag {
namespace {

// Block -> (sample tile, row group).
//
// xcd_group = 1: workgroups are dispatched round-robin over the 8 XCDs (block
// b runs on XCD b % 8), each XCD with its own L2.  All row groups of one
// sample tile go to the same XCD, so the tile's source rows -- read by ~d
// destinations each -- are fetched into one L2 only.  Used when a tile's slice
// of the previous level fits in L2.  Grids are padded to a multiple of 8
// tiles; blocks of a padding tile return at once.
// xcd_group = 0: tile-major order, so the whole GPU works on one tile at a
// time and the tile's slice of the previous level stays in the memory-side
// Infinity Cache while every XCD gathers from it.
// reverse_tiles (tile-major order only): the launch walks the tiles from the
// last to the first, so that it starts on the slice the previous level wrote
// last, which is the one most likely still in the Infinity Cache.
__device__ __forceinline__ bool block_tile(int n_rg, int n_tiles, int xcd_group, int reverse_tiles, int &tile,
                                           int &rg) {
    if (xcd_group) {
        const int xcd = static_cast<int>(blockIdx.x % kXcds);
        const int local = static_cast<int>(blockIdx.x / kXcds);
        const int t = local / n_rg;
        rg = local - t * n_rg;
        tile = t * kXcds + xcd;
    } else {
        tile = static_cast<int>(blockIdx.x) / n_rg;
        rg = static_cast<int>(blockIdx.x) - tile * n_rg;
        if (reverse_tiles)
            tile = n_tiles - 1 - tile;
    }
    return tile < n_tiles;
}

// Interior level.  Workgroup = 4 waves; wave w owns ROWS consecutive
// destination rows of the group's row range, for one tile of 64*K samples
// (lane i handles samples tile*64K + i + 64m, m < K: every load and store
// covers 64 consecutive values of one row); see level_wave_rows.
// RESCALE: the rows are scaled by 2^-e_{l-1}[s], e_{l-1}[s] = ilogb of
// prev_max[s] (the largest |value| of level l-1 for sample s, times the
// headroom of level l), and the largest |value| of this level, times 2^h_next,
// is folded into cur_max[s].  V: storage type of the level values.
template <typename T, int K, int ROWS, bool FROM_ROOT, bool RESCALE, int KIND, typename V>
__global__ __launch_bounds__(kBlock) void level_gather_kernel(
    const int32_t *__restrict__ row_ptr, const typename SweepPath<T, KIND>::Rec *__restrict__ edges, int32_t w_dst, int32_t n_rg,
    int32_t n_tiles, int32_t xcd_group, int32_t reverse_tiles, const V *__restrict__ prev, V *__restrict__ cur, int64_t ld,
    const SampleElem<KIND> *__restrict__ x, int64_t S, int64_t xs, const uint32_t *__restrict__ prev_max,
    uint32_t *__restrict__ cur_max, int32_t h_next, const T *__restrict__ hub_partial) {
    int tile, rg;
    if (!block_tile(n_rg, n_tiles, xcd_group, reverse_tiles, tile, rg))
        return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t tbase = static_cast<int64_t>(tile) * (kWave * K);
    typename SweepPath<T, KIND>::template Samples<K> smp;
    smp.load(x, S, xs, tbase, lane);
    int esh[K];
    uint32_t lmax[K];
#pragma unroll
    for (int m = 0; m < K; ++m) {
        esh[m] = (RESCALE && prev_max) ? ilogb_bits(prev_max[tbase + lane + kWave * m]) : 0;
        lmax[m] = 0u;
    }
    static_assert(ROWS == kWaveRows, "level_wave_rows takes kWaveRows rows per wave");
    const int jbeg = min(rg * (4 * ROWS) + wave * ROWS, w_dst);
    const int jend = min(jbeg + ROWS, w_dst);
    level_wave_rows<T, K, FROM_ROOT, RESCALE, KIND, V>(row_ptr, edges, jbeg, jend, prev, cur, ld, tbase, lane, smp,
                                                       esh, lmax, hub_partial);
    if constexpr (RESCALE) {
        if (cur_max) {
            if (h_next)  // exact: |value| <= 2^15 and h_next <= 96
#pragma unroll
                for (int m = 0; m < K; ++m)
                    lmax[m] = abs_bits(ldexpf(__uint_as_float(lmax[m]), h_next));
            __shared__ uint32_t red[4 * kWave * K];
            fold_max<K, 4>(red, lmax, wave, lane, cur_max + tbase);
        }
    }
}

// Interior rows of high in-degree: block (sample tile, chunk c) sums chunk c
// of the level's list (kFinalChunk edges of one such row; chunks[2c],
// chunks[2c+1] its first and end edge) in the value type T, wave w the w-th
// quarter, and writes ((q0 + q1) + q2) + q3 to partial[c][s] -- hub_sum's
// chunk sums, which the level kernel then adds in ascending order.
template <typename T, int K, bool FROM_ROOT, int KIND, typename V>
__global__ __launch_bounds__(kBlock) void hub_partial_kernel(
    const int32_t *__restrict__ chunks, int32_t n_chunks, const typename SweepPath<T, KIND>::Rec *__restrict__ edges,
    const V *__restrict__ prev, int64_t ld, const SampleElem<KIND> *__restrict__ x, int64_t S, int64_t xs,
    T *__restrict__ partial) {
    using Rec = typename SweepPath<T, KIND>::Rec;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = blockIdx.x / n_chunks;
    const int c = blockIdx.x - tile * n_chunks;
    const int64_t tbase = static_cast<int64_t>(tile) * (kWave * K);
    typename SweepPath<T, KIND>::template Samples<K> smp;
    smp.load(x, S, xs, tbase, lane);
    const ConstPtr<int32_t> ch = as_const(chunks);
    const int c_lo = ch[2 * c], c_hi = ch[2 * c + 1];
    const int e_lo = min(c_lo + wave * kQuarter, c_hi);
    const int e_hi = min(e_lo + kQuarter, c_hi);
    const char *src_tile = reinterpret_cast<const char *>(prev + tbase);
    const uint32_t row_bytes = static_cast<uint32_t>(ld * sizeof(V));
    const uint32_t lane_off = static_cast<uint32_t>(lane * sizeof(V));
    T acc[K];
    edge_sum<T, K, true>(edges, e_lo, e_hi, smp, [&](const Rec &r, int m) -> T {
        if constexpr (FROM_ROOT) {
            return T(1);
        } else {
            const char *row = src_tile + static_cast<uint32_t>(r.src) * row_bytes + lane_off;
            return static_cast<T>(*reinterpret_cast<const V *>(row + m * kWave * sizeof(V)));
        }
    }, acc);
    __shared__ T red[4][kWave * K];
#pragma unroll
    for (int m = 0; m < K; ++m)
        red[wave][lane + kWave * m] = acc[m];
    __syncthreads();
    for (int i = threadIdx.x; i < kWave * K; i += kBlock)
        partial[static_cast<int64_t>(c) * ld + tbase + i] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
}

// Final node, pass 1: block (sample tile, chunk c) sums the edges of chunk c
// (kFinalChunk edges) in binary64; wave w takes the w-th quarter of the chunk;
// the four wave sums are added as ((q0 + q1) + q2) + q3 into partial[c][s].
template <typename TV, int K, bool FROM_ROOT, int KIND>
__global__ __launch_bounds__(kBlock) void final_partial_kernel(
    const typename FinalPath<KIND>::Rec *__restrict__ edges, int32_t n_edges, int32_t n_chunks, const TV *__restrict__ prev, int64_t ld,
    const double *__restrict__ x, int64_t S, int64_t xs, double *__restrict__ partial) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = blockIdx.x / n_chunks;
    const int c = blockIdx.x - tile * n_chunks;
    const int64_t tbase = static_cast<int64_t>(tile) * (kWave * K);
    typename FinalPath<KIND>::template Samples<K> smp;
    smp.load(x, S, xs, tbase, lane);
    const int c_end = min((c + 1) * kFinalChunk, n_edges);
    const int e_lo = min(c * kFinalChunk + wave * kQuarter, c_end);
    const int e_hi = min(e_lo + kQuarter, c_end);
    double acc[K];
    final_quarter<TV, K, FROM_ROOT, KIND>(edges, e_lo, e_hi, prev, ld, tbase, lane, smp, acc);
    __shared__ double red[4][kWave * K];
#pragma unroll
    for (int m = 0; m < K; ++m)
        red[wave][lane + kWave * m] = acc[m];
    __syncthreads();
    for (int i = threadIdx.x; i < kWave * K; i += kBlock)
        partial[static_cast<int64_t>(c) * ld + tbase + i] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
}

// Final node, pass 1, with level L-1 stored tile-major by the panel plan
// (values of type V): as final_partial_kernel, sample s of node src being
// prev[((s / tile) * wbuf + src) * tile + s % tile].
template <int K, typename V, int KIND>
__global__ __launch_bounds__(kBlock) void final_partial_tm_kernel(
    const typename FinalPath<KIND>::Rec *__restrict__ edges, int32_t n_edges, int32_t n_chunks,
    const V *__restrict__ prev, int64_t wbuf, int64_t ld, const double *__restrict__ x, int64_t S, int64_t xs,
    double *__restrict__ partial) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = blockIdx.x / n_chunks;
    const int c = blockIdx.x - tile * n_chunks;
    const int64_t tbase = static_cast<int64_t>(tile) * (kWave * K);
    typename FinalPath<KIND>::template Samples<K> smp;
    smp.load(x, S, xs, tbase, lane);
    const int c_end = min((c + 1) * kFinalChunk, n_edges);
    const int e_lo = min(c * kFinalChunk + wave * kQuarter, c_end);
    const int e_hi = min(e_lo + kQuarter, c_end);
    double acc[K];
    final_sum<K, true>(edges, e_lo, e_hi, smp, [&](const auto &r, int m) -> double {
        const int64_t s = tbase + lane + kWave * m;
        constexpr int kTile = panel_tile(sizeof(V));
        return static_cast<double>(prev[((s / kTile) * wbuf + r.src) * kTile + s % kTile]);
    }, acc);
    __shared__ double red[4][kWave * K];
#pragma unroll
    for (int m = 0; m < K; ++m)
        red[wave][lane + kWave * m] = acc[m];
    __syncthreads();
    for (int i = threadIdx.x; i < kWave * K; i += kBlock)
        partial[static_cast<int64_t>(c) * ld + tbase + i] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
}

__global__ __launch_bounds__(kBlock) void final_combine_kernel(
    const double *__restrict__ partial, int32_t n_chunks, int64_t S_pad, int64_t S,
    const uint32_t *__restrict__ maxbits, int32_t L, double *__restrict__ out, int32_t *__restrict__ out_exp) {
    const int64_t s = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (s < S)
        final_combine_one(partial, n_chunks, S_pad, s, maxbits, L, out, out_exp);
}

__global__ __launch_bounds__(kBlock) void fill_u32_kernel(uint32_t *__restrict__ p, uint32_t v, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock)
        p[i] = v;
}

constexpr int kRows = 8;      // consecutive rows per wave in the interior-level kernel
constexpr int kKFinal = 2;    // samples per lane (final node)
constexpr int64_t kL2Slice = int64_t(4) << 20;  // a tile slice up to this size is kept in one XCD's L2 (4 MB)
constexpr bool kAlternateTiles = true;  // tile-major launches alternate their tile order level by level

// Samples per lane of an interior level (tile = 64 K samples).  When the
// tile's slice of the previous level fits in one XCD's L2, tiles are grouped
// by XCD and the gathers hit L2: binary64 then takes K = 2 (half the registers
// of K = 4, twice the waves per SIMD), 32- and 16-bit storage the largest K in
// {4, 2} whose slice fits.  Otherwise (wide levels) K = 4 amortises each
// record over the most samples.  Measured on the mid and precision workloads.
template <typename T, typename V>
int level_k(int64_t w_src) {
    const auto fits = [&](int K) { return w_src * kWave * K * static_cast<int64_t>(sizeof(V)) <= kL2Slice; };
    if (sizeof(T) == sizeof(double))
        return fits(2) ? 2 : 4;
    if (fits(4))
        return 4;
    return fits(2) ? 2 : 4;
}

// KIND FK_LOOKUP_T32 reads the binary32 tables t32 ([n_slots][ld]) instead of x.
template <typename T, int K, bool RESCALE, int KIND, typename V>
hipError_t launch_level_k(const Graph &g, int l, const void *prev, void *cur, int64_t ld, const double *x_,
                          int64_t S, int64_t xs_, const uint32_t *prev_max, uint32_t *cur_max, int32_t h_next,
                          hipStream_t s, const float *t32, void *hub) {
    const SampleElem<KIND> *x;
    int64_t xs;
    if constexpr (KIND == FK_LOOKUP_T32) {
        x = t32;
        xs = ld;
    } else {
        x = x_;
        xs = xs_;
    }
    const LevelDesc &d = g.levels[l - 1];
    const int32_t rows_per_group = 4 * kRows;
    const int64_t n_rg = (d.w_dst + rows_per_group - 1) / rows_per_group;
    const int64_t n_tiles = ld / (kWave * K);
    const int32_t xcd_group = d.w_src * kWave * K * static_cast<int64_t>(sizeof(V)) <= kL2Slice ? 1 : 0;
    const int32_t reverse_tiles = kAlternateTiles && (l & 1) == 0 ? 1 : 0;
    const int64_t grid = (xcd_group ? round_up(n_tiles, kXcds) : n_tiles) * n_rg;
    if (grid <= 0)
        return hipSuccess;
    if (grid > INT32_MAX)
        return hipErrorInvalidConfiguration;
    const int32_t *rp = g.d_row_ptr + d.rp_begin;
    const typename SweepPath<T, KIND>::Rec *recs;
    if constexpr (KIND != FK_RATIONAL)
        recs = g.d_edgesL;
    else if constexpr (sizeof(T) == sizeof(double))
        recs = g.d_edges;
    else
        recs = g.d_edges32;
    // chunk sums of the level's rows of high in-degree, when there is room for them
    T *hub_partial = nullptr;
    if (d.n_hub_chunks > 0 && hub) {
        hub_partial = static_cast<T *>(hub);
        const int64_t hgrid = n_tiles * d.n_hub_chunks;
        if (hgrid > INT32_MAX)
            return hipErrorInvalidConfiguration;
        const int32_t *chunks = g.d_hub_chunks + 2 * d.hub_begin;
        const int32_t nc = static_cast<int32_t>(d.n_hub_chunks);
        TimedLaunch th(KK_HUB, s);
        if (prev == nullptr)
            hipLaunchKernelGGL((hub_partial_kernel<T, K, true, KIND, V>), dim3(static_cast<unsigned>(hgrid)),
                               dim3(kBlock), 0, s, chunks, nc, recs, static_cast<const V *>(nullptr), ld, x, S, xs,
                               hub_partial);
        else
            hipLaunchKernelGGL((hub_partial_kernel<T, K, false, KIND, V>), dim3(static_cast<unsigned>(hgrid)),
                               dim3(kBlock), 0, s, chunks, nc, recs, static_cast<const V *>(prev), ld, x, S, xs,
                               hub_partial);
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess)
            return err;
    }
    TimedLaunch tl(KK_LEVEL, s);
    if (prev == nullptr)
        hipLaunchKernelGGL((level_gather_kernel<T, K, kRows, true, RESCALE, KIND, V>), dim3(grid), dim3(kBlock), 0, s,
                           rp, recs, static_cast<int32_t>(d.w_dst), static_cast<int32_t>(n_rg),
                           static_cast<int32_t>(n_tiles), xcd_group, reverse_tiles, nullptr, static_cast<V *>(cur), ld,
                           x, S, xs, prev_max, cur_max, h_next, hub_partial);
    else
        hipLaunchKernelGGL((level_gather_kernel<T, K, kRows, false, RESCALE, KIND, V>), dim3(grid), dim3(kBlock), 0, s,
                           rp, recs, static_cast<int32_t>(d.w_dst), static_cast<int32_t>(n_rg),
                           static_cast<int32_t>(n_tiles), xcd_group, reverse_tiles, static_cast<const V *>(prev),
                           static_cast<V *>(cur), ld, x, S, xs, prev_max, cur_max, h_next, hub_partial);
    return hipGetLastError();
}

// LOOKUP_OK: whether the storage type takes lookup factors (binary16 does not:
// its headroom needs a bound on the factors).
template <typename T, bool RESCALE, typename V = T, bool LOOKUP_OK = true>
hipError_t launch_level_t(const Graph &g, int l, const void *prev, void *cur, int64_t ld, const double *x,
                          int64_t S, int64_t xs, const uint32_t *prev_max, uint32_t *cur_max, int32_t h_next,
                          hipStream_t s, const float *t32, void *hub) {
    const bool k2 = level_k<T, V>(g.levels[l - 1].w_src) == 2;
    if (g.kind == FK_LOOKUP) {
        if constexpr (!LOOKUP_OK) {
            return hipErrorInvalidValue;
        } else if constexpr (sizeof(T) == sizeof(float)) {
            if (t32)
                return k2 ? launch_level_k<T, 2, RESCALE, FK_LOOKUP_T32, V>(g, l, prev, cur, ld, x, S, xs, prev_max,
                                                                            cur_max, h_next, s, t32, hub)
                          : launch_level_k<T, 4, RESCALE, FK_LOOKUP_T32, V>(g, l, prev, cur, ld, x, S, xs, prev_max,
                                                                            cur_max, h_next, s, t32, hub);
        }
        if constexpr (LOOKUP_OK)
            return k2 ? launch_level_k<T, 2, RESCALE, FK_LOOKUP, V>(g, l, prev, cur, ld, x, S, xs, prev_max, cur_max,
                                                                    h_next, s, t32, hub)
                      : launch_level_k<T, 4, RESCALE, FK_LOOKUP, V>(g, l, prev, cur, ld, x, S, xs, prev_max, cur_max,
                                                                    h_next, s, t32, hub);
    }
    return k2 ? launch_level_k<T, 2, RESCALE, FK_RATIONAL, V>(g, l, prev, cur, ld, x, S, xs, prev_max, cur_max,
                                                              h_next, s, t32, hub)
              : launch_level_k<T, 4, RESCALE, FK_RATIONAL, V>(g, l, prev, cur, ld, x, S, xs, prev_max, cur_max,
                                                              h_next, s, t32, hub);
}

}  // namespace

int32_t final_chunk_count(int64_t final_in_degree) {
    return static_cast<int32_t>(std::max<int64_t>(1, (final_in_degree + kFinalChunk - 1) / kFinalChunk));
}

hipError_t launch_level(const Graph &g, int l, cos_precision p, const void *prev, void *cur, int64_t ld,
                        const double *x, int64_t S, int64_t xs, const uint32_t *prev_max, uint32_t *cur_max,
                        int32_t h_next, hipStream_t s, const float *t32, void *hub) {
    switch (p) {
    case COS_FP64:
        return launch_level_t<double, false>(g, l, prev, cur, ld, x, S, xs, nullptr, nullptr, 0, s, nullptr, hub);
    case COS_FP32_RESCALED:
        return launch_level_t<float, true>(g, l, prev, cur, ld, x, S, xs, prev_max, cur_max, 0, s, t32, hub);
    case COS_FP32:
        return launch_level_t<float, false>(g, l, prev, cur, ld, x, S, xs, nullptr, nullptr, 0, s, t32, hub);
    case COS_FP16_RESCALED:
        return launch_level_t<float, true, _Float16, false>(g, l, prev, cur, ld, x, S, xs, prev_max, cur_max, h_next,
                                                            s, nullptr, hub);
    case COS_BF16_RESCALED:
        return launch_level_t<float, true, __bf16>(g, l, prev, cur, ld, x, S, xs, prev_max, cur_max, 0, s, t32, hub);
    }
    return hipErrorInvalidValue;
}

namespace {

// t32[i][s] = fl32(x[i][s]) (nearest even) for s < S, 0 for S <= s < ld.
template <bool TILE_MAJOR>
__global__ __launch_bounds__(kBlock) void table32_kernel(const double *__restrict__ x, int64_t xs, int64_t S,
                                                         int32_t n, float *__restrict__ t32, int64_t ld) {
    constexpr int64_t kTile = panel_tile(sizeof(float));
    const int64_t total = static_cast<int64_t>(n) * ld;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < total;
         i += static_cast<int64_t>(gridDim.x) * kBlock) {
        int64_t row, s;
        if constexpr (TILE_MAJOR) {  // i = (tile * n + row) * kTile + j, sample tile * kTile + j
            const int64_t tr = i / kTile;
            row = tr % n;
            s = (tr / n) * kTile + (i - tr * kTile);
        } else {
            row = i / ld;
            s = i - row * ld;
        }
        t32[i] = s < S ? static_cast<float>(x[row * xs + s]) : 0.0f;
    }
}

}  // namespace

hipError_t launch_table32(const double *x, int64_t xs, int64_t S, int32_t n, float *t32, int64_t ld,
                          hipStream_t s, bool tile_major) {
    const int64_t total = static_cast<int64_t>(n) * ld;
    if (total <= 0)
        return hipSuccess;
    TimedLaunch tl(KK_FILL, s);
    const int64_t blocks = std::min<int64_t>((total + kBlock - 1) / kBlock, 8192);
    if (tile_major)
        hipLaunchKernelGGL(table32_kernel<true>, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, x, xs, S, n,
                           t32, ld);
    else
        hipLaunchKernelGGL(table32_kernel<false>, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, x, xs, S,
                           n, t32, ld);
    return hipGetLastError();
}

namespace {

template <int KIND>
hipError_t launch_final_partial(const Graph &g, cos_precision p, const void *prev, int64_t ld, const double *x,
                                int64_t S, int64_t xs, double *partial, int32_t chunks, hipStream_t s) {
    const LevelDesc &d = g.levels[g.L - 1];
    const int64_t n_tiles = ld / (kWave * kKFinal);
    const typename FinalPath<KIND>::Rec *edges;
    if constexpr (KIND == FK_LOOKUP)
        edges = g.d_edgesL + d.e_begin;
    else
        edges = g.d_edges + d.e_begin;
    const int32_t ne = static_cast<int32_t>(d.n_edges);
    TimedLaunch tl(KK_FINAL_PARTIAL, s);
    const dim3 grid(static_cast<unsigned>(n_tiles * chunks));
    if (prev == nullptr)
        hipLaunchKernelGGL((final_partial_kernel<double, kKFinal, true, KIND>), grid, dim3(kBlock), 0, s, edges, ne,
                           chunks, static_cast<const double *>(nullptr), ld, x, S, xs, partial);
    else if (p == COS_FP64)
        hipLaunchKernelGGL((final_partial_kernel<double, kKFinal, false, KIND>), grid, dim3(kBlock), 0, s, edges, ne,
                           chunks, static_cast<const double *>(prev), ld, x, S, xs, partial);
    else if (p == COS_BF16_RESCALED)
        hipLaunchKernelGGL((final_partial_kernel<__bf16, kKFinal, false, KIND>), grid, dim3(kBlock), 0, s, edges, ne,
                           chunks, static_cast<const __bf16 *>(prev), ld, x, S, xs, partial);
    else if (p == COS_FP16_RESCALED && KIND == FK_RATIONAL)
        hipLaunchKernelGGL((final_partial_kernel<_Float16, kKFinal, false, FK_RATIONAL>), grid, dim3(kBlock), 0, s,
                           g.d_edges + d.e_begin, ne, chunks, static_cast<const _Float16 *>(prev), ld, x, S, xs,
                           partial);
    else if (p == COS_FP16_RESCALED)
        return hipErrorInvalidValue;
    else
        hipLaunchKernelGGL((final_partial_kernel<float, kKFinal, false, KIND>), grid, dim3(kBlock), 0, s, edges, ne,
                           chunks, static_cast<const float *>(prev), ld, x, S, xs, partial);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_final(const Graph &g, cos_precision p, const void *prev, int64_t ld, const double *x, int64_t S,
                        int64_t xs, const uint32_t *maxbits, double *partial, int32_t chunks, double *out,
                        int32_t *out_exp, hipStream_t s, bool tile_major) {
    hipError_t err;
    if (tile_major) {
        if (p == COS_FP64 || prev == nullptr || (g.kind == FK_LOOKUP && value_bytes(p) != 4))
            return hipErrorInvalidValue;
        const LevelDesc &d = g.levels[g.L - 1];
        const dim3 grid(static_cast<unsigned>(ld / (kWave * kKFinal) * chunks));
        const EdgeRec *e = g.d_edges + d.e_begin;
        const int32_t ne = static_cast<int32_t>(d.n_edges);
        TimedLaunch tl(KK_FINAL_PARTIAL, s);
        if (g.kind == FK_LOOKUP)
            hipLaunchKernelGGL((final_partial_tm_kernel<kKFinal, float, FK_LOOKUP>), grid, dim3(kBlock), 0, s,
                               g.d_edgesL + d.e_begin, ne, chunks, static_cast<const float *>(prev), g.max_width, ld,
                               x, S, xs, partial);
        else if (p == COS_FP16_RESCALED)
            hipLaunchKernelGGL((final_partial_tm_kernel<kKFinal, _Float16, FK_RATIONAL>), grid, dim3(kBlock), 0, s, e,
                               ne, chunks, static_cast<const _Float16 *>(prev), g.max_width, ld, x, S, xs, partial);
        else if (p == COS_BF16_RESCALED)
            hipLaunchKernelGGL((final_partial_tm_kernel<kKFinal, __bf16, FK_RATIONAL>), grid, dim3(kBlock), 0, s, e,
                               ne, chunks, static_cast<const __bf16 *>(prev), g.max_width, ld, x, S, xs, partial);
        else
            hipLaunchKernelGGL((final_partial_tm_kernel<kKFinal, float, FK_RATIONAL>), grid, dim3(kBlock), 0, s, e,
                               ne, chunks, static_cast<const float *>(prev), g.max_width, ld, x, S, xs, partial);
        err = hipGetLastError();
    } else {
        err = g.kind == FK_LOOKUP ? launch_final_partial<FK_LOOKUP>(g, p, prev, ld, x, S, xs, partial, chunks, s)
                                  : launch_final_partial<FK_RATIONAL>(g, p, prev, ld, x, S, xs, partial, chunks, s);
    }
    if (err != hipSuccess)
        return err;
    TimedLaunch tl(KK_FINAL_COMBINE, s);
    const dim3 grid(static_cast<unsigned>((S + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(final_combine_kernel, grid, dim3(kBlock), 0, s, partial, chunks, ld, S,
                       is_rescaled(p) ? maxbits : nullptr, g.L, out, out_exp);
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
