// Wide levels at binary32 and 16-bit storage: row panels whose edge records sit
// in LDS, swept over narrow sample tiles of the previous level.
//
// On a wide random level every source row is read by about d destinations
// scattered over the level, so a level kernel whose lanes run along 256
// samples at a time fetches each source row about d times from beyond L2.  Here
// the level values are stored tile-major ([tile][node][tile samples], one
// 128-byte line per node and tile: 32 binary32 or 64 16-bit values), and an
// XCD sweeps its sample tiles one after the other, so the gathers of a tile
// fall in that tile's slice of the previous level (width * 128 bytes), a much
// smaller working set for the XCD's L2, and every line fetched is used whole.
// The edge records cannot stream through L2 once per tile as well, so each
// workgroup (one per CU) loads a panel of consecutive destination rows with
// their records into LDS once per level and reuses it for every tile, and the
// tiles' samples are staged in LDS too: inside a tile a lane reads LDS and
// issues gathers only, with the gathers of its next row (or of the next tile's
// first row) in flight while a row is summed.  Level values are written with
// non-temporal stores.
//
// Work split: XCD x (block b runs on XCD b % 8) takes samples of quarter x % 4
// and the rows of half x / 4; its 32 workgroups take that half's panels in
// turn.  Within a workgroup, (tile samples) / 4 lanes share a destination row
// and each lane handles 4 consecutive samples (one 16- or 8-byte gather per
// edge); a lane's rows take their edge ranges from the panel's row offsets in
// LDS.
//
// Arithmetic and order are those of level_wave_rows: per (row, sample) the
// binary32 factor from the binary32 record and the sample rounded to binary32,
// accumulated by fused multiply-adds in canonical edge order from 0 over the
// source values widened exactly to binary32, then the power-of-two rescale and
// one rounding to the storage type -- the results are bit-identical to the
// other plans.
#include <atomic>

#include "sweep_device.h"

namespace cosdag {
namespace {

// One edge in LDS: the binary32 record without its row flags, the source as
// the byte offset of its node's line within a tile's slice of the previous
// level.
struct PanelRec {
    float a, b, k0, k1, k2;
    uint32_t soff;
};
static_assert(sizeof(PanelRec) == 24, "PanelRec layout");
// The same for lookup factors: the binary32 constant and the byte offset of
// the edge's table slot within a tile of the tile-major binary32 tables.
struct PanelRecL {
    float coef;
    uint32_t toff;
    uint32_t unused[3];
    uint32_t soff;
};
static_assert(sizeof(PanelRecL) == sizeof(PanelRec), "PanelRecL layout");

// A sample of the current block of tiles in LDS: its coordinates rounded to
// binary32 and the exponent shift of the previous level (0 without rescale).
struct PanelSample {
    float x0, x1, x2;
    int32_t esh;
};
static_assert(kPanelSampleBytes == kPanelBlockSamples * static_cast<int>(sizeof(PanelSample)), "sample block size");

// Edges of a row gathered together (longer rows take the rest one at a time).
constexpr int kGroup = 6;
static_assert(kGroup <= kPanelPadRecs, "a row's group never reads past the padding");

// A lane's four consecutive values of a node in a tile: loaded as one vector
// (Raw), widened exactly to binary32, stored rounded once to V.
template <typename V>
struct PanelIO;
template <>
struct PanelIO<float> {
    using Raw = float4;
    static __device__ __forceinline__ void widen(const Raw &r, float (&v)[4]) {
        v[0] = r.x;
        v[1] = r.y;
        v[2] = r.z;
        v[3] = r.w;
    }
    static __device__ __forceinline__ void store(float *p, const float (&z)[4]) {
        using F4 = __attribute__((ext_vector_type(4))) float;
        const F4 val = {z[0], z[1], z[2], z[3]};
        __builtin_nontemporal_store(val, reinterpret_cast<F4 *>(p));  // streamed out: L2 keeps the gathered slice
    }
};
template <typename V>
struct PanelIO16 {
    using Raw = uint2;
    static __device__ __forceinline__ float to_float(uint32_t bits) {
        return static_cast<float>(__builtin_bit_cast(V, static_cast<uint16_t>(bits)));
    }
    static __device__ __forceinline__ void widen(const Raw &r, float (&v)[4]) {
        v[0] = to_float(r.x & 0xffffu);
        v[1] = to_float(r.x >> 16);
        v[2] = to_float(r.y & 0xffffu);
        v[3] = to_float(r.y >> 16);
    }
    static __device__ __forceinline__ void store(V *p, const float (&z)[4]) {
        uint32_t h[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            h[j] = __builtin_bit_cast(uint16_t, static_cast<V>(z[j]));
        using U2 = __attribute__((ext_vector_type(2))) uint32_t;
        const U2 val = {h[0] | (h[1] << 16), h[2] | (h[3] << 16)};
        __builtin_nontemporal_store(val, reinterpret_cast<U2 *>(p));
    }
};
template <>
struct PanelIO<_Float16> : PanelIO16<_Float16> {};
template <>
struct PanelIO<__bf16> : PanelIO16<__bf16> {};

// V: storage type of the level values (binary32, or binary16 / bfloat16 under
// RESCALE).  h_next: the next level's headroom exponent (binary16), by which
// this level's largest |value| is raised before it is folded into cur_max.
// LOOKUP: lookup factors coef32 * T_s[slot] at binary32 storage, the tables
// t32 tile-major ([tile][slot][kTile], n_tab lines per tile; a tile's tables
// stay in L2), a row's entries gathered as the row starts.
template <bool FROM_ROOT, bool RESCALE, typename V, bool LOOKUP>
__global__ __launch_bounds__(kPanelThreads) void level_panel_kernel(
    const int32_t *__restrict__ panels, int32_t n_half0, int32_t n_panels, const EdgeRec32 *__restrict__ edges,
    const EdgeRecL *__restrict__ edgesL, const float *__restrict__ t32, int32_t n_tab,
    const int32_t *__restrict__ row_ptr, const V *__restrict__ prev, V *__restrict__ cur, int64_t wbuf,
    int64_t n_tiles, const double *__restrict__ x, int64_t S, int64_t xs, const uint32_t *__restrict__ prev_max,
    uint32_t *__restrict__ cur_max, int32_t h_next) {
    static_assert(!LOOKUP || std::is_same_v<V, float>, "lookup factors on the panel plan at binary32 storage");
    using IO = PanelIO<V>;
    using Rec = std::conditional_t<LOOKUP, PanelRecL, PanelRec>;
    constexpr int kTile = panel_tile(sizeof(V));       // samples per tile
    constexpr int kBlockTiles = kPanelBlockSamples / kTile;
    static_assert(kBlockTiles * kTile == kPanelBlockSamples, "whole tiles per sample block");
    extern __shared__ __align__(16) unsigned char lds[];
    // the workgroup's exponent maxima of a tile, two tables used by alternate tiles: a table is sent out and
    // cleared after the tile's barrier by the threads that read it, and written again two tiles later, after
    // the barrier of the tile between, so one barrier per tile orders every access
    __shared__ uint32_t tmax[2][kTile];
    static_assert(sizeof(tmax) + kPanelLdsBytes <= 160 * 1024, "static and dynamic LDS within a CU's 160 KiB");
    constexpr int kLpr = kTile / 4;  // lanes per row
    constexpr int kRowsPerStep = kPanelThreads / kLpr;
    // a lane's rows: a panel holds at most kPanelMaxRows rows, kRowsPerLane per lane
    constexpr int kRowsPerLane = kPanelMaxRows / kRowsPerStep;
    static_assert(kRowsPerLane % 2 == 0, "rows alternate between two gather buffers");
    const int tid = threadIdx.x;
    const int xcd = static_cast<int>(blockIdx.x % kXcds);
    const int slot = static_cast<int>(blockIdx.x / kXcds);
    const int n_slots = static_cast<int>(gridDim.x / kXcds);
    const int quarter = xcd & 3, half = xcd >> 2;
    const int64_t tpq = n_tiles / 4;  // tiles of each quarter of the samples
    const int64_t t0 = quarter * tpq, t1 = t0 + tpq;
    const int q = tid % kLpr;     // this lane's 4 samples within a tile: 4q .. 4q + 3
    const int rsub = tid / kLpr;  // this lane's rows in a panel: rsub + i * kRowsPerStep
    // the lane's bytes in a node's line; sources and stores are reached from a wave-uniform tile base by
    // 32-bit byte offsets (levels narrower than 2^24 nodes)
    const uint32_t qoff = static_cast<uint32_t>(q) * 4u * sizeof(V);
    const int p_lo = half ? n_half0 : 0, p_hi = half ? n_panels : n_half0;
    if (tid < 2 * kTile)
        tmax[tid / kTile][tid % kTile] = 0u;  // ordered before use by the panel's first barrier
    for (int p = p_lo + slot; p < p_hi; p += n_slots) {
        const ConstPtr<int32_t> pd = as_const(panels) + 4 * p;
        const int rb = pd[0], re = pd[1], eb = pd[2], ee = pd[3];
        const int nr = re - rb, ne = ee - eb;
        // LDS: records from address 0 (a row's records are then reached by instruction offsets), kPanelPadRecs
        // zeroed ones (source 0), the row offsets, then the sample block at the next 16-byte boundary
        Rec *rec = reinterpret_cast<Rec *>(lds);
        const size_t rec_bytes = static_cast<size_t>(ne + kPanelPadRecs) * sizeof(Rec);
        int32_t *off = reinterpret_cast<int32_t *>(lds + rec_bytes);
        PanelSample *smp = reinterpret_cast<PanelSample *>(lds + ((rec_bytes + (nr + 1) * 4 + 15) & ~size_t(15)));
        __syncthreads();  // the previous panel's records are no longer read
        for (int i = tid; i < ne + kPanelPadRecs; i += kPanelThreads) {
            if constexpr (LOOKUP) {
                if (i < ne) {
                    const EdgeRecL &e = edgesL[eb + i];
                    rec[i] = PanelRecL{e.coef32, static_cast<uint32_t>(e.slot) * kPanelLine, {0u, 0u, 0u},
                                       static_cast<uint32_t>(e.src) * kPanelLine};
                } else {
                    rec[i] = PanelRecL{0.0f, 0u, {0u, 0u, 0u}, 0u};
                }
            } else {
                if (i < ne) {
                    const EdgeRec32 &e = edges[eb + i];
                    rec[i] = PanelRec{e.a, e.b, e.k0, e.k1, e.k2, static_cast<uint32_t>(e.src) * kPanelLine};
                } else {
                    rec[i] = PanelRec{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0u};
                }
            }
        }
        for (int i = tid; i <= nr; i += kPanelThreads)
            off[i] = row_ptr[rb + i] - eb;
        __syncthreads();
        // the lane's rows: their edges in LDS
        auto kbf = [&](int i) { const int r = rsub + i * kRowsPerStep; return r < nr ? off[r] : 0; };
        auto kef = [&](int i) { const int r = rsub + i * kRowsPerStep; return r < nr ? off[r + 1] : 0; };
        // source values of LDS edge k for the lane's samples of tile t (level 1: the root's value 1, never
        // loaded)
        using Raw = typename IO::Raw;
        auto gather = [&](int64_t t, int k) -> Raw {
            if constexpr (FROM_ROOT)
                return Raw{};
            else
                return *reinterpret_cast<const Raw *>(reinterpret_cast<const char *>(prev) + t * wbuf * kPanelLine +
                                                      (rec[k].soff + qoff));
        };
        // table entries of LDS edge k for the lane's samples of tile t (lookup factors)
        auto tgather = [&](int64_t t, int k) -> float4 {
            if constexpr (LOOKUP)
                return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(t32) +
                                                         t * n_tab * kPanelLine + (rec[k].toff + qoff));
            else
                return float4{};
        };
        // the first kGroup gathers of row i for tile t, issued unconditionally: records past the row are
        // later records or the zeroed padding, whose sources are rows of the previous level and whose slots
        // are slots of the tables (never summed)
        auto issue = [&](int64_t t, int i, Raw (&v)[kGroup]) {
#pragma unroll
            for (int u = 0; u < kGroup; ++u)
                v[u] = gather(t, kbf(i) + u);
        };
        // the gathers of the next row (or of the next tile's first row) are in flight while a row is summed
        Raw buf[2][kGroup];
        if (t0 < t1)
            issue(t0, 0, buf[0]);
        for (int64_t t = t0; t < t1; ++t) {
            if ((t - t0) % kBlockTiles == 0) {
                // the next kBlockTiles tiles' samples into LDS (rounded to binary32, the exponent shift)
                __syncthreads();  // the previous block is no longer read
                for (int i = tid; i < kPanelBlockSamples; i += kPanelThreads) {
                    const int64_t s = t * kTile + i;
                    PanelSample v{0.0f, 0.0f, 0.0f, 0};
                    if (!LOOKUP && s < S)
                        v = PanelSample{static_cast<float>(x[s]), static_cast<float>(x[xs + s]),
                                        static_cast<float>(x[2 * xs + s]), 0};
                    if (RESCALE && prev_max && s < n_tiles * kTile)
                        v.esh = ilogb_bits(prev_max[s]);
                    smp[i] = v;
                }
                __syncthreads();
            }
            // this lane's samples: LDS reads only, so the gathers in flight are not waited for
            const PanelSample *ms = smp + ((t - t0) % kBlockTiles) * kTile + 4 * q;
            float x0[4], x1[4], x2[4];
            int esh[4];
            uint32_t lmax[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const PanelSample v = ms[j];
                x0[j] = v.x0;
                x1[j] = v.x1;
                x2[j] = v.x2;
                esh[j] = v.esh;
                lmax[j] = 0u;
            }
            char *cslice = reinterpret_cast<char *>(cur) + t * wbuf * kPanelLine;  // tile t of this level
#pragma unroll
            for (int i = 0; i < kRowsPerLane; ++i) {
                if (i + 1 < kRowsPerLane)
                    issue(t, i + 1, buf[(i + 1) & 1]);
                else  // the next tile's first row (on the last tile, an unused repeat of this tile's)
                    issue(min(t + 1, t1 - 1), 0, buf[0]);
                const int kbi = kbf(i), kei = kef(i);
                float4 tbuf[LOOKUP ? kGroup : 1];  // this row's table entries (lookup factors)
                if constexpr (LOOKUP)
#pragma unroll
                    for (int u = 0; u < kGroup; ++u)
                        tbuf[u] = tgather(t, kbi + u);
                float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                // edge k added to the sums when `use` (the group's records past the row are formed and
                // dropped)
                auto add = [&](int k, const Raw &v, const float4 &tv, bool use) {
                    const Rec g = rec[k];
                    float vv[4] = {1.0f, 1.0f, 1.0f, 1.0f};
                    if constexpr (!FROM_ROOT)
                        IO::widen(v, vv);
                    if constexpr (LOOKUP) {
                        const float tt[4] = {tv.x, tv.y, tv.z, tv.w};
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const float f = __builtin_fmaf(g.coef * tt[j], vv[j], acc[j]);
                            acc[j] = use ? f : acc[j];
                        }
                    } else {
                        const EdgeRec32 e{g.a, g.b, g.k0, g.k1, g.k2, 0, 0, 0};
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const float f = __builtin_fmaf(edge_factor32(e, x0[j], x1[j], x2[j]), vv[j], acc[j]);
                            acc[j] = use ? f : acc[j];
                        }
                    }
                };
#pragma unroll
                for (int u = 0; u < kGroup; ++u)
                    add(kbi + u, buf[i & 1][u], tbuf[LOOKUP ? u : 0], kbi + u < kei);
                for (int k = kbi + kGroup; k < kei; ++k)  // rows of more than kGroup edges
                    add(k, gather(t, k), tgather(t, k), true);
                const int r = rsub + i * kRowsPerStep;
                if (r < nr) {
                    float z[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        z[j] = acc[j];
                        if constexpr (RESCALE) {
                            z[j] = scale_pow2(z[j], esh[j]);
                            lmax[j] = max(lmax[j], abs_bits(z[j]));
                        }
                    }
                    IO::store(reinterpret_cast<V *>(cslice + (static_cast<uint32_t>(rb + r) * kPanelLine + qoff)), z);
                }
            }
            if constexpr (RESCALE) {
                if (cur_max) {
                    // lanes of equal q hold the same samples: combine across the wave, then the workgroup
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        for (int d = kLpr; d < kWave; d *= 2)
                            lmax[i] = max(lmax[i], static_cast<uint32_t>(__shfl_xor(static_cast<int>(lmax[i]), d)));
                    if (h_next)  // exact: |value| <= 2^15 and h_next <= 96, and monotone, so the max commutes
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            lmax[i] = abs_bits(ldexpf(__uint_as_float(lmax[i]), h_next));
                    uint32_t *tm = tmax[(t - t0) & 1];
                    if ((tid & (kWave - 1)) < kLpr)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if (lmax[i])
                                atomicMax(&tm[4 * q + i], lmax[i]);
                    __syncthreads();  // the tile's maxima are all in
                    if (tid < kTile) {
                        if (tm[tid])
                            atomicMax(cur_max + t * kTile + tid, tm[tid]);
                        tm[tid] = 0u;
                    }
                }
            }
        }
    }
}

// Allow a panel's dynamic LDS (beyond the default limit) once per instantiation.
template <bool FROM_ROOT, bool RESCALE, typename V, bool LOOKUP>
hipError_t panel_launch(dim3 grid, size_t lds, hipStream_t s, const int32_t *pan, int32_t n0, int32_t n,
                        const Graph &g, const float *t32, const int32_t *rp, const void *prev, void *cur,
                        int64_t ld, const double *x, int64_t S, int64_t xs, const uint32_t *prev_max,
                        uint32_t *cur_max, int32_t h_next) {
    static std::atomic<bool> attr_set{false};
    auto kern = level_panel_kernel<FROM_ROOT, RESCALE, V, LOOKUP>;
    if (!attr_set.load(std::memory_order_acquire)) {
        const hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   static_cast<int>(kPanelLdsBytes));
        if (err != hipSuccess)
            return err;
        attr_set.store(true, std::memory_order_release);  // setting it twice is harmless
    }
    const int64_t n_tiles = ld / panel_tile(sizeof(V));
    hipLaunchKernelGGL(kern, grid, dim3(kPanelThreads), lds, s, pan, n0, n, g.d_edges32, g.d_edgesL, t32,
                       g.n_slots, rp, static_cast<const V *>(prev), static_cast<V *>(cur), g.max_width, n_tiles, x,
                       S, xs, prev_max, cur_max, h_next);
    return hipGetLastError();
}

template <bool RESCALE, typename V, bool LOOKUP = false>
hipError_t panel_launch_level(bool root, dim3 grid, size_t lds, hipStream_t s, const int32_t *pan, int32_t n0,
                              int32_t n, const Graph &g, const float *t32, const int32_t *rp, const void *prev,
                              void *cur, int64_t ld, const double *x, int64_t S, int64_t xs,
                              const uint32_t *prev_max, uint32_t *cur_max, int32_t h_next) {
    return root ? panel_launch<true, RESCALE, V, LOOKUP>(grid, lds, s, pan, n0, n, g, t32, rp, prev, cur, ld, x, S,
                                                         xs, prev_max, cur_max, h_next)
                : panel_launch<false, RESCALE, V, LOOKUP>(grid, lds, s, pan, n0, n, g, t32, rp, prev, cur, ld, x, S,
                                                          xs, prev_max, cur_max, h_next);
}

}  // namespace

bool panel_fits(const Graph &g, cos_precision p) {
    if (g.kind == FK_LOOKUP)
        return g.panel_ok && (p == COS_FP32 || p == COS_FP32_RESCALED);
    return g.panel_ok && (p == COS_FP32 || p == COS_FP32_RESCALED || p == COS_FP16_RESCALED || p == COS_BF16_RESCALED);
}

hipError_t launch_level_panel(const Graph &g, int l, cos_precision p, const void *prev, void *cur, int64_t ld,
                              const double *x, int64_t S, int64_t xs, const uint32_t *prev_max, uint32_t *cur_max,
                              int32_t h_next, const float *t32, hipStream_t s) {
    const LevelDesc &d = g.levels[l - 1];
    const bool lookup = g.kind == FK_LOOKUP;
    if (!panel_fits(g, p) || ld % (4 * panel_tile(value_bytes(p))) != 0 || d.panel_lds > kPanelLdsBytes ||
        (lookup && t32 == nullptr))
        return hipErrorInvalidValue;
    // one workgroup per CU: 32 per XCD
    const dim3 grid(kXcds * 32);
    const int32_t *pan = g.d_panels + 4 * d.panel_begin;
    const int32_t n0 = static_cast<int32_t>(d.n_panel_half0), n = static_cast<int32_t>(d.n_panels);
    const size_t lds = static_cast<size_t>(d.panel_lds);
    const int32_t *rp = g.d_row_ptr + d.rp_begin;
    const bool root = prev == nullptr;
    TimedLaunch tl(KK_LEVEL, s);
    switch (p) {
    case COS_FP32_RESCALED:
        return lookup ? panel_launch_level<true, float, true>(root, grid, lds, s, pan, n0, n, g, t32, rp, prev, cur,
                                                              ld, x, S, xs, prev_max, cur_max, h_next)
                      : panel_launch_level<true, float>(root, grid, lds, s, pan, n0, n, g, t32, rp, prev, cur, ld, x,
                                                        S, xs, prev_max, cur_max, h_next);
    case COS_FP32:
        return lookup ? panel_launch_level<false, float, true>(root, grid, lds, s, pan, n0, n, g, t32, rp, prev, cur,
                                                               ld, x, S, xs, nullptr, nullptr, 0)
                      : panel_launch_level<false, float>(root, grid, lds, s, pan, n0, n, g, t32, rp, prev, cur, ld,
                                                         x, S, xs, nullptr, nullptr, 0);
    case COS_FP16_RESCALED:
        return panel_launch_level<true, _Float16>(root, grid, lds, s, pan, n0, n, g, t32, rp, prev, cur, ld, x, S,
                                                  xs, prev_max, cur_max, h_next);
    case COS_BF16_RESCALED:
        return panel_launch_level<true, __bf16>(root, grid, lds, s, pan, n0, n, g, t32, rp, prev, cur, ld, x, S, xs,
                                                prev_max, cur_max, h_next);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace cosdag
