// Device routines of the level sweep, shared by the standalone kernels
// (kernels_level.hip, kernels_fused.hip) and the serving step kernel
// (serve.hip).  Sharing them is what makes a result bit-identical however the
// work is launched: every node value is one lane's sequential sum over the
// node's edges in canonical order, with the same factor arithmetic.
#pragma once

#include <type_traits>

#include "kernels_common.h"

namespace cosdag {

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Edge records fetched per scalar wait: 256 bytes in a streamed level (four
// binary64 or eight binary32 records), four in the whole-graph sweep and the
// final node.  The record arrays are padded with kEdgePad zeroed records, so a
// full chunk can always be read.
constexpr int kChunk = 4;
template <typename Rec>
constexpr int kStreamChunk = 256 / static_cast<int>(sizeof(Rec));

// The graph's device arrays (row pointers, edge records, level table) are
// written once when the graph is created and only read by kernels, so they are
// read through the constant address space: the compiler then treats a fetch
// from a wave-uniform address as a uniform scalar load wherever the pointer came
// from (a pointer read from memory is otherwise generic, and loads through it
// count as per-lane).
template <typename T>
using ConstPtr = const __attribute__((address_space(4))) T *;
template <typename T>
__device__ __forceinline__ ConstPtr<T> as_const(const T *p) {
    return (ConstPtr<T>)(p);
}

// Level table entry i (fields read one by one: a struct cannot be copied
// through an address-space-qualified reference).
__device__ __forceinline__ LevelDev load_level(const LevelDev *levels, int i) {
    static_assert(sizeof(LevelDev) == 8 * sizeof(int32_t), "five int32 fields and padding");
    const ConstPtr<int32_t> p = as_const(reinterpret_cast<const int32_t *>(levels)) + 8 * i;
    return LevelDev{p[0], p[1], p[2], p[3], p[4], {0, 0, 0}};
}

// Fetch C consecutive records (C * sizeof(Rec) = 128 or 256 bytes) into scalar
// registers.  TOGETHER: an empty asm takes every 16-byte piece as an SGPR
// operand, so all pieces are loaded (one scalar wait) before any field is used
// -- needed where fields are used under per-edge conditions or interleaved with
// vector loads, where the compiler would otherwise fetch each field next to its
// first use (one dependent round trip per edge).  Without it the compiler loads
// only the fields used, which is enough where every use is unconditional.
template <int C, bool TOGETHER, typename Rec>
__device__ __forceinline__ void load_chunk(const Rec *p, Rec (&r)[C]) {
    static_assert(C <= kEdgePad, "a chunk starting at the last edge must stay inside the padded array");
    using V4 = __attribute__((ext_vector_type(4))) unsigned;
    constexpr int kBytes = C * static_cast<int>(sizeof(Rec));
    static_assert(kBytes == 128 || kBytes == 256, "chunks of 128 or 256 bytes");
    const ConstPtr<V4> q = (ConstPtr<V4>)(as_const(p));
    V4 a0 = q[0], a1 = q[1], a2 = q[2], a3 = q[3], a4 = q[4], a5 = q[5], a6 = q[6], a7 = q[7];
    if constexpr (kBytes == 256) {
        V4 b0 = q[8], b1 = q[9], b2 = q[10], b3 = q[11], b4 = q[12], b5 = q[13], b6 = q[14], b7 = q[15];
        if constexpr (TOGETHER)
            asm volatile("" : "+s"(a0), "+s"(a1), "+s"(a2), "+s"(a3), "+s"(a4), "+s"(a5), "+s"(a6), "+s"(a7),
                         "+s"(b0), "+s"(b1), "+s"(b2), "+s"(b3), "+s"(b4), "+s"(b5), "+s"(b6), "+s"(b7));
        const V4 all[16] = {a0, a1, a2, a3, a4, a5, a6, a7, b0, b1, b2, b3, b4, b5, b6, b7};
        __builtin_memcpy(&r[0], all, sizeof(all));
    } else {
        if constexpr (TOGETHER)
            asm volatile("" : "+s"(a0), "+s"(a1), "+s"(a2), "+s"(a3), "+s"(a4), "+s"(a5), "+s"(a6), "+s"(a7));
        const V4 all[8] = {a0, a1, a2, a3, a4, a5, a6, a7};
        __builtin_memcpy(&r[0], all, sizeof(all));
    }
}

// A lane's K samples tbase + lane + 64m: coordinates and |x|^2.  Samples at or
// beyond S (padding) evaluate with x = 0 and are never returned.
template <int K>
struct LaneSamples {
    double x0[K], x1[K], x2[K], q[K];
    __device__ __forceinline__ void load(const double *__restrict__ x, int64_t S, int64_t xs, int64_t tbase,
                                         int lane) {
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const int64_t s = tbase + lane + kWave * m;
            const bool in = s < S;
            x0[m] = in ? x[s] : 0.0;
            x1[m] = in ? x[xs + s] : 0.0;
            x2[m] = in ? x[2 * xs + s] : 0.0;
            q[m] = __builtin_fma(x2[m], x2[m], __builtin_fma(x1[m], x1[m], x0[m] * x0[m]));
        }
    }
};

// The same samples rounded to binary32 (nearest even), for the binary32 factor.
template <int K>
struct LaneSamples32 {
    float x0[K], x1[K], x2[K];
    __device__ __forceinline__ void load(const double *__restrict__ x, int64_t S, int64_t xs, int64_t tbase,
                                         int lane) {
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const int64_t s = tbase + lane + kWave * m;
            const bool in = s < S;
            x0[m] = in ? static_cast<float>(x[s]) : 0.0f;
            x1[m] = in ? static_cast<float>(x[xs + s]) : 0.0f;
            x2[m] = in ? static_cast<float>(x[2 * xs + s]) : 0.0f;
        }
    }
};

// A lane's K samples for lookup factors: pointers to the samples' entries in
// table row 0 (rows [slot][sample], ld apart).  Samples at or beyond S
// (padding) read sample S-1's entries, so every read stays inside the table;
// their results are never returned.
template <int K>
struct LaneTable {
    const double *p[K];
    int64_t ld;
    __device__ __forceinline__ void load(const double *__restrict__ x, int64_t S, int64_t xs, int64_t tbase,
                                         int lane) {
        ld = xs;
#pragma unroll
        for (int m = 0; m < K; ++m)
            p[m] = x + min(tbase + lane + kWave * m, S - 1);
    }
    __device__ __forceinline__ double entry(int32_t slot, int m) const {
        return p[m][static_cast<int64_t>(slot) * ld];
    }
};

// The same with a binary32 copy of the tables, [slot][ld] with ld >= the
// padded sample count (padding columns hold 0), so no clamping is needed.
template <int K>
struct LaneTable32 {
    const float *p[K];
    int64_t ld;
    __device__ __forceinline__ void load(const float *__restrict__ t, int64_t /*S*/, int64_t lt, int64_t tbase,
                                         int lane) {
        ld = lt;
#pragma unroll
        for (int m = 0; m < K; ++m)
            p[m] = t + tbase + lane + kWave * m;
    }
    __device__ __forceinline__ float entry(int32_t slot, int m) const {
        return p[m][static_cast<int64_t>(slot) * ld];
    }
};

template <int K>
__device__ __forceinline__ double factor(const EdgeRec &e, const LaneSamples<K> &xs, int m) {
    return edge_factor64(e, xs.x0[m], xs.x1[m], xs.x2[m], xs.q[m]);
}
template <int K>
__device__ __forceinline__ float factor(const EdgeRec32 &e, const LaneSamples32<K> &xs, int m) {
    return edge_factor32(e, xs.x0[m], xs.x1[m], xs.x2[m]);
}

// Edge factor in the value type T: rational factors by their own formula in T;
// lookup factors as coef * T_s[slot], in binary64, or in binary32 from the
// binary32 constant and the table entry rounded once.
template <typename T, typename Rec, typename Smp>
__device__ __forceinline__ T edge_w(const Rec &r, const Smp &xs, int m) {
    if constexpr (std::is_same_v<Rec, EdgeRecL>) {
        const auto t = xs.entry(r.slot, m);
        if constexpr (sizeof(T) == sizeof(double))
            return r.coef * t;
        else  // the entry rounded once to binary32 (here or when the binary32 table was made)
            return r.coef32 * static_cast<float>(t);
    } else {
        return factor(r, xs, m);
    }
}

// Record and per-lane sample types of the interior levels of a sweep with
// values of type T and factor kind KIND ...
template <typename T, int KIND>
struct SweepPath;
template <>
struct SweepPath<double, FK_RATIONAL> {
    using Rec = EdgeRec;
    template <int K>
    using Samples = LaneSamples<K>;
};
template <>
struct SweepPath<float, FK_RATIONAL> {
    using Rec = EdgeRec32;
    template <int K>
    using Samples = LaneSamples32<K>;
};
template <typename T>
struct SweepPath<T, FK_LOOKUP> {
    using Rec = EdgeRecL;
    template <int K>
    using Samples = LaneTable<K>;
};
template <>
struct SweepPath<float, FK_LOOKUP_T32> {
    using Rec = EdgeRecL;
    template <int K>
    using Samples = LaneTable32<K>;
};
// ... and of the final node, whose factors are binary64 at every precision
// (from the binary64 tables also when the levels read binary32 copies).
template <int KIND>
using FinalPath = SweepPath<double, KIND == FK_LOOKUP_T32 ? FK_LOOKUP : KIND>;
// Element type of the per-sample input the interior levels read.
template <int KIND>
using SampleElem = std::conditional_t<KIND == FK_LOOKUP_T32, float, double>;

// Sum over edges [e_lo, e_hi) of w_e v[src_e] in the type T, sequentially in
// canonical order from T(0): one quarter of a final-node chunk (binary64) or
// of a chunk of an interior node of high in-degree.  The source value of edge
// e comes from src_value(rec, m) (level buffer or LDS).  Full chunks
// accumulate unconditionally, a tail its first n edges only.
template <typename T, int K, bool TOGETHER, typename Rec, typename Smp, typename SrcValue>
__device__ __forceinline__ void edge_sum(const Rec *__restrict__ edges, int e_lo, int e_hi, const Smp &xs,
                                         SrcValue src_value, T (&acc)[K]) {
#pragma unroll
    for (int m = 0; m < K; ++m)
        acc[m] = T(0);
    auto chunk = [&](auto full, int e, int n) {
        Rec r[kChunk];
        load_chunk<kChunk, TOGETHER>(edges + e, r);
        T v[kChunk][K];
#pragma unroll
        for (int u = 0; u < kChunk; ++u)
#pragma unroll
            for (int m = 0; m < K; ++m)
                v[u][m] = src_value(r[u], m);
        T w[kChunk][K];
#pragma unroll
        for (int u = 0; u < kChunk; ++u)
#pragma unroll
            for (int m = 0; m < K; ++m)
                w[u][m] = edge_w<T>(r[u], xs, m);
#pragma unroll
        for (int u = 0; u < kChunk; ++u)
            if (decltype(full)::value || u < n)
#pragma unroll
                for (int m = 0; m < K; ++m)
                    acc[m] = fma_t(w[u][m], v[u][m], acc[m]);
    };
    int e = e_lo;
    for (; e + kChunk <= e_hi; e += kChunk)
        chunk(std::true_type{}, e, kChunk);
    if (e < e_hi)
        chunk(std::false_type{}, e, e_hi - e);
}

// The final node's sum in binary64.
template <int K, bool TOGETHER, typename Rec, typename Smp, typename SrcValue>
__device__ __forceinline__ void final_sum(const Rec *__restrict__ edges, int e_lo, int e_hi, const Smp &xs,
                                          SrcValue src_value, double (&acc)[K]) {
    edge_sum<double, K, TOGETHER>(edges, e_lo, e_hi, xs, src_value, acc);
}

// Interior node of high in-degree (more than kHubEdges in-edges): its edges
// [e_lo, e_hi) are summed in chunks of kFinalChunk, each the four quarters of
// kQuarter edges summed sequentially and added as ((q0 + q1) + q2) + q3 (an
// absent quarter adds T(0)), and the chunk sums added in ascending order to
// T(0) -- the final node's order, in T.  This is the value every plan gives
// such a node; the streamed plan computes the chunks in parallel
// (hub_partial_kernel), the others sequentially with this routine.
template <typename T, int K, bool TOGETHER, typename Rec, typename Smp, typename SrcValue>
__device__ __forceinline__ void hub_sum(const Rec *__restrict__ edges, int e_lo, int e_hi, const Smp &xs,
                                        SrcValue src_value, T (&v)[K]) {
#pragma unroll
    for (int m = 0; m < K; ++m)
        v[m] = T(0);
    for (int c = e_lo; c < e_hi; c += kFinalChunk) {
        T cs[K];
#pragma unroll 1
        for (int i = 0; i < 4; ++i) {
            const int ql = min(c + i * kQuarter, e_hi);
            const int qh = min(ql + kQuarter, e_hi);
            T q[K];
            edge_sum<T, K, TOGETHER>(edges, ql, qh, xs, src_value, q);
#pragma unroll
            for (int m = 0; m < K; ++m)
                cs[m] = i == 0 ? q[m] : cs[m] + q[m];
        }
#pragma unroll
        for (int m = 0; m < K; ++m)
            v[m] = v[m] + cs[m];
    }
}

// One wave computes destination rows [jbeg, jend) (at most kWaveRows) of a
// level for the tile at tbase (64*K samples).  The rows' edges form one
// contiguous stream, walked in chunks: a chunk's records are fetched together
// (one scalar wait), its C*K source values requested together (one vector
// wait), then the factors accumulated.  A row is stored when its flagged last
// edge has been added; rows without in-edges are stored as zeros.
//
// Rows with more than kHubEdges in-edges are taken out of the stream and
// summed in hub_sum's chunked order: from the chunk sums hub_partial_kernel
// left in hub_partial ([chunk][ld], the row's chunks starting at the index its
// first record carries in zero_rows), or, when hub_partial is NULL, by the
// wave itself.
//
// FROM_ROOT: level 1, whose only source is the root (value 1).
// RESCALE:   binary32 with per-(level, sample) power-of-two scaling: each
//            stored value is its sum times 2^-esh[m] (exact), and lmax[m]
//            collects the largest |stored value| bit pattern of the lane
//            (taken before the rounding to V).
// V:         storage type of the level values (T, or a 16-bit format under
//            RESCALE): loads widen V to T exactly, stores round T to V.
// Source rows are reached by 32-bit byte offsets (level buffers < 2 GiB).
constexpr int kWaveRows = 8;
template <typename T, int K, bool FROM_ROOT, bool RESCALE, int KIND, typename V = T>
__device__ __forceinline__ void level_wave_rows(const int32_t *__restrict__ row_ptr,
                                                const typename SweepPath<T, KIND>::Rec *edges, int jbeg, int jend,
                                                const V *__restrict__ prev, V *__restrict__ cur, int64_t ld,
                                                int64_t tbase, int lane,
                                                const typename SweepPath<T, KIND>::template Samples<K> &xs,
                                                const int (&esh)[K], uint32_t (&lmax)[K],
                                                const T *__restrict__ hub_partial = nullptr) {
    using Rec = typename SweepPath<T, KIND>::Rec;
    if (jbeg >= jend)
        return;
    V *const out_base = cur + tbase + lane;
    auto store_row = [&](int j, const T *acc) {
        V *crow = out_base + static_cast<int64_t>(j) * ld;
#pragma unroll
        for (int m = 0; m < K; ++m) {
            T z = acc[m];
            if constexpr (RESCALE) {
                z = scale_pow2(z, esh[m]);
                lmax[m] = max(lmax[m], abs_bits(z));
            }
            crow[kWave * m] = static_cast<V>(z);
        }
    };
    const ConstPtr<int32_t> rp = as_const(row_ptr);
    const char *src_tile = reinterpret_cast<const char *>(prev + tbase);
    const uint32_t row_bytes = static_cast<uint32_t>(ld * sizeof(V));
    const uint32_t lane_off = static_cast<uint32_t>(lane * sizeof(V));
    constexpr int C = kStreamChunk<Rec>;

    // rows [j, j_end), none of high in-degree, as one edge stream
    auto walk = [&](int j, int j_end) {
        int e = rp[j];
        const int e_end = rp[j_end];
        T acc[K];
#pragma unroll
        for (int m = 0; m < K; ++m)
            acc[m] = T(0);
        // rows without in-edges at the start of the range
        while (j < j_end && rp[j + 1] == e) {
            store_row(j, acc);
            ++j;
        }
        const Rec *rec = edges + e;
        // one chunk of the stream: records, source values and factors, then the
        // accumulation edge by edge (every edge of a full chunk, the first n of the
        // tail), storing each row at its flagged last edge
        auto chunk = [&](auto full, int n) {
            Rec r[C];
            load_chunk<C, true>(rec, r);  // past e_end: later edges or the zeroed pad, never used
            // all C*K source values are requested before any is used; records past
            // the end name rows inside the level buffer (src < widest level), so
            // the unused reads stay in bounds
            T v[C][K];
#pragma unroll
            for (int u = 0; u < C; ++u) {
                const char *row = src_tile + static_cast<uint32_t>(r[u].src) * row_bytes + lane_off;
#pragma unroll
                for (int m = 0; m < K; ++m)
                    v[u][m] = FROM_ROOT ? T(1)
                                        : static_cast<T>(*reinterpret_cast<const V *>(row + m * kWave * sizeof(V)));
            }
            T w[C][K];
#pragma unroll
            for (int u = 0; u < C; ++u)
#pragma unroll
                for (int m = 0; m < K; ++m)
                    w[u][m] = edge_w<T>(r[u], xs, m);
#pragma unroll
            for (int u = 0; u < C; ++u) {
                if (decltype(full)::value || u < n) {
#pragma unroll
                    for (int m = 0; m < K; ++m)
                        acc[m] = fma_t(w[u][m], v[u][m], acc[m]);
                    if (r[u].row_end) {
                        store_row(j, acc);
                        ++j;
#pragma unroll
                        for (int m = 0; m < K; ++m)
                            acc[m] = T(0);
                        for (int z = 0; z < r[u].zero_rows && j < j_end; ++z) {
                            store_row(j, acc);
                            ++j;
                        }
                    }
                }
            }
        };
        for (; e + C <= e_end; e += C, rec += C)
            chunk(std::true_type{}, C);
        if (e < e_end)
            chunk(std::false_type{}, e_end - e);
    };

    // a row of high in-degree
    auto hub_row = [&](int h) {
        const int e_lo = rp[h], e_hi = rp[h + 1];
        T v[K];
        if (hub_partial) {
            const int cb = as_const(&edges[e_lo].zero_rows)[0];
            const int nch = (e_hi - e_lo + kFinalChunk - 1) / kFinalChunk;
            const T *pp = hub_partial + static_cast<int64_t>(cb) * ld + tbase + lane;
#pragma unroll
            for (int m = 0; m < K; ++m)
                v[m] = T(0);
            int c = 0;
            for (; c + 8 <= nch; c += 8) {  // loads of a group issued together, additions in order
                T p[8][K];
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int m = 0; m < K; ++m)
                        p[i][m] = pp[static_cast<int64_t>(c + i) * ld + kWave * m];
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int m = 0; m < K; ++m)
                        v[m] = v[m] + p[i][m];
            }
            for (; c < nch; ++c)
#pragma unroll
                for (int m = 0; m < K; ++m)
                    v[m] = v[m] + pp[static_cast<int64_t>(c) * ld + kWave * m];
        } else {
            hub_sum<T, K, true>(edges, e_lo, e_hi, xs, [&](const Rec &r, int m) -> T {
                if constexpr (FROM_ROOT) {
                    return T(1);
                } else {
                    const char *row = src_tile + static_cast<uint32_t>(r.src) * row_bytes + lane_off;
                    return static_cast<T>(*reinterpret_cast<const V *>(row + m * kWave * sizeof(V)));
                }
            }, v);
        }
        store_row(h, v);
    };

    // the rows' bounds, fetched together: bit i of hubs marks row jbeg + i as a
    // row of high in-degree
    int32_t b[kWaveRows + 1];
#pragma unroll
    for (int i = 0; i <= kWaveRows; ++i)
        b[i] = rp[min(jbeg + i, jend)];
    uint32_t hubs = 0u;
#pragma unroll
    for (int i = 0; i < kWaveRows; ++i)
        if (b[i + 1] - b[i] > kHubEdges)
            hubs |= 1u << i;
    // hub-free stretches walked as streams, each row of high in-degree by itself
    int j = jbeg;
    while (true) {
        const uint32_t ahead = hubs >> (j - jbeg);
        const int h = ahead ? j + __builtin_ctz(ahead) : jend;
        walk(j, h);
        if (h == jend)
            break;
        hub_row(h);
        j = h + 1;
    }
}

// Largest |value| bit patterns of NW waves (lmax of each lane) combined in LDS
// and folded into cur_max[0 .. 64K) by integer atomic max (order-free).  All
// threads of the group must call it (it synchronises the group).
template <int K, int NW>
__device__ __forceinline__ void fold_max(uint32_t *red /* LDS [NW][64K] */, const uint32_t (&lmax)[K], int wave,
                                         int lane, uint32_t *__restrict__ cur_max) {
#pragma unroll
    for (int m = 0; m < K; ++m)
        red[wave * (kWave * K) + lane + kWave * m] = lmax[m];
    __syncthreads();
    for (int i = threadIdx.x; i < kWave * K; i += NW * kWave) {
        uint32_t v = 0u;
#pragma unroll
        for (int w = 0; w < NW; ++w)
            v = max(v, red[w * (kWave * K) + i]);
        if (v)
            atomicMax(cur_max + i, v);
    }
    __syncthreads();
}

// final_sum with the level L-1 values in a level buffer (streamed kernels; the
// records are fetched together, ahead of the vector loads).
template <typename TV, int K, bool FROM_ROOT, int KIND>
__device__ __forceinline__ void final_quarter(const typename FinalPath<KIND>::Rec *__restrict__ edges, int e_lo,
                                              int e_hi, const TV *__restrict__ prev, int64_t ld, int64_t tbase,
                                              int lane, const typename FinalPath<KIND>::template Samples<K> &xs,
                                              double (&acc)[K]) {
    const char *src_tile = reinterpret_cast<const char *>(prev + tbase);
    const uint32_t row_bytes = static_cast<uint32_t>(ld * sizeof(TV));
    const uint32_t lane_off = static_cast<uint32_t>(lane * sizeof(TV));
    final_sum<K, true>(edges, e_lo, e_hi, xs, [&](const auto &r, int m) -> double {
        if constexpr (FROM_ROOT) {
            return 1.0;
        } else {
            const char *row = src_tile + static_cast<uint32_t>(r.src) * row_bytes + lane_off;
            return static_cast<double>(*reinterpret_cast<const TV *>(row + m * kWave * sizeof(TV)));
        }
    }, acc);
}

// Final node, second pass for sample s: the chunk partial sums added in
// ascending chunk order, then the rescaled paths' accumulated exponent
// E[s] = sum_{l=0}^{L-2} ilogb(maxbits[l][s]) applied (or returned
// separately).  Row l >= 1 holds the largest |value| of level l (times the
// next level's headroom 2^h, if any); row 0 is 2^h of level 1, or 0 (no
// shift).
__device__ __forceinline__ void final_combine_one(const double *__restrict__ partial, int32_t n_chunks, int64_t S_pad,
                                                  int64_t s, const uint32_t *__restrict__ maxbits, int32_t L,
                                                  double *__restrict__ out, int32_t *__restrict__ out_exp) {
    // the loads of a group are issued together (they are independent); the
    // additions stay in ascending chunk order
    double v = 0.0;
    int c = 0;
    for (; c + 16 <= n_chunks; c += 16) {
        double p[16];
#pragma unroll
        for (int i = 0; i < 16; ++i)
            p[i] = partial[static_cast<int64_t>(c + i) * S_pad + s];
#pragma unroll
        for (int i = 0; i < 16; ++i)
            v += p[i];
    }
    for (; c < n_chunks; ++c)
        v += partial[static_cast<int64_t>(c) * S_pad + s];
    int E = 0;
    if (maxbits) {
        int l = 0;
        for (; l + 8 <= L - 1; l += 8) {
            uint32_t m[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                m[i] = maxbits[static_cast<int64_t>(l + i) * S_pad + s];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                E += ilogb_bits(m[i]);
        }
        for (; l <= L - 2; ++l)
            E += ilogb_bits(maxbits[static_cast<int64_t>(l) * S_pad + s]);
    }
    if (out_exp) {
        out[s] = v;
        out_exp[s] = E;
    } else {
        out[s] = ldexp(v, E);
    }
}

// final_sum with the level L-1 values read from LDS ([node][64K]) or, for
// L = 1, the root's value 1.
template <typename T, int K, bool FROM_ROOT, int KIND>
__device__ __forceinline__ void final_quarter_lds(const typename FinalPath<KIND>::Rec *__restrict__ edges, int e_lo,
                                                  int e_hi, const T *vals, int lane,
                                                  const typename FinalPath<KIND>::template Samples<K> &xs,
                                                  double (&acc)[K]) {
    constexpr int kTile = kWave * K;
    final_sum<K, false>(edges, e_lo, e_hi, xs, [&](const auto &r, int m) -> double {
        if constexpr (FROM_ROOT)
            return 1.0;
        else
            return static_cast<double>(vals[r.src * kTile + lane + kWave * m]);
    }, acc);
}

// ---------------------------------------------------------------- fused sweep

constexpr int kFusedThreads = kFusedWaves * kWave;

// Everything a workgroup needs to sweep one graph for one tile in LDS.
struct FusedGraph {
    const int32_t *row_ptr;
    const EdgeRec *edges;      // binary64 records (binary64 levels, final node)
    const EdgeRec32 *edges32;  // binary32 records (binary32 levels)
    const EdgeRecL *edgesL;    // lookup records (every level)
    const LevelDev *levels;
    int32_t L;
    const double *x;
    int64_t S;
    double *out;
    int32_t *out_exp;
    const float *t32 = nullptr;  // FK_LOOKUP_T32: binary32 tables [n_slots][ld32] for the interior levels
    int64_t ld32 = 0;
};

// One level of the whole-graph sweep for a wave's rows [jb, jb + nb): the
// sums of each row (scaled by 2^-esh when RESCALE) into acc, the largest
// |stored value| bit pattern into lmax.  rpl: lane i (i <= nb) holds the start
// of row jb + i.  FROM_ROOT: level 1, whose only source is the root (value 1).
template <typename T, int K, int RMAX, bool FROM_ROOT, bool RESCALE, int KIND, bool HUBS>
__device__ __forceinline__ void fused_rows(const typename SweepPath<T, KIND>::Rec *edges, const T *vals, int nb,
                                           int rpl, int lane,
                                           const typename SweepPath<T, KIND>::template Samples<K> &xs,
                                           const int (&esh)[K], T (&acc)[RMAX][K], uint32_t (&lmax)[K]) {
    using Rec = typename SweepPath<T, KIND>::Rec;
    constexpr int kTile = kWave * K;
    static_assert(RMAX <= 64, "row mask of 64 bits");
    uint64_t hubs = 0u;  // bit r: row jb + r has more than kHubEdges in-edges
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
            // one chunk of the row: its records, source values and factors, then
            // the accumulation (every edge of a full chunk, the first n of a tail)
            auto chunk = [&](auto full, int e, int n) {
                Rec rr[kChunk];
                load_chunk<kChunk, false>(edges + e, rr);
                // records past the row name rows < widest level: the unused
                // LDS reads stay in bounds
                T v[kChunk][K];
#pragma unroll
                for (int u = 0; u < kChunk; ++u)
#pragma unroll
                    for (int m = 0; m < K; ++m)
                        v[u][m] = FROM_ROOT ? T(1) : vals[rr[u].src * kTile + lane + kWave * m];
                T w[kChunk][K];
#pragma unroll
                for (int u = 0; u < kChunk; ++u)
#pragma unroll
                    for (int m = 0; m < K; ++m)
                        w[u][m] = edge_w<T>(rr[u], xs, m);
#pragma unroll
                for (int u = 0; u < kChunk; ++u)
                    if (decltype(full)::value || u < n)
#pragma unroll
                        for (int m = 0; m < K; ++m)
                            acc[r][m] = fma_t(w[u][m], v[u][m], acc[r][m]);
            };
            int e = __builtin_amdgcn_readlane(rpl, r);
            if constexpr (HUBS) {
                if (e1 - e > kHubEdges) {  // high in-degree: summed below, in hub_sum's order
                    hubs |= uint64_t(1) << r;
                    continue;
                }
            }
            for (; e + kChunk <= e1; e += kChunk)
                chunk(std::true_type{}, e, kChunk);
            if (e < e1)
                chunk(std::false_type{}, e, e1 - e);
            if constexpr (RESCALE) {
#pragma unroll
                for (int m = 0; m < K; ++m) {
                    acc[r][m] = scale_pow2(acc[r][m], esh[m]);
                    lmax[m] = max(lmax[m], abs_bits(acc[r][m]));
                }
            }
        }
    }
    // rows of high in-degree, one at a time (outside the unrolled loop)
    while (HUBS && hubs) {
        const int r = __builtin_ctzll(hubs);
        hubs &= hubs - 1;
        T v[K];
        hub_sum<T, K, false>(edges, __builtin_amdgcn_readlane(rpl, r), __builtin_amdgcn_readlane(rpl, r + 1), xs,
                             [&](const Rec &rr, int m) -> T {
                                 return FROM_ROOT ? T(1) : vals[rr.src * kTile + lane + kWave * m];
                             }, v);
#pragma unroll
        for (int m = 0; m < K; ++m) {
            if constexpr (RESCALE) {
                v[m] = scale_pow2(v[m], esh[m]);
                lmax[m] = max(lmax[m], abs_bits(v[m]));
            }
#pragma unroll
            for (int q = 0; q < RMAX; ++q)
                if (q == r)
                    acc[q][m] = v[m];
        }
    }
}

// Whole-graph sweep for the tile at tbase (64*K samples) by a group of 16
// waves, the level held in LDS as [node][64K] (vals), wave w owning rows
// [w*RMAX, (w+1)*RMAX).  red: [16][64K] uint32 (RESCALE only); part:
// [quarters][64K] binary64.  The final node is reduced in quarters of 64 edges
// combined exactly as final_partial / final_combine do.
template <typename T, int K, int RMAX, bool RESCALE, int KIND>
__device__ __forceinline__ void fused_tile(const FusedGraph &G, int64_t tbase, T *vals, uint32_t *red, double *part,
                                           int wave, int lane) {
    constexpr int kTile = kWave * K;
    typename SweepPath<T, KIND>::template Samples<K> xs;
    if constexpr (KIND == FK_LOOKUP_T32)
        xs.load(G.t32, G.S, G.ld32, tbase, lane);
    else
        xs.load(G.x, G.S, G.S, tbase, lane);
    const typename SweepPath<T, KIND>::Rec *edges;
    if constexpr (KIND != FK_RATIONAL)
        edges = G.edgesL;
    else if constexpr (sizeof(T) == sizeof(double))
        edges = G.edges;
    else
        edges = G.edges32;
    int esh[K], E[K];  // e_{l-1} and the sum of e_1 .. e_{L-2} for this lane's samples
#pragma unroll
    for (int m = 0; m < K; ++m) {
        esh[m] = 0;
        E[m] = 0;
    }
    for (int l = 1; l < G.L; ++l) {
        const LevelDev lv = load_level(G.levels, l - 1);
        const ConstPtr<int32_t> rp = as_const(G.row_ptr) + lv.rp_begin;
        const int jb = min(wave * RMAX, lv.w_dst);
        const int nb = min(jb + RMAX, lv.w_dst) - jb;
        // lane i (i <= nb) holds the start of row jb + i: one load per wave and level
        const int rpl = lane <= nb ? rp[jb + lane] : 0;
        T acc[RMAX][K];
        uint32_t lmax[K];
        // a level with a node of high in-degree takes the variant that sums such rows in chunks
        if (l == 1) {
            if (lv.hubs)
                fused_rows<T, K, RMAX, true, RESCALE, KIND, true>(edges, vals, nb, rpl, lane, xs, esh, acc, lmax);
            else
                fused_rows<T, K, RMAX, true, RESCALE, KIND, false>(edges, vals, nb, rpl, lane, xs, esh, acc, lmax);
        } else {
            if (lv.hubs)
                fused_rows<T, K, RMAX, false, RESCALE, KIND, true>(edges, vals, nb, rpl, lane, xs, esh, acc, lmax);
            else
                fused_rows<T, K, RMAX, false, RESCALE, KIND, false>(edges, vals, nb, rpl, lane, xs, esh, acc, lmax);
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
            if (l <= G.L - 2) {
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

    // final node (binary64 factors from the binary64 records and samples):
    // quarter p holds edges [64p, 64p + 64) of the last level
    const LevelDev lf = load_level(G.levels, G.L - 1);
    const int nq = (lf.n_edges + kQuarter - 1) / kQuarter;
    typename FinalPath<KIND>::template Samples<K> xd;
    if constexpr (KIND == FK_LOOKUP || sizeof(T) == sizeof(double))
        xd = xs;
    else if (wave < nq)
        xd.load(G.x, G.S, G.S, tbase, lane);
    const typename FinalPath<KIND>::Rec *fedges;
    if constexpr (KIND != FK_RATIONAL)
        fedges = G.edgesL + lf.e_begin;
    else
        fedges = G.edges + lf.e_begin;
    for (int p = wave; p < nq; p += kFusedWaves) {
        double acc[K];
        const int e_lo = p * kQuarter;
        const int e_hi = min(e_lo + kQuarter, lf.n_edges);
        if (G.L == 1)
            final_quarter_lds<T, K, true, KIND>(fedges, e_lo, e_hi, vals, lane, xd, acc);
        else
            final_quarter_lds<T, K, false, KIND>(fedges, e_lo, e_hi, vals, lane, xd, acc);
#pragma unroll
        for (int m = 0; m < K; ++m)
            part[p * kTile + lane + kWave * m] = acc[m];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const int64_t s = tbase + lane + kWave * m;
            if (s >= G.S)
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
            if (G.out_exp) {
                G.out[s] = tot;
                G.out_exp[s] = E[m];
            } else {
                G.out[s] = ldexp(tot, E[m]);
            }
        }
    }
    __syncthreads();  // part and vals may be reused by the group's next tile
}

}  // namespace cosdag
