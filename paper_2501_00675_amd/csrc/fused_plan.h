// Host-side planning of the LDS-resident (fused) sweep: LDS layout, the
// rows-per-wave variant and the samples-per-lane K a graph can use.
#pragma once

#include "cos_internal.h"

namespace cosdag {

constexpr size_t kLdsBytes = 160 * 1024;  // LDS per CU on gfx950
constexpr int kMaxRows = 40;              // rows per wave supported (widest level 640)

// Rows-per-wave variants; a (K, RMAX) pair is built only when its register
// accumulators (K * RMAX values per lane) take at most 48 dwords and, with the
// working set of one chunk of four edges (four source values and four factors
// per sample), at most 80: this keeps every variant free of register spills at
// 1024 threads per group (128 VGPRs).
constexpr int kRowVariants[] = {2, 4, 8, 16, 24, kMaxRows};
constexpr bool acc_fits(size_t elem, int K, int rmax) {
    const int dw = static_cast<int>(elem / 4);
    return K * rmax * dw <= 48 && K * rmax * dw + 8 * K * dw <= 80;
}

inline int rows_variant(int64_t rows) {
    for (int r : kRowVariants)
        if (rows <= r)
            return r;
    return 0;
}

struct FusedLayout {
    size_t off_red = 0, off_part = 0, total = 0;
    int32_t n_quarters = 0;
};

// vals [max_width][64K] | red [16][64K] uint32 (rescaled path) | part [quarters][64K] binary64
inline FusedLayout fused_layout(const Graph &g, size_t elem, bool rescale, int K) {
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

// Lookup factors read each sample's table (n_slots entries) for
// every edge; the tables of the tiles resident on one XCD (one workgroup per
// CU, 32 CUs) should stay within half of its 4 MiB L2, else the entries are
// fetched again from the Infinity Cache on every edge.
constexpr int64_t kLookupL2Budget = int64_t(2) << 20;
// entry: bytes of a table entry as the interior levels read it (binary32
// paths read a binary32 copy of the tables).
inline bool lookup_tables_fit(const Graph &g, int K, size_t entry) {
    return g.kind != FK_LOOKUP ||
           static_cast<int64_t>(g.n_slots) * kWave * K * static_cast<int64_t>(entry) * 32 <= kLookupL2Budget;
}

// Largest samples-per-lane K in {4, 2, 1} whose accumulators fit in registers
// and whose layout fits in LDS (0: the graph does not fit the fused plan); for
// lookup factors also the largest whose resident tables fit in L2 (K = 1 is
// always allowed).  16-bit storage is a streamed-plan format (it halves HBM
// bytes; the fused plan keeps levels on chip), so it never takes the fused
// plan.
inline int fused_k(const Graph &g, cos_precision p) {
    if (p != COS_FP64 && p != COS_FP32_RESCALED && p != COS_FP32)
        return 0;
    const int rmax = rows_variant((g.max_width + kFusedWaves - 1) / kFusedWaves);
    if (rmax == 0)
        return 0;
    const size_t elem = p == COS_FP64 ? sizeof(double) : sizeof(float);
    for (int K : {4, 2, 1})
        if (acc_fits(elem, K, rmax) && fused_layout(g, elem, p == COS_FP32_RESCALED, K).total <= kLdsBytes &&
            (K == 1 || lookup_tables_fit(g, K, elem)))
            return K;
    return 0;
}

}  // namespace cosdag
