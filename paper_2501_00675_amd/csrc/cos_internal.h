// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "cos.h"

namespace cosdag {

// Device edge record, one per edge in canonical (dst, src, params) order,
// 64 bytes so a wavefront fetches it with one scalar load: every lane of a
// wave works on the same edge for different samples, so the record is
// wave-uniform.  The denominator of the edge factor is stored expanded,
//     1 + b |x - k|^2 = c0 + cb |x|^2 + g . x,
//     c0 = 1 + b |k|^2,  cb = b,  g = -2 b k,
// so that with |x|^2 kept per lane it costs four fused multiply-adds.
struct alignas(16) EdgeRec {
    double c0, cb, g0, g1, g2;
    double a;
    int32_t src;        // index of the source node within the previous level
    int32_t unused;
    int32_t row_end;    // 1 if this is the last edge into its destination node
    int32_t zero_rows;  // nodes without in-edges that directly follow that destination
};
static_assert(sizeof(EdgeRec) == 64, "EdgeRec layout");

// Binary32 edge record (32 bytes) read by the binary32 level sweeps: a, b and
// k rounded to binary32 (nearest even), the factor being formed directly as
// a / (1 + b |x - k|^2) in binary32; same source index and row flags as EdgeRec.
struct alignas(16) EdgeRec32 {
    float a, b, k0, k1, k2;
    int32_t src;
    int32_t row_end;
    int32_t zero_rows;
};
static_assert(sizeof(EdgeRec32) == 32, "EdgeRec32 layout");

// The device edge arrays carry this many zeroed records after the last edge,
// so that kernels may fetch records in fixed-size chunks without bounds tests.
constexpr int kEdgePad = 8;

// Lookup edge record (32 bytes): w_e(s) = coef * T_s[slot], the per-sample
// table T given at evaluation as rows [slot][sample]; coef in binary64 and
// rounded to binary32, same source index and row flags as EdgeRec.
struct alignas(16) EdgeRecL {
    double coef;
    float coef32;
    int32_t slot;
    int32_t src;
    int32_t row_end;
    int32_t zero_rows;
    int32_t unused;
};
static_assert(sizeof(EdgeRecL) == 32, "EdgeRecL layout");

// Edge-factor kinds (cos_graph_info.factor_kind).
enum FactorKind : int32_t { FK_RATIONAL = 0, FK_LOOKUP = 1 };
// Kernel-only kind: lookup factors whose interior levels read a binary32 copy
// of the sample tables (the binary32 paths of cos_evaluate).
constexpr int32_t FK_LOOKUP_T32 = 2;

// Per edge level l = 1..L (stored at index l-1).
struct LevelDesc {
    int64_t w_src;     // widths[l-1]
    int64_t w_dst;     // widths[l]
    int64_t e_begin;   // first edge of the level (global canonical index)
    int64_t n_edges;
    int64_t rp_begin;  // offset of this level's row_ptr[w_dst + 1] in the row_ptr array
    int64_t max_deg;   // largest in-degree in this level
    // rows of more than kHubEdges in-edges (interior levels): their chunks of
    // kFinalChunk edges are entries [hub_begin, hub_begin + n_hub_chunks) of
    // Graph::d_hub_chunks, row by row; the first record of such a row holds,
    // in zero_rows, the index of its first chunk relative to hub_begin
    int64_t hub_begin = 0;
    int64_t n_hub_chunks = 0;
    // panel plan (interior levels): panels [panel_begin, panel_begin + n_panels)
    // of Graph::d_panels, the first n_panel_half0 covering the first half of
    // the rows; panel_lds: the largest panel's LDS bytes
    int64_t panel_begin = 0;
    int64_t n_panel_half0 = 0;
    int64_t n_panels = 0;
    int64_t panel_lds = 0;
};

// Compact level table read by the fused kernel (device copy).
struct LevelDev {
    int32_t w_dst;
    int32_t rp_begin;
    int32_t e_begin;
    int32_t n_edges;
    int32_t hubs;  // 1 if an interior level has a node of more than kHubEdges in-edges
    int32_t pad[3];
};

struct Graph {
    int32_t kind = FK_RATIONAL;       // edge-factor kind
    int32_t n_slots = 0;              // lookup: entries of each sample's table
    int32_t L = 0;
    std::vector<int64_t> widths;      // L+1
    std::vector<int64_t> level_first; // L+2, first global node id of each level
    std::vector<LevelDesc> levels;    // L
    int64_t n_nodes = 0, n_edges = 0;
    int64_t max_width = 0;            // interior levels 1..L-1
    int64_t max_in_degree = 0;        // interior levels 1..L-1
    // binary16 storage: headroom exponent h[l] of node level l = 1..L-1
    // (h[0] unused); empty when the graph's factors have no bound (lookup)
    std::vector<int32_t> h16;
    // whether every binary32 record field is finite: a finite binary64
    // parameter beyond the binary32 range rounds to +-inf, and the binary32
    // sweeps then refuse the graph
    bool f32_ok = true;
    // canonical host copy (for export)
    std::vector<int32_t> h_src, h_dst;
    std::vector<double> h_a, h_b, h_k;       // rational factors
    std::vector<int32_t> h_slot;              // lookup factors
    std::vector<double> h_coef;
    // device copies
    void *d_base = nullptr;
    size_t d_bytes = 0;
    int32_t *d_row_ptr = nullptr;     // global edge indices, per level w_dst+1 entries
    EdgeRec *d_edges = nullptr;       // binary64 records (binary64 sweeps, every final node)
    EdgeRec32 *d_edges32 = nullptr;   // binary32 records (interior levels of the binary32 sweeps)
    EdgeRecL *d_edgesL = nullptr;     // lookup records (every level, every precision)
    LevelDev *d_levels = nullptr;     // L entries
    int32_t *d_h16 = nullptr;         // h16 on the device (L entries; NULL when h16 is empty)
    int32_t *d_hub_chunks = nullptr;  // (first edge, end edge) pairs of the chunks of high in-degree rows
    bool panel_ok = false;            // every interior level has a panel table (binary32 panel plan)
    int32_t *d_panels = nullptr;      // (first row, end row, first edge, end edge) per panel, level after level
    int64_t max_hub_chunks = 0;       // most chunks of such rows in one level
    int device = 0;
    cos_path path = COS_PATH_AUTO;    // kernel plan chosen by cos_graph_set_path
};

const Graph &graph_of(const cos_graph *h);
// COS_OK if the graph's records can be evaluated at precision p, else the
// refusal (COS_EINVAL, message prefixed with who): binary32 sweeps need every
// binary32 record field finite.
cos_status check_precision_range(const Graph &g, cos_precision p, const char *who);

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
cos_status fail(cos_status st, const std::string &msg);
cos_status hip_fail(hipError_t err, const char *what);

// ---------------------------------------------------------------- timing probe
enum KernelKind { KK_LEVEL = 0, KK_FUSED = 1, KK_FINAL_PARTIAL = 2, KK_FINAL_COMBINE = 3,
                  KK_FILL = 4, KK_SERVE = 5, KK_HUB = 6, KK_COUNT = 7 };
bool timing_on();
void timing_begin(int kind, hipStream_t s);
void timing_end(int kind, hipStream_t s);

// Brackets one kernel launch with timing events while the probe is enabled.
struct TimedLaunch {
    int kind;
    hipStream_t s;
    TimedLaunch(int k, hipStream_t st) : kind(k), s(st) { timing_begin(kind, s); }
    ~TimedLaunch() { timing_end(kind, s); }
};

// ---------------------------------------------------------------- launch plans
constexpr int kWave = 64;
constexpr int kBlock = 256;          // 4 wavefronts per workgroup (streamed kernels)
constexpr int kSamplePad = 256;      // S is padded to a multiple of this
constexpr int kXcds = 8;             // MI355X: 8 accelerator dies, one L2 each
constexpr int kFinalChunk = 256;     // final-node edges per partial sum (4 quarters of 64)
constexpr int kQuarter = kFinalChunk / 4;
// An interior node with more in-edges than this is summed in chunks of
// kFinalChunk edges (the final node's order) instead of edge after edge.
constexpr int kHubEdges = 1024;
// Panel plan: bytes of a node's values in one tile of the tile-major level
// buffers (one 128-byte line: 32 binary32 or 64 16-bit samples per tile),
// threads per workgroup, samples staged in LDS at a time, LDS a panel's records
// and row offsets may take, and the narrowest level width for which the plan is
// built (narrower levels keep a 256-sample tile's slice in L2 on the plain
// streamed plan).
constexpr int kPanelLine = 128;
constexpr int kPanelThreads = 1024;
constexpr int kPanelBlockSamples = 256;
constexpr int kPanelSampleBytes = kPanelBlockSamples * 16;
constexpr int64_t kPanelLdsBytes = 160 * 1024 - 512;       // the dynamic LDS of a workgroup (512 B static)
constexpr int64_t kPanelRecBytes = kPanelLdsBytes - kPanelSampleBytes;  // a panel's records and offsets
constexpr int64_t kPanelMinWidth = 4097;
constexpr int kPanelMaxRows = 1024;  // rows of one panel (8 per lane at binary32, 16 at 16 bits)
constexpr int kPanelPadRecs = 8;     // zeroed records after a panel's own in LDS
constexpr int kFusedWaves = 16;      // wavefronts per workgroup of the LDS-resident sweep

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
// Samples per tile of the panel plan for stored values of vb bytes.
__host__ __device__ constexpr int panel_tile(int vb) { return kPanelLine / vb; }

// Precisions whose interior levels carry the per-(level, sample) exponent.
__host__ __device__ inline bool is_rescaled(cos_precision p) {
    return p == COS_FP32_RESCALED || p == COS_FP16_RESCALED || p == COS_BF16_RESCALED;
}
// Bytes of one stored level value.
inline size_t value_bytes(cos_precision p) {
    return p == COS_FP64 ? 8 : (p == COS_FP16_RESCALED || p == COS_BF16_RESCALED) ? 2 : 4;
}
// Largest headroom exponent of binary16 storage (row sums of |a| up to 2^110).
constexpr int32_t kMaxHeadroom16 = 96;

// Workspace layout of one evaluate call.  The streamed plan sweeps the graph
// once per chunk of S_chunk samples (S_pad = S_chunk rounded to kSamplePad);
// a chunk's level buffer stays below kMaxLevelBytes so kernels can address
// rows with 32-bit byte offsets.
struct Workspace {
    size_t bytes = 0;
    size_t off_buf0 = 0, off_buf1 = 0, off_maxbits = 0, off_partial = 0;
    size_t off_table32 = 0;    // binary32 sample tables [n_slots][S_pad] (lookup, binary32 paths), if used
    size_t off_hub = 0;        // chunk sums of high in-degree rows [chunk][S_pad] in the value type, if any
    bool table32 = false;
    int64_t S_chunk = 0;       // samples per sweep
    int64_t S_pad = 0;         // row length of the level buffers
    int32_t final_chunks = 0;  // partial sums of the final node
    bool fused = false;        // whole sweep in the LDS-resident kernel
};
constexpr int64_t kMaxLevelBytes = int64_t(1) << 31;
// Whether the sweep of a graph at precision p reads binary32 copies of the
// sample tables (lookup factors, binary32 arithmetic).
inline bool uses_table32(const Graph &g, cos_precision p) {
    return g.kind == FK_LOOKUP && (p == COS_FP32 || p == COS_FP32_RESCALED || p == COS_BF16_RESCALED);
}
// Layout for sweeps of at most S_chunk samples (S_chunk > 0); with_table32
// false leaves out the binary32 tables (the serving runtime reads binary64 ones).
Workspace layout_for_chunk(const Graph &g, int64_t S_chunk, cos_precision p, bool with_table32 = true);
// Natural plan for S samples: fused if it fits, else the largest chunk allowed.
Workspace plan_workspace(const Graph &g, int64_t S, cos_precision p);
// Largest sample chunk whose level buffer stays below kMaxLevelBytes.
int64_t max_chunk(const Graph &g, cos_precision p);

// Kernel launchers.  All return hipSuccess or the launch error.  x points at
// the chunk's first sample; xs is the distance between coordinate rows of x.
// Rescaled precisions: prev_max / cur_max are the maxbits rows l-1 and l,
// h_next the headroom exponent folded into cur_max (0 unless binary16).
// t32 (nullable): binary32 sample tables [n_slots][ld] of a lookup graph,
// read instead of x by the interior levels.
// hub (nullable): room for the level's chunk sums of high in-degree rows,
// computed by a launch of their own before the level's; NULL: the level
// kernel sums such rows itself (the same bits).
hipError_t launch_level(const Graph &g, int l, cos_precision p, const void *prev, void *cur,
                        int64_t ld, const double *x, int64_t S, int64_t xs, const uint32_t *prev_max,
                        uint32_t *cur_max, int32_t h_next, hipStream_t s, const float *t32 = nullptr,
                        void *hub = nullptr);
// t32[i][s] = fl32(x[i][s]) for s < S, 0 for S <= s < ld (n rows); tile_major:
// the same values stored [tile][i][panel_tile(4)] (the binary32 panel plan's
// tables, one 128-byte line per slot and tile).
hipError_t launch_table32(const double *x, int64_t xs, int64_t S, int32_t n, float *t32, int64_t ld,
                          hipStream_t s, bool tile_major = false);
// tile_major: the last interior level is stored [tile][node][panel_tile(value
// bytes)] (panel plan), with max_width rows per tile.
hipError_t launch_final(const Graph &g, cos_precision p, const void *prev, int64_t ld,
                        const double *x, int64_t S, int64_t xs, const uint32_t *maxbits, double *partial,
                        int32_t chunks, double *out, int32_t *out_exp, hipStream_t s, bool tile_major = false);
// Panel plan: whether it applies to graph g at precision p, and one interior
// level (level buffers tile-major, ld = the padded sample count).
bool panel_fits(const Graph &g, cos_precision p);
// Lookup factors read t32, the tile-major binary32 tables (launch_table32 with tile_major).
hipError_t launch_level_panel(const Graph &g, int l, cos_precision p, const void *prev, void *cur, int64_t ld,
                              const double *x, int64_t S, int64_t xs, const uint32_t *prev_max, uint32_t *cur_max,
                              int32_t h_next, const float *t32, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);

// A whole run of Monte Carlo walkers (cos_mc_run): state x [3][C], v [C],
// proposals xp [3][C] and their values vp [C], per-walker sums.
struct McArgs {
    double *x, *v, *xp, *vp;
    int64_t C, step0, n_steps;
    uint64_t seed;
    double sigma;
    int64_t *accepted;
    double *acc;
};

// LDS-resident whole-graph sweep (kernels_fused.hip).  With mc, one launch
// runs every step of the walkers instead (rational factors).
bool fused_fits(const Graph &g, cos_precision p);
hipError_t launch_fused(const Graph &g, cos_precision p, const double *x, int64_t S, double *out,
                        int32_t *out_exp, hipStream_t s, const McArgs *mc = nullptr, const float *t32 = nullptr,
                        int64_t ld32 = 0);

int32_t final_chunk_count(int64_t final_in_degree);

}  // namespace cosdag
