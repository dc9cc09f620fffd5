// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "cos.h"

namespace cosdag {

// Device edge records, one per edge in canonical (dst, src, params) order.
// Each is read with scalar loads by a whole wavefront: every lane of a wave
// works on the same edge for different samples, so the record is uniform.
struct alignas(16) EdgeF64 {
    double k0, k1, k2, b, a;
    int32_t src;  // index of the source node within the previous level
    int32_t pad;
};
static_assert(sizeof(EdgeF64) == 48, "EdgeF64 layout");

struct alignas(16) EdgeF32 {
    float k0, k1, k2, b, a;
    int32_t src;
    int32_t pad0, pad1;
};
static_assert(sizeof(EdgeF32) == 32, "EdgeF32 layout");

// Per edge level l = 1..L (stored at index l-1).
struct LevelDesc {
    int64_t w_src;     // widths[l-1]
    int64_t w_dst;     // widths[l]
    int64_t e_begin;   // first edge of the level (global canonical index)
    int64_t n_edges;
    int64_t rp_begin;  // offset of this level's row_ptr[w_dst + 1] in the row_ptr array
    int64_t max_deg;   // largest in-degree in this level
};

struct Graph {
    int32_t L = 0;
    std::vector<int64_t> widths;      // L+1
    std::vector<int64_t> level_first; // L+2, first global node id of each level
    std::vector<LevelDesc> levels;    // L
    int64_t n_nodes = 0, n_edges = 0;
    int64_t max_width = 0;            // interior levels 1..L-1
    int64_t max_in_degree = 0;        // interior levels 1..L-1
    // canonical host copy (for export)
    std::vector<int32_t> h_src, h_dst;
    std::vector<double> h_a, h_b, h_k;
    // device copies
    void *d_base = nullptr;
    size_t d_bytes = 0;
    int32_t *d_row_ptr = nullptr;     // global edge indices, per level w_dst+1 entries
    EdgeF64 *d_e64 = nullptr;
    EdgeF32 *d_e32 = nullptr;
    int device = 0;
};

const Graph &graph_of(const cos_graph *h);

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
cos_status fail(cos_status st, const std::string &msg);
cos_status hip_fail(hipError_t err, const char *what);

// ---------------------------------------------------------------- timing probe
enum KernelKind { KK_LEVEL = 0, KK_FUSED = 1, KK_FINAL_PARTIAL = 2, KK_FINAL_COMBINE = 3,
                  KK_FILL = 4, KK_SERVE = 5, KK_COUNT = 6 };
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
constexpr int kBlock = 256;          // 4 wavefronts per workgroup
constexpr int kSamplePad = 256;      // S is padded to a multiple of this

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Workspace layout of one evaluate call.
struct Workspace {
    size_t bytes = 0;
    size_t off_buf0 = 0, off_buf1 = 0, off_maxbits = 0, off_partial = 0;
    int64_t S_pad = 0;
    int64_t level_elems = 0;   // max_width * S_pad
    int32_t final_chunks = 0;  // partial sums of the final node
};
Workspace plan_workspace(const Graph &g, int64_t S, cos_precision p);

// Kernel launchers (kernels_level.hip).  All return hipSuccess or the launch error.
hipError_t launch_level(const Graph &g, int l, cos_precision p, const void *prev, void *cur,
                        int64_t ld, const double *x, int64_t S, const uint32_t *prev_max,
                        uint32_t *cur_max, hipStream_t s);
hipError_t launch_final(const Graph &g, cos_precision p, const void *prev, int64_t ld,
                        const double *x, int64_t S, const uint32_t *maxbits, double *partial,
                        int32_t chunks, double *out, int32_t *out_exp, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);

int32_t final_chunk_count(int64_t final_in_degree);

}  // namespace cosdag
