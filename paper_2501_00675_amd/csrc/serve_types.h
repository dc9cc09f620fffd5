// Types shared by the serving runtime (server.cpp) and its step kernels
// (serve.hip).
#pragma once

#include "cos_internal.h"

namespace cosdag {

// Work a request contributes to one step.
enum ServeKind : uint32_t {
    SK_FUSED = 0,    // the whole graph for 64-sample tiles, levels in LDS (one step per request)
    SK_LEVEL = 1,    // one interior level: items = (row group of 32 rows) x (tile of 256 samples)
    SK_FINAL = 2,    // final-node partial sums: items = (chunk of 256 edges) x (tile of 128 samples)
    SK_COMBINE = 3,  // final-node combine: items = tiles of 256 samples
    SK_TABLE32 = 4,  // binary32 copy of a lookup request's tables: items = 256 entries
};

constexpr int kServeLevelK = 4;                            // samples per lane, level items
constexpr int kServeLevelRows = 8;                         // rows per wave, level items
constexpr int kServeLevelRowsPerItem = 4 * kServeLevelRows;  // 4 waves per streamed-kernel workgroup
constexpr int kServeFinalK = 2;                            // samples per lane, final-node items
constexpr int kServeCombineTile = kBlock;                  // samples per combine item
constexpr int kServeMaxEntries = 512;                      // requests per step (upper bound on slots)

// One admitted request as the step kernels see it (device copy per slot).
struct ServeReqDev {
    const int32_t *row_ptr;
    const EdgeRec *edges;
    const EdgeRec32 *edges32;
    const EdgeRecL *edgesL;   // lookup factors (x is then the sample's table, [n_slots][S])
    const LevelDev *levels;
    const int32_t *h16;       // binary16 storage: the graph's headroom exponents per node level
    const double *x;
    double *out;
    int32_t *out_exp;
    char *ws;                 // workspace of a streamed request (level buffers, exponents, partials)
    float *t32;               // streamed lookup request at binary32: its tables' binary32 copy [n_slots][S_pad]
    int64_t S;
    int64_t S_pad;
    uint64_t off_buf0, off_buf1, off_maxbits, off_partial;
    int32_t L;
    int32_t precision;        // cos_precision
    int32_t rows_variant;     // fused requests: rows per wave (compile-time variant)
    int32_t final_chunks;     // streamed requests: final-node partial rows
    int32_t n_slots;          // lookup factors: table entries per sample
    uint32_t off_red, off_part;  // fused requests: LDS layout (one sample per lane)
};

struct StepEntry {
    uint32_t slot;
    uint32_t kind;        // ServeKind
    uint32_t level;       // SK_LEVEL: the level l
    uint32_t n_items;
    uint32_t item_base;   // items of earlier entries of the same section
    uint32_t n_rg;        // SK_LEVEL: row groups; SK_FINAL: chunks
    uint32_t pad[2];
};

// Sections of a step, each run by its own kernel: whole-graph (fused) work and
// level / final / combine (streamed) work, for rational and for lookup
// factors.  Entries are stored section by section; each section numbers its
// items from 0.
enum ServeSection : uint32_t { SS_FUSED = 0, SS_STREAMED = 1, SS_FUSED_LOOKUP = 2, SS_STREAMED_LOOKUP = 3,
                               SS_COUNT = 4 };

// A newly admitted request's slot entry and the initial value of its exponent
// rows, carried by the first step that includes the request: the step's set-up
// kernel writes them before the step kernels run.
struct StepSetup {
    uint32_t slot;
    uint32_t fill;  // 1: set the exponent rows (a streamed request at a rescaled precision)
    uint32_t row0;  // exponent row 0: 2^h_1 as binary32 bits for binary16 storage, else 0 (rows 1..L: 0)
    uint32_t pad;
    ServeReqDev req;
};

struct StepTable {
    uint32_t n[SS_COUNT];      // entries per section
    uint32_t items[SS_COUNT];  // items per section
    uint32_t n_setup;            // newly admitted requests whose set-up this step carries
    uint32_t pad[3];
    // item counters of the streamed sections, one per XCD and section, a cache
    // line each (uploaded as 0 with the table)
    struct alignas(128) Counter {
        uint32_t v;
    } claimed[SS_COUNT][kXcds];
    StepEntry e[kServeMaxEntries];
    StepSetup setup[kServeMaxEntries];
};
// First entry of section sec.
__host__ __device__ inline uint32_t section_begin(const StepTable &t, uint32_t sec) {
    uint32_t b = 0;
    for (uint32_t i = 0; i < sec; ++i)
        b += t.n[i];
    return b;
}

// Build the executable graph of one step: upload of the host table h_tab to
// d_tab, the set-up kernel (slot entries and exponent rows of the newly
// admitted requests), then one kernel per section as independent branches
// reading d_tab and the slot table d_reqs -- the two rational-factor sections
// only (with_lookup false) or all four.
hipError_t serve_build_step_graph(StepTable *d_tab, const StepTable *h_tab, ServeReqDev *d_reqs,
                                  bool with_lookup, hipGraphExec_t *exec);

}  // namespace cosdag
