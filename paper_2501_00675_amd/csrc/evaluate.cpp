// cos_evaluate: plan (fused or streamed, sample chunks), workspace layout and
// the per-level launch sequence.
#include <algorithm>
#include <map>
#include <mutex>
#include <string>

#include "cos_internal.h"

namespace cosdag {

namespace {
size_t elem_size(cos_precision p) { return value_bytes(p); }
}  // namespace

// Largest chunk (multiple of kSamplePad) whose level buffer stays below
// kMaxLevelBytes; 0 if even kSamplePad samples do not.
int64_t max_chunk(const Graph &g, cos_precision p) {
    const int64_t w = std::max<int64_t>(g.max_width, 1);
    const int64_t cap = (kMaxLevelBytes - 1) / (w * static_cast<int64_t>(elem_size(p)));
    return cap / kSamplePad * kSamplePad;
}

Workspace layout_for_chunk(const Graph &g, int64_t S_chunk, cos_precision p, bool with_table32) {
    Workspace w;
    w.S_chunk = S_chunk;
    w.S_pad = round_up(std::max<int64_t>(S_chunk, 1), kSamplePad);
    const size_t level_bytes = static_cast<size_t>(g.max_width * w.S_pad) * elem_size(p);
    size_t off = 0;
    auto take = [&](size_t n) {
        const size_t o = off;
        off = static_cast<size_t>(round_up(static_cast<int64_t>(off + n), 256));
        return o;
    };
    w.off_buf0 = take(level_bytes);
    w.off_buf1 = take(level_bytes);
    w.off_maxbits = is_rescaled(p) ? take(static_cast<size_t>(g.L + 1) * w.S_pad * sizeof(uint32_t)) : 0;
    w.final_chunks = final_chunk_count(g.levels.back().n_edges);
    w.off_partial = take(static_cast<size_t>(w.final_chunks) * w.S_pad * sizeof(double));
    w.table32 = with_table32 && uses_table32(g, p);
    if (w.table32)
        w.off_table32 = take(static_cast<size_t>(g.n_slots) * w.S_pad * sizeof(float));
    if (g.max_hub_chunks > 0)  // chunk sums of rows of high in-degree, binary64 or binary32
        w.off_hub = take(static_cast<size_t>(g.max_hub_chunks) * w.S_pad * (p == COS_FP64 ? 8 : 4));
    w.bytes = std::max<size_t>(off, 256);
    return w;
}

Workspace plan_workspace(const Graph &g, int64_t S, cos_precision p) {
    Workspace w;
    w.fused = g.path == COS_PATH_FUSED || (g.path == COS_PATH_AUTO && fused_fits(g, p));
    if (w.fused) {  // levels live in LDS: device scratch only for binary32 tables
        w.S_chunk = S;
        w.S_pad = round_up(std::max<int64_t>(S, 1), kSamplePad);
        w.table32 = uses_table32(g, p);
        const size_t t32 = w.table32 ? static_cast<size_t>(g.n_slots) * w.S_pad * sizeof(float) : 0;
        w.bytes = std::max<size_t>(static_cast<size_t>(round_up(static_cast<int64_t>(t32), 256)), 256);
        return w;
    }
    const int64_t cap = max_chunk(g, p);
    return layout_for_chunk(g, std::min<int64_t>(std::max<int64_t>(S, 1), std::max<int64_t>(cap, 1)), p);
}

}  // namespace cosdag

using namespace cosdag;

namespace {
bool valid_precision(cos_precision p) {
    return p == COS_FP64 || p == COS_FP32_RESCALED || p == COS_FP32 || p == COS_FP16_RESCALED ||
           p == COS_BF16_RESCALED;
}

// Headroom exponent of node level l under precision p (binary16 only).
int32_t headroom(const Graph &g, cos_precision p, int l) {
    return p == COS_FP16_RESCALED ? g.h16[static_cast<size_t>(l)] : 0;
}

// One streamed sweep of the graph for samples [0, S) of the chunk starting at x.
hipError_t sweep_chunk(const Graph &g, cos_precision p, const Workspace &w, char *base, const double *x,
                       int64_t S, int64_t xs, double *out, int32_t *out_exp, hipStream_t st) {
    void *bufs[2] = {base + w.off_buf0, base + w.off_buf1};
    uint32_t *maxbits = is_rescaled(p) ? reinterpret_cast<uint32_t *>(base + w.off_maxbits) : nullptr;
    double *partial = reinterpret_cast<double *>(base + w.off_partial);
    float *t32 = w.table32 ? reinterpret_cast<float *>(base + w.off_table32) : nullptr;
    hipError_t err = hipSuccess;
    // lookup factors at binary32: the chunk's tables rounded once, read by the interior levels
    // wide graphs at binary32 or 16-bit storage: level buffers tile-major, levels by row panels
    // (kernels_panel.hip); lookup factors then read the binary32 tables tile-major too
    const bool panel = (g.path == COS_PATH_AUTO || g.path == COS_PATH_PANEL) && panel_fits(g, p);
    if (t32)
        err = launch_table32(x, xs, S, g.n_slots, t32, w.S_pad, st, panel);
    // row 0: the root's value 1 times level 1's headroom 2^h (0 = no shift);
    // rows 1..L: zero, for the atomic max of each level
    const int32_t h1 = g.L >= 2 ? headroom(g, p, 1) : 0;
    if (maxbits && err == hipSuccess)
        err = launch_fill_u32(maxbits, h1 ? static_cast<uint32_t>(127 + h1) << 23 : 0u, w.S_pad, st);
    if (maxbits && err == hipSuccess)
        err = launch_fill_u32(maxbits + w.S_pad, 0u, static_cast<int64_t>(g.L) * w.S_pad, st);
    const void *prev = nullptr;  // level 0: the root, value 1
    for (int l = 1; l <= g.L - 1 && err == hipSuccess; ++l) {
        void *cur = bufs[(l - 1) & 1];
        const uint32_t *pm = maxbits ? maxbits + static_cast<int64_t>(l - 1) * w.S_pad : nullptr;
        uint32_t *cm = (maxbits && l <= g.L - 2) ? maxbits + static_cast<int64_t>(l) * w.S_pad : nullptr;
        const int32_t h_next = l <= g.L - 2 ? headroom(g, p, l + 1) : 0;
        if (panel)
            err = launch_level_panel(g, l, p, prev, cur, w.S_pad, x, S, xs, pm, cm, h_next, t32, st);
        else
            err = launch_level(g, l, p, prev, cur, w.S_pad, x, S, xs, pm, cm, h_next, st, t32,
                               g.max_hub_chunks > 0 ? base + w.off_hub : nullptr);
        prev = cur;
    }
    if (err == hipSuccess)
        err = launch_final(g, p, prev, w.S_pad, x, S, xs, maxbits, partial, w.final_chunks, out, out_exp, st,
                           panel && g.L >= 2);
    return err;
}
}  // namespace

extern "C" cos_status cos_evaluate_workspace_size(const cos_graph *h, int64_t S, cos_precision p, uint64_t *bytes) {
    if (!h || !bytes)
        return fail(COS_EINVAL, "cos_evaluate_workspace_size: NULL argument");
    if (S < 0 || !valid_precision(p))
        return fail(COS_EINVAL, "cos_evaluate_workspace_size: bad S or precision");
    *bytes = plan_workspace(graph_of(h), S, p).bytes;
    return COS_OK;
}

namespace {

// The checks and launches of one evaluate call.  ws == NULL: the workspace is
// allocated and freed in stream order.  `who` prefixes error messages.
cos_status evaluate_with(const cos_graph *h, const double *x_dev, int64_t S, cos_precision p, double *out_dev,
                         int32_t *out_exp_dev, void *ws, uint64_t workspace_bytes, hipStream_t st,
                         const char *who) {
    const std::string w_ = who;
    if (!h)
        return fail(COS_EINVAL, w_ + ": graph is NULL");
    if (S < 0 || S > (int64_t(1) << 40))
        return fail(COS_EINVAL, w_ + ": S out of range");
    if (!valid_precision(p))
        return fail(COS_EINVAL, w_ + ": unknown precision");
    if (S == 0)
        return COS_OK;
    if (!x_dev || !out_dev)
        return fail(COS_EINVAL, w_ + ": x or out is NULL");
    const Graph &g = graph_of(h);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != g.device)
        return fail(COS_EINVAL, w_ + ": the current device is not the graph's device");
    if (check_precision_range(g, p, who) != COS_OK)
        return COS_EINVAL;
    if (value_bytes(p) == 2 && g.path == COS_PATH_FUSED)
        return fail(COS_EINVAL, w_ + ": 16-bit level storage runs on the streamed plan only");
    if (p == COS_FP16_RESCALED && g.h16.empty())
        return fail(COS_EINVAL, w_ + ": binary16 storage needs rational factors with level row sums of "
                                     "|a| below 2^110 (use COS_BF16_RESCALED or COS_FP32_RESCALED)");
    Workspace w = plan_workspace(g, S, p);
    if (w.fused && !fused_fits(g, p))
        return fail(COS_EINVAL, w_ + ": the fused plan was requested but the graph does not fit in LDS");
    if (g.path == COS_PATH_PANEL && !panel_fits(g, p))
        return fail(COS_EINVAL, w_ + ": the panel plan was requested but applies only to graphs wider than 4096 "
                                     "nodes without nodes of more than 1024 in-edges, at binary32 and (rational "
                                     "factors) 16-bit storage precisions");
    if (!w.fused && max_chunk(g, p) < kSamplePad)
        return fail(COS_EINVAL, w_ + ": a level is too wide for the streamed plan");

    bool owned = false;
    if (ws) {
        if (reinterpret_cast<uintptr_t>(ws) % 256)
            return fail(COS_EINVAL, w_ + ": workspace must be 256-byte aligned");
        if (workspace_bytes < w.bytes) {
            // a smaller workspace: sweep in smaller sample chunks that fit in it
            if (w.fused)
                return fail(COS_EINVAL, w_ + ": workspace of " + std::to_string(workspace_bytes) +
                                            " bytes is smaller than the " + std::to_string(w.bytes) +
                                            " bytes the fused plan needs");
            int64_t c = w.S_pad - kSamplePad;
            while (c >= kSamplePad && layout_for_chunk(g, c, p).bytes > workspace_bytes)
                c -= kSamplePad;
            if (c < kSamplePad)
                return fail(COS_EINVAL, w_ + ": workspace of " + std::to_string(workspace_bytes) +
                                            " bytes is too small for even " + std::to_string(kSamplePad) +
                                            " samples per sweep (" +
                                            std::to_string(layout_for_chunk(g, kSamplePad, p).bytes) +
                                            " bytes)");
            w = layout_for_chunk(g, c, p);
        }
    } else {
        hipError_t err = hipMallocAsync(&ws, w.bytes, st);
        if (err != hipSuccess)
            return hip_fail(err, "hipMallocAsync(workspace)");
        owned = true;
    }

    hipError_t err = hipSuccess;
    if (w.fused) {
        float *t32 = w.table32 ? static_cast<float *>(ws) : nullptr;
        if (t32)
            err = launch_table32(x_dev, S, S, g.n_slots, t32, w.S_pad, st);
        if (err == hipSuccess)
            err = launch_fused(g, p, x_dev, S, out_dev, out_exp_dev, st, nullptr, t32, w.S_pad);
    } else {
        for (int64_t s0 = 0; s0 < S && err == hipSuccess; s0 += w.S_chunk) {
            const int64_t n = std::min(w.S_chunk, S - s0);
            err = sweep_chunk(g, p, w, static_cast<char *>(ws), x_dev + s0, n, S, out_dev + s0,
                              out_exp_dev ? out_exp_dev + s0 : nullptr, st);
        }
    }
    if (owned) {
        hipError_t ferr = hipFreeAsync(ws, st);
        if (err == hipSuccess)
            err = ferr;
    }
    if (err != hipSuccess)
        return hip_fail(err, (w_ + ": kernel launch").c_str());
    return COS_OK;
}

// Fixed workspace of cos_evaluate_no_alloc, one copy per device.  In host code
// `scratch` names a host-side stand-in, not device memory: kernels are given
// the device address hipGetSymbolAddress returns, looked up once per device.
constexpr uint64_t kScratchBytes = uint64_t(COS_NO_ALLOC_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device -> address of that device's copy of scratch

// The calling thread's current device must be dev.
cos_status scratch_of_device(int dev, void **ptr) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *p = nullptr;
        const hipError_t err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (err != hipSuccess)
            return hip_fail(err, "cos_evaluate_no_alloc: hipGetSymbolAddress(scratch)");
        if (p == nullptr || reinterpret_cast<uintptr_t>(p) % 256)
            return fail(COS_EDEVICE, "cos_evaluate_no_alloc: the scratch array has no usable device address");
        it = g_scratch_ptr.emplace(dev, p).first;
    }
    *ptr = it->second;
    return COS_OK;
}

}  // namespace

extern "C" cos_status cos_evaluate(const cos_graph *h, const double *x_dev, int64_t S, cos_precision p,
                                   double *out_dev, int32_t *out_exp_dev, void *workspace_dev,
                                   uint64_t workspace_bytes, void *stream) {
    return evaluate_with(h, x_dev, S, p, out_dev, out_exp_dev, workspace_dev, workspace_bytes,
                         static_cast<hipStream_t>(stream), "cos_evaluate");
}

extern "C" cos_status cos_evaluate_no_alloc(const cos_graph *h, const double *x_dev, int64_t S, cos_precision p,
                                            double *out_dev, int32_t *out_exp_dev, void *stream) {
    if (!h)
        return fail(COS_EINVAL, "cos_evaluate_no_alloc: graph is NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != graph_of(h).device)
        return fail(COS_EINVAL, "cos_evaluate_no_alloc: the current device is not the graph's device");
    void *ws = nullptr;
    const cos_status st = scratch_of_device(dev, &ws);
    if (st != COS_OK)
        return st;
    return evaluate_with(h, x_dev, S, p, out_dev, out_exp_dev, ws, kScratchBytes, static_cast<hipStream_t>(stream),
                         "cos_evaluate_no_alloc");
}
