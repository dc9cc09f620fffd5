// cos_evaluate: workspace planning and the per-level launch sequence.
#include <algorithm>

#include "cos_internal.h"

namespace cosdag {

Workspace plan_workspace(const Graph &g, int64_t S, cos_precision p) {
    Workspace w;
    w.S_pad = round_up(std::max<int64_t>(S, 1), kSamplePad);
    const size_t elem = p == COS_FP64 ? sizeof(double) : sizeof(float);
    w.level_elems = g.max_width * w.S_pad;
    size_t off = 0;
    auto take = [&](size_t n) {
        const size_t o = off;
        off = round_up(static_cast<int64_t>(off + n), 256);
        return o;
    };
    w.off_buf0 = take(w.level_elems * elem);
    w.off_buf1 = take(w.level_elems * elem);
    w.off_maxbits = p == COS_FP32_RESCALED ? take(static_cast<size_t>(g.L + 1) * w.S_pad * sizeof(uint32_t)) : 0;
    w.final_chunks = final_chunk_count(g.levels.back().n_edges);
    w.off_partial = take(static_cast<size_t>(w.final_chunks) * w.S_pad * sizeof(double));
    w.bytes = std::max<size_t>(off, 256);
    return w;
}

}  // namespace cosdag

using namespace cosdag;

namespace {
bool valid_precision(cos_precision p) { return p == COS_FP64 || p == COS_FP32_RESCALED || p == COS_FP32; }
}  // namespace

extern "C" cos_status cos_evaluate_workspace_size(const cos_graph *h, int64_t S, cos_precision p, uint64_t *bytes) {
    if (!h || !bytes)
        return fail(COS_EINVAL, "cos_evaluate_workspace_size: NULL argument");
    if (S < 0 || !valid_precision(p))
        return fail(COS_EINVAL, "cos_evaluate_workspace_size: bad S or precision");
    *bytes = plan_workspace(graph_of(h), S, p).bytes;
    return COS_OK;
}

extern "C" cos_status cos_evaluate(const cos_graph *h, const double *x_dev, int64_t S, cos_precision p,
                                   double *out_dev, int32_t *out_exp_dev, void *workspace_dev,
                                   uint64_t workspace_bytes, void *stream) {
    if (!h)
        return fail(COS_EINVAL, "cos_evaluate: graph is NULL");
    if (S < 0 || S > (int64_t(1) << 40))
        return fail(COS_EINVAL, "cos_evaluate: S out of range");
    if (!valid_precision(p))
        return fail(COS_EINVAL, "cos_evaluate: unknown precision");
    if (S == 0)
        return COS_OK;
    if (!x_dev || !out_dev)
        return fail(COS_EINVAL, "cos_evaluate: x or out is NULL");
    const Graph &g = graph_of(h);
    const Workspace w = plan_workspace(g, S, p);
    if (w.S_pad * std::max<int64_t>(g.max_width, 1) > (int64_t(1) << 40))
        return fail(COS_EINVAL, "cos_evaluate: level buffer too large");
    hipStream_t st = static_cast<hipStream_t>(stream);

    void *ws = workspace_dev;
    bool owned = false;
    if (ws) {
        if (workspace_bytes < w.bytes)
            return fail(COS_EINVAL, "cos_evaluate: workspace smaller than cos_evaluate_workspace_size");
        if (reinterpret_cast<uintptr_t>(ws) % 256)
            return fail(COS_EINVAL, "cos_evaluate: workspace must be 256-byte aligned");
    } else {
        hipError_t err = hipMallocAsync(&ws, w.bytes, st);
        if (err != hipSuccess)
            return hip_fail(err, "hipMallocAsync(workspace)");
        owned = true;
    }
    char *base = static_cast<char *>(ws);
    void *bufs[2] = {base + w.off_buf0, base + w.off_buf1};
    uint32_t *maxbits = p == COS_FP32_RESCALED ? reinterpret_cast<uint32_t *>(base + w.off_maxbits) : nullptr;
    double *partial = reinterpret_cast<double *>(base + w.off_partial);

    hipError_t err = hipSuccess;
    if (maxbits)
        err = launch_fill_u32(maxbits, 0u, static_cast<int64_t>(g.L + 1) * w.S_pad, st);
    const void *prev = nullptr;  // level 0: the root, value 1
    for (int l = 1; l <= g.L - 1 && err == hipSuccess; ++l) {
        void *cur = bufs[(l - 1) & 1];
        const uint32_t *pm = (maxbits && l >= 2) ? maxbits + static_cast<int64_t>(l - 1) * w.S_pad : nullptr;
        uint32_t *cm = (maxbits && l <= g.L - 2) ? maxbits + static_cast<int64_t>(l) * w.S_pad : nullptr;
        err = launch_level(g, l, p, prev, cur, w.S_pad, x_dev, S, pm, cm, st);
        prev = cur;
    }
    if (err == hipSuccess)
        err = launch_final(g, p, prev, w.S_pad, x_dev, S, maxbits, partial, w.final_chunks, out_dev, out_exp_dev, st);
    if (owned) {
        hipError_t ferr = hipFreeAsync(ws, st);
        if (err == hipSuccess)
            err = ferr;
    }
    if (err != hipSuccess)
        return hip_fail(err, "cos_evaluate: kernel launch");
    return COS_OK;
}
