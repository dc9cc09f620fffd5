// Monte Carlo over sample configurations: C Markov-chain walkers, one per
// sample lane of the level sweep.  The paper integrates the diagram sum over
// the vertex coordinates by Monte Carlo (Sec. II.B), evaluates the many
// walkers' configurations together (Sec. II.C, "Distributing the task on a
// grid of blocks") and keeps proposal and acceptance on the device with a
// device random-number generator (Sec. IV).  One step of every walker:
//
//   r0..r3 = Philox4x64-10(counter (c, t, 0, 0), key (seed, 0))
//   u_i    = (r_i >> 11) 2^-53
//   x'     = x + sigma (2 u_{0..2} - 1)          proposal (product, then sum)
//   v'     = V(x')                              the level sweep
//   accept iff u_3 |v| < |v'|                   Metropolis for the density |V|
//   acc[0] += sign v, acc[1] += |x|^2, accepted += take   (at the new state)
//
// Every random number is a function of (seed, walker, step) only, so a run
// split into several calls, or over a subset of walkers, is bit-identical to
// one call.  Graphs that take the fused plan run the whole call in one
// launch (mc_fused_kernel: the walkers of a tile stay with one workgroup for
// every step); others take three launches per step (propose, cos_evaluate,
// accept).  Both give the same bits.
#include <cmath>

#include "mc_device.h"

namespace cosdag {
namespace {

__global__ __launch_bounds__(kBlock) void mc_propose_kernel(const double *__restrict__ x, double *__restrict__ xp,
                                                            int64_t C, int64_t t, uint64_t seed, double sigma) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (c < C)
        mc_propose(x, xp, C, c, t, seed, sigma);
}

__global__ __launch_bounds__(kBlock) void mc_accept_kernel(double *__restrict__ x, double *__restrict__ v,
                                                           const double *__restrict__ xp,
                                                           const double *__restrict__ vp, int64_t C, int64_t t,
                                                           uint64_t seed, int64_t *__restrict__ accepted,
                                                           double *__restrict__ acc) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (c < C)
        mc_accept(x, v, xp, vp, C, c, t, seed, accepted, acc);
}

struct McLayout {
    size_t off_xp = 0, off_vp = 0, off_eval = 0, eval_bytes = 0, total = 0;
};

McLayout mc_layout(const cos_graph *h, int64_t C, cos_precision p, cos_status &st) {
    McLayout m;
    auto up = [](size_t n) { return static_cast<size_t>(round_up(static_cast<int64_t>(n), 256)); };
    m.off_xp = 0;
    m.off_vp = up(3 * static_cast<size_t>(C) * sizeof(double));
    m.off_eval = m.off_vp + up(static_cast<size_t>(C) * sizeof(double));
    uint64_t eb = 0;
    st = cos_evaluate_workspace_size(h, C, p, &eb);
    m.eval_bytes = eb;
    m.total = m.off_eval + up(eb);
    return m;
}

}  // namespace
}  // namespace cosdag

using namespace cosdag;

extern "C" cos_status cos_mc_workspace_size(const cos_graph *h, int64_t C, cos_precision p, uint64_t *bytes) {
    if (!h || !bytes)
        return fail(COS_EINVAL, "cos_mc_workspace_size: NULL argument");
    if (C < 1 || C > (int64_t(1) << 31))
        return fail(COS_EINVAL, "cos_mc_workspace_size: C must be in 1..2^31");
    cos_status st = COS_OK;
    const McLayout m = mc_layout(h, C, p, st);
    if (st != COS_OK)
        return st;
    *bytes = m.total;
    return COS_OK;
}

extern "C" cos_status cos_mc_run(const cos_graph *h, cos_precision p, int64_t C, double *x_dev, double *v_dev,
                                 int64_t step0, int64_t n_steps, uint64_t seed, double sigma,
                                 int64_t *accepted_dev, double *acc_dev, void *workspace_dev,
                                 uint64_t workspace_bytes, void *stream) {
    if (!h)
        return fail(COS_EINVAL, "cos_mc_run: graph is NULL");
    if (C < 1 || C > (int64_t(1) << 31))
        return fail(COS_EINVAL, "cos_mc_run: C must be in 1..2^31");
    if (step0 < 0 || n_steps < 0)
        return fail(COS_EINVAL, "cos_mc_run: step0 and n_steps must be >= 0");
    if (!std::isfinite(sigma) || sigma < 0.0)
        return fail(COS_EINVAL, "cos_mc_run: sigma must be finite and >= 0");
    if (!x_dev || !v_dev || !accepted_dev || !acc_dev)
        return fail(COS_EINVAL, "cos_mc_run: NULL device pointer");
    const Graph &g = graph_of(h);
    if (g.kind != FK_RATIONAL)
        return fail(COS_EINVAL, "cos_mc_run: the walkers move coordinates x, so the graph needs rational factors");
    // the conditions cos_evaluate would refuse inside the loop, checked before anything is queued
    if (check_precision_range(g, p, "cos_mc_run") != COS_OK)
        return COS_EINVAL;
    if (value_bytes(p) == 2 && g.path == COS_PATH_FUSED)
        return fail(COS_EINVAL, "cos_mc_run: 16-bit level storage runs on the streamed plan only");
    if (p == COS_FP16_RESCALED && g.h16.empty())
        return fail(COS_EINVAL, "cos_mc_run: binary16 storage needs level row sums of |a| below 2^110");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != g.device)
        return fail(COS_EINVAL, "cos_mc_run: the current device is not the graph's device");
    cos_status st = COS_OK;
    const McLayout m = mc_layout(h, C, p, st);
    if (st != COS_OK)
        return st;
    if (n_steps == 0)
        return COS_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *ws = workspace_dev;
    bool owned = false;
    if (ws) {
        if (reinterpret_cast<uintptr_t>(ws) % 256)
            return fail(COS_EINVAL, "cos_mc_run: workspace must be 256-byte aligned");
        if (workspace_bytes < m.total)
            return fail(COS_EINVAL, "cos_mc_run: workspace smaller than cos_mc_workspace_size");
    } else {
        const hipError_t err = hipMallocAsync(&ws, m.total, s);
        if (err != hipSuccess)
            return hip_fail(err, "hipMallocAsync(mc workspace)");
        owned = true;
    }
    char *base = static_cast<char *>(ws);
    double *xp = reinterpret_cast<double *>(base + m.off_xp);
    double *vp = reinterpret_cast<double *>(base + m.off_vp);
    void *ew = base + m.off_eval;
    const dim3 grid(static_cast<unsigned>((C + kBlock - 1) / kBlock));
    hipError_t err = hipSuccess;
    // graphs on the fused plan: the whole run in one launch (persistent walkers)
    const bool fused = (g.path == COS_PATH_AUTO || g.path == COS_PATH_FUSED) && fused_fits(g, p);
    if (fused) {
        const McArgs a{x_dev, v_dev, xp, vp, C, step0, n_steps, seed, sigma, accepted_dev, acc_dev};
        err = launch_fused(g, p, xp, C, vp, nullptr, s, &a);
    }
    for (int64_t t = step0; !fused && t < step0 + n_steps && st == COS_OK && err == hipSuccess; ++t) {
        hipLaunchKernelGGL(mc_propose_kernel, grid, dim3(kBlock), 0, s, x_dev, xp, C, t, seed, sigma);
        err = hipGetLastError();
        if (err != hipSuccess)
            break;
        st = cos_evaluate(h, xp, C, p, vp, nullptr, ew, m.eval_bytes, stream);
        if (st != COS_OK)
            break;
        hipLaunchKernelGGL(mc_accept_kernel, grid, dim3(kBlock), 0, s, x_dev, v_dev, xp, vp, C, t, seed,
                           accepted_dev, acc_dev);
        err = hipGetLastError();
    }
    if (owned) {
        const hipError_t ferr = hipFreeAsync(ws, s);
        if (err == hipSuccess)
            err = ferr;
    }
    if (st != COS_OK)
        return st;
    if (err != hipSuccess)
        return hip_fail(err, "cos_mc_run: kernel launch");
    return COS_OK;
}
