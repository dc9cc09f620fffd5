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
//   v'     = V(x')                              the level sweep (cos_evaluate)
//   accept iff u_3 |v| < |v'|                   Metropolis for the density |V|
//   acc[0] += sign v, acc[1] += |x|^2, accepted += take   (at the new state)
//
// Every random number is a function of (seed, walker, step) only, so a run
// split into several calls, or over a subset of walkers, is bit-identical to
// one call.
#include <cmath>

#include "cos_internal.h"

namespace cosdag {
namespace {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull, kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull, kPhiloxW1 = 0xBB67AE8584CAA73Bull;

// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two
// 64x64->128 multiplies, the key bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint64_t hi0 = __umul64hi(kPhiloxM0, c[0]), lo0 = kPhiloxM0 * c[0];
        const uint64_t hi1 = __umul64hi(kPhiloxM1, c[2]), lo1 = kPhiloxM1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ __forceinline__ double unit_uniform(uint64_t r) { return static_cast<double>(r >> 11) * 0x1.0p-53; }

__device__ __forceinline__ void walker_uniforms(uint64_t seed, int64_t c, int64_t t, double (&u)[4]) {
    uint64_t w[4] = {static_cast<uint64_t>(c), static_cast<uint64_t>(t), 0ull, 0ull};
    philox4x64_10(w, seed, 0ull);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        u[i] = unit_uniform(w[i]);
}

// x' = x + sigma (2 u - 1): the product and the sum each rounded (no fusion).
__global__ __launch_bounds__(kBlock) void mc_propose_kernel(const double *__restrict__ x, double *__restrict__ xp,
                                                            int64_t C, int64_t t, uint64_t seed, double sigma) {
#pragma clang fp contract(off)
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (c >= C)
        return;
    double u[4];
    walker_uniforms(seed, c, t, u);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double step = sigma * (2.0 * u[i] - 1.0);
        xp[i * C + c] = x[i * C + c] + step;
    }
}

// Metropolis decision for |V| and the per-walker sums at the resulting state.
__global__ __launch_bounds__(kBlock) void mc_accept_kernel(double *__restrict__ x, double *__restrict__ v,
                                                           const double *__restrict__ xp,
                                                           const double *__restrict__ vp, int64_t C, int64_t t,
                                                           uint64_t seed, int64_t *__restrict__ accepted,
                                                           double *__restrict__ acc) {
#pragma clang fp contract(off)
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (c >= C)
        return;
    double u[4];
    walker_uniforms(seed, c, t, u);
    double v0 = v[c];
    const double v1 = vp[c];
    double x0 = x[c], x1 = x[C + c], x2 = x[2 * C + c];
    if (u[3] * fabs(v0) < fabs(v1)) {
        x0 = xp[c];
        x1 = xp[C + c];
        x2 = xp[2 * C + c];
        x[c] = x0;
        x[C + c] = x1;
        x[2 * C + c] = x2;
        v[c] = v1;
        v0 = v1;
        accepted[c] += 1;
    }
    acc[c] += static_cast<double>((v0 > 0.0) - (v0 < 0.0));
    const double r2 = x0 * x0 + x1 * x1 + x2 * x2;
    acc[C + c] += r2;
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
    for (int64_t t = step0; t < step0 + n_steps && st == COS_OK && err == hipSuccess; ++t) {
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
