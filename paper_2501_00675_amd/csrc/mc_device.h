// Device routines of the Monte Carlo walkers, shared by the step-by-step
// kernels (mc.hip) and the persistent whole-run kernel for graphs that take
// the fused plan (kernels_fused.hip): the same counter-based generator and
// the same unfused arithmetic, so both give the same bits.
#pragma once

#include "cos_internal.h"

namespace cosdag {

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

// The four uniforms (r >> 11) 2^-53 of walker c at step t.
__device__ __forceinline__ void walker_uniforms(uint64_t seed, int64_t c, int64_t t, double (&u)[4]) {
    uint64_t w[4] = {static_cast<uint64_t>(c), static_cast<uint64_t>(t), 0ull, 0ull};
    philox4x64_10(w, seed, 0ull);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        u[i] = static_cast<double>(w[i] >> 11) * 0x1.0p-53;
}

// Walker c's proposal x' = x + sigma (2 u - 1), the product and the sum each
// rounded (no fusion); x and xp are [3][C].
__device__ __forceinline__ void mc_propose(const double *__restrict__ x, double *__restrict__ xp, int64_t C,
                                           int64_t c, int64_t t, uint64_t seed, double sigma) {
#pragma clang fp contract(off)
    double u[4];
    walker_uniforms(seed, c, t, u);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double step = sigma * (2.0 * u[i] - 1.0);
        xp[i * C + c] = x[i * C + c] + step;
    }
}

// Walker c's Metropolis decision for |V| (accept iff u_3 |v| < |v'|) and its
// sums at the resulting state: acc[0][c] += sign v, acc[1][c] += |x|^2.
__device__ __forceinline__ void mc_accept(double *__restrict__ x, double *__restrict__ v,
                                          const double *__restrict__ xp, const double *__restrict__ vp, int64_t C,
                                          int64_t c, int64_t t, uint64_t seed, int64_t *__restrict__ accepted,
                                          double *__restrict__ acc) {
#pragma clang fp contract(off)
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

}  // namespace cosdag
