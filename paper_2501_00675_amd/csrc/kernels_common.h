// Device helpers shared by the level-sweep kernels.
#pragma once

#include "cos_internal.h"

namespace cosdag {

// Denominator 1 + b|x - k|^2 from the expanded record: c0 + cb q + g . x with
// q = |x|^2 (binary64; on CDNA a binary64 FMA issues at the binary32 rate when
// packed FP32 math is not used).
__device__ __forceinline__ double edge_denom(const EdgeRec &e, double x0, double x1, double x2, double q) {
    return __builtin_fma(e.g2, x2, __builtin_fma(e.g1, x1, __builtin_fma(e.g0, x0, __builtin_fma(e.cb, q, e.c0))));
}

// w = a / D in binary64: v_rcp_f64 (about 2^-24 accurate) followed by one
// residual correction w = w0 + (a - D w0) r, which squares the reciprocal's
// relative error (measured worst case 2.2e-15 for D in [1, 1000]).  D >= 1,
// so no scaling of the operands is needed.
__device__ __forceinline__ double edge_factor64(const EdgeRec &e, double x0, double x1, double x2, double q) {
    const double D = edge_denom(e, x0, x1, x2, q);
    const double r = __builtin_amdgcn_rcp(D);
    const double w0 = e.a * r;
    return __builtin_fma(__builtin_fma(-D, w0, e.a), r, w0);
}

// binary32 factor from the binary32 record and the sample rounded to binary32:
// r = x - k, D = 1 + b |r|^2 by fused multiply-adds, then v_rcp_f32 (1.5 ulp,
// measured) and the product with a.  D >= 1 up to rounding, so the reciprocal
// needs no scaling.
__device__ __forceinline__ float edge_factor32(const EdgeRec32 &e, float x0, float x1, float x2) {
    const float r0 = x0 - e.k0, r1 = x1 - e.k1, r2 = x2 - e.k2;
    const float s = __builtin_fmaf(r2, r2, __builtin_fmaf(r1, r1, r0 * r0));
    return e.a * __builtin_amdgcn_rcpf(__builtin_fmaf(e.b, s, 1.0f));
}

// ilogb of a non-negative binary32 given by its bit pattern; 0, inf and NaN
// give 0 (no rescale).
__device__ __forceinline__ int ilogb_bits(uint32_t u) {
    if (u == 0u || u >= 0x7f800000u)
        return 0;
    const uint32_t ex = u >> 23;
    if (ex)
        return static_cast<int>(ex) - 127;
    return (31 - __clz(u)) - 149;  // subnormal
}

__device__ __forceinline__ uint32_t abs_bits(float v) { return __float_as_uint(v) & 0x7fffffffu; }

// Scale by 2^-e (exact for normal results).
__device__ __forceinline__ float scale_pow2(float v, int e) { return ldexpf(v, -e); }
__device__ __forceinline__ double scale_pow2(double v, int e) { return ldexp(v, -e); }

}  // namespace cosdag
