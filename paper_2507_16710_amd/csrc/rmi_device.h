// Device evaluation of the learned CDF model (two-level RMI).
//
// Model buffer (floats): head [rc, ra, rb, leaves, 0, 0, 0, 0], then one
// 8-float record per leaf [a, b, x0, lo, hi, 0, 0, 0].  For a key with
// order-preserving image t:
//   x = float(t)              round to nearest even
//   r = float(bits(x))        x >= 0, so its bits grow with x: a log-like feature
//   leaf = clamp(floor(ra*(r - rc) + rb), 0, L-1)
//   F = clamp(a*(x - x0) + b, lo, hi)          (a >= 0, hi_i <= lo_{i+1})
//   code = min(floor(F * 2^cb), 2^cb - 1)
// Every step is a nondecreasing function of t, so the code never decreases
// as the key grows.  Products and sums are rounded separately (__fmul_rn,
// __fadd_rn) so the compiler cannot fuse them: the integer results must not
// depend on contraction.
#pragma once

#include "ak_internal.h"

namespace ak {

struct RmiHead {
    float rc, ra, rb, L;
    float pad[4];
};
struct RmiLeaf {
    float a, b, x0, lo, hi, pad0, pad1, pad2;
};

__device__ __forceinline__ float to_f32(uint32_t t) { return (float)t; }
__device__ __forceinline__ float to_f32(uint64_t t) { return (float)t; }

template <typename U>
__device__ __forceinline__ int rmi_leaf(const RmiHead &h, U t, float &x) {
    x = to_f32(t);
    const float r = (float)__float_as_uint(x);
    float p = __fadd_rn(__fmul_rn(h.ra, __fsub_rn(r, h.rc)), h.rb);
    p = fminf(fmaxf(p, 0.0f), __fsub_rn(h.L, 1.0f));
    return (int)p;
}

template <typename U>
__device__ __forceinline__ float rmi_cdf(const RmiHead &h, const RmiLeaf *leaves, U t) {
    float x;
    const int leaf = rmi_leaf(h, t, x);
    const float4 p0 = *reinterpret_cast<const float4 *>(&leaves[leaf].a);
    const float hi = leaves[leaf].hi;
    float F = __fadd_rn(__fmul_rn(p0.x, __fsub_rn(x, p0.z)), p0.y);
    return fminf(fmaxf(F, p0.w), hi);
}

template <typename U>
__device__ __forceinline__ uint32_t rmi_code(const RmiHead &h, const RmiLeaf *leaves, U t, int cb, float scale) {
    const float F = rmi_cdf(h, leaves, t);
    const uint32_t c = (uint32_t)__fmul_rn(F, scale);
    const uint32_t top = (1u << cb) - 1u;
    return c < top ? c : top;
}

}  // namespace ak
