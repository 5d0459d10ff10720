// Device evaluation of the learned CDF model (two-level RMI).
//
// Model buffer (floats): head [rc, ra, rb, L, 0, 0, 0, 0], then L+1 leaf
// records [a, b, x0, lo] (16 bytes each; record L is a sentinel whose lo is
// 1).  For a key with order-preserving image t:
//   x = float(t)              round to nearest even
//   r = float(bits(x))        x >= 0, so its bits grow with x: a log-like feature
//   leaf = clamp(floor(ra*(r - rc) + rb), 0, L-1)
//   F = clamp(a*(x - x0) + b, lo[leaf], lo[leaf+1])     (a >= 0)
//   code = min(floor(F * 2^cb), 2^cb - 1)
// The upper clamp of a leaf is the lower clamp of the next one, so the leaf
// ranges nest by construction and every step is a nondecreasing function
// of t: the code never decreases as the key grows.  Products and sums are
// rounded separately (the library is built without FMA contraction): the
// integer results must not depend on fusing.
#pragma once

#include "ak_internal.h"

namespace ak {

struct RmiHead {
    float rc, ra, rb, L;
    float pad[4];
};
using RmiLeaf = float4;  // a, b, x0, lo

constexpr int RMI_LDS_LEAVES = 4096;  // tables up to this size are staged in LDS

__device__ __forceinline__ float to_f32(uint32_t t) { return (float)t; }
__device__ __forceinline__ float to_f32(uint64_t t) { return (float)t; }

__device__ __forceinline__ const RmiHead &rmi_head(const float *model) {
    return *reinterpret_cast<const RmiHead *>(model);
}
__device__ __forceinline__ const RmiLeaf *rmi_leaves(const float *model) {
    return reinterpret_cast<const RmiLeaf *>(model + 8);
}

template <typename U>
__device__ __forceinline__ int rmi_leaf(const RmiHead &h, U t, float &x) {
    x = to_f32(t);
    const float r = (float)__float_as_uint(x);
    float p = __fadd_rn(__fmul_rn(h.ra, __fsub_rn(r, h.rc)), h.rb);
    p = fminf(fmaxf(p, 0.0f), __fsub_rn(h.L, 1.0f));
    return (int)p;
}

// F of a key whose leaf record p and upper clamp hi are already read
__device__ __forceinline__ float rmi_cdf_at(const RmiLeaf &p, float hi, float x) {
    const float F = __fadd_rn(__fmul_rn(p.x, __fsub_rn(x, p.z)), p.y);
    return fminf(fmaxf(F, p.w), hi);
}

__device__ __forceinline__ uint32_t rmi_code_at(const RmiLeaf &p, float hi, float x, int cb, float scale) {
    const uint32_t c = (uint32_t)__fmul_rn(rmi_cdf_at(p, hi, x), scale);
    const uint32_t top = (1u << cb) - 1u;
    return c < top ? c : top;
}

template <typename U>
__device__ __forceinline__ float rmi_cdf(const RmiHead &h, const RmiLeaf *leaves, U t) {
    float x;
    const int leaf = rmi_leaf(h, t, x);
    return rmi_cdf_at(leaves[leaf], leaves[leaf + 1].w, x);
}

template <typename U>
__device__ __forceinline__ uint32_t rmi_code(const RmiHead &h, const RmiLeaf *leaves, U t, int cb, float scale) {
    float x;
    const int leaf = rmi_leaf(h, t, x);
    return rmi_code_at(leaves[leaf], leaves[leaf + 1].w, x, cb, scale);
}

// Codes of G keys: every leaf is located and its records requested before
// any code is formed, so the table reads of the G keys are in flight
// together.
template <int G, typename U>
__device__ __forceinline__ void rmi_code_group(const RmiHead &h, const RmiLeaf *leaves, const U (&t)[G], int cb,
                                               float scale, uint32_t (&c)[G]) {
    float x[G];
    int leaf[G];
#pragma unroll
    for (int g = 0; g < G; ++g) leaf[g] = rmi_leaf(h, t[g], x[g]);
    RmiLeaf p[G];
    float hi[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        p[g] = leaves[leaf[g]];
        hi[g] = leaves[leaf[g] + 1].w;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) c[g] = rmi_code_at(p[g], hi[g], x[g], cb, scale);
}

// Copies the L+1 leaf records into LDS (`dst`, room for L+1 float4) with
// the whole block, then waits for the block.  Returns the table to use:
// the LDS copy if L <= RMI_LDS_LEAVES, else the global one.
__device__ __forceinline__ const RmiLeaf *rmi_stage(const float *model, RmiLeaf *dst) {
    const int L = (int)rmi_head(model).L;
    const RmiLeaf *src = rmi_leaves(model);
    if (L > RMI_LDS_LEAVES || dst == nullptr) return src;
    for (int i = threadIdx.x; i <= L; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
    return dst;
}

// LDS bytes a kernel needs to stage the table of an L-leaf model.
inline size_t rmi_stage_bytes(int L) { return L <= RMI_LDS_LEAVES ? (size_t)(L + 1) * sizeof(float4) : 0; }

}  // namespace ak
