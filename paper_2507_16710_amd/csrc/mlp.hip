// The second learned CDF model: a 1-64-64-1 network, trained on the GPU by
// the kernels of this file and tabulated into the two-level model's table
// so that the per-key inference of the sort stays one leaf lookup.
//
//   input    u = (r - r_first) * s in [0, 1]: the log-like key feature of
//            the model's root (bits of float32(image(key)) as a float),
//            over the sample's feature range, s = 1 / (r_last - r_first)
//   network  f(u) = w3 . tanh(W2 tanh(W1 u + c1) + c2) + c3
//            W1 = sp(A1), W2 = sp(A2), w3 = sp(a3) with sp = softplus: the
//            weights are positive and tanh increases, so f increases with u
//   loss     mean over K training points of (f(u_k) - y_k)^2, the points
//            taken at evenly spaced ranks j_k of the sorted sample (m keys),
//            y_k = j_k / m
//   training Adam on the raw parameters (A1, c1, A2, c2, a3, c3) from a
//            start placed at the quantiles of the training inputs
//   table    f at the left edges u_i = i / L of the root's L equal feature
//            widths, clamped to [0, 1] and made nondecreasing, becomes leaf
//            i's lower clamp lo_i; leaf i interpolates linearly in x =
//            float32(image) between its knot x_i (the float whose bits are
//            the knot's feature) and the next knot.
//
// Parameter layout (floats): A1[64] | c1[64] | A2[64 x 64] (row: layer-2
// unit, column: layer-1 unit) | c2[64] | a3[64] | c3.
//
// One training step is two launches: k_mlp_grad (one workgroup per 64
// points: forward, loss and backward through both layers with the weights
// and activations in LDS, writing that workgroup's gradient sums), then
// k_mlp_adam (one thread per parameter: the sums over the workgroups in a
// fixed order, the softplus chain rule, the Adam update, the new effective
// weights).  The contraction over the 64 x 64 layer is done by VALU FMAs
// from LDS: a step is about 0.1 GFLOP over 4096 points, a few microseconds
// of arithmetic, so the step time is launch latency either way.
#include <algorithm>
#include <cmath>

#include "ak_internal.h"
#include "rmi_device.h"

namespace ak {

constexpr int MH = 64;
constexpr int MP = AK_MLP_PARAMS;
constexpr int MO_A1 = 0, MO_C1 = MH, MO_A2 = 2 * MH, MO_C2 = MO_A2 + MH * MH, MO_A3 = MO_C2 + MH,
              MO_C3 = MO_A3 + MH;
static_assert(MO_C3 + 1 == MP, "parameter layout");
constexpr int MLP_PTS = 64;    // training points per workgroup
constexpr int MLP_K = 4096;    // training points taken from the sample
constexpr float MLP_LR = 1e-2f, MLP_B1 = 0.9f, MLP_B2 = 0.999f, MLP_EPS = 1e-8f;

__device__ __forceinline__ bool mlp_is_weight(int q) {
    return q < MO_C1 || (q >= MO_A2 && q < MO_C2) || (q >= MO_A3 && q < MO_C3);
}
__device__ __forceinline__ float softplus_f(float x) { return fmaxf(x, 0.f) + log1pf(expf(-fabsf(x))); }
__device__ __forceinline__ float sigmoid_f(float x) { return 1.f / (1.f + expf(-x)); }

// Feature of a key (the root's input): bits of float32(image) as a float.
template <int DT>
__device__ __forceinline__ float mlp_feature(typename KT<DT>::U key) {
    const float x = to_f32(KT<DT>::image(key));
    return (float)__float_as_uint(x);
}

// Training points: j_k = floor((2k+1) m / (2K)), u_k = (r(j_k) - r0) * s,
// y_k = float(j_k) / float(m), with s = 1 / (r(m-1) - r0) (0 if flat).
template <int DT>
__global__ __launch_bounds__(256) void k_mlp_points(const typename KT<DT>::U *sorted, uint32_t m, uint32_t K,
                                                    float *u, float *y) {
    const uint32_t k = blockIdx.x * 256u + threadIdx.x;
    if (k >= K) return;
    const float r0 = mlp_feature<DT>(sorted[0]);
    const float width = __fsub_rn(mlp_feature<DT>(sorted[m - 1]), r0);
    const float s = width > 0.f ? __fdiv_rn(1.0f, width) : 0.f;
    const uint32_t j = (uint32_t)(((2ull * k + 1ull) * m) / (2ull * K));
    u[k] = __fmul_rn(__fsub_rn(mlp_feature<DT>(sorted[j]), r0), s);
    y[k] = __fdiv_rn((float)j, (float)m);
}

// Effective parameters: softplus of the weights, biases as they are.
__device__ __forceinline__ float mlp_eff(int q, float raw) { return mlp_is_weight(q) ? softplus_f(raw) : raw; }

// Start: layer-1 unit i steps at c_i = u[floor((2i+1) K / 128)] with slope
// s_i = clamp(4 / (c_{i+1} - c_{i-1}), 16, 4096) (one-sided at the ends),
// A1 = s_i, c1 = -(s_i c_i); A2 = 2 on the diagonal, -7 elsewhere; a3 = -5;
// c2 = 0; c3 = 1/2.  Adam moments zero.
__global__ __launch_bounds__(256) void k_mlp_init(const float *u, uint32_t K, float *raw, float *eff, float *mo,
                                                  float *vo) {
    for (int q = blockIdx.x * 256 + threadIdx.x; q < MP; q += gridDim.x * 256) {
        float v;
        if (q < MO_A2) {
            const int i = q % MH;
            auto ctr = [&](int t) { return u[((2ull * (uint32_t)t + 1ull) * K) / (2ull * MH)]; };
            const float c = ctr(i);
            const float gap = __fsub_rn(ctr(min(i + 1, MH - 1)), ctr(max(i - 1, 0)));
            float sl = gap > 0.f ? __fdiv_rn(4.0f, gap) : 4096.f;
            sl = fminf(fmaxf(sl, 16.f), 4096.f);
            v = q < MO_C1 ? sl : -__fmul_rn(sl, c);
        } else if (q < MO_C2) {
            const int r = (q - MO_A2) / MH, c = (q - MO_A2) % MH;
            v = r == c ? 2.f : -7.f;
        } else if (q < MO_A3) {
            v = 0.f;
        } else if (q < MO_C3) {
            v = -5.f;
        } else {
            v = 0.5f;
        }
        raw[q] = v;
        eff[q] = mlp_eff(q, v);
        mo[q] = 0.f;
        vo[q] = 0.f;
    }
}

__global__ __launch_bounds__(256) void k_mlp_effective(const float *raw, float *eff) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q < MP) eff[q] = mlp_eff(q, raw[q]);
}

// Forward and backward over the 64 points of this workgroup.  part[g] gets
// the gradient sums with respect to the EFFECTIVE parameters (the softplus
// chain rule is applied after the sums) and, last, the sum of squared
// residuals.  Points past K contribute nothing.
__global__ __launch_bounds__(256) void k_mlp_grad(const float *u, const float *y, uint32_t K, const float *eff,
                                                  float *part) {
    constexpr int LD = MH + 1;  // padded rows
    __shared__ float sW2[MH * LD], sH1[MLP_PTS * LD], sH2[MLP_PTS * LD];
    __shared__ float sW1[MH], sC1[MH], sC2[MH], sW3[MH], sU[MLP_PTS], sY[MLP_PTS], sDF[MLP_PTS];
    __shared__ float sRed[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const uint32_t p0 = blockIdx.x * MLP_PTS;
    float *out = part + (size_t)blockIdx.x * (MP + 1);
    for (int q = t; q < MH * MH; q += 256) sW2[(q / MH) * LD + (q % MH)] = eff[MO_A2 + q];
    if (t < MH) {
        sW1[t] = eff[MO_A1 + t];
        sC1[t] = eff[MO_C1 + t];
        sC2[t] = eff[MO_C2 + t];
        sW3[t] = eff[MO_A3 + t];
        const uint32_t k = p0 + (uint32_t)t;
        sU[t] = k < K ? u[k] : 0.f;
        sY[t] = k < K ? y[k] : 0.f;
    }
    const float c3 = eff[MO_C3];
    __syncthreads();
    // layer 1
    for (int e = t; e < MLP_PTS * MH; e += 256) {
        const int p = e / MH, j = e % MH;
        sH1[p * LD + j] = tanhf(__fadd_rn(__fmul_rn(sW1[j], sU[p]), sC1[j]));
    }
    __syncthreads();
    // layer 2: every thread a 4 x 4 block (points pa.., units ia..)
    const int pa = 4 * (t / 16), ia = 4 * (t % 16);
    {
        float acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = sC2[ia + b];
        for (int j = 0; j < MH; ++j) {
            float h[4], wv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) h[a] = sH1[(pa + a) * LD + j];
#pragma unroll
            for (int b = 0; b < 4; ++b) wv[b] = sW2[(ia + b) * LD + j];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = __fadd_rn(acc[a][b], __fmul_rn(h[a], wv[b]));
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) sH2[(pa + a) * LD + ia + b] = tanhf(acc[a][b]);
    }
    __syncthreads();
    // output, residual, dL/df = 2 r / K, squared residuals
    if (w == 0) {
        float f = c3;
        for (int i = 0; i < MH; ++i) f = __fadd_rn(f, __fmul_rn(sW3[i], sH2[lane * LD + i]));
        const bool valid = p0 + (uint32_t)lane < K;
        const float r = valid ? __fsub_rn(f, sY[lane]) : 0.f;
        sDF[lane] = __fdiv_rn(__fmul_rn(2.f, r), (float)K);
        float sq = __fmul_rn(r, r);
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) sq += __shfl_xor(sq, d, 64);
        if (lane == 0) sRed[0] = sq;
    }
    __syncthreads();
    // dw3 and dc3 (need the activations of layer 2 before they are replaced)
    if (w == 1) {
        const int i = lane;
        float s = 0.f;
        for (int p = 0; p < MLP_PTS; ++p) s = __fadd_rn(s, __fmul_rn(sDF[p], sH2[p * LD + i]));
        out[MO_A3 + i] = s;
        float d = sDF[lane];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) d += __shfl_xor(d, o, 64);
        if (lane == 0) out[MO_C3] = d;
    }
    __syncthreads();
    // dz2 = df * w3 * (1 - h2^2), in place of h2
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            float &h = sH2[(pa + a) * LD + ia + b];
            h = __fmul_rn(__fmul_rn(sDF[pa + a], sW3[ia + b]), __fsub_rn(1.f, __fmul_rn(h, h)));
        }
    __syncthreads();
    // dc2, dW2 = dz2^T h1 (blocks of 4 layer-2 units x 4 layer-1 units)
    if (w == 0) {
        float s = 0.f;
        for (int p = 0; p < MLP_PTS; ++p) s = __fadd_rn(s, sH2[p * LD + lane]);
        out[MO_C2 + lane] = s;
    }
    {
        const int ib = 4 * (t / 16), jb = 4 * (t % 16);
        float acc[4][4] = {};
        for (int p = 0; p < MLP_PTS; ++p) {
            float d[4], h[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) d[a] = sH2[p * LD + ib + a];
#pragma unroll
            for (int b = 0; b < 4; ++b) h[b] = sH1[p * LD + jb + b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = __fadd_rn(acc[a][b], __fmul_rn(d[a], h[b]));
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) out[MO_A2 + (ib + a) * MH + jb + b] = acc[a][b];
    }
    __syncthreads();
    // dh1 = dz2 W2, dz1 = dh1 (1 - h1^2) in place of h1 (points x layer-1 units)
    {
        const int jb = ia;
        float acc[4][4] = {};
        for (int i = 0; i < MH; ++i) {
            float d[4], wv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) d[a] = sH2[(pa + a) * LD + i];
#pragma unroll
            for (int b = 0; b < 4; ++b) wv[b] = sW2[i * LD + jb + b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = __fadd_rn(acc[a][b], __fmul_rn(d[a], wv[b]));
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                float &h = sH1[(pa + a) * LD + jb + b];
                h = __fmul_rn(acc[a][b], __fsub_rn(1.f, __fmul_rn(h, h)));
            }
    }
    __syncthreads();
    // dW1 = sum dz1 u, dc1 = sum dz1
    if (w == 0) {
        float s1 = 0.f, s0 = 0.f;
        for (int p = 0; p < MLP_PTS; ++p) {
            const float d = sH1[p * LD + lane];
            s1 = __fadd_rn(s1, __fmul_rn(d, sU[p]));
            s0 = __fadd_rn(s0, d);
        }
        out[MO_A1 + lane] = s1;
        out[MO_C1 + lane] = s0;
    }
    if (t == 0) out[MP] = sRed[0];
}

// Gradient with respect to the raw parameters (sums over the workgroups in
// order, softplus chain rule) and the loss, into g[0..MP] (the parity entry).
__global__ __launch_bounds__(256) void k_mlp_reduce(const float *part, int G, uint32_t K, const float *raw,
                                                    float *g) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q > MP) return;
    float s = 0.f;
    for (int b = 0; b < G; ++b) s = __fadd_rn(s, part[(size_t)b * (MP + 1) + q]);
    if (q == MP) g[q] = __fdiv_rn(s, (float)K);
    else g[q] = mlp_is_weight(q) ? __fmul_rn(s, sigmoid_f(raw[q])) : s;
}

// One Adam step of every parameter (t >= 1; bc1 = 1 - b1^t, bc2 = 1 - b2^t).
__global__ __launch_bounds__(256) void k_mlp_adam(const float *part, int G, uint32_t K, float *raw, float *eff,
                                                  float *mo, float *vo, float bc1, float bc2, float *loss_out) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q > MP) return;
    float s = 0.f;
    for (int b = 0; b < G; ++b) s = __fadd_rn(s, part[(size_t)b * (MP + 1) + q]);
    if (q == MP) {
        if (loss_out) *loss_out = __fdiv_rn(s, (float)K);
        return;
    }
    const float x = raw[q];
    const float g = mlp_is_weight(q) ? __fmul_rn(s, sigmoid_f(x)) : s;
    const float m = __fadd_rn(__fmul_rn(MLP_B1, mo[q]), __fmul_rn(1.f - MLP_B1, g));
    const float v = __fadd_rn(__fmul_rn(MLP_B2, vo[q]), __fmul_rn(1.f - MLP_B2, __fmul_rn(g, g)));
    mo[q] = m;
    vo[q] = v;
    const float mh = __fdiv_rn(m, bc1), vh = __fdiv_rn(v, bc2);
    const float nx = __fsub_rn(x, __fdiv_rn(__fmul_rn(MLP_LR, mh), __fadd_rn(sqrtf(vh), MLP_EPS)));
    raw[q] = nx;
    eff[q] = mlp_eff(q, nx);
}

// f(u) in float32 from the effective parameters.
__device__ float mlp_forward(const float *eff, float u) {
    float h1[MH];
#pragma unroll
    for (int j = 0; j < MH; ++j) h1[j] = tanhf(__fadd_rn(__fmul_rn(eff[MO_A1 + j], u), eff[MO_C1 + j]));
    float f = eff[MO_C3];
    for (int i = 0; i < MH; ++i) {
        float z = eff[MO_C2 + i];
#pragma unroll
        for (int j = 0; j < MH; ++j) z = __fadd_rn(z, __fmul_rn(eff[MO_A2 + i * MH + j], h1[j]));
        f = __fadd_rn(f, __fmul_rn(eff[MO_A3 + i], tanhf(z)));
    }
    return f;
}

// Table of the trained network in the two-level model's format (the head,
// rc and ra, is already written by the root kernel).  One workgroup: every
// knot evaluated into LDS, a running maximum (per-thread runs, then a scan
// of the run maxima across the workgroup), then the leaf records.
__global__ __launch_bounds__(1024) void k_mlp_tabulate(const float *eff, int L, float *model) {
    extern __shared__ float sF[];  // L + 1 knot values
    __shared__ float sE[MP];
    __shared__ float sWave[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int q = t; q < MP; q += 1024) sE[q] = eff[q];
    __syncthreads();
    const float invL = __fdiv_rn(1.0f, (float)L);
    for (int i = t; i <= L; i += 1024) {
        const float f = mlp_forward(sE, __fmul_rn((float)i, invL));
        sF[i] = fminf(fmaxf(f, 0.f), 1.f);
    }
    __syncthreads();
    if (t == 0) {
        sF[0] = 0.f;
        sF[L] = 1.f;
    }
    __syncthreads();
    // thread t owns the run [t*C, t*C + C) of the L+1 values
    const int C = (L + 1 + 1023) / 1024;
    const int b0 = t * C, b1 = min(b0 + C, L + 1);
    float run = 0.f;
    for (int i = b0; i < b1; ++i) run = fmaxf(run, sF[i]);
    // inclusive max-scan of the run maxima: waves, then across waves
    float inc = run;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const float o = __shfl_up(inc, d, 64);
        if (lane >= d) inc = fmaxf(inc, o);
    }
    if (lane == 63) sWave[w] = inc;
    __syncthreads();
    float carry = 0.f;
    for (int ww = 0; ww < w; ++ww) carry = fmaxf(carry, sWave[ww]);
    const float before = fmaxf(carry, __shfl_up(inc, 1, 64) * (lane > 0 ? 1.f : 0.f));
    float cur = before;
    for (int i = b0; i < b1; ++i) {
        cur = fmaxf(cur, sF[i]);
        sF[i] = cur;
    }
    __syncthreads();
    const RmiHead h = rmi_head(model);
    const float step = h.ra > 0.f ? __fdiv_rn(1.0f, h.ra) : 0.f;
    auto knot_x = [&](int i) {
        const float r = __fadd_rn(h.rc, __fmul_rn((float)i, step));
        return __uint_as_float((uint32_t)r);
    };
    RmiLeaf *lv = reinterpret_cast<RmiLeaf *>(model + 8);
    for (int i = t; i < L; i += 1024) {
        const float x0 = knot_x(i), x1 = knot_x(i + 1);
        const float dx = __fsub_rn(x1, x0);
        const float a = dx > 0.f ? __fdiv_rn(__fsub_rn(sF[i + 1], sF[i]), dx) : 0.f;
        lv[i] = make_float4(a, sF[i], x0, sF[i]);
    }
    if (t == 0) lv[L] = make_float4(0.f, 1.f, 0.f, 1.f);
}

// Scratch of a fit: points (u, y), raw and effective parameters, Adam
// moments, the workgroups' gradient sums, and (debug) the last loss.
struct MlpBufs {
    float *u, *y, *raw, *eff, *mo, *vo, *part, *loss;
};

size_t mlp_scratch_bytes(int64_t m) {
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t K = (size_t)std::min<int64_t>(m, MLP_K);
    const size_t G = (K + MLP_PTS - 1) / MLP_PTS;
    return 2 * al(K * 4) + 4 * al((size_t)MP * 4) + al(G * (MP + 1) * 4) + 256;
}

static ak_status mlp_bufs(Workspace *ws, int64_t m, MlpBufs *b) {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t K = (size_t)std::min<int64_t>(m, MLP_K);
    const size_t G = (K + MLP_PTS - 1) / MLP_PTS;
    ak_status r = ws_reserve(ws, &ws->aux[1], &ws->aux_bytes[1], mlp_scratch_bytes(m));
    if (r != AK_OK) return r;
    char *p = (char *)ws->aux[1];
    b->u = (float *)p;
    p += al(K * 4);
    b->y = (float *)p;
    p += al(K * 4);
    b->raw = (float *)p;
    p += al((size_t)MP * 4);
    b->eff = (float *)p;
    p += al((size_t)MP * 4);
    b->mo = (float *)p;
    p += al((size_t)MP * 4);
    b->vo = (float *)p;
    p += al((size_t)MP * 4);
    b->part = (float *)p;
    p += al(G * (MP + 1) * 4);
    b->loss = (float *)p;
    return AK_OK;
}

// Fits the network to the ascending sample (m keys) with `iters` Adam steps
// and writes its table (L leaves) into `model`; `params_out` (optional)
// gets the trained raw parameters.
template <int DT>
static ak_status mlp_fit_t(Workspace *ws, const void *sorted, int64_t m64, int L, int iters, float *model,
                           float *params_out) {
    using U = typename KT<DT>::U;
    hipStream_t s = ws->stream;
    const uint32_t m = (uint32_t)m64;
    const uint32_t K = std::min<uint32_t>(m, MLP_K);
    const int G = (int)((K + MLP_PTS - 1) / MLP_PTS);
    MlpBufs b;
    ak_status r = mlp_bufs(ws, m64, &b);
    if (r != AK_OK) return r;
    ProfScope ps("mlp_fit", s);
    hipLaunchKernelGGL((k_mlp_points<DT>), dim3((K + 255) / 256), dim3(256), 0, s, (const U *)sorted, m, K, b.u,
                       b.y);
    AK_LAUNCH_CHECK("k_mlp_points");
    const unsigned pg = (unsigned)((MP + 1 + 255) / 256);
    hipLaunchKernelGGL(k_mlp_init, dim3(pg), dim3(256), 0, s, (const float *)b.u, K, b.raw, b.eff, b.mo, b.vo);
    AK_LAUNCH_CHECK("k_mlp_init");
    double p1 = 1.0, p2 = 1.0;
    for (int t = 1; t <= iters; ++t) {
        p1 *= (double)MLP_B1;
        p2 *= (double)MLP_B2;
        hipLaunchKernelGGL(k_mlp_grad, dim3(G), dim3(256), 0, s, (const float *)b.u, (const float *)b.y, K,
                           (const float *)b.eff, b.part);
        hipLaunchKernelGGL(k_mlp_adam, dim3(pg), dim3(256), 0, s, (const float *)b.part, G, K, b.raw, b.eff, b.mo,
                           b.vo, (float)(1.0 - p1), (float)(1.0 - p2), b.loss);
    }
    AK_LAUNCH_CHECK("k_mlp_adam");
    if ((r = rmi_root(s, DT, sorted, m, L, model)) != AK_OK) return r;
    hipLaunchKernelGGL(k_mlp_tabulate, dim3(1), dim3(1024), (size_t)(L + 1) * 4, s, (const float *)b.eff, L, model);
    AK_LAUNCH_CHECK("k_mlp_tabulate");
    if (params_out) AK_HIP(hipMemcpyAsync(params_out, b.raw, (size_t)MP * 4, hipMemcpyDeviceToDevice, s));
    return AK_OK;
}

ak_status mlp_fit(Workspace *ws, int dt, const void *sorted, int64_t m, int L, int iters, float *model,
                  float *params_out) {
    switch (dt) {
    case AK_I32: return mlp_fit_t<AK_I32>(ws, sorted, m, L, iters, model, params_out);
    case AK_I64: return mlp_fit_t<AK_I64>(ws, sorted, m, L, iters, model, params_out);
    case AK_U32: return mlp_fit_t<AK_U32>(ws, sorted, m, L, iters, model, params_out);
    case AK_U64: return mlp_fit_t<AK_U64>(ws, sorted, m, L, iters, model, params_out);
    case AK_F32: return mlp_fit_t<AK_F32>(ws, sorted, m, L, iters, model, params_out);
    case AK_F64: return mlp_fit_t<AK_F64>(ws, sorted, m, L, iters, model, params_out);
    }
    set_error("mlp_fit: unsupported dtype");
    return AK_ERR_UNSUPPORTED_DTYPE;
}

// Loss and gradient (raw parameters) at `params` over K given points.
ak_status mlp_loss_grad(Workspace *ws, const float *u, const float *y, int64_t K, const float *params, float *out) {
    hipStream_t s = ws->stream;
    const int G = (int)((K + MLP_PTS - 1) / MLP_PTS);
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t need = al((size_t)MP * 4) + al((size_t)G * (MP + 1) * 4);
    ak_status r = ws_reserve(ws, &ws->aux[1], &ws->aux_bytes[1], need);
    if (r != AK_OK) return r;
    float *eff = (float *)ws->aux[1];
    float *part = (float *)((char *)ws->aux[1] + al((size_t)MP * 4));
    const unsigned pg = (unsigned)((MP + 1 + 255) / 256);
    hipLaunchKernelGGL(k_mlp_effective, dim3(pg), dim3(256), 0, s, params, eff);
    AK_LAUNCH_CHECK("k_mlp_effective");
    hipLaunchKernelGGL(k_mlp_grad, dim3(G), dim3(256), 0, s, u, y, (uint32_t)K, (const float *)eff, part);
    AK_LAUNCH_CHECK("k_mlp_grad");
    hipLaunchKernelGGL(k_mlp_reduce, dim3(pg), dim3(256), 0, s, (const float *)part, G, (uint32_t)K, params, out);
    AK_LAUNCH_CHECK("k_mlp_reduce");
    return AK_OK;
}

}  // namespace ak
