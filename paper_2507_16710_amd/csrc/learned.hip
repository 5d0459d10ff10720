// Learned-CDF partition sort: same output as the radix sort, reached by
// ordering the keys by a learned estimate of their CDF first.
//
//   1. sample m keys at SplitMix64-hashed positions, sort the sample;
//   2. fit a two-level RMI to the sorted sample: a fixed root spreading the
//      sample's log-like feature range over L leaves, and per leaf a linear
//      CDF trained by Newton steps built from a forward kernel (residuals,
//      loss) and a backward kernel (gradient, curvature);
//   3. stable LSD passes over the model's cb-bit code of every key (the
//      one-sweep kernel with code digits): keys ordered by code;
//   4. cut the code-ordered array at code changes into chunks that fit one
//      workgroup and sort each chunk on chip (keys of different codes never
//      need to cross a cut, because the code grows with the key);
//   5. runs of a single code longer than a chunk fall back to radix passes
//      (after a check that skips runs of one repeated key).
// The paper's sorter is a merge sort (Sec. II-B); the learned partition is
// this library's own design for the same result.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "lds_sort.h"
#include "long_sort.h"
#include "radix_kernels.h"
#include "rmi_device.h"

namespace ak {

constexpr uint64_t SM64_GAMMA = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t j) {
    uint64_t z = seed + (j + 1) * SM64_GAMMA;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename U>
__global__ __launch_bounds__(256) void k_sample(const U *keys, uint64_t n, uint64_t seed, uint32_t m, U *out) {
    const uint32_t j = blockIdx.x * 256u + threadIdx.x;
    if (j >= m) return;
    const uint64_t pos = __umul64hi(splitmix64_at(seed, j), n);
    out[j] = keys[pos];
}

// ------------------------------------------------------------- fitting
// Scratch layout of a fit (floats / ints in one buffer):
struct FitScratch {
    uint32_t *st;    // L+1 leaf sample starts
    float *resid;    // m residuals
    float *stats;    // L x 8 per-leaf sums
};

template <int DT>
__global__ void k_rmi_root(const typename KT<DT>::U *sorted, uint32_t m, int L, float *model) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const float x0 = to_f32(KT<DT>::image(sorted[0]));
    const float x1 = to_f32(KT<DT>::image(sorted[m - 1]));
    const float r0 = (float)__float_as_uint(x0), r1 = (float)__float_as_uint(x1);
    const float width = __fsub_rn(r1, r0);
    RmiHead h;
    h.rc = r0;
    h.ra = width > 0.f ? __fdiv_rn((float)L, width) : 0.f;
    h.rb = 0.f;
    h.L = (float)L;
    for (int i = 0; i < 4; ++i) h.pad[i] = 0.f;
    *reinterpret_cast<RmiHead *>(model) = h;
}

// Model of the method without training: every key in leaf 0, F linear from
// the smallest to the largest sampled key (equal-width key ranges).
template <int DT>
__global__ void k_rmi_untrained(const typename KT<DT>::U *sorted, uint32_t m, int L, float *model) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const float x0 = to_f32(KT<DT>::image(sorted[0]));
    const float x1 = to_f32(KT<DT>::image(sorted[m - 1]));
    if (i == 0) {
        RmiHead h{};
        h.L = (float)L;
        *reinterpret_cast<RmiHead *>(model) = h;
    }
    if (i <= L) {
        const float width = __fsub_rn(x1, x0);
        RmiLeaf lf;
        if (i == 0) lf = make_float4(width > 0.f ? __fdiv_rn(1.0f, width) : 0.f, 0.f, x0, 0.f);
        else lf = make_float4(0.f, 1.f, 0.f, 1.f);
        reinterpret_cast<RmiLeaf *>(model + 8)[i] = lf;
    }
}

// st[i] = first sample routed to leaf >= i (routing is monotone, so every
// leaf owns a contiguous range of the sorted sample).
template <int DT>
__global__ void k_rmi_bounds(const typename KT<DT>::U *sorted, uint32_t m, const float *model, uint32_t *st) {
    const int L = (int)reinterpret_cast<const RmiHead *>(model)->L;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > L) return;
    const RmiHead h = *reinterpret_cast<const RmiHead *>(model);
    uint32_t lo = 0, hi = m;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        float x;
        if (rmi_leaf(h, KT<DT>::image(sorted[mid]), x) < i) lo = mid + 1;
        else hi = mid;
    }
    st[i] = lo;
}

// Leaf setup: lower clamp st/m (the upper one is the next leaf's lower
// clamp, en/m; the sentinel record L has lo = 1), centre x0 = middle
// sample, a = b = 0, and the slope scale s = 2^-e with 2^e <= max |x - x0|
// < 2^(e+1) over the leaf's samples (a power of two, so scaled and
// unscaled products round identically; 1 for an empty or flat leaf).
template <int DT>
__device__ __forceinline__ float leaf_scale_of(const typename KT<DT>::U *sorted, uint32_t s, uint32_t e, float x0) {
    if (e <= s) return 1.f;
    const float d0 = fabsf(__fsub_rn(to_f32(KT<DT>::image(sorted[s])), x0));
    const float d1 = fabsf(__fsub_rn(to_f32(KT<DT>::image(sorted[e - 1])), x0));
    const float dm = fmaxf(d0, d1);
    return dm > 0.f ? ldexpf(1.0f, -ilogbf(dm)) : 1.f;
}

template <int DT>
__global__ void k_rmi_leaf_init(const typename KT<DT>::U *sorted, uint32_t m, const uint32_t *st, float *model,
                                float *scales) {
    const int L = (int)reinterpret_cast<const RmiHead *>(model)->L;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > L) return;
    RmiLeaf *lf = reinterpret_cast<RmiLeaf *>(model + 8) + i;
    if (i == L) {
        *lf = make_float4(0.f, 1.f, 0.f, __fdiv_rn((float)m, (float)m));
        return;
    }
    const uint32_t s = st[i], e = st[i + 1];
    const float lo = __fdiv_rn((float)s, (float)m);
    float x0 = 0.f;
    if (e > s) x0 = to_f32(KT<DT>::image(sorted[s + (e - s - 1) / 2]));
    *lf = make_float4(0.f, e > s ? 0.f : lo, x0, lo);
    scales[i] = leaf_scale_of<DT>(sorted, s, e, x0);
}

// Scale of every leaf for given parameters (as in k_rmi_leaf_init).
template <int DT>
__global__ void k_leaf_scale(const typename KT<DT>::U *sorted, const uint32_t *st, const float *model,
                             float *scales) {
    const int L = (int)reinterpret_cast<const RmiHead *>(model)->L;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L) return;
    scales[i] = leaf_scale_of<DT>(sorted, st[i], st[i + 1], reinterpret_cast<const RmiLeaf *>(model + 8)[i].z);
}

template <int B>
__device__ __forceinline__ float block_sum_f(float v, float *s_red) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) s_red[w] = v;
    __syncthreads();
    float t = 0.f;
#pragma unroll
    for (int i = 0; i < B / 64; ++i) t += s_red[i];
    __syncthreads();
    return t;
}

// The leaf sums run over work items of at most FIT_CH samples (a leaf's
// samples split into consecutive pieces), so one leaf holding a large
// share of the sample (a repeated key) does not leave one workgroup walking
// it alone.  Every item writes its partial sums, and k_rmi_sum adds a
// leaf's items in order: the result does not depend on scheduling.
constexpr uint32_t FIT_CH = 8192;

// item prefix: ipre[i] = first item of leaf i (ipre[L] = item count), one
// workgroup of 1024 threads
__global__ __launch_bounds__(1024) void k_fit_items(const uint32_t *st, int L, uint32_t *ipre) {
    __shared__ uint32_t s_wsum[16];
    __shared__ uint32_t s_carry;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_carry = 0;
    __syncthreads();
    for (int base = 0; base < L; base += 1024) {
        const int i = base + tid;
        const uint32_t v = i < L ? (st[i + 1] - st[i] + FIT_CH - 1) / FIT_CH : 0u;
        const uint32_t incl = wave_incl_scan(v);
        if (lane == 63) s_wsum[w] = incl;
        __syncthreads();
        uint32_t run = s_carry;
        for (int ww = 0; ww < w; ++ww) run += s_wsum[ww];
        if (i < L) ipre[i] = run + incl - v;
        __syncthreads();
        if (tid == 1023) s_carry = run + incl;
        __syncthreads();
    }
    if (tid == 0) ipre[L] = s_carry;
}

__global__ __launch_bounds__(256) void k_fit_itemmap(const uint32_t *ipre, int L, uint32_t *item_leaf) {
    for (int i = blockIdx.x; i < L; i += gridDim.x)
        for (uint32_t k = ipre[i] + threadIdx.x; k < ipre[i + 1]; k += 256) item_leaf[k] = (uint32_t)i;
}

// the samples [j0, j1) of work item blockIdx.x and its leaf (false: no item)
__device__ __forceinline__ bool fit_item(const uint32_t *st, const uint32_t *ipre, const uint32_t *item_leaf, int L,
                                         uint32_t &leaf, uint32_t &j0, uint32_t &j1) {
    const uint32_t item = blockIdx.x;
    if (item >= ipre[L]) return false;
    leaf = item_leaf[item];
    j0 = st[leaf] + (item - ipre[leaf]) * FIT_CH;
    j1 = min(j0 + FIT_CH, st[leaf + 1]);
    return true;
}

// Forward: residual of every sample, r = a*dx + b - j/m (in the leaf's
// scaled coordinates a' = a/s, dx' = dx*s), and the item's partial loss.
template <int DT>
__global__ __launch_bounds__(256) void k_rmi_fwd(const typename KT<DT>::U *sorted, uint32_t m, const uint32_t *st,
                                                 const uint32_t *ipre, const uint32_t *item_leaf, int L,
                                                 const float *model, const float *scales, float *resid,
                                                 float *part) {
    __shared__ float s_red[4];
    uint32_t i, j0, j1;
    if (!fit_item(st, ipre, item_leaf, L, i, j0, j1)) return;
    const RmiLeaf lf = reinterpret_cast<const RmiLeaf *>(model + 8)[i];  // a, b, x0, lo
    const float sc = scales[i];
    const float a_s = __fdiv_rn(lf.x, sc);  // exact: sc is a power of two
    const float fm = (float)m;
    float loss = 0.f;
    for (uint32_t j = j0 + threadIdx.x; j < j1; j += 256) {
        const float dx = __fmul_rn(__fsub_rn(to_f32(KT<DT>::image(sorted[j])), lf.z), sc);
        const float y = __fdiv_rn((float)j, fm);
        const float r = __fsub_rn(__fadd_rn(__fmul_rn(a_s, dx), lf.y), y);
        resid[j] = r;
        loss = __fadd_rn(loss, __fmul_rn(r, r));
    }
    loss = block_sum_f<256>(loss, s_red);
    if (threadIdx.x == 0) part[8 * blockIdx.x + 0] = loss;
}

// Backward: the item's partial gradient of the loss w.r.t. (a', b) and
// curvature terms (Gauss-Newton = exact Hessian for this least-squares loss).
template <int DT>
__global__ __launch_bounds__(256) void k_rmi_bwd(const typename KT<DT>::U *sorted, const uint32_t *st,
                                                 const uint32_t *ipre, const uint32_t *item_leaf, int L,
                                                 const float *model, const float *scales, const float *resid,
                                                 float *part) {
    __shared__ float s_red[4];
    uint32_t i, j0, j1;
    if (!fit_item(st, ipre, item_leaf, L, i, j0, j1)) return;
    const RmiLeaf lf = reinterpret_cast<const RmiLeaf *>(model + 8)[i];
    const float sc = scales[i];
    float ga = 0.f, gb = 0.f, hxx = 0.f, hx = 0.f;
    for (uint32_t j = j0 + threadIdx.x; j < j1; j += 256) {
        const float dx = __fmul_rn(__fsub_rn(to_f32(KT<DT>::image(sorted[j])), lf.z), sc);
        const float r = resid[j];
        ga = __fadd_rn(ga, __fmul_rn(r, dx));
        gb = __fadd_rn(gb, r);
        hxx = __fadd_rn(hxx, __fmul_rn(dx, dx));
        hx = __fadd_rn(hx, dx);
    }
    ga = block_sum_f<256>(ga, s_red);
    gb = block_sum_f<256>(gb, s_red);
    hxx = block_sum_f<256>(hxx, s_red);
    hx = block_sum_f<256>(hx, s_red);
    if (threadIdx.x == 0) {
        float *o = part + 8 * blockIdx.x;
        o[1] = ga;
        o[2] = gb;
        o[3] = hxx;
        o[4] = hx;
    }
}

// Per leaf: its items' partial sums added in item order, as
// stats[8i..8i+7] = loss, dL/da', dL/db, 2*sum dx'^2, 2*sum dx', 2*count, s, 0.
__global__ void k_rmi_sum(const uint32_t *st, const uint32_t *ipre, int L, const float *scales, const float *part,
                          float *stats) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L) return;
    float loss = 0.f, ga = 0.f, gb = 0.f, hxx = 0.f, hx = 0.f;
    for (uint32_t k = ipre[i]; k < ipre[i + 1]; ++k) {
        const float *q = part + 8 * k;
        loss = __fadd_rn(loss, q[0]);
        ga = __fadd_rn(ga, q[1]);
        gb = __fadd_rn(gb, q[2]);
        hxx = __fadd_rn(hxx, q[3]);
        hx = __fadd_rn(hx, q[4]);
    }
    float *o = stats + 8 * i;
    o[0] = loss;
    o[1] = 2.f * ga;
    o[2] = 2.f * gb;
    o[3] = 2.f * hxx;
    o[4] = 2.f * hx;
    o[5] = 2.f * (float)(st[i + 1] - st[i]);
    o[6] = scales[i];
    o[7] = 0.f;
}

// Newton step per leaf on the quadratic loss, projected onto a' >= 0 (the
// monotone set): if the step would make the slope negative, the slope is
// set to 0 and b takes its optimum for that slope.
__global__ void k_rmi_update(float *model, const uint32_t *st, const float *scales, const float *stats) {
    const int L = (int)reinterpret_cast<const RmiHead *>(model)->L;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L || st[i + 1] == st[i]) return;
    RmiLeaf *lf = reinterpret_cast<RmiLeaf *>(model + 8) + i;
    const float *g = stats + 8 * i;
    const float sc = scales[i];
    float a = __fdiv_rn(lf->x, sc), b = lf->y;
    const float ga = g[1], gb = g[2], h00 = g[3], h01 = g[4], h11 = g[5];
    const float det = h00 * h11 - h01 * h01;
    float na, nb;
    if (det > 1e-6f * h00 * h11 && h00 > 0.f) {
        na = a - (h11 * ga - h01 * gb) / det;
        nb = b - (h00 * gb - h01 * ga) / det;
    } else {
        na = a;
        nb = b - gb / h11;
    }
    if (!(na >= 0.f)) {
        nb = b - (gb - h01 * a) / h11;
        na = 0.f;
    }
    lf->x = __fmul_rn(na, sc);
    lf->y = nb;
}

// ------------------------------------------------------------ inference
template <int DT>
__global__ __launch_bounds__(256) void k_rmi_codes(const typename KT<DT>::U *keys, uint32_t n, const float *model,
                                                   int cb, uint32_t *codes, int staged) {
    extern __shared__ float4 s_leaves[];
    const RmiHead h = rmi_head(model);
    const RmiLeaf *lv = rmi_stage(model, staged ? s_leaves : nullptr);
    const float scale = (float)(1u << cb);
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u)
        codes[i] = rmi_code(h, lv, KT<DT>::image(keys[i]), cb, scale);
}

// ------------------------------------------------------ chunk sorting
struct LearnedState {
    uint32_t fb_count;      // fallback runs found
    uint32_t fb_next;       // fallback work counter
    uint32_t chunks;        // on-chip chunk sorts
    uint32_t pad;
    unsigned long long fb_keys;
    unsigned long long const_keys;
};

struct FbRun {
    uint32_t start, len;
};

// What a chunk sort orders by: the model code of a key (learned sort) or a
// bit field of its order-preserving image (prefix-partitioned radix sort).
// Both are nondecreasing in the key, so the code-ordered array is ordered
// by code and its equal-code runs are contiguous.
template <int DT>
struct RmiCoder {
    RmiHead h;
    const RmiLeaf *lv;
    int cb;
    float scale;
    __device__ uint32_t operator()(typename KT<DT>::U key) const {
        return rmi_code(h, lv, KT<DT>::image(key), cb, scale);
    }
};
template <int DT>
struct PrefixCoder {
    int shift;
    uint32_t mask;
    __device__ uint32_t operator()(typename KT<DT>::U key) const {
        return (uint32_t)((uint64_t)KT<DT>::image(key) >> shift) & mask;
    }
};

// Smallest i >= q with code(i) != c (or n); codes are nondecreasing in the
// position.  Called by all 64 lanes of one wave (same arguments, same
// result in every lane): a 64-ary search.  Each round probes 64 positions
// at once; while none differs the stride grows 64-fold, then each round
// narrows the bracket [first unknown, first known different] 64-fold.  A
// run of up to 63 keys takes one round trip, a run of L keys about
// 2 log64(L) (a one-thread gallop-and-bisect takes 2 log2(L) dependent
// loads).
template <int DT, typename CD>
__device__ uint32_t next_code_change(const typename KT<DT>::U *keys, uint32_t n, uint32_t q, uint32_t c,
                                     const CD &cd) {
    const uint64_t lane = threadIdx.x & 63;
    uint64_t lo = q, hi = n;  // the answer lies in [lo, hi]; hi differs (or is n)
    uint64_t stride = 1;
    bool growing = true;
    while (true) {
        const uint64_t i = lo + lane * stride;
        const bool diff = i >= hi || cd(keys[i]) != c;
        const uint64_t m = ballot64(diff);
        if (m == 0) {
            // lo + 63 * stride has code c
            lo += 63 * stride + 1;
            if (growing) stride *= 64;
            continue;
        }
        const uint64_t j = (uint64_t)__builtin_ctzll(m);
        const uint64_t cand = lo + j * stride < hi ? lo + j * stride : hi;
        if (j == 0 || stride == 1) return (uint32_t)cand;
        // lo + (j - 1) * stride has code c, cand differs
        hi = cand;
        lo += (j - 1) * stride + 1;
        growing = false;
        stride = stride / 64 > 0 ? stride / 64 : 1;
    }
}

// A piece boundary: p itself if p is 0, n, or the first key of a code run;
// otherwise the start of the next code run (one wave, as above).
template <int DT, typename CD>
__device__ uint32_t piece_boundary(const typename KT<DT>::U *keys, uint32_t n, uint32_t p, const CD &cd) {
    if (p == 0 || p >= n) return p >= n ? n : 0;
    return next_code_change<DT>(keys, n, p, cd(keys[p - 1]), cd);
}

template <typename U, int W, int IPT, int MR>
struct ChunkSmem {
    SmallSmem<U, false, W, IPT> sort;
    uint32_t mtot[MR], mstart[MR];  // top-digit buckets of the prefix finish
    uint32_t clast;  // code of the chunk's last element
    uint32_t cut;
    uint32_t bound[2];
    uint32_t code0;
    uint32_t code_next;  // code of the key after the chunk
};

// One workgroup per piece of the code-ordered array: cuts it at code
// changes into chunks of at most W*64*IPT keys and sorts each on chip.
// PREFIX: the code is the key-prefix field the run state describes, and the
// kernel exits at once if the run took plain passes instead; otherwise the
// model code.
// Register budget: WPE waves per SIMD (8: 64 VGPRs, so two 16-wave or four
// 8-wave workgroups per CU), so one workgroup's barriers overlap the
// others' loads.
template <int DT, int W, int IPT, int WPE, bool PREFIX, int MB = 9>
__global__ __launch_bounds__(W * 64) __attribute__((amdgpu_waves_per_eu(WPE))) void k_chunk_sort(typename KT<DT>::U *keys, uint32_t n, const float *model,
                                                       int cb, uint32_t piece, FbRun *fb, LearnedState *ls,
                                                       const RunState *st) {
    using U = typename KT<DT>::U;
    using CD = typename std::conditional<PREFIX, PrefixCoder<DT>, RmiCoder<DT>>::type;
    constexpr int B = W * 64, CAP = B * IPT;
    __shared__ ChunkSmem<U, W, IPT, (PREFIX && MB > 0) ? (1 << MB) : 1> sm;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    CD cd;
    if constexpr (PREFIX) {
        if (!st->pfx_active) return;
        cd.shift = st->pfx_shift;
        cd.mask = st->pfx_mask;
    } else {
        // the keys of a chunk lie in a narrow code range, so their leaf
        // records stay in cache: the table is read from global memory
        cd.h = rmi_head(model);
        cd.lv = rmi_leaves(model);
        cd.cb = cb;
        cd.scale = (float)(1u << cb);
    }
    const uint64_t p0 = (uint64_t)blockIdx.x * piece;
    const uint64_t p1 = std::min<uint64_t>(p0 + piece, n);
    // the two ends at once, one wave each
    if (w < 2) {
        const uint32_t b = piece_boundary<DT>(keys, n, (uint32_t)(w == 0 ? p0 : p1), cd);
        if (lane == 0) sm.bound[w] = b;
    }
    __syncthreads();
    uint32_t pos = sm.bound[0];
    const uint32_t end = sm.bound[1];
    uint32_t nchunks = 0;
    while (pos < end) {
        // per-thread indices re-derived per chunk from an opaque copy of the
        // thread id (hoisted out of the loop they would hold registers)
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int lane = tid & 63, w = tid >> 6;
        const uint32_t len = std::min<uint32_t>(CAP, end - pos);
        // one read of the chunk: registers (striped) for the sort and the cut
        U k[IPT];
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t e = striped_elem<IPT>(w, j, lane);
            k[j] = e < len ? keys[pos + e] : U(0);
        }
        uint32_t cut = end;
        if (pos + len < end) {
            // Here len == CAP.  Codes do not decrease along the chunk, so its
            // last code change is where the run of its last code starts.
            // Wave 0 forms the code of every SPAN-th element, then of each
            // element of the SPAN-wide gap in which that run starts (two
            // model rounds in one wave instead of one per key); wave 1
            // forms the codes of the chunk's first key and of the key after
            // the chunk.  The keys come from the cache (just loaded).
            constexpr uint32_t SPAN = CAP / 64;
            static_assert(CAP % 64 == 0 && SPAN <= 64 && W >= 2, "one wave covers the samples and a gap");
            if (w == 0) {
                const uint32_t c = cd(keys[pos + (uint32_t)(lane + 1) * SPAN - 1]);
                const uint32_t clast = __shfl(c, 63, 64);
                const uint32_t g = (uint32_t)__builtin_ctzll(ballot64(c == clast));  // lane 63 matches
                // the run starts in [g*SPAN, (g+1)*SPAN): its last element
                // is sample g, which has the last code
                const uint32_t c2 = (uint32_t)lane < SPAN ? cd(keys[pos + g * SPAN + (uint32_t)lane]) : clast;
                const uint64_t m2 = ballot64((uint32_t)lane < SPAN && c2 == clast);
                if (lane == 0) {
                    sm.clast = clast;
                    sm.cut = g * SPAN + (uint32_t)__builtin_ctzll(m2);
                }
            } else if (w == 1 && lane < 2) {
                const uint32_t c = cd(keys[pos + (lane == 0 ? len : 0u)]);
                if (lane == 0) sm.code_next = c;
                else sm.code0 = c;
            }
            __syncthreads();
            // the chunk ends at its own end if its last code differs from
            // the next key's
            const uint32_t q = sm.clast != sm.code_next ? len : sm.cut;
            if (q == 0) {
                // one code spans past the chunk: hand the whole run to the fallback
                if (w == 0) {
                    const uint32_t run_end = next_code_change<DT>(keys, end, pos + len, sm.code0, cd);
                    if (lane == 0) {
                        const uint32_t slot = atomicAdd(&ls->fb_count, 1u);
                        fb[slot] = FbRun{pos, run_end - pos};
                        sm.cut = run_end;
                    }
                }
                __syncthreads();
                pos = sm.cut;
                __syncthreads();
                continue;
            }
            cut = pos + q;
            __syncthreads();
        }
        // the group finish (passes over the top 16 varying bits, then
        // comparisons inside the short groups of equal top bits they leave;
        // LSD passes over every varying bit for chunks of few varying bits
        // or long groups), or for prefix chunks optionally one pass on the
        // top MB varying bits and comparisons inside its buckets
        if constexpr (PREFIX && MB > 0) lds_sort_chunk<DT, W, IPT, MB>(k, keys + pos, cut - pos, sm.sort, sm.mtot, sm.mstart, tid);
        else lds_sort_top<DT, W, IPT>(k, keys + pos, cut - pos, sm.sort, tid);
        ++nchunks;
        pos = cut;
        __syncthreads();
    }
    if (tid == 0 && nchunks) atomicAdd(&ls->chunks, nchunks);
}

// Fallback, step 1: flag runs holding more than one distinct key (every
// workgroup scans a slice of every run).
template <int DT>
__global__ __launch_bounds__(256) void k_fb_check(const typename KT<DT>::U *keys, const FbRun *fb,
                                                  const LearnedState *ls, uint32_t *nonconst) {
    using U = typename KT<DT>::U;
    const uint32_t nr = ls->fb_count;
    for (uint32_t r = 0; r < nr; ++r) {
        const FbRun run = fb[r];
        const U first = keys[run.start];
        bool diff = false;
        for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < run.len; i += (uint64_t)gridDim.x * 256)
            diff |= keys[run.start + i] != first;
        if (__syncthreads_or(diff) && threadIdx.x == 0) atomicOr(&nonconst[r], 1u);
    }
}

// Fallback: the runs become [lo, hi) ranges for the segmented sort (unused
// slots up to the capacity are empty ranges).
__global__ void k_fb_ranges(const FbRun *fb, LearnedState *ls, int64_t *lo, int64_t *hi, uint32_t cap) {
    const uint32_t nr = ls->fb_count;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += gridDim.x * blockDim.x) {
        if (i < nr) {
            const FbRun r = fb[i];
            lo[i] = r.start;
            hi[i] = (int64_t)r.start + r.len;
            atomicAdd(&ls->fb_keys, (unsigned long long)r.len);
        } else {
            lo[i] = 0;
            hi[i] = 0;
        }
    }
}

// Statistics only: keys of fallback runs that hold one repeated key.
__global__ void k_fb_const(const FbRun *fb, LearnedState *ls, const uint32_t *nonconst) {
    const uint32_t nr = ls->fb_count;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nr; i += gridDim.x * blockDim.x)
        if (!nonconst[i]) atomicAdd(&ls->const_keys, (unsigned long long)fb[i].len);
}

__global__ void k_learned_reset(LearnedState *ls, uint32_t *nonconst, uint32_t cap) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *ls = LearnedState{};
    for (uint32_t k = i; k < cap; k += gridDim.x * blockDim.x) nonconst[k] = 0;
}

// Top-level bucket histogram (statistics only); the counters follow the
// staged leaf table in dynamic LDS.
template <int DT>
__global__ __launch_bounds__(256) void k_bucket_hist(const typename KT<DT>::U *keys, uint32_t n, const float *model,
                                                     int cb, int shift, int nb, uint32_t *hist, int staged) {
    extern __shared__ float4 s_dyn[];
    const int L = (int)rmi_head(model).L;
    uint32_t *s_h = reinterpret_cast<uint32_t *>(s_dyn + (staged ? L + 1 : 0));
    for (int i = threadIdx.x; i < nb; i += 256) s_h[i] = 0;
    const RmiHead h = rmi_head(model);
    const RmiLeaf *lv = rmi_stage(model, staged ? s_dyn : nullptr);
    __syncthreads();
    const float scale = (float)(1u << cb);
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u)
        atomicAdd(&s_h[rmi_code(h, lv, KT<DT>::image(keys[i]), cb, scale) >> shift], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += 256)
        if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
}

// ------------------------------------------------------------ drivers
static int64_t sample_count(int64_t n, float frac) {
    int64_t m = (int64_t)((double)n * (double)frac);
    m = std::max<int64_t>(m, 4096);
    return std::min<int64_t>(m, n);
}

static int code_bits(int64_t n) {
    int lg = 1;
    while (lg < 40 && (int64_t(1) << lg) < n) ++lg;
    return std::min(24, std::max(12, lg - 7));
}

static inline size_t model_floats(int L) { return 8 + 4 * ((size_t)L + 1); }

// Fit scratch: leaf starts (L+1), scales (L), residuals (m), per-leaf sums
// (8 L); 256-byte aligned pieces in aux[1].
struct FitBufs {
    uint32_t *st;
    float *scales, *resid, *stats;
    uint32_t *ipre, *item_leaf;  // work items of the leaf sums
    float *part;                 // 8 partial sums per item
    uint32_t max_items;
    float *model_copy;
};
// upper bound of the fit's work items (every leaf adds at most one partial piece)
static inline size_t fit_max_items(uint32_t m, int L) { return (size_t)m / FIT_CH + (size_t)L + 1; }

static size_t fit_scratch_bytes(uint32_t m, int L, bool with_model) {
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t mi = fit_max_items(m, L);
    return al((size_t)(L + 1) * 4) + al((size_t)L * 4) + al((size_t)m * 4) + al((size_t)L * 32) +
           al((size_t)(L + 1) * 4) + al(mi * 4) + al(mi * 32) + (with_model ? model_floats(L) * 4 : 0) + 256;
}

static ak_status fit_scratch(Workspace *ws, uint32_t m, int L, bool with_model, FitBufs *f) {
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t mi = fit_max_items(m, L);
    const size_t o_sc = al((size_t)(L + 1) * 4);
    const size_t o_res = o_sc + al((size_t)L * 4);
    const size_t o_stats = o_res + al((size_t)m * 4);
    const size_t o_ipre = o_stats + al((size_t)L * 32);
    const size_t o_ileaf = o_ipre + al((size_t)(L + 1) * 4);
    const size_t o_part = o_ileaf + al(mi * 4);
    const size_t o_model = o_part + al(mi * 32);
    const size_t need = fit_scratch_bytes(m, L, with_model);
    ak_status r = ws_reserve(ws, &ws->aux[1], &ws->aux_bytes[1], need);
    if (r != AK_OK) return r;
    char *base = (char *)ws->aux[1];
    f->st = (uint32_t *)base;
    f->scales = (float *)(base + o_sc);
    f->resid = (float *)(base + o_res);
    f->stats = (float *)(base + o_stats);
    f->ipre = (uint32_t *)(base + o_ipre);
    f->item_leaf = (uint32_t *)(base + o_ileaf);
    f->part = (float *)(base + o_part);
    f->max_items = (uint32_t)mi;
    f->model_copy = (float *)(base + o_model);
    return AK_OK;
}

// Work items of the leaf sums, from the leaf starts f.st.
static ak_status fit_items(hipStream_t s, int L, const FitBufs &f) {
    hipLaunchKernelGGL(k_fit_items, dim3(1), dim3(1024), 0, s, (const uint32_t *)f.st, L, f.ipre);
    AK_LAUNCH_CHECK("k_fit_items");
    hipLaunchKernelGGL(k_fit_itemmap, dim3((unsigned)std::min(L, 4096)), dim3(256), 0, s, (const uint32_t *)f.ipre, L,
                       f.item_leaf);
    AK_LAUNCH_CHECK("k_fit_itemmap");
    return AK_OK;
}

// Loss, gradient and curvature of every leaf into `stats` (8 per leaf).
template <int DT>
static ak_status leaf_sums(hipStream_t s, const typename KT<DT>::U *srt, uint32_t m, int L, const float *model,
                           const FitBufs &f, float *stats) {
    hipLaunchKernelGGL((k_rmi_fwd<DT>), dim3(f.max_items), dim3(256), 0, s, srt, m, (const uint32_t *)f.st,
                       (const uint32_t *)f.ipre, (const uint32_t *)f.item_leaf, L, model, (const float *)f.scales,
                       f.resid, f.part);
    AK_LAUNCH_CHECK("k_rmi_fwd");
    hipLaunchKernelGGL((k_rmi_bwd<DT>), dim3(f.max_items), dim3(256), 0, s, srt, (const uint32_t *)f.st,
                       (const uint32_t *)f.ipre, (const uint32_t *)f.item_leaf, L, model, (const float *)f.scales,
                       (const float *)f.resid, f.part);
    AK_LAUNCH_CHECK("k_rmi_bwd");
    hipLaunchKernelGGL(k_rmi_sum, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, s, (const uint32_t *)f.st,
                       (const uint32_t *)f.ipre, L, (const float *)f.scales, (const float *)f.part, stats);
    AK_LAUNCH_CHECK("k_rmi_sum");
    return AK_OK;
}

template <int DT>
static ak_status fit_t(Workspace *ws, const void *sorted, uint32_t m, int L, int iters, float *model,
                       bool untrained) {
    using U = typename KT<DT>::U;
    hipStream_t s = ws->stream;
    const U *srt = (const U *)sorted;
    const unsigned lg = (unsigned)((L + 256) / 256);
    ProfScope ps("rmi_fit", s);
    if (untrained) {
        hipLaunchKernelGGL((k_rmi_untrained<DT>), dim3(lg), dim3(256), 0, s, srt, m, L, model);
        AK_LAUNCH_CHECK("k_rmi_untrained");
        return AK_OK;
    }
    FitBufs f;
    ak_status r = fit_scratch(ws, m, L, false, &f);
    if (r != AK_OK) return r;
    hipLaunchKernelGGL((k_rmi_root<DT>), dim3(1), dim3(64), 0, s, srt, m, L, model);
    AK_LAUNCH_CHECK("k_rmi_root");
    hipLaunchKernelGGL((k_rmi_bounds<DT>), dim3(lg), dim3(256), 0, s, srt, m, (const float *)model, f.st);
    AK_LAUNCH_CHECK("k_rmi_bounds");
    hipLaunchKernelGGL((k_rmi_leaf_init<DT>), dim3(lg), dim3(256), 0, s, srt, m, (const uint32_t *)f.st, model,
                       f.scales);
    AK_LAUNCH_CHECK("k_rmi_leaf_init");
    if ((r = fit_items(s, L, f)) != AK_OK) return r;
    for (int it = 0; it < iters; ++it) {
        if ((r = leaf_sums<DT>(s, srt, m, L, model, f, f.stats)) != AK_OK) return r;
        hipLaunchKernelGGL(k_rmi_update, dim3(lg), dim3(256), 0, s, model, (const uint32_t *)f.st,
                           (const float *)f.scales, (const float *)f.stats);
        AK_LAUNCH_CHECK("k_rmi_update");
    }
    return AK_OK;
}

template <int DT>
static ak_status root_t(hipStream_t s, const void *sorted, uint32_t m, int L, float *model) {
    hipLaunchKernelGGL((k_rmi_root<DT>), dim3(1), dim3(64), 0, s, (const typename KT<DT>::U *)sorted, m, L, model);
    AK_LAUNCH_CHECK("k_rmi_root");
    return AK_OK;
}

static ak_status read_leaves(hipStream_t s, const float *model, int *L) {
    float head[8];
    AK_HIP(hipMemcpyAsync(head, model, sizeof(head), hipMemcpyDeviceToHost, s));
    AK_HIP(hipStreamSynchronize(s));
    const float lf = head[3];
    if (!(lf >= 1.f && lf <= 65536.f) || lf != (float)(int)lf) {
        set_error("model has a bad leaf count");
        return AK_ERR_INVALID_ARG;
    }
    *L = (int)lf;
    return AK_OK;
}

template <int DT>
static ak_status leaf_grad_t(Workspace *ws, const void *sorted, uint32_t m, const float *model_in, float *out) {
    using U = typename KT<DT>::U;
    hipStream_t s = ws->stream;
    int L = 0;
    ak_status r = read_leaves(s, model_in, &L);
    if (r != AK_OK) return r;
    FitBufs f;
    if ((r = fit_scratch(ws, m, L, false, &f)) != AK_OK) return r;
    const U *srt = (const U *)sorted;
    const unsigned lg = (unsigned)((L + 256) / 256);
    // leaf ranges and scales come from the samples (as in a fit); the given
    // parameters (a, b, x0) are used as they are
    hipLaunchKernelGGL((k_rmi_bounds<DT>), dim3(lg), dim3(256), 0, s, srt, m, model_in, f.st);
    AK_LAUNCH_CHECK("k_rmi_bounds");
    hipLaunchKernelGGL((k_leaf_scale<DT>), dim3(lg), dim3(256), 0, s, srt, (const uint32_t *)f.st, model_in,
                       f.scales);
    AK_LAUNCH_CHECK("k_leaf_scale");
    if ((r = fit_items(s, L, f)) != AK_OK) return r;
    return leaf_sums<DT>(s, srt, m, L, model_in, f, out);
}

// Pieces of the code-ordered array per CU for the chunk sorts (one
// workgroup per piece, at least four chunks each; $AK_PIECES_PER_CU
// overrides the default).  Smaller pieces even out the tail of the launch:
// on 2^31 mixture keys the learned sort took 63.6-63.8 ms at 16 per CU,
// 61.3-62.4 at 64, 61.1-61.5 at 128 and 61.4-61.7 at 256.
static uint32_t pieces_per_cu() {
    static const uint32_t v = [] {
        const char *e = getenv("AK_PIECES_PER_CU");
        const int x = (e && *e) ? atoi(e) : 128;
        return (uint32_t)(x >= 1 && x <= 4096 ? x : 128);
    }();
    return v;
}

// On-chip chunk shapes (waves, keys per lane, register budget in waves per
// SIMD); $AK_CHUNK_VARIANT picks one (default 2).  The smallest capacity
// sizes the fallback bookkeeping: a fallback run is longer than a chunk.
struct ChunkShape {
    int w, ipt, wpe;
};
constexpr ChunkShape CHUNK_SHAPES[3] = {{16, 4, 8}, {8, 4, 8}, {4, 8, 6}};
constexpr int LEARNED_CAP_MIN = 2048;

static int chunk_variant() {
    static const int v = [] {
        const char *e = getenv("AK_CHUNK_VARIANT");
        const int x = (e && *e) ? atoi(e) : 2;  // 4 waves x 8 keys: fastest on the 2^31 mixture
        return x >= 0 && x < 3 ? x : 2;
    }();
    return v;
}

template <int DT, int V>
static void launch_chunk_sort(hipStream_t s, uint32_t npieces, typename KT<DT>::U *keys, uint32_t n,
                              const float *model, int cb, uint32_t piece, FbRun *fb, LearnedState *ls) {
    constexpr ChunkShape c = CHUNK_SHAPES[V];
    hipLaunchKernelGGL((k_chunk_sort<DT, c.w, c.ipt, c.wpe, false>), dim3(npieces), dim3(c.w * 64), 0, s, keys, n,
                       model, cb, piece, fb, ls, (const RunState *)nullptr);
}

// dtype dispatch of a templated driver
#define AK_DT_SWITCH(dt, FN, ...)                          \
    switch (dt) {                                          \
    case AK_I32: return FN<AK_I32>(__VA_ARGS__);           \
    case AK_I64: return FN<AK_I64>(__VA_ARGS__);           \
    case AK_U32: return FN<AK_U32>(__VA_ARGS__);           \
    case AK_U64: return FN<AK_U64>(__VA_ARGS__);           \
    case AK_F32: return FN<AK_F32>(__VA_ARGS__);           \
    case AK_F64: return FN<AK_F64>(__VA_ARGS__);           \
    }                                                      \
    return AK_ERR_UNSUPPORTED_DTYPE;

// ------------------------------------------- prefix-partitioned finish
// The plain radix sort of a key-only run whose top places spread the keys
// stops after the passes over those places; these launches finish it (they
// exit at once when the run took all its passes).
// Chunk shapes of the prefix finish (2048 keys each: waves, keys per lane,
// register budget, and how a chunk is finished: 0 = the group finish of
// lds_sort_top, else the bits of the one top-digit pass of lds_sort_chunk;
// $AK_PFX_CHUNK_VARIANT picks one).  2^30 uniform int64 keys: 27.6 ms with
// the first, 30.1 ms with the second, 30.5-30.7 ms with the one-pass
// finishes.
struct PfxShape {
    int w, ipt, wpe, mb;
};
constexpr PfxShape PFX_SHAPES[5] = {{4, 8, 6, 0}, {8, 4, 8, 0}, {8, 4, 8, 9}, {4, 8, 6, 9}, {4, 8, 6, 8}};
constexpr int PFX_CAP = 2048;
static_assert(PFX_SHAPES[0].w * 64 * PFX_SHAPES[0].ipt == PFX_CAP && PFX_SHAPES[1].w * 64 * PFX_SHAPES[1].ipt == PFX_CAP &&
                  PFX_SHAPES[2].w * 64 * PFX_SHAPES[2].ipt == PFX_CAP && PFX_SHAPES[3].w * 64 * PFX_SHAPES[3].ipt == PFX_CAP &&
                  PFX_SHAPES[4].w * 64 * PFX_SHAPES[4].ipt == PFX_CAP,
              "prefix chunk shapes hold PFX_CAP keys");

static int pfx_variant() {
    static const int v = [] {
        const char *e = getenv("AK_PFX_CHUNK_VARIANT");
        const int x = (e && *e) ? atoi(e) : 0;
        return x >= 0 && x < 5 ? x : 0;
    }();
    return v;
}

int prefix_chunk_keys() { return PFX_CAP; }

// a fallback run is longer than a chunk
static uint32_t prefix_fb_cap(int64_t n) { return (uint32_t)(n / prefix_chunk_keys() + 2); }

// aux[5]: state | fallback runs | range bounds (lo, hi)
static size_t prefix_aux_bytes(uint32_t cap) {
    return 256 + (((size_t)cap * sizeof(FbRun) + 255) & ~size_t(255)) + (size_t)cap * 16;
}

size_t prefix_finish_bytes(int dt, int64_t n, bool small) {
    const uint32_t cap = prefix_fb_cap(n);
    return ((prefix_aux_bytes(cap) + 255) & ~size_t(255)) + (small ? 0 : segmented_scratch_bytes(dt, n, cap, false));
}

ak_status prefix_reserve(Workspace *ws, int, int64_t n) {
    return ws_reserve(ws, &ws->aux[5], &ws->aux_bytes[5], prefix_aux_bytes(prefix_fb_cap(n)));
}

// Fallback of the prefix finish of small runs (at most a few million keys):
// every workgroup takes fallback runs from the list and sorts each with the
// one-workgroup LSD sort through the scratch copy.  One fixed launch, so a
// small sort's whole launch sequence can be captured and replayed; the runs
// a chunk cannot hold are rare there (the route is chosen only when the
// expected run is a quarter chunk).
constexpr int PFX_FB_W = 16, PFX_FB_IPT = 4;
template <int DT>
__global__ __launch_bounds__(PFX_FB_W * 64) void k_pfx_fallback(typename KT<DT>::U *keys, typename KT<DT>::U *tmp,
                                                                const FbRun *fb, LearnedState *ls) {
    using U = typename KT<DT>::U;
    __shared__ LongSmem<U, PFX_FB_W, PFX_FB_IPT> sm;
    __shared__ uint32_t s_r;
    while (true) {
        if (threadIdx.x == 0) s_r = atomicAdd(&ls->fb_next, 1u);
        __syncthreads();
        const uint32_t r = s_r;
        __syncthreads();
        if (r >= ls->fb_count) break;
        const FbRun run = fb[r];
        if (threadIdx.x == 0) atomicAdd(&ls->fb_keys, (unsigned long long)run.len);
        sort_long<DT, PFX_FB_W, PFX_FB_IPT>(keys + run.start, tmp + run.start, run.len, sm);
    }
}

template <int DT>
static ak_status prefix_finish_t(Workspace *ws, hipStream_t s, void *keys, int64_t n64, const RunState *st,
                                 bool small) {
    using U = typename KT<DT>::U;
    const uint32_t n = (uint32_t)n64;
    const uint32_t cap = prefix_fb_cap(n64);
    char *base = (char *)ws->aux[5];
    LearnedState *ls = (LearnedState *)base;
    FbRun *fb = (FbRun *)(base + 256);
    int64_t *lo = (int64_t *)(base + 256 + (((size_t)cap * sizeof(FbRun) + 255) & ~size_t(255)));
    int64_t *hi = lo + cap;
    hipLaunchKernelGGL(k_learned_reset, dim3(1), dim3(256), 0, s, ls, (uint32_t *)nullptr, 0u);
    AK_LAUNCH_CHECK("k_learned_reset");
    // small runs: one chunk per workgroup, so every CU works at once
    const uint32_t pieces_target = (uint32_t)num_cus() * pieces_per_cu();
    const uint32_t piece =
        small ? PFX_CAP : std::max<uint32_t>(PFX_CAP * 4, (n + pieces_target - 1) / pieces_target);
    const uint32_t npieces = (n + piece - 1) / piece;
    {
        ProfScope ps("prefix_chunk_sort", s);
        auto launch = [&](auto shape) {
            constexpr PfxShape c = PFX_SHAPES[decltype(shape)::value];
            hipLaunchKernelGGL((k_chunk_sort<DT, c.w, c.ipt, c.wpe, true, c.mb>), dim3(npieces), dim3(c.w * 64), 0, s,
                               (U *)keys, n, (const float *)nullptr, 0, piece, fb, ls, st);
        };
        switch (pfx_variant()) {
        case 0: launch(std::integral_constant<int, 0>{}); break;
        case 1: launch(std::integral_constant<int, 1>{}); break;
        case 2: launch(std::integral_constant<int, 2>{}); break;
        case 3: launch(std::integral_constant<int, 3>{}); break;
        default: launch(std::integral_constant<int, 4>{}); break;
        }
    }
    AK_LAUNCH_CHECK("k_chunk_sort");
    if (small) {
        ProfScope ps("prefix_fallback", s);
        hipLaunchKernelGGL((k_pfx_fallback<DT>), dim3((unsigned)num_cus()), dim3(PFX_FB_W * 64), 0, s, (U *)keys,
                           (U *)ws->keys0, (const FbRun *)fb, ls);
        AK_LAUNCH_CHECK("k_pfx_fallback");
        return AK_OK;
    }
    const uint32_t fgrid = std::min<uint32_t>((cap + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fb_ranges, dim3(fgrid), dim3(256), 0, s, (const FbRun *)fb, ls, lo, hi, cap);
    AK_LAUNCH_CHECK("k_fb_ranges");
    ProfScope ps("prefix_fallback", s);
    return segmented_sort_ranges(ws, DT, keys, lo, hi, cap, n64, ws->keys0);
}

ak_status prefix_counts(Workspace *ws, int64_t out[3]) {
    LearnedState ls{};
    AK_HIP(hipMemcpy(&ls, ws->aux[5], sizeof(ls), hipMemcpyDeviceToHost));
    out[0] = ls.chunks;
    out[1] = ls.fb_count;
    out[2] = (int64_t)ls.fb_keys;
    return AK_OK;
}

ak_status prefix_finish(Workspace *ws, hipStream_t s, int dt, void *keys, int64_t n, const RunState *st, bool small) {
    AK_DT_SWITCH(dt, prefix_finish_t, ws, s, keys, n, st, small)
}

// aux[0] of one learned call: sample keys | model | learned state |
// fallback runs | flags | fallback range bounds
static size_t learned_aux0_bytes(size_t kb, uint32_t m, int L, uint32_t fb_cap) {
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    return al((size_t)m * kb) + al(model_floats(L) * 4) + 256 + al((size_t)fb_cap * sizeof(FbRun)) +
           al((size_t)fb_cap * 4) + (size_t)fb_cap * 16 + 256;
}

template <int DT>
static ak_status learned_t(Workspace *ws, void *keys, int64_t n64, const ak_learned_cfg *cfg,
                           ak_learned_stats *stats) {
    using U = typename KT<DT>::U;
    hipStream_t s = ws->stream;
    const uint32_t n = (uint32_t)n64;
    if (n64 <= small_sort_capacity(DT)) {  // one workgroup sorts it on chip
        ak_status r = radix_sort(ws, DT, keys, nullptr, n64, 1);
        if (r == AK_OK && stats) {
            *stats = ak_learned_stats{};
            stats->n = n64;
            AK_HIP(hipStreamSynchronize(s));
        }
        return r;
    }
    const int L = cfg->leaves;
    const uint32_t m = (uint32_t)sample_count(n64, cfg->sample_frac);
    const int cb = code_bits(n64);
    const int cvar = chunk_variant();
    const int CAP = CHUNK_SHAPES[cvar].w * 64 * CHUNK_SHAPES[cvar].ipt;
    const uint32_t fb_cap = n / LEARNED_CAP_MIN + 2;
    ak_status r;
    // aux[0]: sample keys | model | learned state | fallback runs | flags
    const size_t off_model = ((size_t)m * sizeof(U) + 255) & ~size_t(255);
    const size_t off_state = off_model + ((model_floats(L) * 4 + 255) & ~size_t(255));
    const size_t off_fb = off_state + 256;
    const size_t off_nc = off_fb + (((size_t)fb_cap * sizeof(FbRun) + 255) & ~size_t(255));
    const size_t off_lo = off_nc + (((size_t)fb_cap * 4 + 255) & ~size_t(255));
    const size_t off_hi = off_lo + (size_t)fb_cap * 8;
    const size_t need = learned_aux0_bytes(sizeof(U), m, L, fb_cap);
    if ((r = ws_reserve(ws, &ws->aux[0], &ws->aux_bytes[0], need)) != AK_OK) return r;
    char *base = (char *)ws->aux[0];
    U *sample = (U *)base;
    float *model = (float *)(base + off_model);
    LearnedState *ls = (LearnedState *)(base + off_state);
    FbRun *fb = (FbRun *)(base + off_fb);
    uint32_t *nonconst = (uint32_t *)(base + off_nc);
    int64_t *fb_lo = (int64_t *)(base + off_lo);
    int64_t *fb_hi = (int64_t *)(base + off_hi);

    hipLaunchKernelGGL(k_learned_reset, dim3(std::min<uint32_t>((fb_cap + 255) / 256, 1024)), dim3(256), 0, s, ls,
                       nonconst, fb_cap);
    AK_LAUNCH_CHECK("k_learned_reset");
    // 1. sample + sort the sample
    hipLaunchKernelGGL((k_sample<U>), dim3((m + 255) / 256), dim3(256), 0, s, (const U *)keys, (uint64_t)n,
                       cfg->seed, m, sample);
    AK_LAUNCH_CHECK("k_sample");
    if ((r = radix_sort(ws, DT, sample, nullptr, m, 1)) != AK_OK) return r;
    // 2. fit (the untrained model is the same for both model kinds)
    if (cfg->model == AK_MODEL_MLP && !cfg->untrained) {
        if ((r = mlp_fit(ws, DT, sample, m, L, cfg->train_iters, model, nullptr)) != AK_OK) return r;
    } else if ((r = fit_t<DT>(ws, sample, m, L, cfg->train_iters, model, cfg->untrained != 0)) != AK_OK) {
        return r;
    }
    // 3. order by code
    if ((r = code_partition(ws, DT, keys, n, model, L, cb, 2)) != AK_OK) return r;
    // 4. chunks on chip
    const uint32_t pieces_target = (uint32_t)num_cus() * pieces_per_cu();
    uint32_t piece = std::max<uint32_t>((uint32_t)CAP * 4, (n + pieces_target - 1) / pieces_target);
    const uint32_t npieces = (n + piece - 1) / piece;
    // The keys of a chunk lie in a narrow code range, so its model reads hit
    // one or two leaf records in cache: the table is not staged here, which
    // keeps the workgroup's LDS small enough for several per CU.
    const size_t stage = rmi_stage_bytes(L);
    {
        ProfScope ps_chunk("chunk_sort", s);
        switch (cvar) {
        case 0: launch_chunk_sort<DT, 0>(s, npieces, (U *)keys, n, (const float *)model, cb, piece, fb, ls); break;
        case 1: launch_chunk_sort<DT, 1>(s, npieces, (U *)keys, n, (const float *)model, cb, piece, fb, ls); break;
        default: launch_chunk_sort<DT, 2>(s, npieces, (U *)keys, n, (const float *)model, cb, piece, fb, ls); break;
        }
    }
    AK_LAUNCH_CHECK("k_chunk_sort");
    // 5. fallback runs: radix-sorted as segments (runs of one repeated key
    // only cost the histogram read there: every digit place is trivial)
    const uint32_t fgrid = std::min<uint32_t>((fb_cap + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fb_ranges, dim3(fgrid), dim3(256), 0, s, (const FbRun *)fb, ls, fb_lo, fb_hi, fb_cap);
    AK_LAUNCH_CHECK("k_fb_ranges");
    if ((r = ws_reserve(ws, &ws->keys0, &ws->keys0_bytes, (size_t)n * sizeof(U))) != AK_OK) return r;
    {
        ProfScope ps_fb("fallback_segmented", s);
        if ((r = segmented_sort_ranges(ws, DT, keys, fb_lo, fb_hi, fb_cap, n, ws->keys0)) != AK_OK) return r;
    }

    if (stats) {
        const int bl = std::min(std::min(cfg->buckets_log2, cb), 14);
        const int nb = 1 << bl;
        if ((r = ws_reserve(ws, &ws->aux[2], &ws->aux_bytes[2], (size_t)nb * 4)) != AK_OK) return r;
        uint32_t *hist = (uint32_t *)ws->aux[2];
        if ((r = zero_fill(s, hist, (size_t)nb * 4)) != AK_OK) return r;
        hipLaunchKernelGGL((k_fb_check<DT>), dim3(num_cus() * 4), dim3(256), 0, s, (const U *)keys,
                           (const FbRun *)fb, (const LearnedState *)ls, nonconst);
        AK_LAUNCH_CHECK("k_fb_check");
        hipLaunchKernelGGL(k_fb_const, dim3(fgrid), dim3(256), 0, s, (const FbRun *)fb, ls,
                           (const uint32_t *)nonconst);
        AK_LAUNCH_CHECK("k_fb_const");
        hipLaunchKernelGGL((k_bucket_hist<DT>), dim3(num_cus() * 4), dim3(256), stage + (size_t)nb * 4, s,
                           (const U *)keys, n, (const float *)model, cb, cb - bl, nb, hist, (int)(stage > 0));
        AK_LAUNCH_CHECK("k_bucket_hist");
        LearnedState hls;
        std::vector<uint32_t> hh(nb);
        AK_HIP(hipMemcpyAsync(&hls, ls, sizeof(hls), hipMemcpyDeviceToHost, s));
        AK_HIP(hipMemcpyAsync(hh.data(), hist, (size_t)nb * 4, hipMemcpyDeviceToHost, s));
        AK_HIP(hipStreamSynchronize(s));
        ak_learned_stats st{};
        st.n = n64;
        st.sample_size = m;
        st.leaves = L;
        st.code_bits = cb;
        st.max_bucket = *std::max_element(hh.begin(), hh.end());
        st.imbalance = (double)st.max_bucket / ((double)n64 / nb);
        st.fallback_keys = (int64_t)hls.fb_keys;
        st.constant_keys = (int64_t)hls.const_keys;
        st.fallback_runs = hls.fb_count;
        st.chunks = hls.chunks;
        *stats = st;
    }
    return AK_OK;
}


ak_status learned_sort(Workspace *ws, int dt, void *keys, int64_t n, const ak_learned_cfg *cfg,
                       ak_learned_stats *stats) {
    AK_DT_SWITCH(dt, learned_t, ws, keys, n, cfg, stats)
}

// Sum of what one call reserves, in order: sample, model and fallback
// bookkeeping; fit scratch; the sample's radix sort; the code passes; the
// fallback's segmented sort over fb_cap ranges (its key scratch is keys0);
// the statistics histogram.  Buffers that grow within the call (sample
// sort, then the code passes) are counted at both sizes, which is what a
// caller arena needs (the library's own buffers grow in place).
size_t learned_temp_bytes(int dt, int64_t n, const ak_learned_cfg *cfg) {
    if (n <= small_sort_capacity(dt)) return 0;
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const int64_t m = sample_count(n, cfg->sample_frac);
    const int L = cfg->leaves;
    const size_t kb = (size_t)dtype_bytes(dt);
    const uint32_t fb_cap = (uint32_t)(n / LEARNED_CAP_MIN + 2);
    const size_t aux0 = al(learned_aux0_bytes(kb, (uint32_t)m, L, fb_cap));
    const size_t aux1 = al(cfg->model == AK_MODEL_MLP ? mlp_scratch_bytes(m) : fit_scratch_bytes((uint32_t)m, L, false));
    return aux0 + aux1 + radix_temp_bytes(dt, m, false) + code_partition_bytes(dt, n) +
           segmented_scratch_bytes(dt, n, fb_cap, false) + al((size_t)4 << 14);
}

template <int DT>
static ak_status sample_t(hipStream_t s, const void *keys, int64_t n, uint64_t seed, int64_t m, void *out) {
    using U = typename KT<DT>::U;
    hipLaunchKernelGGL((k_sample<U>), dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, (const U *)keys,
                       (uint64_t)n, seed, (uint32_t)m, (U *)out);
    AK_LAUNCH_CHECK("k_sample");
    return AK_OK;
}

ak_status learned_sample(hipStream_t s, int dt, const void *keys, int64_t n, uint64_t seed, int64_t m, void *out) {
    AK_DT_SWITCH(dt, sample_t, s, keys, n, seed, m, out)
}

template <int DT>
static ak_status fit_entry_t(Workspace *ws, const void *sorted, int64_t m, int L, int iters, float *model) {
    return fit_t<DT>(ws, sorted, (uint32_t)m, L, iters, model, false);
}

ak_status rmi_fit(Workspace *ws, int dt, const void *sorted, int64_t m, int leaves, int iters, float *model) {
    AK_DT_SWITCH(dt, fit_entry_t, ws, sorted, m, leaves, iters, model)
}

template <int DT>
static ak_status grad_entry_t(Workspace *ws, const void *sorted, int64_t m, const float *model, float *out) {
    return leaf_grad_t<DT>(ws, sorted, (uint32_t)m, model, out);
}

ak_status rmi_leaf_grad(Workspace *ws, int dt, const void *sorted, int64_t m, const float *model, float *out) {
    AK_DT_SWITCH(dt, grad_entry_t, ws, sorted, m, model, out)
}

template <int DT>
static ak_status codes_t(hipStream_t s, const void *keys, int64_t n, const float *model, int cb, uint32_t *codes) {
    using U = typename KT<DT>::U;
    int L = 0;
    ak_status r = read_leaves(s, model, &L);
    if (r != AK_OK) return r;
    const size_t stage = rmi_stage_bytes(L);
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, (int64_t)num_cus() * 8);
    hipLaunchKernelGGL((k_rmi_codes<DT>), dim3(grid), dim3(256), stage, s, (const U *)keys, (uint32_t)n, model, cb,
                       codes, (int)(stage > 0));
    AK_LAUNCH_CHECK("k_rmi_codes");
    return AK_OK;
}

ak_status rmi_codes(hipStream_t s, int dt, const void *keys, int64_t n, const float *model, int cb,
                    uint32_t *codes) {
    AK_DT_SWITCH(dt, codes_t, s, keys, n, model, cb, codes)
}

ak_status rmi_root(hipStream_t s, int dt, const void *sorted, uint32_t m, int L, float *model) {
    AK_DT_SWITCH(dt, root_t, s, sorted, m, L, model)
}

}  // namespace ak
