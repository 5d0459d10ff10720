// Batched segmented sort: every segment [off[s], off[s+1]) sorted on its own,
// all segments of a class in one persistent launch.
//
// Segments are binned by length into work buckets processed largest first:
//   huge   (>= xl_min keys)       many workgroups: per-segment digit
//                                 histograms, then one-sweep passes whose
//                                 look-back stays inside the segment (tiles of
//                                 all huge segments share persistent grids)
//   long   (c_max < len < xl_min) one 1024-thread workgroup, multi-pass LSD
//                                 radix through a scratch copy (one bucket per
//                                 power of two, longest first, so the tail is
//                                 short ones); its own persistent kernel
//   big    (b_max < len <= c_max) one 512-thread workgroup, on-chip sort of
//                                 up to 16384 keys (one read, one write; 32
//                                 keys per lane, 256 registers); its own
//                                 persistent kernel, segments above 8192 keys
//                                 first
//   medium (a_max < len <= b_max) one workgroup, on-chip sort
//   short  (2 <= len <= a_max)    one wave per segment, on-chip sort
// The on-chip classes share a second persistent kernel.  Their tile shapes
// (keys per lane of the short and medium classes) are
// template variants chosen from a tuning table written by the autotuner;
// the class limits and the persistent grid are runtime knobs of the same
// table.  The launch sequence (reset, count, scan, place, sort) is captured
// once per (dtype, segment count, tuning) into a HIP graph and replayed; the
// kernels read every pointer from a device-side argument block that a tiny
// kernel rewrites before each replay.
#include <dlfcn.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "lds_sort.h"
#include "long_sort.h"

namespace ak {

constexpr int SEG_W = 4;              // waves of a persistent workgroup
constexpr int B_XL = 0;               // huge segments
constexpr int NB_LONG = 24;           // long buckets 1..24: 32 - floor(log2(len))
constexpr int B_BIG2 = NB_LONG + 1;   // big bucket, above BIG_SPLIT keys
constexpr int B_BIG1 = NB_LONG + 2;   // big bucket, up to BIG_SPLIT keys
constexpr int B_MED = NB_LONG + 3;    // medium bucket
constexpr int B_SHORT = NB_LONG + 4;  // short bucket
constexpr int NB = NB_LONG + 5;
constexpr int BIG_W = 8;              // waves of the big class's workgroup (256 VGPRs each)
constexpr int BIG_SPLIT = BIG_W * 64 * 16;
// keys per lane of the big class's largest tile (LDS: 128 KB of keys)
template <typename U>
constexpr int big_ipt() { return 32; }
inline uint32_t big_cap(int) { return (uint32_t)BIG_W * 64u * 32u; }
// Huge-class tile shapes (W waves x IPT keys per lane); xl_variant() picks
// one per key width ($AK_XL_VARIANT overrides the default), and the tile
// size travels in the argument block.  Defaults from the sweeps: 32-bit
// keys on the 100,000-segment batch (65% of the keys in huge segments):
// 8 x 12 keys 9.28 ms, 8 x 10 9.89 ms, 8 x 8 10.51 ms, 8 x 14 11.55 ms,
// 16 x 8 and 8 x 16 11.15 ms (8 x 16 holds 162 registers, three waves per
// SIMD); 64-bit keys (the learned sort's fallback runs of 2^31 mixture
// keys, whole learned sort): 8 x 8 68.2 ms, 8 x 12 68.9 ms.
struct XlShape {
    int w, ipt;
};
constexpr int XL_NVAR = 4;
constexpr XlShape XL_SHAPES[XL_NVAR] = {{8, 12}, {8, 10}, {8, 14}, {8, 8}};
constexpr int XL_HT = 16;             // tiles per histogram work item
static int xl_variant(int dt) {
    static const int forced = [] {
        const char *e = getenv("AK_XL_VARIANT");
        const int x = (e && *e) ? atoi(e) : -1;
        return x >= 0 && x < XL_NVAR ? x : -1;
    }();
    if (forced >= 0) return forced;
    return key_bits(dt) == 64 ? 3 : 0;
}
static uint32_t xl_tile(int dt) {
    const XlShape sh = XL_SHAPES[xl_variant(dt)];
    return (uint32_t)(sh.w * 64 * sh.ipt);
}

// per huge segment: active digit places and the index of each active pass
struct XlDesc {
    uint8_t j[8];
    uint32_t mask;
    uint32_t q;
};

struct SegArgs {
    void *keys;
    const int64_t *off;  // segment s is keys[off[s] .. hi[s])
    const int64_t *hi;   // (CSR offsets: hi = off + 1)
    void *tmp;          // scratch, same layout as keys[off[0] ..)
    int32_t *list;      // segment ids, grouped by bucket
    int64_t nseg;
    int64_t base;       // off[0]
    int64_t end;        // off[nseg]
    uint32_t a_max, b_max, c_max, xl_min;
    uint32_t xl_tile;   // keys per huge-class tile
    uint32_t xl_cap;    // room for huge segments in the arrays below
    uint32_t *xl_pre;   // xl_cap+1 tile prefix of the huge segments
    uint32_t *xl_tseg;  // huge segment of every tile
    uint32_t xl_tcap;   // room for tiles in xl_tseg and per place in xl_amap
    uint32_t *xl_apre;  // (places+1) x (xl_cap+1): tile prefix of the segments with work there
    uint32_t *xl_amap;  // (places+1) x xl_tcap: segment of every such tile
    uint32_t *xl_hist;  // xl_cap x places x RADIX digit counts
    XlDesc *xl_desc;    // xl_cap descriptors
    uint64_t *xl_lb;    // look-back words, tiles x RADIX
    uint64_t xl_lb_words;
};

struct SegState {
    uint32_t count[NB];
    uint32_t start[NB + 1];
    uint32_t cursor[NB];
    uint32_t next_item;     // work counter of the on-chip classes
    uint32_t nitems;
    uint32_t next_long;     // work counter of the long class
    uint32_t next_big;      // work counter of the big class
    uint32_t error;
    uint32_t xl_count;      // huge segments (<= xl_cap)
    uint32_t xl_tiles;      // their tiles
    uint32_t xl_ctr[12];    // work counters: hist, scan, 8 passes, final
    uint32_t xl_atiles[9];  // tiles with work per place (index 8: the copy back)
    uint32_t epoch;         // look-back epoch base of this call
    uint32_t lb_clear;      // 1: epochs wrapped, clear the look-back words
};

struct SegTune {
    int ipt_a = 4;        // short class: 64*ipt_a keys per wave
    int ipt_b = 16;       // medium class and long-class tiles: 256*ipt_b keys
    int grid_mult = 4;    // persistent workgroups per CU
    int b_max = 0;        // 0: the medium capacity
    int xl_min = 32768;   // shortest segment of the huge class
};

__device__ __forceinline__ int seg_bucket(uint32_t len, uint32_t a_max, uint32_t b_max, uint32_t c_max,
                                          uint32_t xl_min) {
    if (len <= 1) return -1;
    if (len <= a_max) return B_SHORT;
    if (len <= b_max) return B_MED;
    if (len >= xl_min) return B_XL;
    if (len <= c_max) return len > (uint32_t)BIG_SPLIT ? B_BIG2 : B_BIG1;
    const int lg = 31 - __builtin_clz(len);
    return 32 - lg < NB_LONG ? 32 - lg : NB_LONG;
}

// Writes the argument block.  With device_bounds the batch's ends are read
// here from the CSR offsets, base = off[0] and end = off[nseg], and checked
// against the key count `bound`: ends outside [0, bound] or decreasing set
// the error word and empty the batch (every kernel then finds no work).
__global__ void k_seg_setargs(SegArgs *a, SegArgs v, SegState *st, int device_bounds, int64_t bound) {
    if (device_bounds) {
        const int64_t b = v.off[0], e = v.hi[v.nseg - 1];
        if (b < 0 || e < b || e > bound) {
            atomicOr(&st->error, 1u);
            v.nseg = 0;
            v.base = v.end = 0;
        } else {
            v.base = b;
            v.end = e;
        }
    }
    *a = v;
}

// Also advances the look-back epoch (30-bit; 16 per call): on wrap the
// words are cleared by k_xl_lbclear before any pass uses them.
__global__ void k_seg_reset(SegState *st) {
    const int t = threadIdx.x;
    if (t < NB) {
        st->count[t] = 0;
        st->cursor[t] = 0;
    }
    if (t < 12) st->xl_ctr[t] = 0;
    if (t == 0) {
        st->next_item = 0;
        st->nitems = 0;
        st->next_long = 0;
        st->next_big = 0;
        uint32_t e = st->epoch + 16;
        st->lb_clear = 0;
        if (e < 16 || e + 16 >= (1u << 30)) {
            e = 16;
            st->lb_clear = 1;
        }
        st->epoch = e;
    }
}

__global__ __launch_bounds__(256) void k_seg_count(const SegArgs *ap, SegState *st) {
    const SegArgs a = *ap;
    __shared__ uint32_t s_c[NB];
    if (threadIdx.x < NB) s_c[threadIdx.x] = 0;
    __syncthreads();
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s < a.nseg) {
        const int64_t lo = a.off[s], hi = a.hi[s];
        if (hi < lo || lo < a.base || hi > a.end) {
            atomicOr(&st->error, 1u);
        } else {
            const int b = seg_bucket((uint32_t)(hi - lo), a.a_max, a.b_max, a.c_max, a.xl_min);
            if (b >= 0) atomicAdd(&s_c[b], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < NB && s_c[threadIdx.x]) atomicAdd(&st->count[threadIdx.x], s_c[threadIdx.x]);
}

__global__ void k_seg_scan(SegState *st) {
    if (threadIdx.x != 0) return;
    uint32_t run = 0;
    for (int b = 0; b < NB; ++b) {
        st->start[b] = run;
        run += st->count[b];
    }
    st->start[NB] = run;
    // short segments are taken SEG_W at a time (one per wave)
    st->nitems = st->start[B_SHORT] + (st->count[B_SHORT] + SEG_W - 1) / SEG_W;
    st->xl_count = st->count[B_XL];
}

__global__ __launch_bounds__(256) void k_seg_place(const SegArgs *ap, SegState *st) {
    const SegArgs a = *ap;
    __shared__ uint32_t s_c[NB], s_base[NB];
    if (threadIdx.x < NB) s_c[threadIdx.x] = 0;
    __syncthreads();
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int b = -1;
    uint32_t mine = 0;
    if (s < a.nseg) {
        const int64_t lo = a.off[s], hi = a.hi[s];
        if (hi >= lo && lo >= a.base && hi <= a.end)
            b = seg_bucket((uint32_t)(hi - lo), a.a_max, a.b_max, a.c_max, a.xl_min);
        if (b >= 0) mine = atomicAdd(&s_c[b], 1u);
    }
    __syncthreads();
    if (threadIdx.x < NB && s_c[threadIdx.x])
        s_base[threadIdx.x] = atomicAdd(&st->cursor[threadIdx.x], s_c[threadIdx.x]);
    __syncthreads();
    if (b >= 0) a.list[st->start[b] + s_base[b] + mine] = (int32_t)s;
}

// The long class and the on-chip classes run as two persistent kernels so
// that each gets its own register budget (one kernel holding all three
// sorts would need the largest of them, with spills).
constexpr int LONG_W = 16, LONG_IPT = 4;  // long-class tile: 4096 keys

// WPE: waves per SIMD the register allocation aims for: 8 fits two
// workgroups per CU (a few registers spill), 4 fits one without spills.
template <int DT, int WPE>
__global__ __launch_bounds__(LONG_W * 64) __attribute__((amdgpu_waves_per_eu(WPE))) void k_seg_long(
    const SegArgs *ap, SegState *st) {
    using U = typename KT<DT>::U;
    __shared__ LongSmem<U, LONG_W, LONG_IPT> sm;
    __shared__ uint32_t s_item;
    const SegArgs a = *ap;
    U *keys = (U *)a.keys;
    U *tmp = (U *)a.tmp;
    const uint32_t first = st->start[B_XL + 1], med0 = st->start[B_BIG2];
    while (true) {
        if (threadIdx.x == 0) s_item = first + atomicAdd(&st->next_long, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= med0) break;
        const int64_t s = a.list[item];
        const int64_t lo = a.off[s], len = a.hi[s] - lo;
        sort_long<DT, LONG_W, LONG_IPT>(keys + lo, tmp + (lo - a.base), (uint32_t)len, sm);
    }
}

// Big class: one 1024-thread workgroup per segment, sorted on chip; the
// smaller tile shape for segments up to BIG_SPLIT keys (fewer idle lanes per
// ranking step), the 128 KB one above.
template <typename U>
union BigSmem {
    SmallSmem<U, false, BIG_W, 16> lo;
    SmallSmem<U, false, BIG_W, big_ipt<U>()> hi;
};

template <int DT>
__global__ __launch_bounds__(BIG_W * 64) void k_seg_big(const SegArgs *ap, SegState *st) {
    using U = typename KT<DT>::U;
    __shared__ BigSmem<U> sm;
    __shared__ uint32_t s_item;
    const SegArgs a = *ap;
    U *keys = (U *)a.keys;
    const uint32_t first = st->start[B_BIG2], end = st->start[B_MED];
    while (true) {
        if (threadIdx.x == 0) s_item = first + atomicAdd(&st->next_big, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= end) break;
        const int64_t s = a.list[item];
        const int64_t lo = a.off[s];
        const uint32_t len = (uint32_t)(a.hi[s] - lo);
        if (len <= (uint32_t)BIG_SPLIT) lds_sort_tile_top<DT, BIG_W, 16>(keys + lo, keys + lo, len, sm.lo, threadIdx.x);
        else lds_sort_tile_top<DT, BIG_W, big_ipt<U>()>(keys + lo, keys + lo, len, sm.hi, threadIdx.x);
        __syncthreads();
    }
}

template <typename U, int IPT_A, int IPT_B>
union SegSmem {
    SmallSmem<U, false, SEG_W, IPT_B> med;
    SmallSmem<U, false, 1, IPT_A> shrt[SEG_W];
};

// Register budget: three workgroups per CU for the medium tiles up to 16
// keys per lane (the group finish would otherwise take the kernel just past
// the 168 registers that allow it).
template <int DT, int IPT_A, int IPT_B>
__global__ __launch_bounds__(SEG_W * 64) __attribute__((amdgpu_waves_per_eu(IPT_B <= 16 ? 3 : 1))) void k_seg_sort(const SegArgs *ap, SegState *st) {
    using U = typename KT<DT>::U;
    __shared__ SegSmem<U, IPT_A, IPT_B> sm;
    __shared__ uint32_t s_item;
    const SegArgs a = *ap;
    U *keys = (U *)a.keys;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t nitems = st->nitems;
    const uint32_t med0 = st->start[B_MED], short0 = st->start[B_SHORT], nshort = st->count[B_SHORT];
    while (true) {
        if (tid == 0) s_item = med0 + atomicAdd(&st->next_item, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= nitems) break;
        if (item < short0) {
            const int64_t s = a.list[item];
            const int64_t lo = a.off[s], len = a.hi[s] - lo;
            lds_sort_tile_top<DT, SEG_W, IPT_B>(keys + lo, keys + lo, (uint32_t)len, sm.med, tid);
        } else {
            const uint32_t g = (item - short0) * SEG_W + w;
            if (g < nshort) {
                const int64_t s = a.list[short0 + g];
                const int64_t lo = a.off[s], len = a.hi[s] - lo;
                lds_sort_tile_top<DT, 1, IPT_A>(keys + lo, keys + lo, (uint32_t)len, sm.shrt[w], lane);
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------- huge segments
// Tiles of all huge segments are numbered consecutively, segment by
// segment; xl_pre[i] is the first tile of huge segment i.

__global__ __launch_bounds__(1024) void k_xl_prefix(const SegArgs *ap, SegState *st) {
    const SegArgs a = *ap;
    __shared__ uint32_t s_wsum[16];
    __shared__ uint32_t s_carry;
    const uint32_t cnt = min(st->xl_count, a.xl_cap);
    const uint32_t first = st->start[B_XL];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < cnt; base += 1024) {
        const uint32_t i = base + tid;
        uint32_t v = 0;
        if (i < cnt) {
            const int64_t s = a.list[first + i];
            const int64_t len = a.hi[s] - a.off[s];
            v = (uint32_t)((len + a.xl_tile - 1) / a.xl_tile);
        }
        const uint32_t incl = wave_incl_scan(v);
        if (lane == 63) s_wsum[w] = incl;
        __syncthreads();
        uint32_t pre = s_carry;
        for (int ww = 0; ww < w; ++ww) pre += s_wsum[ww];
        if (i < cnt) a.xl_pre[i] = pre + incl - v;
        __syncthreads();
        if (tid == 1023) s_carry = pre + incl;
        __syncthreads();
    }
    if (tid == 0) {
        a.xl_pre[cnt] = s_carry;
        st->xl_tiles = s_carry;
        st->xl_count = cnt;
    }
}

// Segment of every tile (one entry per tile, so the passes find their
// segment with one load instead of a search).
__global__ __launch_bounds__(256) void k_xl_tilemap(const SegArgs *ap, const SegState *st) {
    const SegArgs a = *ap;
    const uint32_t cnt = st->xl_count;
    for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x)
        for (uint32_t t = a.xl_pre[i] + threadIdx.x; t < a.xl_pre[i + 1]; t += 256) a.xl_tseg[t] = i;
}

// A huge segment has work at place p < P if that place is active for it,
// and at "place" P (the copy back) if it ran an odd number of passes.
template <int P>
__device__ __forceinline__ bool xl_has_work(const XlDesc &d, int p) {
    return p < P ? ((d.mask >> p) & 1u) != 0 : (d.q & 1u) != 0;
}

// Per place, numbers the tiles of the segments with work there
// consecutively (so a pass claims only tiles it has to process): one
// workgroup, a running prefix over the segments for each place.
template <int P>
__global__ __launch_bounds__(1024) void k_xl_active(const SegArgs *ap, SegState *st) {
    const SegArgs a = *ap;
    __shared__ uint32_t s_wsum[16];
    __shared__ uint32_t s_carry;
    const uint32_t cnt = st->xl_count;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int p = 0; p <= P; ++p) {
        uint32_t *pre = a.xl_apre + (size_t)p * (a.xl_cap + 1);
        if (tid == 0) s_carry = 0;
        __syncthreads();
        for (uint32_t base = 0; base < cnt; base += 1024) {
            const uint32_t i = base + tid;
            uint32_t v = 0;
            if (i < cnt && xl_has_work<P>(a.xl_desc[i], p)) v = a.xl_pre[i + 1] - a.xl_pre[i];
            const uint32_t incl = wave_incl_scan(v);
            if (lane == 63) s_wsum[w] = incl;
            __syncthreads();
            uint32_t run = s_carry;
            for (int ww = 0; ww < w; ++ww) run += s_wsum[ww];
            if (i < cnt) pre[i] = run + incl - v;
            __syncthreads();
            if (tid == 1023) s_carry = run + incl;
            __syncthreads();
        }
        if (tid == 0) {
            pre[cnt] = s_carry;
            st->xl_atiles[p] = s_carry;
        }
        __syncthreads();
    }
}

template <int P>
__global__ __launch_bounds__(256) void k_xl_amap(const SegArgs *ap, const SegState *st) {
    const SegArgs a = *ap;
    const uint32_t cnt = st->xl_count;
    for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
        const XlDesc d = a.xl_desc[i];
        for (int p = 0; p <= P; ++p) {
            if (!xl_has_work<P>(d, p)) continue;
            const uint32_t *pre = a.xl_apre + (size_t)p * (a.xl_cap + 1);
            uint32_t *map = a.xl_amap + (size_t)p * a.xl_tcap;
            for (uint32_t t = pre[i] + threadIdx.x; t < pre[i + 1]; t += 256) map[t] = i;
        }
    }
}

template <int P>
__global__ __launch_bounds__(256) void k_xl_zero(const SegArgs *ap, const SegState *st) {
    const SegArgs a = *ap;
    const size_t words = (size_t)st->xl_count * P * RADIX;
    for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < words; i += (size_t)gridDim.x * 256) a.xl_hist[i] = 0;
    if (st->lb_clear) {
        for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < a.xl_lb_words; i += (size_t)gridDim.x * 256)
            a.xl_lb[i] = 0;
    }
}

// Digit counts of every place per huge segment: work items of XL_HT tiles,
// counted in lane-private LDS counters (lane l adds to copy l mod 32 of a
// counter word; 16-bit halves for bins d and d + 128), so a wave's LDS
// atomics never meet in a bank whatever the digits; the copies are folded
// and added to the segment's global counts whenever the item's tiles move
// to another segment and at the item's end (an item adds at most
// XL_HT * tile / 32 to one 16-bit count, below 2^15 for every tile shape).
// A wave whose 64 keys are all equal (runs of one repeated key, as in the
// learned sort's fallback) adds its count once per place to a separate
// 32-bit array instead.
template <int DT>
__global__ __launch_bounds__(1024) void k_xl_hist(const SegArgs *ap, SegState *st) {
    using U = typename KT<DT>::U;
    constexpr int B = 1024;
    constexpr int P = (int)sizeof(U);
    constexpr int ROWS = P * 128, NR = (ROWS + B - 1) / B;
    __shared__ uint32_t s_h[ROWS * 32];
    __shared__ uint32_t s_eq[P * RADIX];
    __shared__ uint32_t s_item;
    const SegArgs a = *ap;
    const U *keys = (const U *)a.keys;
    const uint32_t ntiles = st->xl_tiles, first = st->start[B_XL];
    const uint32_t nitems = (ntiles + XL_HT - 1) / XL_HT;
    const int tid = threadIdx.x;
    const uint32_t copy = (uint32_t)tid & 31u;
    {
        uint4 *z = reinterpret_cast<uint4 *>(s_h);
        for (int i = tid; i < ROWS * 8; i += B) z[i] = make_uint4(0, 0, 0, 0);
        for (int i = tid; i < P * RADIX; i += B) s_eq[i] = 0;
    }
    // folds the copies of every counter word (lane r starts at copy r mod
    // 32: distinct banks), adds the totals to segment `seg`, clears
    auto flush = [&](int seg) {
        uint32_t *gh = a.xl_hist + (size_t)seg * P * RADIX;
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            const int r = j * B + tid;
            if (r < ROWS) {
                uint32_t lo = 0, hi = 0;
#pragma unroll 8
                for (int k = 0; k < 32; ++k) {
                    const int idx = r * 32 + ((k + r) & 31);
                    const uint32_t v = s_h[idx];
                    lo += v & 0xFFFFu;
                    hi += v >> 16;
                    s_h[idx] = 0;
                }
                const int p = r >> 7, w = r & 127;
                lo += s_eq[p * RADIX + w];
                hi += s_eq[p * RADIX + w + 128];
                s_eq[p * RADIX + w] = 0;
                s_eq[p * RADIX + w + 128] = 0;
                if (lo) atomicAdd(&gh[p * RADIX + w], lo);
                if (hi) atomicAdd(&gh[p * RADIX + w + 128], hi);
            }
        }
    };
    auto count4 = [&](uint32_t x, int p0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (p0 + q >= P) break;
            const uint32_t w = (x >> (8 * q)) & 127u;
            const uint32_t half = (x >> (8 * q + 7)) & 1u;
            atomicAdd(&s_h[((p0 + q) * 128 + w) * 32 + copy], half * 0xFFFFu + 1u);
        }
    };
    __syncthreads();
    while (true) {
        if (tid == 0) s_item = atomicAdd(&st->xl_ctr[0], 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= nitems) break;
        const uint32_t g0 = item * XL_HT, g1 = min(g0 + XL_HT, ntiles);
        int cur = -1;
        for (uint32_t g = g0; g < g1; ++g) {
            const int i = (int)a.xl_tseg[g];
            if (cur >= 0 && i != cur) {
                __syncthreads();
                flush(cur);
                __syncthreads();
            }
            cur = i;
            const int64_t s = a.list[first + i];
            const int64_t lo = a.off[s], len = a.hi[s] - lo;
            const uint32_t tb = (g - a.xl_pre[i]) * a.xl_tile;
            const uint32_t tv = (uint32_t)min((int64_t)a.xl_tile, len - (int64_t)tb);
            // XI keys per thread in flight before they are counted
            constexpr int XI = 4;
            for (uint32_t e0 = 0; e0 < tv; e0 += B * XI) {
                U v[XI];
#pragma unroll
                for (int it = 0; it < XI; ++it) {
                    const uint32_t e = e0 + it * B + tid;
                    v[it] = e < tv ? keys[lo + tb + e] : U(0);
                }
#pragma unroll
                for (int it = 0; it < XI; ++it) {
                    if (e0 + it * B + tid >= tv) break;
                    const U t = KT<DT>::image(v[it]);
                    const uint64_t act = ballot64(true);
                    const uint64_t t64 = (uint64_t)t;
                    const uint32_t tl = __builtin_amdgcn_readfirstlane((uint32_t)t64);
                    const uint32_t th = __builtin_amdgcn_readfirstlane((uint32_t)(t64 >> 32));
                    if (ballot64((uint32_t)t64 == tl && (uint32_t)(t64 >> 32) == th) == act) {
                        if (count_below(act) == 0) {
                            const uint32_t c = (uint32_t)__popcll(act);
#pragma unroll
                            for (int p = 0; p < P; ++p)
                                atomicAdd(&s_eq[p * RADIX + ((uint32_t)(t64 >> (8 * p)) & (RADIX - 1))], c);
                        }
                        continue;
                    }
                    count4((uint32_t)t64, 0);
                    if constexpr (P > 4) count4((uint32_t)(t64 >> 32), 4);
                }
            }
        }
        __syncthreads();
        if (cur >= 0) flush(cur);
        __syncthreads();
    }
}

// Per huge segment: exclusive digit offsets (in place of the counts),
// trivial places, and the index of every active pass.
template <int P>
__global__ __launch_bounds__(256) void k_xl_scan(const SegArgs *ap, SegState *st) {
    __shared__ uint32_t s_buf[RADIX], s_wsum[4];
    __shared__ int s_active[8];
    const SegArgs a = *ap;
    const uint32_t cnt = st->xl_count, first = st->start[B_XL];
    const int tid = threadIdx.x;
    for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
        const int64_t s = a.list[first + i];
        const uint32_t len = (uint32_t)(a.hi[s] - a.off[s]);
        for (int p = 0; p < P; ++p) {
            uint32_t *h = a.xl_hist + ((size_t)i * P + p) * RADIX;
            const uint32_t c = h[tid];
            const int trivial = __syncthreads_or(c == len);
            s_buf[tid] = c;
            __syncthreads();
            block_exscan<256, RADIX>(s_buf, s_buf, s_wsum, tid);
            h[tid] = s_buf[tid];
            if (tid == 0) s_active[p] = !trivial;
            __syncthreads();
        }
        if (tid == 0) {
            XlDesc d{};
            uint32_t q = 0;
            for (int p = 0; p < P; ++p) {
                if (s_active[p]) {
                    d.j[p] = (uint8_t)q++;
                    d.mask |= 1u << p;
                }
            }
            d.q = q;
            a.xl_desc[i] = d;
        }
        __syncthreads();
    }
}

// One digit place over the tiles of every huge segment (persistent grid,
// tiles taken in order).  Same tile work as the global one-sweep pass, with
// the look-back stopping at the segment's first tile and offsets relative
// to the segment; the segment ping-pongs with its scratch copy.
template <int DT, int W, int IPT>
__global__ __launch_bounds__(W * 64) void k_xl_pass(const SegArgs *ap, SegState *st, int place) {
    using U = typename KT<DT>::U;
    constexpr int B = W * 64, TILE = W * 64 * IPT;
    constexpr int P = (int)sizeof(U);
    constexpr size_t RAW = (size_t)TILE * sizeof(U) > (size_t)W * RADIX * 2 ? (size_t)TILE * sizeof(U)
                                                                            : (size_t)W * RADIX * 2;
    __shared__ __align__(16) uint8_t s_raw[RAW];
    __shared__ uint32_t s_tot[RADIX], s_start[RADIX], s_glob[RADIX], s_wsum[W];
    __shared__ uint32_t s_tile, s_seg;
    uint16_t *s_cnt = reinterpret_cast<uint16_t *>(s_raw);
    U *s_keys = reinterpret_cast<U *>(s_raw);
    const SegArgs a = *ap;
    U *keys = (U *)a.keys;
    U *tmp = (U *)a.tmp;
    const uint32_t ntiles = st->xl_atiles[place], first = st->start[B_XL];
    const uint32_t *amap = a.xl_amap + (size_t)place * a.xl_tcap;
    const uint32_t *apre = a.xl_apre + (size_t)place * (a.xl_cap + 1);
    const uint32_t epoch = st->epoch + (uint32_t)place;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // tiles of the segments active at this place only, in segment order
    while (true) {
        if (tid == 0) {
            s_tile = atomicAdd(&st->xl_ctr[2 + place], 1u);
            s_seg = s_tile < ntiles ? amap[s_tile] : 0u;
        }
        __syncthreads();
        const uint32_t tile = s_tile, i = s_seg;
        __syncthreads();
        if (tile >= ntiles) break;
        const XlDesc desc = a.xl_desc[i];
        const int64_t s = a.list[first + i];
        const int64_t lo = a.off[s], len = a.hi[s] - lo;
        const uint32_t lt = tile - apre[i];
        const uint32_t tbase = lt * (uint32_t)TILE;
        const uint32_t tvalid = (uint32_t)min((int64_t)TILE, len - (int64_t)tbase);
        const int jj_pass = desc.j[place];
        const U *src = (jj_pass & 1) ? tmp + (lo - a.base) : keys + lo;
        U *dst = (jj_pass & 1) ? keys + lo : tmp + (lo - a.base);
        const int shift = 8 * place;

        U k[IPT];
        uint32_t rd[IPT];  // digit, then rank | digit << 16
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t e = striped_elem<IPT>(w, j, lane);
            k[j] = e < tvalid ? src[tbase + e] : U(0);
            rd[j] = e < tvalid ? (uint32_t)(KT<DT>::image(k[j]) >> shift) & (RADIX - 1) : 0u;
        }
        rank_match_packed<RADIX_BITS, W, IPT, uint16_t>(rd, tvalid, s_cnt, s_tot, tid);
        uint64_t *lb = a.xl_lb + (size_t)tile * RADIX;
        for (int d = tid; d < RADIX; d += B)
            lb_store(lb + d, lb_pack(epoch, lt == 0 ? LB_INC : LB_AGG, s_tot[d]));
        block_exscan<B, RADIX>(s_tot, s_start, s_wsum, tid);
        rank_finish_packed<RADIX_BITS, W, IPT, uint16_t>(rd, s_cnt, s_start, tid);
        // staged by tile position before the look-back, as in the one-sweep
        // pass (the counters are dead after the barrier)
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t e = striped_elem<IPT>(w, j, lane);
            if (e < tvalid) s_keys[rd[j] & 0xFFFFu] = k[j];
        }
        {
            constexpr int K = B / RADIX;
            const int d = tid / K, kk = tid % K;
            uint32_t excl = 0;
            if (lt > 0) {
                excl = lookback_prefix<K, 4>(a.xl_lb + (size_t)(tile - lt) * RADIX + d, (int64_t)lt - 1, epoch, kk);
                if (kk == 0) lb_store(lb + d, lb_pack(epoch, LB_INC, excl + s_tot[d]));
            }
            if (kk == 0) s_glob[d] = a.xl_hist[((size_t)i * P + place) * RADIX + d] + excl - s_start[d];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t e = (uint32_t)(j * B + tid);
            if (e < tvalid) {
                const U key = s_keys[e];
                const uint32_t d = (uint32_t)(KT<DT>::image(key) >> shift) & (RADIX - 1);
                dst[s_glob[d] + e] = key;
            }
        }
        __syncthreads();
    }
}

// Huge segments that ran an odd number of passes end in the scratch copy.
template <int DT>
__global__ __launch_bounds__(256) void k_xl_final(const SegArgs *ap, SegState *st) {
    using U = typename KT<DT>::U;
    __shared__ uint32_t s_tile, s_seg;
    const SegArgs a = *ap;
    U *keys = (U *)a.keys;
    const U *tmp = (const U *)a.tmp;
    constexpr int P = (int)sizeof(U);
    const uint32_t ntiles = st->xl_atiles[P], first = st->start[B_XL];
    const uint32_t *amap = a.xl_amap + (size_t)P * a.xl_tcap;
    const uint32_t *apre = a.xl_apre + (size_t)P * (a.xl_cap + 1);
    while (true) {
        if (threadIdx.x == 0) {
            s_tile = atomicAdd(&st->xl_ctr[10], 1u);
            s_seg = s_tile < ntiles ? amap[s_tile] : 0u;
        }
        __syncthreads();
        const uint32_t tile = s_tile, i = s_seg;
        __syncthreads();
        if (tile >= ntiles) break;
        const int64_t s = a.list[first + i];
        const int64_t lo = a.off[s], len = a.hi[s] - lo;
        const uint32_t tbase = (tile - apre[i]) * a.xl_tile;
        const uint32_t tv = (uint32_t)min((int64_t)a.xl_tile, len - (int64_t)tbase);
        for (uint32_t e = threadIdx.x; e < tv; e += 256) keys[lo + tbase + e] = tmp[lo - a.base + tbase + e];
    }
}

// ------------------------------------------------------------ tuning
static std::mutex g_tune_mu;
static SegTune g_tune[2];  // [0]: 32-bit keys, [1]: 64-bit keys
static bool g_tune_loaded = false;

static int json_int(const std::string &txt, const std::string &obj, const char *field, int dflt) {
    const size_t o = txt.find("\"" + obj + "\"");
    if (o == std::string::npos) return dflt;
    const size_t e = txt.find('}', o);
    const size_t f = txt.find(std::string("\"") + field + "\"", o);
    if (f == std::string::npos || f > e) return dflt;
    const size_t c = txt.find(':', f);
    if (c == std::string::npos) return dflt;
    return atoi(txt.c_str() + c + 1);
}

// Reads the tuning table: $AK_TUNE_TABLE, else tune_gfx950.json next to
// libak.so.  Missing file or fields keep the built-in defaults.
static void load_tune_table() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    std::string path;
    if (const char *env = getenv("AK_TUNE_TABLE")) path = env;
    if (path.empty()) {
        Dl_info info;
        if (dladdr((void *)&load_tune_table, &info) && info.dli_fname) {
            std::string so = info.dli_fname;
            path = so.substr(0, so.find_last_of('/') + 1) + "tune_gfx950.json";
        }
    }
    FILE *f = path.empty() ? nullptr : fopen(path.c_str(), "rb");
    if (!f) return;
    std::string txt;
    char buf[4096];
    size_t r;
    while ((r = fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, r);
    fclose(f);
    const char *names[2] = {"seg32", "seg64"};
    for (int i = 0; i < 2; ++i) {
        g_tune[i].ipt_a = json_int(txt, names[i], "ipt_a", g_tune[i].ipt_a);
        g_tune[i].ipt_b = json_int(txt, names[i], "ipt_b", g_tune[i].ipt_b);
        g_tune[i].grid_mult = json_int(txt, names[i], "grid_mult", g_tune[i].grid_mult);
        g_tune[i].b_max = json_int(txt, names[i], "b_max", g_tune[i].b_max);
        g_tune[i].xl_min = json_int(txt, names[i], "xl_min", g_tune[i].xl_min);
    }
}

static bool tune_valid(int kb, const SegTune &t) {
    const bool a_ok = t.ipt_a == 2 || t.ipt_a == 4;
    const bool b_ok = t.ipt_b == 8 || t.ipt_b == 16 || (kb == 32 && t.ipt_b == 32);
    return a_ok && b_ok && t.grid_mult >= 1 && t.grid_mult <= 16 && t.b_max >= 0 && t.xl_min >= 4096;
}

}  // namespace ak

// Sets the segmented-sort tuning for 32- or 64-bit keys (autotuner hook).
extern "C" ak_status ak_seg_set_tuning(int key_bits, int ipt_a, int ipt_b, int grid_mult, int b_max,
                                       int xl_min) {
    using namespace ak;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_table();
    SegTune t{ipt_a, ipt_b, grid_mult, b_max, xl_min};
    if ((key_bits != 32 && key_bits != 64) || !tune_valid(key_bits, t)) {
        set_error("invalid segmented-sort tuning");
        return AK_ERR_INVALID_ARG;
    }
    g_tune[key_bits == 64] = t;
    return AK_OK;
}

namespace ak {

struct SegPlanKey {
    int dtype;
    int64_t nseg;
    int ipt_a, ipt_b, grid;
    bool operator<(const SegPlanKey &o) const {
        return std::tie(dtype, nseg, ipt_a, ipt_b, grid) < std::tie(o.dtype, o.nseg, o.ipt_a, o.ipt_b, o.grid);
    }
};

struct SegCache {
    SegArgs *args = nullptr;
    SegState *state = nullptr;
    hipStream_t capture = nullptr;
    std::map<SegPlanKey, hipGraphExec_t> graphs;
};
static std::mutex g_seg_mu;
static std::map<Workspace *, SegCache> g_seg;

template <int DT, int IA, int IB>
static void launch_sort_kernel(dim3 grid, hipStream_t s, const SegArgs *a, SegState *st) {
    hipLaunchKernelGGL((k_seg_sort<DT, IA, IB>), grid, dim3(SEG_W * 64), 0, s, a, st);
}

template <int DT>
static ak_status launch_seg_sort(const SegTune &t, dim3 grid, hipStream_t s, const SegArgs *a, SegState *st) {
    if (t.ipt_a == 2 && t.ipt_b == 8) launch_sort_kernel<DT, 2, 8>(grid, s, a, st);
    else if (t.ipt_a == 2 && t.ipt_b == 16) launch_sort_kernel<DT, 2, 16>(grid, s, a, st);
    else if (t.ipt_a == 4 && t.ipt_b == 8) launch_sort_kernel<DT, 4, 8>(grid, s, a, st);
    else if (t.ipt_a == 4 && t.ipt_b == 16) launch_sort_kernel<DT, 4, 16>(grid, s, a, st);
    else if constexpr (key_bits(DT) == 32) {
        if (t.ipt_a == 2 && t.ipt_b == 32) launch_sort_kernel<DT, 2, 32>(grid, s, a, st);
        else if (t.ipt_a == 4 && t.ipt_b == 32) launch_sort_kernel<DT, 4, 32>(grid, s, a, st);
        else return AK_ERR_INTERNAL;
    } else {
        return AK_ERR_INTERNAL;
    }
    AK_LAUNCH_CHECK("k_seg_sort");
    return AK_OK;
}

// Long-class kernel variant: 0 = two workgroups per CU, 1 = one
// ($AK_SEG_LONG_VARIANT overrides the default).
static int seg_long_variant() {
    static const int v = [] {
        const char *e = getenv("AK_SEG_LONG_VARIANT");
        return (e && *e) ? (atoi(e) == 1 ? 1 : 0) : 0;
    }();
    return v;
}

template <int DT>
static ak_status launch_seg_big(hipStream_t s, const SegArgs *a, SegState *st) {
    // 256 registers per lane: one workgroup per CU
    hipLaunchKernelGGL((k_seg_big<DT>), dim3((unsigned)num_cus()), dim3(BIG_W * 64), 0, s, a, st);
    AK_LAUNCH_CHECK("k_seg_big");
    return AK_OK;
}

template <int DT>
static ak_status launch_seg_long(hipStream_t s, const SegArgs *a, SegState *st) {
    if (seg_long_variant() == 0)
        hipLaunchKernelGGL((k_seg_long<DT, LONG_W / 2>), dim3((unsigned)num_cus() * 2), dim3(LONG_W * 64), 0, s, a,
                           st);
    else
        hipLaunchKernelGGL((k_seg_long<DT, LONG_W / 4>), dim3((unsigned)num_cus()), dim3(LONG_W * 64), 0, s, a,
                           st);
    AK_LAUNCH_CHECK("k_seg_long");
    return AK_OK;
}

template <int DT>
static ak_status launch_xl(int grid, hipStream_t s, SegArgs *a, SegState *st) {
    constexpr int P = key_bits(DT) / 8;
    hipLaunchKernelGGL(k_xl_prefix, dim3(1), dim3(1024), 0, s, a, st);
    AK_LAUNCH_CHECK("k_xl_prefix");
    hipLaunchKernelGGL(k_xl_tilemap, dim3(grid), dim3(256), 0, s, a, st);
    AK_LAUNCH_CHECK("k_xl_tilemap");
    hipLaunchKernelGGL((k_xl_zero<P>), dim3(grid), dim3(256), 0, s, a, st);
    AK_LAUNCH_CHECK("k_xl_zero");
    // one 1024-thread workgroup per CU for 64-bit keys (128 KB of counters), two for 32-bit keys
    hipLaunchKernelGGL((k_xl_hist<DT>), dim3((unsigned)num_cus() * (key_bits(DT) == 64 ? 1 : 2)), dim3(1024), 0, s,
                       a, st);
    AK_LAUNCH_CHECK("k_xl_hist");
    hipLaunchKernelGGL((k_xl_scan<P>), dim3(grid), dim3(256), 0, s, a, st);
    AK_LAUNCH_CHECK("k_xl_scan");
    hipLaunchKernelGGL((k_xl_active<P>), dim3(1), dim3(1024), 0, s, a, st);
    AK_LAUNCH_CHECK("k_xl_active");
    hipLaunchKernelGGL((k_xl_amap<P>), dim3(grid), dim3(256), 0, s, a, st);
    AK_LAUNCH_CHECK("k_xl_amap");
    for (int p = 0; p < P; ++p) {
        auto pass = [&](auto vc) {
            constexpr XlShape sh = XL_SHAPES[decltype(vc)::value];
            hipLaunchKernelGGL((k_xl_pass<DT, sh.w, sh.ipt>), dim3(grid), dim3(sh.w * 64), 0, s, a, st, p);
        };
        switch (xl_variant(DT)) {
        case 0: pass(std::integral_constant<int, 0>{}); break;
        case 1: pass(std::integral_constant<int, 1>{}); break;
        case 2: pass(std::integral_constant<int, 2>{}); break;
        default: pass(std::integral_constant<int, 3>{}); break;
        }
        AK_LAUNCH_CHECK("k_xl_pass");
    }
    hipLaunchKernelGGL((k_xl_final<DT>), dim3(grid), dim3(256), 0, s, a, st);
    AK_LAUNCH_CHECK("k_xl_final");
    return AK_OK;
}

static ak_status seg_launch_all(int dt, const SegTune &t, int64_t nseg, int grid, hipStream_t s, SegArgs *a,
                                SegState *st) {
    const unsigned g = (unsigned)((nseg + 255) / 256);
    hipLaunchKernelGGL(k_seg_reset, dim3(1), dim3(64), 0, s, st);
    AK_LAUNCH_CHECK("k_seg_reset");
    hipLaunchKernelGGL(k_seg_count, dim3(g), dim3(256), 0, s, a, st);
    AK_LAUNCH_CHECK("k_seg_count");
    hipLaunchKernelGGL(k_seg_scan, dim3(1), dim3(64), 0, s, st);
    AK_LAUNCH_CHECK("k_seg_scan");
    hipLaunchKernelGGL(k_seg_place, dim3(g), dim3(256), 0, s, a, st);
    AK_LAUNCH_CHECK("k_seg_place");
    ak_status r;
    switch (dt) {
    case AK_I32: r = launch_xl<AK_I32>(grid, s, a, st); break;
    case AK_I64: r = launch_xl<AK_I64>(grid, s, a, st); break;
    case AK_U32: r = launch_xl<AK_U32>(grid, s, a, st); break;
    case AK_U64: r = launch_xl<AK_U64>(grid, s, a, st); break;
    case AK_F32: r = launch_xl<AK_F32>(grid, s, a, st); break;
    case AK_F64: r = launch_xl<AK_F64>(grid, s, a, st); break;
    default: r = AK_ERR_UNSUPPORTED_DTYPE;
    }
    if (r != AK_OK) return r;
    switch (dt) {
    case AK_I32: r = launch_seg_long<AK_I32>(s, a, st); break;
    case AK_I64: r = launch_seg_long<AK_I64>(s, a, st); break;
    case AK_U32: r = launch_seg_long<AK_U32>(s, a, st); break;
    case AK_U64: r = launch_seg_long<AK_U64>(s, a, st); break;
    case AK_F32: r = launch_seg_long<AK_F32>(s, a, st); break;
    case AK_F64: r = launch_seg_long<AK_F64>(s, a, st); break;
    default: r = AK_ERR_UNSUPPORTED_DTYPE;
    }
    if (r != AK_OK) return r;
    switch (dt) {
    case AK_I32: r = launch_seg_big<AK_I32>(s, a, st); break;
    case AK_I64: r = launch_seg_big<AK_I64>(s, a, st); break;
    case AK_U32: r = launch_seg_big<AK_U32>(s, a, st); break;
    case AK_U64: r = launch_seg_big<AK_U64>(s, a, st); break;
    case AK_F32: r = launch_seg_big<AK_F32>(s, a, st); break;
    case AK_F64: r = launch_seg_big<AK_F64>(s, a, st); break;
    default: r = AK_ERR_UNSUPPORTED_DTYPE;
    }
    if (r != AK_OK) return r;
    switch (dt) {
    case AK_I32: return launch_seg_sort<AK_I32>(t, dim3(grid), s, a, st);
    case AK_I64: return launch_seg_sort<AK_I64>(t, dim3(grid), s, a, st);
    case AK_U32: return launch_seg_sort<AK_U32>(t, dim3(grid), s, a, st);
    case AK_U64: return launch_seg_sort<AK_U64>(t, dim3(grid), s, a, st);
    case AK_F32: return launch_seg_sort<AK_F32>(t, dim3(grid), s, a, st);
    case AK_F64: return launch_seg_sort<AK_F64>(t, dim3(grid), s, a, st);
    }
    return AK_ERR_UNSUPPORTED_DTYPE;
}

// Scratch layout of one call: the class limits from the tuning, and the
// pieces of misc2 (segment list, huge-segment tile prefix, descriptors,
// digit counts, tile maps) plus the huge segments' look-back words.
struct SegLayout {
    SegTune t;
    uint32_t a_max, b_max, c_max, xl_min, xl_cap, xl_tile;
    size_t off_pre, off_desc, off_hist, off_tseg, off_apre, off_amap, misc2_need;
    size_t max_tiles, lb_words;
};

static SegLayout seg_layout(int dt, int64_t n, int64_t nseg) {
    SegLayout L;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_tune_table();
        L.t = g_tune[key_bits(dt) == 64];
    }
    if (!tune_valid(key_bits(dt), L.t)) L.t = SegTune{};
    const SegTune &t = L.t;
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const int P = dtype_bytes(dt);
    L.a_max = 64u * (uint32_t)t.ipt_a;
    const uint32_t cap_b = 256u * (uint32_t)t.ipt_b;
    L.b_max = t.b_max > 0 ? std::min<uint32_t>((uint32_t)t.b_max, cap_b) : cap_b;
    L.xl_min = (uint32_t)std::max(t.xl_min, (int)L.b_max + 1);
    L.c_max = big_cap(dt);
    L.xl_cap = (uint32_t)std::min<int64_t>(nseg, n / L.xl_min + 1);
    L.xl_tile = xl_tile(dt);
    L.max_tiles = (size_t)n / L.xl_tile + L.xl_cap + 1;
    L.off_pre = al((size_t)nseg * 4);
    L.off_desc = L.off_pre + al((size_t)(L.xl_cap + 1) * 4);
    L.off_hist = L.off_desc + al((size_t)L.xl_cap * sizeof(XlDesc));
    L.off_tseg = L.off_hist + al((size_t)L.xl_cap * P * RADIX * 4);
    L.off_apre = L.off_tseg + al(L.max_tiles * 4);
    L.off_amap = L.off_apre + al((size_t)(P + 1) * (L.xl_cap + 1) * 4);
    L.misc2_need = L.off_amap + (size_t)(P + 1) * L.max_tiles * 4;
    L.lb_words = L.max_tiles * RADIX;
    return L;
}

// Scratch of one batched call over n keys in nseg segments (with_tmp: the
// key-sized scratch copy too).
size_t segmented_scratch_bytes(int dt, int64_t n, int64_t nseg, bool with_tmp) {
    if (n <= 0 || nseg <= 0) return 0;
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const SegLayout L = seg_layout(dt, n, nseg);
    return (with_tmp ? al((size_t)n * dtype_bytes(dt)) : 0) + al(L.misc2_need) + al(L.lb_words * 8);
}

size_t segmented_temp_bytes(int dt, int64_t n, int64_t nseg) { return segmented_scratch_bytes(dt, n, nseg, true); }

// Sorts the ranges keys[lo[s] .. hi[s]) (base <= lo <= hi <= end, ranges
// disjoint) through the captured launch sequence; `tmp` holds end - base
// keys of scratch laid out like keys[base ..).
// device_bounds: base and end are read from the offsets on the device (the
// caller gives only the key count as `end`, base 0), so the call never
// waits for the device unless scratch must grow.
static ak_status seg_run(Workspace *ws, int dt, void *keys, const int64_t *lo, const int64_t *hi, int64_t nseg,
                         int64_t base, int64_t end, void *tmp, bool device_bounds = false) {
    hipStream_t s = ws->stream;
    const int64_t n = end - base;
    const SegLayout L = seg_layout(dt, n, nseg);
    const SegTune &t = L.t;
    const int grid = num_cus() * t.grid_mult;
    ak_status r;
    const size_t kb = (size_t)dtype_bytes(dt);
    if (!tmp) {
        if ((r = ws_reserve(ws, &ws->misc, &ws->misc_bytes, (size_t)n * kb)) != AK_OK) return r;
        tmp = ws->misc;
    }
    if ((r = ws_reserve(ws, &ws->misc2, &ws->misc2_bytes, L.misc2_need)) != AK_OK) return r;
    if (L.lb_words * 8 > ws->aux_bytes[3]) {
        if ((r = ws_reserve(ws, &ws->aux[3], &ws->aux_bytes[3], L.lb_words * 8)) != AK_OK) return r;
        if ((r = zero_fill(s, ws->aux[3], ws->aux_bytes[3])) != AK_OK) return r;
    }

    std::lock_guard<std::mutex> lk(g_seg_mu);
    SegCache &c = g_seg[ws];
    if (!c.args) {
        AK_HIP(hipMalloc((void **)&c.args, sizeof(SegArgs)));
        AK_HIP(hipMalloc((void **)&c.state, sizeof(SegState)));
        if ((r = zero_fill(s, c.state, sizeof(SegState))) != AK_OK) return r;
        AK_HIP(hipStreamCreateWithFlags(&c.capture, hipStreamNonBlocking));
    }
    SegArgs v{};
    v.keys = keys;
    v.off = lo;
    v.hi = hi;
    v.tmp = tmp;
    v.list = (int32_t *)ws->misc2;
    v.nseg = nseg;
    v.base = base;
    v.end = end;
    v.a_max = L.a_max;
    v.b_max = L.b_max;
    v.xl_min = L.xl_min;
    v.c_max = L.c_max;
    v.xl_cap = L.xl_cap;
    v.xl_tile = L.xl_tile;
    v.xl_pre = (uint32_t *)((char *)ws->misc2 + L.off_pre);
    v.xl_desc = (XlDesc *)((char *)ws->misc2 + L.off_desc);
    v.xl_hist = (uint32_t *)((char *)ws->misc2 + L.off_hist);
    v.xl_tseg = (uint32_t *)((char *)ws->misc2 + L.off_tseg);
    v.xl_tcap = (uint32_t)L.max_tiles;
    v.xl_apre = (uint32_t *)((char *)ws->misc2 + L.off_apre);
    v.xl_amap = (uint32_t *)((char *)ws->misc2 + L.off_amap);
    v.xl_lb = (uint64_t *)ws->aux[3];
    v.xl_lb_words = ws->aux_bytes[3] / 8;
    hipLaunchKernelGGL(k_seg_setargs, dim3(1), dim3(1), 0, s, c.args, v, c.state, (int)device_bounds, end);
    AK_LAUNCH_CHECK("k_seg_setargs");

    SegPlanKey key{dt, nseg, t.ipt_a, t.ipt_b, grid};
    auto it = c.graphs.find(key);
    if (it == c.graphs.end()) {
        hipGraph_t g = nullptr;
        AK_HIP(hipStreamBeginCapture(c.capture, hipStreamCaptureModeRelaxed));
        ak_status lr = seg_launch_all(dt, t, nseg, grid, c.capture, c.args, c.state);
        hipError_t ce = hipStreamEndCapture(c.capture, &g);
        if (lr != AK_OK) {
            if (g) (void)hipGraphDestroy(g);
            return lr;
        }
        if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate");
        it = c.graphs.emplace(key, ex).first;
    }
    ProfScope ps("segmented_graph", s);
    AK_HIP(hipGraphLaunch(it->second, s));
    return AK_OK;
}

ak_status segmented_sort(Workspace *ws, int dt, void *keys, const int64_t *offsets, int64_t nseg) {
    hipStream_t s = ws->stream;
    if (nseg >= (int64_t(1) << 31)) {
        set_error("nseg >= 2^31");
        return AK_ERR_INVALID_ARG;
    }
    int64_t ends[2] = {0, 0};
    AK_HIP(hipMemcpyAsync(&ends[0], offsets, 8, hipMemcpyDeviceToHost, s));
    AK_HIP(hipMemcpyAsync(&ends[1], offsets + nseg, 8, hipMemcpyDeviceToHost, s));
    AK_HIP(hipStreamSynchronize(s));
    const int64_t n = ends[1] - ends[0];
    if (ends[0] < 0 || n < 0 || n > AK_MAX_KEYS) {
        set_error("offsets[nseg] - offsets[0] must be in [0, 2^31] and offsets[0] >= 0");
        return AK_ERR_INVALID_ARG;
    }
    if (n == 0) return AK_OK;
    ak_status r = ws_arena_fits(ws, segmented_temp_bytes(dt, n, nseg));
    if (r != AK_OK) return r;
    return seg_run(ws, dt, keys, offsets, offsets + 1, nseg, ends[0], ends[1], nullptr);
}

ak_status segmented_sort_n(Workspace *ws, int dt, void *keys, int64_t n, const int64_t *offsets, int64_t nseg) {
    if (nseg >= (int64_t(1) << 31)) {
        set_error("nseg >= 2^31");
        return AK_ERR_INVALID_ARG;
    }
    if (n == 0) return AK_OK;
    ak_status r = ws_arena_fits(ws, segmented_temp_bytes(dt, n, nseg));
    if (r != AK_OK) return r;
    return seg_run(ws, dt, keys, offsets, offsets + 1, nseg, 0, n, nullptr, true);
}

ak_status segmented_sort_ranges(Workspace *ws, int dt, void *keys, const int64_t *lo, const int64_t *hi,
                                int64_t nseg, int64_t end, void *tmp) {
    if (nseg <= 0 || end <= 0) return AK_OK;
    return seg_run(ws, dt, keys, lo, hi, nseg, 0, end, tmp);
}

// Device error flag of the segmented sort on this workspace (cleared).
uint32_t segmented_take_error(Workspace *ws) {
    std::lock_guard<std::mutex> lk(g_seg_mu);
    auto it = g_seg.find(ws);
    if (it == g_seg.end() || !it->second.state) return 0;
    uint32_t f = 0;
    if (hipMemcpy(&f, &it->second.state->error, 4, hipMemcpyDeviceToHost) != hipSuccess) return 0;
    if (f) {
        const uint32_t z = 0;
        (void)hipMemcpy(&it->second.state->error, &z, 4, hipMemcpyHostToDevice);
    }
    return f;
}

void segmented_release(Workspace *ws) {
    std::lock_guard<std::mutex> lk(g_seg_mu);
    auto it = g_seg.find(ws);
    if (it == g_seg.end()) return;
    for (auto &kv : it->second.graphs) (void)hipGraphExecDestroy(kv.second);
    if (it->second.args) (void)hipFree(it->second.args);
    if (it->second.state) (void)hipFree(it->second.state);
    if (it->second.capture) (void)hipStreamDestroy(it->second.capture);
    g_seg.erase(it);
}

}  // namespace ak
