// Kernels and launch sequences of the LSD radix sort (gfx950): up-front
// multi-place histogram, digit-offset scan with device-side pass skipping,
// one-sweep digit passes (stable in-tile ranking by wave ballots, decoupled
// look-back across tiles, LDS-staged coalesced scatter), the finishing
// copy, and the single-workgroup on-chip sort for small inputs.  Templated
// over the key type and over what the run carries with the keys (nothing,
// indices, a payload, or indices alone with the keys fetched through them),
// and included by the translation units that instantiate them.
//
// What is computed is the paper's sort / sortperm / sort by key
// (Sec. II-B): a stable ascending sort under the Julia Base order.  The
// paper builds its sorter as a merge sort in a portable kernel language;
// this library uses 8-bit LSD radix passes because ballots and per-wave LDS
// counters are available on gfx950 (the paper names wave-level intrinsics
// as what radix sort needs, Sec. I-B), and the prefix scan across tiles is
// the decoupled look-back scan that the paper cites for its accumulate
// (Sec. II-B).
#pragma once

#include <algorithm>
#include <functional>

#include "radix_common.h"
#include "radix_kernels.h"
#include "lds_sort.h"
#include "rmi_device.h"

namespace ak {

// ---------------------------------------------------------------- init
// Zeroes the run's counters (the digit counts are zero already: the digit
// scan of the previous run cleared them) and takes the next 16 look-back
// epochs from the workspace counter (restarting at 16 before 2^30; the host
// mirrors this and clears the look-back words at that point).
static __global__ void k_run_init(RunState *st, uint32_t *epoch_dev) {
    const int tid = threadIdx.x;
    if (tid < MAX_PLACES) st->tile_ctr[tid] = 0;
    if (tid == 0) {
        uint32_t e = *epoch_dev + 16;
        if (e + 16 >= (1u << 30)) e = 16;
        *epoch_dev = e;
        st->epoch_base = e;
    }
}

// Exclusive digit offsets per place; a place where one digit holds every
// key is inactive (its pass would be a copy).  Active passes are numbered
// so that each pass kernel can pick its source and destination buffers
// without a host round trip.  One 1024-thread workgroup, in its own launch
// after the histogram (the kernel boundary makes every workgroup's counts
// visible: a "last workgroup finishes" handoff inside the histogram needs a
// device-scope release fence in every workgroup, which on gfx950 writes
// back the L2 of its XCD, about 50 us at one million keys); it sums the
// HIST_REP copies, clears them for the next run, and scans four places at
// a time.
//
// pfx_cap > 0 (key-only runs that can finish on chip): if the top k = 2..4
// places spread the keys so that the expected largest run of equal prefix,
// n * prod over those places of (largest digit count / n), is at most
// pfx_cap keys, and the run then saves at least two passes, only the active
// places among those k keep their passes and the run is marked prefix-
// partitioned: the keys leave the passes ordered by their top k places,
// and the chunk sort finishes each run of equal prefix.  The estimate
// assumes independent places; a wrong guess costs time (longer runs go to
// the segmented fallback), never order.
template <int MAXP>
__global__ __launch_bounds__(1024) void k_scan_places(RunState *st, uint32_t n, int nplaces, uint32_t pfx_cap) {
    // four groups of 256 threads, one place each at a time
    constexpr int G = 4, PG = (MAXP + G - 1) / G;
    __shared__ uint32_t s_buf[G][RADIX];
    __shared__ uint32_t s_wsum[G][4];
    __shared__ int s_active[MAX_PLACES], s_triv[MAX_PLACES];
    __shared__ uint32_t s_pmax[MAX_PLACES];
    const int tid = threadIdx.x, g = tid >> 8, t = tid & (RADIX - 1);
    if (tid < MAX_PLACES) {
        s_pmax[tid] = 0;
        s_triv[tid] = 0;
    }
    // every copy of every place of this group in flight at once (one round
    // trip; the places a run does not have hold zeros), then cleared
    uint32_t cnt[PG];
    {
        uint32_t v[PG][HIST_REP];
#pragma unroll
        for (int k = 0; k < PG; ++k)
#pragma unroll
            for (int r = 0; r < HIST_REP; ++r) v[k][r] = g + G * k < MAXP ? st->hist[r][g + G * k][t] : 0u;
#pragma unroll
        for (int k = 0; k < PG; ++k) {
            cnt[k] = 0;
#pragma unroll
            for (int r = 0; r < HIST_REP; ++r) {
                cnt[k] += v[k][r];
                if (g + G * k < MAXP) st->hist[r][g + G * k][t] = 0;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PG; ++k) {
        const int p = g + G * k;
        const bool live = p < nplaces;
        const uint32_t c = live ? cnt[k] : 0u;
        if (live && c == n) s_triv[p] = 1;
        uint32_t m = c;   // the wave's largest count, then one LDS atomic
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, 64));
        if (live && (t & 63) == 0 && m) atomicMax(&s_pmax[p], m);
        s_buf[g][t] = c;
        __syncthreads();
        block_exscan<RADIX, RADIX>(s_buf[g], s_buf[g], s_wsum[g], t);
        if (live) st->base[p][t] = s_buf[g][t];
        __syncthreads();
    }
    if (tid < MAX_PLACES) s_active[tid] = tid < nplaces ? !s_triv[tid] : 0;
    __syncthreads();
    if (tid == 0) {
        int q = 0, top = -1;
        for (int p = 0; p < nplaces; ++p) {
            q += s_active[p];
            if (s_active[p]) top = p;
        }
        int lo = 0, qk = q;  // lowest place that keeps its pass; passes kept
        uint32_t kp = 0;
        if (pfx_cap > 0 && top >= 1) {
            for (int k = 2; k <= 4 && k <= top + 1; ++k) {
                double e = (double)n;
                for (int i = 0; i < k; ++i) e *= (double)s_pmax[top - i] / (double)n;
                if (e <= (double)pfx_cap) {
                    int qa = 0;
                    for (int p = top - k + 1; p <= top; ++p) qa += s_active[p];
                    if (qa + 2 <= q) {
                        kp = (uint32_t)k;
                        lo = top - k + 1;
                        qk = qa;
                    }
                    break;
                }
            }
        }
        int j = 0;
        for (int p = 0; p < MAX_PLACES; ++p) {
            PassDesc d;
            d.active = (p < nplaces && p >= lo) ? s_active[p] : 0;
            d.j = d.active ? j++ : -1;
            d.q = qk;
            d.shift = p * RADIX_BITS;
            st->desc[p] = d;
        }
        st->q = qk;
        st->pfx_active = kp != 0;
        st->pfx_places = kp;
        st->pfx_shift = lo * RADIX_BITS;
        st->pfx_mask = kp >= 4 ? 0xFFFFFFFFu : ((1u << (kp * RADIX_BITS)) - 1u);
    }
}

// ---------------------------------------------------------- histogram
// Histogram of code digits (learned sort) and of 128-bit keys: one read of
// the keys, counting the digit of every place in LDS counters shared by the
// workgroup, then one global atomic per nonzero bin.  The lanes of a wave
// that hold the first lane's digit add their count once instead of as
// conflicting LDS atomics on one address (all 64 for a constant high place
// of small keys, the frequent digit of a skewed place).
// Code digits use 1024-thread workgroups: the staged model table (64 KB at
// 4096 leaves) leaves room for two workgroups per CU.
template <int DT, bool CODE>
__global__ __launch_bounds__(CODE ? 1024 : 256) void k_hist(const typename KT<DT>::U *__restrict__ keys, uint32_t n,
                                                            int nplaces, RunState *st, const float *model, int cb,
                                                            int staged) {
    extern __shared__ float4 s_leaves[];
    using U = typename KT<DT>::U;
    constexpr int B = CODE ? 1024 : 256, ITEMS = 8;
    // code digits have at most 3 places (24 code bits); key digits one per
    // byte of the key
    constexpr int HP = CODE ? 4 : (int)sizeof(U);
    __shared__ uint32_t s_h[HP * RADIX];
    const int tid = threadIdx.x;
    for (int i = tid; i < HP * RADIX; i += B) s_h[i] = 0;
    RmiHead h;
    const RmiLeaf *leaves = nullptr;
    float scale = 0.f;
    if (CODE) {
        h = rmi_head(model);
        leaves = rmi_stage(model, staged ? s_leaves : nullptr);
        scale = (float)(1u << cb);
    }
    __syncthreads();
    const uint32_t stride = gridDim.x * B * ITEMS;
    for (uint32_t base = blockIdx.x * B * ITEMS; base < n; base += stride) {
        U v[ITEMS];
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const uint32_t i = base + it * B + tid;
            v[it] = i < n ? __builtin_nontemporal_load(keys + i) : U(0);
        }
        // model codes: one uniform branch per batch, so the staged table is
        // read with LDS instructions (not flat loads through a pointer that
        // may be LDS or global)
        U cv[ITEMS];
        if constexpr (CODE) {
            auto codes = [&](const RmiLeaf *lv) {
#pragma unroll
                for (int it = 0; it < ITEMS; ++it) cv[it] = (U)rmi_code(h, lv, KT<DT>::image(v[it]), cb, scale);
            };
            if (staged) codes(reinterpret_cast<const RmiLeaf *>(s_leaves));
            else codes(rmi_leaves(model));
        }
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const uint32_t i = base + it * B + tid;
            if (i >= n) break;
            const U t = CODE ? cv[it] : KT<DT>::image(v[it]);
            const uint64_t act = ballot64(true);
            // key digits: every place of the key, unrolled (constant shifts)
            constexpr int KP = (int)sizeof(U);
#pragma unroll
            for (int p = 0; p < (CODE ? HP : KP); ++p) {
                if (CODE && p >= nplaces) break;
                const uint32_t d = (uint32_t)(t >> (p * RADIX_BITS)) & (RADIX - 1);
                // the lanes that share the first lane's digit add once when
                // there are many of them (all lanes of a constant place, the
                // frequent digit of a skewed one); otherwise every lane adds
                // one (a single atomic instruction)
                const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
                const uint64_t m0 = ballot64(d == d0);
                if (__popcll(m0) > 8) {
                    if (count_below(act) == 0) atomicAdd(&s_h[p * RADIX + d0], (uint32_t)__popcll(m0));
                    if (d != d0) atomicAdd(&s_h[p * RADIX + d], 1u);
                } else {
                    atomicAdd(&s_h[p * RADIX + d], 1u);
                }
            }
        }
    }
    __syncthreads();
    uint32_t(*gh)[RADIX] = st->hist[blockIdx.x % HIST_REP];
    for (int i = tid; i < nplaces * RADIX; i += B)
        if (s_h[i]) atomicAdd(&gh[i / RADIX][i % RADIX], s_h[i]);
}

// Histogram of the keys of 16-, 32- and 64-bit key types.  Every lane of a
// wave adds to its own copy of the counters (copy = lane % 32, 32 copies of
// every counter word), so the 32 lanes that one LDS cycle serves always hit
// 32 distinct banks, whatever their digits; shared counters make random
// digits collide in banks (about 3 conflict cycles per access measured on
// 2^28 float32 keys).  The copies hold 16-bit counts, bins d and d + 128 of
// a place in the two halves of one word (16 KB of LDS per digit place);
// they are folded into 32-bit registers often enough that no 16-bit count
// can wrap, and added to the global copies once per workgroup.  One
// workgroup of B threads per CU for 64-bit keys (128 KB), two for narrower
// keys; ITEMS keys per lane per batch.
// CODE: the digits of the model codes (at most 24 bits: three places, of
// which the first `nplaces` are counted), with the model's leaf table staged
// in dynamic LDS when `staged`.
template <int DT, int B, int ITEMS, bool CODE = false>
__global__ __launch_bounds__(B) void k_hist_lp(const typename KT<DT>::U *__restrict__ keys, uint32_t n,
                                               RunState *st, int nplaces = 0, const float *model = nullptr,
                                               int cb = 0, int staged = 0) {
    extern __shared__ float4 s_leaves[];
    using U = typename KT<DT>::U;
    constexpr int NP = CODE ? 3 : (int)sizeof(U);   // digit places
    constexpr int ROWS = NP * 128;       // counter words per copy
    constexpr int NR = (ROWS + B - 1) / B;
    // adds one 16-bit count takes per batch at most: two lanes of every wave
    // share a copy, ITEMS keys each
    constexpr int PER_BATCH = (B / 32) * ITEMS;
    constexpr int FOLD = 32768 / PER_BATCH;  // batches between folds
    static_assert(FOLD >= 1, "16-bit counts must not wrap");
    __shared__ uint32_t s_h[ROWS * 32];
    const int tid = threadIdx.x;
    const uint32_t copy = (uint32_t)tid & 31u;
    {
        uint4 *z = reinterpret_cast<uint4 *>(s_h);
        for (int i = tid; i < ROWS * 8; i += B) z[i] = make_uint4(0, 0, 0, 0);
    }
    uint32_t lo[NR], hi[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) lo[j] = hi[j] = 0;
    // every copy of a counter word summed into registers (and cleared when
    // more keys follow); lane r starts at copy r % 32, so a wave's 32 lanes
    // of one LDS cycle read 32 distinct banks
    auto fold = [&](bool clear) {
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            const int r = j * B + tid;
            if (r < ROWS) {
                uint32_t a = 0, b = 0;
#pragma unroll 8
                for (int k = 0; k < 32; ++k) {
                    const int idx = r * 32 + ((k + r) & 31);
                    const uint32_t v = s_h[idx];
                    a += v & 0xFFFFu;
                    b += v >> 16;
                    if (clear) s_h[idx] = 0;
                }
                lo[j] += a;
                hi[j] += b;
            }
        }
    };
    // the digits of four places held in one 32-bit word of the key image
    auto count4 = [&](uint32_t x, int p0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (p0 + q >= NP) break;
            const uint32_t w = (x >> (8 * q)) & 127u;
            const uint32_t half = (x >> (8 * q + 7)) & 1u;
            atomicAdd(&s_h[((p0 + q) * 128 + w) * 32 + copy], half * 0xFFFFu + 1u);
        }
    };
    auto count = [&](U v) {
        const U t = KT<DT>::image(v);
        count4((uint32_t)t, 0);
        if constexpr (NP > 4) count4((uint32_t)((uint64_t)t >> 32), 4);
    };
    RmiHead h{};
    float scale = 0.f;
    if constexpr (CODE) {
        h = rmi_head(model);
        rmi_stage(model, staged ? s_leaves : nullptr);
        scale = (float)(1u << cb);
    }
    // model codes of a batch: one uniform branch per batch, so the staged
    // table is read with LDS instructions
    auto codes = [&](const U (&v)[ITEMS], uint32_t (&c)[ITEMS]) {
        if constexpr (CODE) {
            auto run = [&](const RmiLeaf *lv) {
#pragma unroll
                for (int it = 0; it < ITEMS; ++it) c[it] = rmi_code(h, lv, KT<DT>::image(v[it]), cb, scale);
            };
            if (staged) run(reinterpret_cast<const RmiLeaf *>(s_leaves));
            else run(rmi_leaves(model));
        }
    };
    __syncthreads();
    const uint32_t per = (uint32_t)B * ITEMS;
    const uint32_t stride = gridDim.x * per;
    int batches = 0;
    for (uint32_t base = blockIdx.x * per; base < n; base += stride) {
        U v[ITEMS];
        const bool full = base + per <= n;
        if (full) {
#pragma unroll
            for (int it = 0; it < ITEMS; ++it) v[it] = __builtin_nontemporal_load(keys + base + it * B + tid);
        } else {
#pragma unroll
            for (int it = 0; it < ITEMS; ++it) {
                const uint32_t i = base + it * B + tid;
                v[it] = i < n ? __builtin_nontemporal_load(keys + i) : U(0);
            }
        }
        if constexpr (CODE) {
            uint32_t c[ITEMS];
            codes(v, c);
#pragma unroll
            for (int it = 0; it < ITEMS; ++it)
                if (full || base + it * B + tid < n) count4(c[it], 0);
        } else if (full) {
#pragma unroll
            for (int it = 0; it < ITEMS; ++it) count(v[it]);
        } else {
#pragma unroll
            for (int it = 0; it < ITEMS; ++it)
                if (base + it * B + tid < n) count(v[it]);
        }
        if (++batches == FOLD) {
            __syncthreads();
            fold(true);
            __syncthreads();
            batches = 0;
        }
    }
    __syncthreads();
    fold(false);
    uint32_t(*gh)[MAX_PLACES][RADIX] = st->hist;
    const int rep = blockIdx.x % HIST_REP;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int r = j * B + tid;
        // (code digits: only the places the run has; the others stay zero)
        if (r < ROWS && (!CODE || (r >> 7) < nplaces)) {
            const int p = r >> 7, w = r & 127;
            if (lo[j]) atomicAdd(&gh[rep][p][w], lo[j]);
            if (hi[j]) atomicAdd(&gh[rep][p][w + 128], hi[j]);
        }
    }
}

// ----------------------------------------------------- one-sweep pass
// One workgroup per tile of W*64*IPT keys, tiles taken in launch order from
// an atomic counter (so every tile's predecessors are already running).
// LDS: the per-wave 16-bit digit counters of the ranking phase share their
// bytes with the key staging buffer of the scatter phase.
// Sort mode with a second scratch buffer and an odd number q >= 3 of
// active passes: route the passes through both scratch buffers so the last
// one writes the caller's keys.
__device__ __forceinline__ bool odd_route(int q, const void *t1) { return t1 != nullptr && (q & 1) && q >= 3; }

// Keys whose model codes a code pass forms together (their table reads in
// flight at once; the persistent code passes run two waves per SIMD, too
// few to hide one read's latency behind another wave).
#ifndef AK_CODE_GROUP
#define AK_CODE_GROUP 2
#endif
constexpr int CODE_GROUP = AK_CODE_GROUP;

template <typename U, typename V, bool VAL, bool CODE, int W, int IPT>
struct OsSmem {
    static constexpr int TILE = W * 64 * IPT;
    static constexpr size_t KEYS =
        (size_t)TILE * sizeof(U) + (VAL ? (size_t)TILE * sizeof(V) : 0) + (CODE ? TILE : 0);
    static constexpr size_t CNT = (size_t)W * RADIX * 2;
    static constexpr size_t RAW = KEYS > CNT ? KEYS : CNT;
};

// Register budget: for 64-bit keys two workgroups per CU (W/2 waves per
// SIMD) for one-tile workgroups, one for the persistent ones (W/4); 32-bit
// keys use larger tiles that would spill under the tighter budget.
template <int DT, int MODE, int W, int IPT, bool CODE, bool PERS>
__global__ __launch_bounds__(W * 64) __attribute__((amdgpu_waves_per_eu(
    PERS ? W / 4 : (key_bits(DT) >= 64 ? W / 2 : 1)))) void k_onesweep(OnesweepArgs a) {
    using U = typename KT<DT>::U;
    using V = typename ModeT<MODE>::V;
    constexpr bool VAL = ModeT<MODE>::VAL;
    constexpr bool PAIRS = ModeT<MODE>::PAIRS;
    constexpr bool LOWMEM = MODE == M_LOWMEM;
    using SM = OsSmem<U, V, VAL, CODE, W, IPT>;
    constexpr int B = W * 64, TILE = B * IPT;
    constexpr int K = B / RADIX;  // threads per digit in the look-back
    static_assert(B >= RADIX && B % RADIX == 0, "block must cover the radix");
    const PassDesc pd = a.st->desc[a.place];
    if (!pd.active) return;

    __shared__ __align__(16) uint8_t s_raw[SM::RAW];
    __shared__ uint32_t s_tot[RADIX], s_start[RADIX], s_glob[RADIX];
    __shared__ uint32_t s_wsum[W];
    __shared__ uint32_t s_tile;
    uint16_t *s_cnt = reinterpret_cast<uint16_t *>(s_raw);
    U *s_keys = reinterpret_cast<U *>(s_raw);
    V *s_vals = reinterpret_cast<V *>(s_raw + (size_t)TILE * sizeof(U));
    uint8_t *s_dig = s_raw + (size_t)TILE * sizeof(U) + (VAL ? (size_t)TILE * sizeof(V) : 0);

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    extern __shared__ float4 s_leaves[];

    // buffers of this pass.  Sort (and the keys and payloads of a sort by
    // key) ping-pong between the caller's buffer and t0 (with t1 and an odd
    // number q >= 3 of passes: keys -> t0 -> t1 -> ... -> keys, so the last
    // pass writes the caller's buffer).  Sortperm reads the const keys first,
    // then t0/t1, and its indices end in the permutation after the last
    // pass; the low-memory sortperm moves only indices (same buffers) and
    // reads every key from the const array through them.
    const int j = pd.j, q = pd.q;
    const U *src;
    U *dst = nullptr;
    const V *vsrc = nullptr;
    V *vdst = nullptr;
    if (!VAL || PAIRS) {
        if (odd_route(q, a.t1)) {
            auto buf = [&](int i) { return (U *)((i == 0 || i == q) ? a.keys : ((i & 1) ? a.t0 : a.t1)); };
            src = buf(j);
            dst = buf(j + 1);
            if (PAIRS) {
                auto vb = [&](int i) { return (V *)((i == 0 || i == q) ? a.vals : ((i & 1) ? a.v0 : a.v1)); };
                vsrc = vb(j);
                vdst = vb(j + 1);
            }
        } else {
            src = (const U *)((j & 1) ? a.t0 : a.keys);
            dst = (U *)((j & 1) ? a.keys : a.t0);
            if (PAIRS) {
                vsrc = (const V *)((j & 1) ? a.v0 : a.vals);
                vdst = (V *)((j & 1) ? a.vals : a.v0);
            }
        }
    } else {
        if (LOWMEM) src = (const U *)a.keys;
        else {
            src = (const U *)(j == 0 ? a.keys : (((j - 1) & 1) ? a.t1 : a.t0));
            dst = (U *)((j & 1) ? a.t1 : a.t0);
        }
        auto vb = [&](int i) { return (V *)((((q - 1 - i) & 1) == 0) ? a.vals : a.v0); };
        vsrc = j == 0 ? nullptr : vb(j - 1);
        vdst = vb(j);
    }
    const bool last = (j == q - 1);
    const int shift = pd.shift;

    RmiHead h;
    const RmiLeaf *leaves = nullptr;
    float scale = 0.f;
    if (CODE) {
        h = rmi_head(a.model);
        leaves = rmi_stage(a.model, a.staged ? s_leaves : nullptr);
        scale = (float)(1u << a.cb);
    }
    // Tiles are claimed in order from the pass counter, so a tile's
    // predecessors are always held by running workgroups.  PERS = false: one
    // tile per workgroup (grid = tiles).  PERS (always for code digits, whose
    // persistent grid reuses the staged model table): each workgroup claims
    // its next tile and issues that tile's loads before it waits in the
    // look-back, so the HBM latency overlaps the wait.  A workgroup holds at
    // most two claims, the tile it works on and the next, so the smallest
    // unfinished tile always belongs to a workgroup that can finish it.
    const uint32_t ntiles = (a.n + TILE - 1) / TILE;
    auto load_tile = [&](uint32_t t, int w_, int lane_, U(&kk)[IPT], V(&vv)[IPT]) {
        const uint32_t tb = t * (uint32_t)TILE;
        const uint32_t tv = min((uint32_t)TILE, a.n - tb);
        if constexpr (LOWMEM) {
            // indices first (made in the first pass), then each index's key
#pragma unroll
            for (int jj = 0; jj < IPT; ++jj) {
                const uint32_t e = striped_elem<IPT>(w_, jj, lane_);
                vv[jj] = e >= tv ? 0u : (vsrc ? __builtin_nontemporal_load(vsrc + tb + e) : tb + e);
            }
#pragma unroll
            for (int jj = 0; jj < IPT; ++jj) {
                const uint32_t e = striped_elem<IPT>(w_, jj, lane_);
                kk[jj] = e < tv ? src[vv[jj]] : U(0);
            }
            return;
        }
        const U *sp = src + tb + w_ * 64 * IPT + lane_;
        if (tv == (uint32_t)TILE) {
#pragma unroll
            for (int jj = 0; jj < IPT; ++jj) kk[jj] = __builtin_nontemporal_load(sp + jj * 64);
        } else {
#pragma unroll
            for (int jj = 0; jj < IPT; ++jj) {
                const uint32_t e = striped_elem<IPT>(w_, jj, lane_);
                kk[jj] = e < tv ? __builtin_nontemporal_load(sp + jj * 64) : U(0);
            }
        }
        if (VAL) {
#pragma unroll
            for (int jj = 0; jj < IPT; ++jj) {
                const uint32_t e = striped_elem<IPT>(w_, jj, lane_);
                vv[jj] = e >= tv ? V(0) : (vsrc ? __builtin_nontemporal_load(vsrc + tb + e) : (V)(tb + e));
            }
        }
    };
    if (tid == 0) s_tile = atomicAdd(&a.st->tile_ctr[a.place], 1u);
    __syncthreads();
    uint32_t tile = s_tile;
    if (tile >= ntiles) return;
    U k[IPT];
    V v[IPT];
    load_tile(tile, w, lane, k, v);
    while (true) {
    // Per-thread indices are re-derived each iteration from an opaque copy
    // of the thread id: hoisted out of the loop they would stay live across
    // tiles and cost registers (occupancy).
    int tid = threadIdx.x;
    if (PERS) asm volatile("" : "+v"(tid));
    const int lane = tid & 63, w = tid >> 6;
    const uint32_t tbase = tile * (uint32_t)TILE;
    const uint32_t tvalid = min((uint32_t)TILE, a.n - tbase);
    uint32_t rd[IPT];  // digit, then rank | digit << 16
    if constexpr (CODE) {
        // one uniform branch: the staged table is read with LDS
        // instructions (a pointer that may be LDS or global would be read
        // with slower flat loads).  No per-key bounds test: the ranking
        // ignores the digits past the tile's end (keys there are zero, and
        // the clamped leaf index keeps their table reads in bounds), and a
        // test would become a branch around each key's table reads that
        // serialises their latency.
        auto code_digits = [&](const RmiLeaf *lv) {
            constexpr int G = IPT % CODE_GROUP == 0 ? CODE_GROUP : (IPT % 2 == 0 ? 2 : 1);
#pragma unroll
            for (int j0 = 0; j0 < IPT; j0 += G) {
                U t[G];
                uint32_t c[G];
#pragma unroll
                for (int g = 0; g < G; ++g) t[g] = KT<DT>::image(k[j0 + g]);
                rmi_code_group<G>(h, lv, t, a.cb, scale, c);
#pragma unroll
                for (int g = 0; g < G; ++g) rd[j0 + g] = (c[g] >> shift) & (RADIX - 1);
            }
        };
        if (a.staged) code_digits(reinterpret_cast<const RmiLeaf *>(s_leaves));
        else code_digits(rmi_leaves(a.model));
    } else {
#pragma unroll
        for (int jj = 0; jj < IPT; ++jj) {
            const uint32_t e = striped_elem<IPT>(w, jj, lane);
            const U t = KT<DT>::image(k[jj]);
            rd[jj] = e < tvalid ? (uint32_t)(t >> shift) & (RADIX - 1) : 0u;
        }
    }

    rank_match_packed<RADIX_BITS, W, IPT, uint16_t>(rd, tvalid, s_cnt, s_tot, tid);

    // publish this tile's digit counts first, so successors can look back
    // (the first tile of a group is inclusive within its group)
    uint64_t *lb = a.lookback + (size_t)tile * RADIX;
    const uint32_t epoch = a.st->epoch_base + (uint32_t)a.place;
    for (int d = tid; d < RADIX; d += B)
        lb_store(lb + d, lb_pack(epoch, tile % LB_GROUP == 0 ? LB_INC : LB_AGG, s_tot[d]));
    // the next claim (every thread read s_tile before rank_match's barriers;
    // block_exscan's barriers publish the new value)
    if (PERS && tid == 0) s_tile = atomicAdd(&a.st->tile_ctr[a.place], 1u);

    block_exscan<B, RADIX>(s_tot, s_start, s_wsum, tid);
    rank_finish_packed<RADIX_BITS, W, IPT, uint16_t>(rd, s_cnt, s_start, tid);

    uint32_t next = ntiles;
    U kn[IPT];
    V vn[IPT];
    if (PERS) {
        next = s_tile;
        if (next < ntiles) load_tile(next, w, lane, kn, vn);
    }

    // The keys are staged in LDS by their tile positions before the
    // look-back (the positions do not depend on it): that work then lies
    // between publishing this tile's counts and reading its predecessors'
    // (2^31-key learned sort: code passes 46.2 -> 44.2 ms; 2^30 lognormal
    // int64 keys 37.4 -> 36.1 ms).
    __syncthreads();  // counters are dead from here on: their bytes hold keys
#pragma unroll
    for (int jj = 0; jj < IPT; ++jj) {
        const uint32_t e = striped_elem<IPT>(w, jj, lane);
        if (e < tvalid) {
            const uint32_t r = rd[jj] & 0xFFFFu;
            s_keys[r] = k[jj];
            if (CODE) s_dig[r] = (uint8_t)(rd[jj] >> 16);
            if (VAL) s_vals[r] = v[jj];
        }
    }
    // two-level decoupled look-back (K*LB_M words per round trip): inside
    // the tile's group, then over the words of the groups before it
    {
        const int d = tid / K, kk = tid % K;
        const uint32_t g = tile / LB_GROUP, jl = tile % LB_GROUP;
        uint64_t *lbg = a.lookback + (size_t)ntiles * RADIX;
        uint32_t lexcl = 0, gexcl = 0;
        if (jl > 0) {
            // stops at the group's first tile at the latest (inclusive word)
            lexcl = lookback_prefix<K, LB_M>(a.lookback + d, (int64_t)tile - 1, epoch, kk);
            if (kk == 0) lb_store(lb + d, lb_pack(epoch, LB_INC, lexcl + s_tot[d]));
        }
        const bool glast = jl == LB_GROUP - 1;
        if (glast && kk == 0)
            lb_store(lbg + (size_t)g * RADIX + d, lb_pack(epoch, g == 0 ? LB_INC : LB_AGG, lexcl + s_tot[d]));
        if (g > 0) {
            gexcl = lookback_prefix<K, LB_M>(lbg + d, (int64_t)g - 1, epoch, kk);
            if (glast && kk == 0)
                lb_store(lbg + (size_t)g * RADIX + d, lb_pack(epoch, LB_INC, gexcl + lexcl + s_tot[d]));
        }
        if (kk == 0) s_glob[d] = a.st->base[a.place][d] + gexcl + lexcl - s_start[d];
    }
    __syncthreads();

    // coalesced scatter: consecutive threads write consecutive slots of a
    // digit's run
#pragma unroll
    for (int jj = 0; jj < IPT; ++jj) {
        const uint32_t i = (uint32_t)(jj * B + tid);
        if (i < tvalid) {
            const U key = s_keys[i];
            const uint32_t d = CODE ? (uint32_t)s_dig[i] : (uint32_t)(KT<DT>::image(key) >> shift) & (RADIX - 1);
            const uint32_t pos = s_glob[d] + i;
            // sortperm: keys are not needed after the last pass; the
            // low-memory sortperm never writes keys
            if (!LOWMEM && (MODE != M_PERM || !last)) __builtin_nontemporal_store(key, dst + pos);
            if (VAL) __builtin_nontemporal_store(s_vals[i], vdst + pos);
        }
    }
    if (!PERS || next >= ntiles) break;
    __syncthreads();  // the tile's LDS is reused by the next one
    tile = next;
#pragma unroll
    for (int jj = 0; jj < IPT; ++jj) {
        k[jj] = kn[jj];
        if (VAL) v[jj] = vn[jj];
    }
    }
}

// ------------------------------------------- reduce-then-scan passes
// The same stable digit pass without any waiting between workgroups: a
// read-only kernel counts every chunk's digits, a scan turns the counts
// into each chunk's output offset per digit (global digit offset plus the
// counts of the chunks before it), and the scatter kernel walks its chunk's
// tiles in order, carrying the running offsets in LDS.  One more read of
// the keys per pass than the one-sweep pass, no look-back.

// Source and destination of pass pd (the one-sweep pass's routing).
template <typename U, bool VAL>
__device__ __forceinline__ void pass_route(const OnesweepArgs &a, const PassDesc &pd, const U *&src, U *&dst,
                                           const uint32_t *&vsrc, uint32_t *&vdst) {
    const int j = pd.j, q = pd.q;
    vsrc = nullptr;
    vdst = nullptr;
    if (!VAL) {
        if (odd_route(q, a.t1)) {
            auto buf = [&](int i) { return (U *)((i == 0 || i == q) ? a.keys : ((i & 1) ? a.t0 : a.t1)); };
            src = buf(j);
            dst = buf(j + 1);
        } else {
            src = (const U *)((j & 1) ? a.t0 : a.keys);
            dst = (U *)((j & 1) ? a.keys : a.t0);
        }
    } else {
        src = (const U *)(j == 0 ? a.keys : (((j - 1) & 1) ? a.t1 : a.t0));
        dst = (U *)((j & 1) ? a.t1 : a.t0);
        auto vb = [&](int i) { return (uint32_t *)((((q - 1 - i) & 1) == 0) ? a.vals : a.v0); };
        vsrc = j == 0 ? nullptr : vb(j - 1);
        vdst = vb(j);
    }
}

// Digit counts of chunk blockIdx.x (TILE * chunk_tiles keys) at this place.
template <int DT, bool VAL, bool CODE, int TILE>
__global__ __launch_bounds__(256) void k_rts_count(OnesweepArgs a) {
    using U = typename KT<DT>::U;
    constexpr int B = 256;
    const PassDesc pd = a.st->desc[a.place];
    if (!pd.active) return;
    __shared__ uint32_t s_h[RADIX];
    extern __shared__ float4 s_leaves[];
    const int tid = threadIdx.x;
    s_h[tid] = 0;
    RmiHead h;
    const RmiLeaf *leaves = nullptr;
    float scale = 0.f;
    if (CODE) {
        h = rmi_head(a.model);
        leaves = rmi_stage(a.model, a.staged ? s_leaves : nullptr);
        scale = (float)(1u << a.cb);
    }
    const U *src;
    U *dst;
    const uint32_t *vsrc;
    uint32_t *vdst;
    pass_route<U, VAL>(a, pd, src, dst, vsrc, vdst);
    const int shift = pd.shift;
    __syncthreads();
    const uint32_t c = blockIdx.x;
    const uint32_t lo = c * a.chunk_tiles * (uint32_t)TILE;
    const uint32_t hi = min(a.n, lo + a.chunk_tiles * (uint32_t)TILE);
    constexpr int ITEMS = 8;
    for (uint32_t base = lo; base < hi; base += B * ITEMS) {
        U v[ITEMS];
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const uint32_t i = base + it * B + tid;
            v[it] = i < hi ? __builtin_nontemporal_load(src + i) : U(0);
        }
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const uint32_t i = base + it * B + tid;
            if (i >= hi) break;
            U t = KT<DT>::image(v[it]);
            if constexpr (CODE) t = (U)rmi_code(h, leaves, t, a.cb, scale);
            const uint32_t d = (uint32_t)(t >> shift) & (RADIX - 1);
            const uint64_t act = ballot64(true);
            const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
            if (ballot64(d == d0) == act) {
                if (count_below(act) == 0) atomicAdd(&s_h[d0], (uint32_t)__popcll(act));
            } else {
                atomicAdd(&s_h[d], 1u);
            }
        }
    }
    __syncthreads();
    a.ccnt[(size_t)tid * a.nchunks + c] = s_h[tid];
}

// Per digit (one workgroup each): exclusive scan of the chunk counts plus
// the digit's global offset, in place.
static __global__ __launch_bounds__(1024) void k_rts_scan(OnesweepArgs a) {
    const PassDesc pd = a.st->desc[a.place];
    if (!pd.active) return;
    __shared__ uint32_t s_wsum[16];
    __shared__ uint32_t s_carry;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int d = blockIdx.x;
    uint32_t *row = a.ccnt + (size_t)d * a.nchunks;
    if (tid == 0) s_carry = a.st->base[a.place][d];
    __syncthreads();
    for (uint32_t b0 = 0; b0 < a.nchunks; b0 += 1024) {
        const uint32_t i = b0 + tid;
        const uint32_t v = i < a.nchunks ? row[i] : 0u;
        const uint32_t incl = wave_incl_scan(v);
        if (lane == 63) s_wsum[w] = incl;
        __syncthreads();
        uint32_t run = s_carry;
        for (int ww = 0; ww < w; ++ww) run += s_wsum[ww];
        if (i < a.nchunks) row[i] = run + incl - v;
        __syncthreads();
        if (tid == 1023) s_carry = run + incl;
        __syncthreads();
    }
}

// Scatter of chunk blockIdx.x: its tiles in order, each ranked stably on
// chip and written to the chunk's running digit offsets.
template <int DT, bool VAL, int W, int IPT, bool CODE>
__global__ __launch_bounds__(W * 64) __attribute__((amdgpu_waves_per_eu(
    CODE ? W / 4 : (key_bits(DT) == 64 ? W / 2 : 1)))) void k_rts_scatter(OnesweepArgs a) {
    using U = typename KT<DT>::U;
    using SM = OsSmem<U, uint32_t, VAL, CODE, W, IPT>;
    constexpr int B = W * 64, TILE = B * IPT;
    const PassDesc pd = a.st->desc[a.place];
    if (!pd.active) return;
    __shared__ __align__(16) uint8_t s_raw[SM::RAW];
    __shared__ uint32_t s_tot[RADIX], s_start[RADIX], s_glob[RADIX], s_run[RADIX];
    __shared__ uint32_t s_wsum[W];
    uint16_t *s_cnt = reinterpret_cast<uint16_t *>(s_raw);
    U *s_keys = reinterpret_cast<U *>(s_raw);
    uint32_t *s_vals = reinterpret_cast<uint32_t *>(s_raw + (size_t)TILE * sizeof(U));
    uint8_t *s_dig = s_raw + (size_t)TILE * sizeof(U) + (VAL ? (size_t)TILE * 4 : 0);
    extern __shared__ float4 s_leaves[];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const U *src;
    U *dst;
    const uint32_t *vsrc;
    uint32_t *vdst;
    pass_route<U, VAL>(a, pd, src, dst, vsrc, vdst);
    const bool last = pd.j == pd.q - 1;
    const int shift = pd.shift;
    RmiHead h;
    const RmiLeaf *leaves = nullptr;
    float scale = 0.f;
    if (CODE) {
        h = rmi_head(a.model);
        leaves = rmi_stage(a.model, a.staged ? s_leaves : nullptr);
        scale = (float)(1u << a.cb);
    }
    const uint32_t c = blockIdx.x;
    for (int d = tid; d < RADIX; d += B) s_run[d] = a.ccnt[(size_t)d * a.nchunks + c];
    const uint32_t t0 = c * a.chunk_tiles;
    const uint32_t t1 = min((a.n + TILE - 1) / TILE, t0 + a.chunk_tiles);
    // tile t's keys (and values) in registers, striped; the next tile's are
    // loaded before tile t is ranked, so their latency overlaps the work
    auto load_tile = [&](uint32_t t, int w_, int lane_, U(&kk)[IPT], uint32_t(&vv)[IPT]) {
        const uint32_t tb = t * (uint32_t)TILE;
        const uint32_t tv = min((uint32_t)TILE, a.n - tb);
        const U *sp = src + tb + w_ * 64 * IPT + lane_;
#pragma unroll
        for (int jj = 0; jj < IPT; ++jj) {
            const uint32_t e = striped_elem<IPT>(w_, jj, lane_);
            kk[jj] = e < tv ? __builtin_nontemporal_load(sp + jj * 64) : U(0);
            if (VAL) vv[jj] = e >= tv ? 0u : (vsrc ? __builtin_nontemporal_load(vsrc + tb + e) : tb + e);
        }
    };
    U k[IPT];
    uint32_t v[IPT];
    if (t0 < t1) load_tile(t0, w, lane, k, v);
    for (uint32_t tile = t0; tile < t1; ++tile) {
        // per-thread indices re-derived each tile from an opaque copy of the
        // thread id (hoisted out of the loop they would be spilled)
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int lane = tid & 63, w = tid >> 6;
        const uint32_t tbase = tile * (uint32_t)TILE;
        const uint32_t tvalid = min((uint32_t)TILE, a.n - tbase);
        U kn[IPT];
        uint32_t vn[IPT], rd[IPT];
        if (tile + 1 < t1) load_tile(tile + 1, w, lane, kn, vn);
#pragma unroll
        for (int jj = 0; jj < IPT; ++jj) {
            const uint32_t e = striped_elem<IPT>(w, jj, lane);
            U t = KT<DT>::image(k[jj]);
            if constexpr (CODE) t = (U)rmi_code(h, leaves, t, a.cb, scale);
            rd[jj] = e < tvalid ? (uint32_t)(t >> shift) & (RADIX - 1) : 0u;
        }
        rank_match_packed<RADIX_BITS, W, IPT, uint16_t>(rd, tvalid, s_cnt, s_tot, tid);
        block_exscan<B, RADIX>(s_tot, s_start, s_wsum, tid);
        rank_finish_packed<RADIX_BITS, W, IPT, uint16_t>(rd, s_cnt, s_start, tid);
        for (int d = tid; d < RADIX; d += B) {
            s_glob[d] = s_run[d] - s_start[d];
            s_run[d] += s_tot[d];
        }
        __syncthreads();  // counters are dead from here on: their bytes hold keys
#pragma unroll
        for (int jj = 0; jj < IPT; ++jj) {
            const uint32_t e = striped_elem<IPT>(w, jj, lane);
            if (e < tvalid) {
                const uint32_t r = rd[jj] & 0xFFFFu;
                s_keys[r] = k[jj];
                if (CODE) s_dig[r] = (uint8_t)(rd[jj] >> 16);
                if (VAL) s_vals[r] = v[jj];
            }
        }
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < IPT; ++jj) {
            const uint32_t i = (uint32_t)(jj * B + tid);
            if (i < tvalid) {
                const U key = s_keys[i];
                const uint32_t d = CODE ? (uint32_t)s_dig[i] : (uint32_t)(KT<DT>::image(key) >> shift) & (RADIX - 1);
                const uint32_t pos = s_glob[d] + i;
                if (!VAL || !last) __builtin_nontemporal_store(key, dst + pos);
                if (VAL) __builtin_nontemporal_store(s_vals[i], vdst + pos);
            }
        }
        __syncthreads();  // the tile's LDS is reused by the next one
#pragma unroll
        for (int jj = 0; jj < IPT; ++jj) {
            k[jj] = kn[jj];
            if (VAL) v[jj] = vn[jj];
        }
    }
}

// ---------------------------------------------------------- finalize
// After the passes.  Sort and sort by key: a single active pass (or an odd
// number without the second scratch buffers) leaves the keys in t0 and the
// payloads in v0, which are copied back.  Sortperm (both kinds): with no
// active pass (all keys equal) the permutation is the identity.
template <typename U, int MODE>
__global__ __launch_bounds__(256) void k_finalize(const RunState *st, OnesweepArgs a) {
    using V = typename ModeT<MODE>::V;
    const int q = st->q;
    const uint32_t n = a.n, stride = gridDim.x * blockDim.x;
    const uint32_t i0 = blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (MODE == M_KEYS || ModeT<MODE>::PAIRS) {
        if ((q & 1) == 0 || odd_route(q, a.t1)) return;
        for (uint32_t i = i0; i < n; i += stride) {
            __builtin_nontemporal_store(__builtin_nontemporal_load((const U *)a.t0 + i), (U *)a.keys + i);
            if (ModeT<MODE>::PAIRS)
                __builtin_nontemporal_store(__builtin_nontemporal_load((const V *)a.v0 + i), (V *)a.vals + i);
        }
    } else {
        if (q != 0) return;
        for (uint32_t i = i0; i < n; i += stride) ((uint32_t *)a.vals)[i] = i;
    }
}

// One workgroup sorts up to W*64*IPT keys on chip in one launch: keys in
// place, or the permutation into vals, or keys and payloads in place.
template <int DT, int MODE, int W, int IPT>
__global__ __launch_bounds__(W * 64) void k_small_sort(typename KT<DT>::U *keys, void *vals, uint32_t n) {
    using U = typename KT<DT>::U;
    constexpr bool VAL = ModeT<MODE>::VAL;
    __shared__ SmallSmem<U, VAL, W, IPT> sm;
    if constexpr (MODE == M_KEYS) lds_sort_tile_top<DT, W, IPT>(keys, keys, n, sm, threadIdx.x);
    else if constexpr (ModeT<MODE>::PAIRS)
        lds_sort_pairs<DT, typename ModeT<MODE>::V, W, IPT>(keys, (typename ModeT<MODE>::V *)vals, n, sm, threadIdx.x);
    else lds_sort_tile<DT, true, W, IPT>(keys, nullptr, (uint32_t *)vals, n, sm, threadIdx.x);
}


// ------------------------------------------------------- launch sequence
template <int DT, bool VAL, bool CODE, int V>
static void launch_rts_v(hipStream_t s, uint32_t tiles, OnesweepArgs a, size_t stage) {
    constexpr OsShape sh = CODE ? OS_CODE_SHAPES[key_bits(DT) == 64][V] : OS_SHAPES[key_class(DT)][VAL ? 1 : 0][V];
    constexpr int TILE = sh.w * 64 * sh.ipt;
    a.chunk_tiles = rts_chunk_tiles(tiles);
    a.nchunks = (tiles + a.chunk_tiles - 1) / a.chunk_tiles;
    hipLaunchKernelGGL((k_rts_count<DT, VAL, CODE, TILE>), dim3(a.nchunks), dim3(256), stage, s, a);
    hipLaunchKernelGGL(k_rts_scan, dim3(RADIX), dim3(1024), 0, s, a);
    hipLaunchKernelGGL((k_rts_scatter<DT, VAL, sh.w, sh.ipt, CODE>), dim3(a.nchunks), dim3(sh.w * 64), stage, s, a);
}

template <int DT, int MODE, bool CODE, int V>
static void launch_pass_v(hipStream_t s, uint32_t tiles, const OnesweepArgs &a, size_t stage) {
    if constexpr (MODE <= M_PERM) {
        if (os_rts()) {
            launch_rts_v<DT, MODE == M_PERM, CODE, V>(s, tiles, a, stage);
            return;
        }
    }
    constexpr OsShape sh =
        CODE ? OS_CODE_SHAPES[key_bits(DT) == 64][V] : OS_SHAPES[key_class(DT)][ModeT<MODE>::VCLASS][V];
    // code digits: persistent grid (the staged table leaves room for one
    // workgroup per CU); key digits: a persistent grid of at most two
    // workgroups per CU (the shapes' LDS admits one or two), or one
    // workgroup per tile
    if constexpr (CODE) {
        const uint32_t grid = std::min<uint32_t>(tiles, (uint32_t)num_cus() * (stage ? 1 : 2));
        hipLaunchKernelGGL((k_onesweep<DT, MODE, sh.w, sh.ipt, true, true>), dim3(grid), dim3(sh.w * 64), stage, s,
                           a);
    } else if constexpr (sh.pers) {
        const uint32_t grid = std::min<uint32_t>(tiles, (uint32_t)num_cus() * 2);
        hipLaunchKernelGGL((k_onesweep<DT, MODE, sh.w, sh.ipt, false, true>), dim3(grid), dim3(sh.w * 64), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_onesweep<DT, MODE, sh.w, sh.ipt, false, false>), dim3(tiles), dim3(sh.w * 64), 0, s,
                           a);
    }
}

static inline const char *pass_name(int mode, bool code) {
    if (code) return "onesweep_code_pass";
    switch (mode) {
    case M_PERM: return "onesweep_pair_pass";
    case M_PAIRS4:
    case M_PAIRS8: return "onesweep_kv_pass";
    case M_LOWMEM: return "onesweep_lowmem_pass";
    }
    return "onesweep_pass";
}

template <int DT, int MODE, bool CODE>
static ak_status launch_passes(hipStream_t stream, Workspace *ws, OnesweepArgs a, int nplaces, size_t stage) {
    static_assert(!CODE || MODE == M_KEYS, "code digits order keys only");
    const int var = CODE ? os_code_variant(DT) : os_variant(DT, MODE, a.n);
    const int TILE = CODE ? os_code_tile(DT) : os_tile(DT, MODE, a.n);
    const uint32_t tiles = (a.n + TILE - 1) / TILE;
    constexpr int DEF = OS_DEFAULT[key_class(DT)][ModeT<MODE>::VCLASS];
    for (int p = 0; p < nplaces; ++p) {
        a.place = p;
        ProfScope ps(pass_name(MODE, CODE), stream);
        if constexpr (CODE || os_all_variants(DT, MODE)) {
            switch (var) {
            case 0: launch_pass_v<DT, MODE, CODE, 0>(stream, tiles, a, stage); break;
            case 1: launch_pass_v<DT, MODE, CODE, 1>(stream, tiles, a, stage); break;
            case 2: launch_pass_v<DT, MODE, CODE, 2>(stream, tiles, a, stage); break;
            default: launch_pass_v<DT, MODE, CODE, 3>(stream, tiles, a, stage); break;
            }
        } else if constexpr (MODE == M_KEYS) {
            // the small-input shape (variant 0) and the default
            if (var == 0) launch_pass_v<DT, MODE, false, 0>(stream, tiles, a, stage);
            else launch_pass_v<DT, MODE, false, DEF>(stream, tiles, a, stage);
        } else {
            launch_pass_v<DT, MODE, false, DEF>(stream, tiles, a, stage);
        }
        AK_LAUNCH_CHECK("k_onesweep");
    }
    return AK_OK;
}

// The whole multi-workgroup run: init (epochs, counters), histogram, digit
// scan, one pass per place (inactive ones exit at once), and the device-
// decided copy-back / identity.  `vals`
// is the permutation output (sortperm), the payload (sort by key) or null.
template <int DT, int MODE, bool CODE>
static ak_status launch_run(hipStream_t s, Workspace *ws, RunState *st, void *keys, void *vals, uint32_t n,
                            int nplaces, const float *model, int cb, size_t stage = 0, uint32_t pfx_cap = 0) {
    using U = typename KT<DT>::U;
    hipLaunchKernelGGL(k_run_init, dim3(1), dim3(256), 0, s, st, ws->epoch_dev);
    AK_LAUNCH_CHECK("k_run_init");
    {
        ProfScope ps(CODE ? "code_hist" : "digit_hist", s);
        // the lane-private histogram for 16- to 64-bit key digits (shape
        // $AK_HIST_VARIANT 0..2; 3: the shared-counter kernel)
        const int hv = hist_variant();
        bool done = false;
        if constexpr (!CODE && key_bits(DT) <= 64) {
            if (hv < 3) {
                done = true;
                constexpr int NP = (int)sizeof(U);
                auto launch = [&](auto bc, auto ic) {
                    constexpr int B = decltype(bc)::value, IT = decltype(ic)::value;
                    // workgroups per CU: 160 KB of LDS, 2048 threads
                    const int per_cu = std::min(160 / (NP * 16), 2048 / B);
                    const uint32_t grid = (uint32_t)std::min<int64_t>(((int64_t)n + B * IT - 1) / (B * IT),
                                                                      (int64_t)num_cus() * per_cu);
                    hipLaunchKernelGGL((k_hist_lp<DT, B, IT>), dim3(grid), dim3(B), 0, s, (const U *)keys, n, st);
                };
                if (hv == 0) launch(std::integral_constant<int, 1024>{}, std::integral_constant<int, 8>{});
                else if (hv == 1) launch(std::integral_constant<int, 1024>{}, std::integral_constant<int, 16>{});
                else launch(std::integral_constant<int, 512>{}, std::integral_constant<int, 16>{});
                AK_LAUNCH_CHECK("k_hist_lp");
            }
        }
        // code digits: the lane-private kernel next to the staged table (one
        // workgroup per CU: 48 KB of counters, up to 64 KB of table)
        if constexpr (CODE) {
            if (hv < 3 && nplaces <= 3) {
                done = true;
                constexpr int B = 1024, IT = 8;
                const uint32_t grid =
                    (uint32_t)std::min<int64_t>(((int64_t)n + B * IT - 1) / (B * IT), (int64_t)num_cus());
                hipLaunchKernelGGL((k_hist_lp<DT, B, IT, true>), dim3(grid), dim3(B), stage, s, (const U *)keys, n,
                                   st, nplaces, model, cb, (int)(stage > 0));
                AK_LAUNCH_CHECK("k_hist_lp");
            }
        }
        if (!done) {
            constexpr int HB = CODE ? 1024 : 256;
            const uint32_t hgrid = (uint32_t)std::min<int64_t>(((int64_t)n + HB * 8 - 1) / (HB * 8),
                                                               (int64_t)num_cus() * (CODE ? 2 : 8));
            hipLaunchKernelGGL((k_hist<DT, CODE>), dim3(hgrid), dim3(HB), stage, s, (const U *)keys, n, nplaces,
                               st, model, cb, (int)(stage > 0));
            AK_LAUNCH_CHECK("k_hist");
        }
    }
    constexpr int HP = CODE ? 4 : (int)sizeof(U);
    hipLaunchKernelGGL((k_scan_places<HP>), dim3(1), dim3(1024), 0, s, st, n, nplaces, pfx_cap);
    AK_LAUNCH_CHECK("k_scan_places");
    OnesweepArgs a{};
    a.keys = keys;
    a.t0 = ws->keys0;
    a.t1 = ws->keys1;
    a.v0 = ws->vals0;
    a.v1 = ws->vals1;
    a.vals = vals;
    a.lookback = ws->lookback;
    a.ccnt = (uint32_t *)ws->aux[4];
    a.st = st;
    a.n = n;
    a.model = model;
    a.cb = cb;
    a.staged = stage > 0;
    ak_status r = launch_passes<DT, MODE, CODE>(s, ws, a, nplaces, stage);
    if (r != AK_OK) return r;
    const uint32_t fgrid = (uint32_t)std::min<int64_t>(((int64_t)n + 1023) / 1024, (int64_t)num_cus() * 8);
    hipLaunchKernelGGL((k_finalize<U, MODE>), dim3(fgrid), dim3(256), 0, s, (const RunState *)st, a);
    AK_LAUNCH_CHECK("k_finalize");
    return AK_OK;
}

// --------------------------------------------------------------- driver
constexpr int SMALL_W = 4, SMALL_IPT = 16;
// Key-only runs above this size may take the prefix-partitioned finish.
constexpr int64_t PREFIX_MIN = int64_t(1) << 16;
// Runs of up to GRAPH_MAX keys are latency-bound (about p+3 launches of a
// few microseconds of work each), so their launch sequence is captured once
// per (dtype, mode, n, pointers, workspace generation) and replayed.
// Epochs come from the device counter, so replays never meet stale words.
constexpr int64_t GRAPH_MAX = int64_t(1) << 22;

struct GraphKey {
    int dt, mode, slot;
    uint32_t n;
    const void *keys;
    const void *vals;
    uint32_t gen;
    bool operator<(const GraphKey &o) const {
        if (dt != o.dt) return dt < o.dt;
        if (mode != o.mode) return mode < o.mode;
        if (slot != o.slot) return slot < o.slot;
        if (n != o.n) return n < o.n;
        if (keys != o.keys) return keys < o.keys;
        if (vals != o.vals) return vals < o.vals;
        return gen < o.gen;
    }
};
// Replays the cached graph of `key` on the workspace's stream, recording it
// first with `record` (on a capture stream) if there is none.
ak_status graph_run(Workspace *ws, const GraphKey &key, const std::function<ak_status(hipStream_t)> &record);

// The key types whose key-only runs may take the prefix-partitioned finish
// (its chunk sort handles 32- and 64-bit keys).
constexpr bool prefix_dtype(int dt) { return dt >= AK_I32 && dt <= AK_F64; }

static inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }
// Bytes of the chunk counts of a reduce-then-scan pass over `tiles` tiles
// (at most one chunk per tile).
static inline size_t rts_bytes(size_t tiles) { return tiles * RADIX * 4; }

template <int DT, int MODE>
static ak_status radix_sort_t(Workspace *ws, void *keys, void *vals, int64_t n64, int slot) {
    using U = typename KT<DT>::U;
    using V = typename ModeT<MODE>::V;
    hipStream_t s = ws->stream;
    const uint32_t n = (uint32_t)n64;
    if (n64 <= small_sort_capacity(DT)) {
        hipLaunchKernelGGL((k_small_sort<DT, MODE, SMALL_W, SMALL_IPT>), dim3(1), dim3(SMALL_W * 64), 0, s, (U *)keys,
                           vals, n);
        AK_LAUNCH_CHECK("k_small_sort");
        return AK_OK;
    }
    const size_t kb = sizeof(U);
    ak_status r;
    if (MODE != M_LOWMEM) {
        if ((r = ws_reserve(ws, &ws->keys0, &ws->keys0_bytes, (size_t)n * kb)) != AK_OK) return r;
        if ((r = ws_reserve(ws, &ws->keys1, &ws->keys1_bytes, (size_t)n * kb)) != AK_OK) return r;
    }
    if (ModeT<MODE>::VAL && (r = ws_reserve(ws, &ws->vals0, &ws->vals0_bytes, (size_t)n * sizeof(V))) != AK_OK)
        return r;
    if (ModeT<MODE>::PAIRS && (r = ws_reserve(ws, &ws->vals1, &ws->vals1_bytes, (size_t)n * sizeof(V))) != AK_OK)
        return r;
    const int TILE = os_tile(DT, MODE, n64);
    const size_t tiles = (n + TILE - 1) / TILE;
    if ((r = ws_reserve_lookback(ws, lookback_words(tiles) * 8)) != AK_OK) return r;
    if ((r = ws_reserve(ws, &ws->aux[4], &ws->aux_bytes[4], rts_bytes(tiles))) != AK_OK) return r;
    // key-only runs may finish on chip once their top places are placed
    // (decided on the device from the digit counts; plain passes otherwise).
    // Small runs finish with fixed launches only (captured with the rest);
    // larger ones hand long runs to the segmented sort, which captures its
    // own launch graph, so they cannot be recorded into a caller's graph.
    const bool small = n64 <= GRAPH_MAX;
    const bool pfx = MODE == M_KEYS && prefix_dtype(DT) && n64 > PREFIX_MIN && (small || !stream_capturing(s));
    if (pfx && (r = prefix_reserve(ws, DT, n64)) != AK_OK) return r;
    if (slot == 0) ws->last_route = pfx ? 2 : 1;
    uint32_t epoch;
    if ((r = ws_next_epoch(ws, &epoch)) != AK_OK) return r;
    RunState *st = ws->state + slot;
    const int nplaces = (int)sizeof(U);
    const uint32_t pfx_cap = pfx ? (uint32_t)(prefix_chunk_keys() / 4) : 0u;
    auto run = [&](hipStream_t cs) -> ak_status {
        ak_status rr = launch_run<DT, MODE, false>(cs, ws, st, keys, vals, n, nplaces, nullptr, 0, 0, pfx_cap);
        if (rr != AK_OK || !pfx) return rr;
        return prefix_finish(ws, cs, DT, keys, n64, st, small);
    };
    if (!small || ws->no_graph || stream_capturing(s)) return run(s);
    return graph_run(ws, GraphKey{DT, MODE, slot, n, keys, vals, ws->gen}, run);
}

}  // namespace ak
