// Block-level building blocks of the radix kernels: exclusive scans and the
// stable in-tile digit ranking (wave ballot match + per-wave LDS counters).
#pragma once

#include "ak_internal.h"

namespace ak {

// Barrier of a cooperating group of W waves.  A group of one wave (several
// independent single-wave groups share a block) only needs its own LDS
// accesses ordered: a wavefront fence and a wave barrier.
template <int W>
__device__ __forceinline__ void grp_sync() {
    if constexpr (W == 1) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Exclusive scan of R counters held in LDS (`in`, may alias `out`) by the B
// threads of a group (tid = thread index within the group).  s_wsum needs
// B/64 words.  Ends with a group barrier.
template <int B, int R>
__device__ __forceinline__ void block_exscan(const uint32_t *in, uint32_t *out, uint32_t *s_wsum, int tid) {
    constexpr int K = (R + B - 1) / B;
    constexpr int W = B / 64;
    const int lane = tid & 63, w = tid >> 6;
    uint32_t v[K];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int idx = tid * K + k;
        v[k] = idx < R ? in[idx] : 0u;
        sum += v[k];
    }
    const uint32_t incl = wave_incl_scan(sum);
    if (lane == 63) s_wsum[w] = incl;
    grp_sync<W>();
    uint32_t run = incl - sum;
    for (int ww = 0; ww < w; ++ww) run += s_wsum[ww];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int idx = tid * K + k;
        if (idx < R) out[idx] = run;
        run += v[k];
    }
    grp_sync<W>();
}

// Tile layout used by every ranking kernel: "wave-striped".  Item j of lane
// l in wave w is tile element w*64*IPT + j*64 + l, so each item is one
// coalesced 64-lane access and processing items j = 0..IPT-1 in order walks
// the wave's elements in input order (which makes the ranking stable).
template <int IPT>
__device__ __forceinline__ uint32_t striped_elem(int w, int j, int lane) {
    return (uint32_t)(w * 64 * IPT + j * 64 + lane);
}

// Phase 1 of the stable ranking.  For every valid item, finds the lanes of
// its wave holding the same digit (RB ballots), and gives the item its rank
// among equal digits of earlier items of the wave.  Per-wave digit counters
// live in s_cnt[w*R + d]; afterwards (and a barrier) s_cnt holds, per
// digit, the exclusive prefix over waves and s_tot the tile's digit totals.
// Each item's digit and rank share one register (rd[j] = rank | digit <<
// 16; ranks stay below 2^16), which saves IPT registers per lane: on input
// rd[j] holds the digit, afterwards the wave-local rank and the digit.
template <int RB, int W, int IPT, typename C = uint32_t>
__device__ __forceinline__ void rank_match_packed(uint32_t (&rd)[IPT], uint32_t nvalid, C *s_cnt, uint32_t *s_tot,
                                                  int tid) {
    constexpr int R = 1 << RB;
    constexpr int B = W * 64;
    const int lane = tid & 63, w = tid >> 6;
    for (int i = tid; i < W * R; i += B) s_cnt[i] = 0;
    grp_sync<W>();
    C *cnt = s_cnt + w * R;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t dg = rd[j];
        const bool valid = striped_elem<IPT>(w, j, lane) < nvalid;
        const uint64_t vm = ballot64(valid);
        // lanes that differ from this one in some bit: per bit b, with t
        // all ones where this lane's bit is set, mis |= ballot ^ t (one
        // three-input op per half: 0xF6 is S0 | (S1 ^ S2))
        uint32_t mlo = 0u, mhi = 0u;
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            uint32_t t = (uint32_t)__builtin_amdgcn_sbfe((int32_t)dg, b, 1);
            asm("" : "+v"(t));  // the ballot tests t itself, not a second shift of dg
            const uint64_t m = ballot64(t != 0u);
            mlo = __builtin_amdgcn_bitop3_b32(mlo, (uint32_t)m, t, 0xF6);
            mhi = __builtin_amdgcn_bitop3_b32(mhi, (uint32_t)(m >> 32), t, 0xF6);
        }
        const uint64_t peers = ((uint64_t)((uint32_t)(vm >> 32) & ~mhi) << 32) | ((uint32_t)vm & ~mlo);
        const uint32_t below = count_below(peers);
        const uint32_t c = cnt[dg];
        rd[j] = (c + below) | (dg << 16);
        if (valid && below == 0) cnt[dg] = (C)(c + (uint32_t)__popcll(peers));
    }
    grp_sync<W>();
    if constexpr (B >= R && W % (B / R) == 0) {
        constexpr int TPD = B / R, WPT = W / TPD;
        const int d = tid / TPD, g = tid % TPD;
        uint32_t c[WPT];
#pragma unroll
        for (int i = 0; i < WPT; ++i) c[i] = s_cnt[(g * WPT + i) * R + d];
        uint32_t sum = 0;
#pragma unroll
        for (int i = 0; i < WPT; ++i) {
            const uint32_t t = c[i];
            c[i] = sum;
            sum += t;
        }
        uint32_t incl = sum;
#pragma unroll
        for (int o = 1; o < TPD; o <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)incl, o, TPD);
            if (g >= o) incl += y;
        }
        const uint32_t base = incl - sum;
#pragma unroll
        for (int i = 0; i < WPT; ++i) s_cnt[(g * WPT + i) * R + d] = (C)(base + c[i]);
        if (g == TPD - 1) s_tot[d] = incl;
    } else {
        for (int d = tid; d < R; d += B) {
            uint32_t run = 0;
#pragma unroll
            for (int ww = 0; ww < W; ++ww) {
                const uint32_t c = s_cnt[ww * R + d];
                s_cnt[ww * R + d] = (C)run;
                run += c;
            }
            s_tot[d] = run;
        }
    }
    grp_sync<W>();
}

// Phase 2: with s_start = exclusive scan of s_tot over digits, turns the
// wave-local ranks into tile positions.
template <int RB, int W, int IPT, typename C = uint32_t>
__device__ __forceinline__ void rank_finish_packed(uint32_t (&rd)[IPT], const C *s_cnt, const uint32_t *s_start,
                                                   int tid) {
    constexpr int R = 1 << RB;
    const int w = tid >> 6;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t dg = rd[j] >> 16;
        rd[j] += s_start[dg] + (uint32_t)s_cnt[w * R + dg];
    }
}

// Decoupled look-back of one digit by a group of K adjacent threads (kk =
// rank in the group).  lbd[p * RADIX] is the word of the tile at local index
// p; `first` is the local index of the nearest predecessor (>= 0).  The
// first round reads the K nearest predecessors (one word per thread: the
// common case ends there); later rounds read M words per thread, K*M tiles
// per round trip.  Sums counts down to (and including) the nearest
// inclusive prefix and returns that exclusive prefix.  Every predecessor
// publishes, and local tile 0 publishes an inclusive prefix, so the walk
// ends.
template <int K, int M>
__device__ __forceinline__ uint32_t lookback_prefix(const uint64_t *lbd, int64_t first, uint32_t epoch, int kk) {
    uint32_t excl = 0;
    int64_t p0 = first;
    int mw = 1;  // words per thread this round
    while (true) {
        const uint32_t win = (uint32_t)(K * mw);
        uint64_t wv[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int64_t p = p0 - (int64_t)(kk * mw + m);
            wv[m] = (m < mw && p >= 0) ? lb_load(lbd + (size_t)p * RADIX) : lb_pack(epoch, LB_INC, 0u);
        }
        uint32_t inc_at = win, notready_at = win;
#pragma unroll
        for (int m = M - 1; m >= 0; --m) {
            if (m >= mw) continue;
            uint32_t fl = (uint32_t)(wv[m] >> 32) & 3u;
            if ((uint32_t)(wv[m] >> 34) != epoch) fl = 0;
            if (fl == LB_INC) inc_at = (uint32_t)(kk * mw + m);
            if (fl == 0) notready_at = (uint32_t)(kk * mw + m);
        }
#pragma unroll
        for (int o = 1; o < K; o <<= 1) {
            inc_at = min(inc_at, (uint32_t)__shfl_xor((int)inc_at, o, 64));
            notready_at = min(notready_at, (uint32_t)__shfl_xor((int)notready_at, o, 64));
        }
        const uint32_t need = inc_at < win ? inc_at : win - 1;
        if (notready_at <= need) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        uint32_t c = 0;
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (m < mw && (uint32_t)(kk * mw + m) <= need) c += (uint32_t)wv[m];
#pragma unroll
        for (int o = 1; o < K; o <<= 1) c += (uint32_t)__shfl_xor((int)c, o, 64);
        excl += c;
        if (inc_at < win) return excl;
        p0 -= win;
        mw = M;
    }
}

// OR and AND of a 64-bit value over the valid lanes of the block.
template <int W>
__device__ __forceinline__ void block_or_and(uint64_t vor, uint64_t vand, uint64_t *s_red, uint64_t &ror,
                                             uint64_t &rand_, int tid) {
    const int lane = tid & 63, w = tid >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t olo = __shfl_xor((uint32_t)vor, d, 64), ohi = __shfl_xor((uint32_t)(vor >> 32), d, 64);
        const uint32_t alo = __shfl_xor((uint32_t)vand, d, 64), ahi = __shfl_xor((uint32_t)(vand >> 32), d, 64);
        vor |= ((uint64_t)ohi << 32) | olo;
        vand &= ((uint64_t)ahi << 32) | alo;
    }
    if (lane == 0) {
        s_red[w] = vor;
        s_red[W + w] = vand;
    }
    grp_sync<W>();
    ror = 0;
    rand_ = ~0ull;
#pragma unroll
    for (int ww = 0; ww < W; ++ww) {
        ror |= s_red[ww];
        rand_ &= s_red[W + ww];
    }
    grp_sync<W>();
}

}  // namespace ak
