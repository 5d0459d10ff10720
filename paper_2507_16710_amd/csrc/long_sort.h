// Single-workgroup LSD radix sort of a long key range through a scratch
// copy (used for long segments and for the learned sort's fallback runs).
#pragma once

#include "radix_common.h"

namespace ak {

// ------------------------------------------------------- long segments
template <typename U, int W, int IPT>
struct LongSmem {
    U keys[W * 64 * IPT];
    uint8_t dig[W * 64 * IPT];
    uint32_t cnt[W * RADIX];
    uint32_t tot[RADIX], start[RADIX], run[RADIX];
    uint32_t hist[8][RADIX];
    uint32_t wsum[W];
    int32_t places[8];
    int32_t q;
};

// One workgroup sorts a long segment: one read for the histograms of every
// digit place, then per non-trivial place a stable pass over the segment's
// tiles in order (running digit offsets carried in LDS from tile to tile),
// ping-ponging between the segment and its scratch copy.
template <int DT, int W, int IPT>
__device__ void sort_long(typename KT<DT>::U *keys, typename KT<DT>::U *tmp, uint32_t len,
                          LongSmem<typename KT<DT>::U, W, IPT> &sm) {
    using U = typename KT<DT>::U;
    constexpr int B = W * 64, TILE = B * IPT;
    constexpr int P = (int)sizeof(U);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int i = tid; i < 8 * RADIX; i += B) (&sm.hist[0][0])[i] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < len; i += B) {
        const U t = KT<DT>::image(keys[i]);
        const uint64_t act = ballot64(true);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const uint32_t d = (uint32_t)(t >> (8 * p)) & (RADIX - 1);
            const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
            if (ballot64(d == d0) == act) {
                if (count_below(act) == 0) atomicAdd(&sm.hist[p][d0], (uint32_t)__popcll(act));
            } else {
                atomicAdd(&sm.hist[p][d], 1u);
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        int q = 0;
        for (int p = 0; p < P; ++p) {
            bool trivial = false;
            for (int d = 0; d < RADIX; ++d) trivial |= (sm.hist[p][d] == len);
            if (!trivial) sm.places[q++] = p;
        }
        sm.q = q;
    }
    __syncthreads();
    const int q = sm.q;
    for (int j = 0; j < q; ++j) {
        const int p = sm.places[j];
        const U *src = (j & 1) ? tmp : keys;
        U *dst = (j & 1) ? keys : tmp;
        block_exscan<B, RADIX>(sm.hist[p], sm.run, sm.wsum, tid);
        // tiles in order; the next tile's keys are loaded while this one is
        // ranked and scattered
        U kn[IPT];
#pragma unroll
        for (int jj = 0; jj < IPT; ++jj) {
            const uint32_t e = striped_elem<IPT>(w, jj, lane);
            kn[jj] = e < len ? src[e] : U(0);
        }
        for (uint32_t tb = 0; tb < len; tb += TILE) {
            const uint32_t tvalid = min((uint32_t)TILE, len - tb);
            U k[IPT];
            uint32_t rd[IPT];  // digit, then rank | digit << 16
#pragma unroll
            for (int jj = 0; jj < IPT; ++jj) k[jj] = kn[jj];
            const uint32_t nb = tb + TILE;
            if (nb < len) {
#pragma unroll
                for (int jj = 0; jj < IPT; ++jj) {
                    const uint32_t e = striped_elem<IPT>(w, jj, lane);
                    kn[jj] = nb + e < len ? src[nb + e] : U(0);
                }
            }
#pragma unroll
            for (int jj = 0; jj < IPT; ++jj) {
                const uint32_t e = striped_elem<IPT>(w, jj, lane);
                rd[jj] = e < tvalid ? (uint32_t)(KT<DT>::image(k[jj]) >> (8 * p)) & (RADIX - 1) : 0u;
            }
            rank_match_packed<RADIX_BITS, W, IPT>(rd, tvalid, sm.cnt, sm.tot, tid);
            block_exscan<B, RADIX>(sm.tot, sm.start, sm.wsum, tid);
            rank_finish_packed<RADIX_BITS, W, IPT>(rd, sm.cnt, sm.start, tid);
#pragma unroll
            for (int jj = 0; jj < IPT; ++jj) {
                const uint32_t e = striped_elem<IPT>(w, jj, lane);
                if (e < tvalid) {
                    sm.keys[rd[jj] & 0xFFFFu] = k[jj];
                    sm.dig[rd[jj] & 0xFFFFu] = (uint8_t)(rd[jj] >> 16);
                }
            }
            __syncthreads();
#pragma unroll
            for (int jj = 0; jj < IPT; ++jj) {
                const uint32_t i = (uint32_t)(jj * B + tid);
                if (i < tvalid) {
                    const uint32_t d = sm.dig[i];
                    dst[sm.run[d] + i - sm.start[d]] = sm.keys[i];
                }
            }
            __syncthreads();
            for (int d = tid; d < RADIX; d += B) sm.run[d] += sm.tot[d];
            __syncthreads();
        }
    }
    if (q & 1) {
        for (uint32_t i = tid; i < len; i += B) keys[i] = tmp[i];
    }
    __syncthreads();
}

}  // namespace ak
