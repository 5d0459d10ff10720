// On-chip sort of one tile by a group of waves (used for small inputs, for
// short segments and for the learned sort's chunks).
#pragma once

#include "radix_common.h"
#include "radix_kernels.h"

namespace ak {

// ------------------------------------------------ single-workgroup sort
// Sorts up to W*64*IPT keys on chip with a group of W waves (tid = thread
// index within the group): load once, skip the bits that do not vary
// (OR/AND reduction of the images), one stable ranking per 8-bit digit
// between the lowest and highest varying bit, store once.  `in` may equal
// `out`: every key is read before any is written.  With VAL the output is
// the permutation (vout[i] = input index of the i-th smallest key).
// Sorts the first `len` keys of a tile already held in registers in the
// wave-striped layout (k[j] of lane l in wave w is element w*64*IPT + j*64
// + l); writes them sorted to out[0..len) (or, with VAL, the input indices
// to vout).
template <int DT, bool VAL, int W, int IPT>
__device__ __forceinline__ void lds_sort_regs(typename KT<DT>::U (&k)[IPT], typename KT<DT>::U *out,
                                              uint32_t *vout, uint32_t len,
                                              SmallSmem<typename KT<DT>::U, VAL, W, IPT> &sm, int tid) {
    using U = typename KT<DT>::U;
    constexpr int B = W * 64;
    const int lane = tid & 63, w = tid >> 6;
    uint32_t v[IPT], rd[IPT];  // digit, then rank | digit << 16
    uint64_t vor = 0, vand = ~0ull;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t e = striped_elem<IPT>(w, j, lane);
        if (e < len) {
            const uint64_t t = (uint64_t)KT<DT>::image(k[j]);
            vor |= t;
            vand &= t;
        }
        if (VAL) v[j] = e;
    }
    uint64_t ror, rand_;
    block_or_and<W>(vor, vand, sm.red, ror, rand_, tid);
    const uint64_t diff = ror ^ rand_;
    if (diff != 0) {
        const int lo = __builtin_ctzll(diff), hi = 63 - __builtin_clzll(diff);
        for (int shift = lo; shift <= hi; shift += RADIX_BITS) {
#pragma unroll
            for (int j = 0; j < IPT; ++j) {
                const uint32_t e = striped_elem<IPT>(w, j, lane);
                rd[j] = e < len ? (uint32_t)(KT<DT>::image(k[j]) >> shift) & (RADIX - 1) : 0u;
            }
            rank_match_packed<RADIX_BITS, W, IPT>(rd, len, sm.cnt, sm.tot, tid);
            block_exscan<B, RADIX>(sm.tot, sm.start, sm.wsum, tid);
            rank_finish_packed<RADIX_BITS, W, IPT>(rd, sm.cnt, sm.start, tid);
#pragma unroll
            for (int j = 0; j < IPT; ++j) {
                const uint32_t e = striped_elem<IPT>(w, j, lane);
                if (e < len) {
                    sm.keys[rd[j] & 0xFFFFu] = k[j];
                    if (VAL) sm.vals[rd[j] & 0xFFFFu] = v[j];
                }
            }
            grp_sync<W>();
#pragma unroll
            for (int j = 0; j < IPT; ++j) {
                const uint32_t e = striped_elem<IPT>(w, j, lane);
                if (e < len) {
                    k[j] = sm.keys[e];
                    if (VAL) v[j] = sm.vals[e];
                }
            }
            grp_sync<W>();
        }
    }
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t e = striped_elem<IPT>(w, j, lane);
        if (e < len) {
            if (!VAL) out[e] = k[j];
            else vout[e] = v[j];
        }
    }
}

// Loads up to W*64*IPT keys from `in` and sorts them on chip (`in` may
// equal `out`: every key is read before any is written).
template <int DT, bool VAL, int W, int IPT>
__device__ __forceinline__ void lds_sort_tile(const typename KT<DT>::U *in, typename KT<DT>::U *out,
                                              uint32_t *vout, uint32_t len,
                                              SmallSmem<typename KT<DT>::U, VAL, W, IPT> &sm, int tid) {
    using U = typename KT<DT>::U;
    const int lane = tid & 63, w = tid >> 6;
    U k[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t e = striped_elem<IPT>(w, j, lane);
        k[j] = e < len ? in[e] : U(0);
    }
    lds_sort_regs<DT, VAL, W, IPT>(k, out, vout, len, sm, tid);
}

}  // namespace ak
