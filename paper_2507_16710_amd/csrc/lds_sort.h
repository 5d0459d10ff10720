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
__device__ __forceinline__ void lds_sort_core(typename KT<DT>::U (&k)[IPT], uint32_t (&v)[IPT], uint32_t len,
                                              SmallSmem<typename KT<DT>::U, VAL, W, IPT> &sm, int tid) {
    using U = typename KT<DT>::U;
    constexpr int B = W * 64;
    const int lane = tid & 63, w = tid >> 6;
    uint32_t rd[IPT];  // digit, then rank | digit << 16
    // the bits that vary over the tile: OR and AND of the images, in two
    // 64-bit halves (the high half is zero below 128-bit keys)
    uint64_t olo = 0, alo = ~0ull, ohi = 0, ahi = ~0ull;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t e = striped_elem<IPT>(w, j, lane);
        if (e < len) {
            const auto t = KT<DT>::image(k[j]);
            olo |= img_lo(t);
            alo &= img_lo(t);
            ohi |= img_hi(t);
            ahi &= img_hi(t);
        }
        if (VAL) v[j] = e;
    }
    uint64_t ror, rand_;
    block_or_and<W>(olo, alo, sm.red, ror, rand_, tid);
    const uint64_t dlo = ror ^ rand_;
    uint64_t dhi = 0;
    if constexpr (key_bits(DT) > 64) {
        block_or_and<W>(ohi, ahi, sm.red, ror, rand_, tid);
        dhi = ror ^ rand_;
    }
    if (dlo != 0 || dhi != 0) {
        const int lo = dlo ? __builtin_ctzll(dlo) : 64 + __builtin_ctzll(dhi);
        const int hi = dhi ? 127 - __builtin_clzll(dhi) : 63 - __builtin_clzll(dlo);
        for (int shift = lo; shift <= hi; shift += RADIX_BITS) {
            // per-thread indices re-derived every pass from an opaque copy
            // of the thread id: hoisted out of the loop they would hold one
            // register per key
            int tq = tid;
            asm volatile("" : "+v"(tq));
            const int lane = tq & 63, w = tq >> 6;
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
}

template <int DT, bool VAL, int W, int IPT>
__device__ __forceinline__ void lds_sort_regs(typename KT<DT>::U (&k)[IPT], typename KT<DT>::U *out,
                                              uint32_t *vout, uint32_t len,
                                              SmallSmem<typename KT<DT>::U, VAL, W, IPT> &sm, int tid) {
    const int lane = tid & 63, w = tid >> 6;
    uint32_t v[IPT];
    lds_sort_core<DT, VAL, W, IPT>(k, v, len, sm, tid);
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t e = striped_elem<IPT>(w, j, lane);
        if (e < len) {
            if (!VAL) out[e] = k[j];
            else vout[e] = v[j];
        }
    }
}

// Sort by key of up to W*64*IPT keys on chip, in place: the keys sorted,
// and the payloads vals[0..len) reordered the same way (every payload is
// read through the tile's permutation before any is written).
template <int DT, typename V, int W, int IPT>
__device__ __forceinline__ void lds_sort_pairs(typename KT<DT>::U *keys, V *vals, uint32_t len,
                                               SmallSmem<typename KT<DT>::U, true, W, IPT> &sm, int tid) {
    using U = typename KT<DT>::U;
    const int lane = tid & 63, w = tid >> 6;
    U k[IPT];
    uint32_t v[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t e = striped_elem<IPT>(w, j, lane);
        k[j] = e < len ? keys[e] : U(0);
    }
    lds_sort_core<DT, true, W, IPT>(k, v, len, sm, tid);
    V pv[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t e = striped_elem<IPT>(w, j, lane);
        pv[j] = e < len ? vals[v[j]] : V(0);
    }
    __syncthreads();  // every payload read before any is written
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t e = striped_elem<IPT>(w, j, lane);
        if (e < len) {
            keys[e] = k[j];
            vals[e] = pv[j];
        }
    }
}

// Keys-only on-chip sort of a chunk of a code-ordered array (the chunk sorts
// of the prefix-partitioned radix sort), stable, same result as
// lds_sort_regs.  When more than 24 bits vary, one stable pass orders the
// chunk by its top MB varying bits (most significant digit first; 16-bit
// counters in the counter space, 2^MB-entry bucket totals and starts in
// mtot / mstart); if every bucket then holds at most BMAX keys, each key's
// final place is its bucket's start plus the number of keys of its bucket
// that precede it in the total order: a smaller image, or an equal image at
// an earlier place (the pass kept input order).  They are counted by
// comparing against the bucket's keys in LDS, and the key is stored at its
// place in `out`, which must not overlap keys other threads still read (the
// whole chunk is on chip by then).  A chunk of nearly uniform keys has
// about len / 2^MB keys per bucket, so this costs one ranking pass plus a
// few comparisons per key instead of one ranking pass per varying digit.
// Chunks with a larger bucket take the LSD passes of lds_sort_regs over
// the keys in their bucket order.
template <int DT, int W, int IPT, int MB, int BMAX = 64>
__device__ __forceinline__ void lds_sort_chunk(typename KT<DT>::U (&k)[IPT], typename KT<DT>::U *out, uint32_t len,
                                               SmallSmem<typename KT<DT>::U, false, W, IPT> &sm, uint32_t *mtot,
                                               uint32_t *mstart, int tid) {
    using U = typename KT<DT>::U;
    using I = decltype(KT<DT>::image(k[0]));
    constexpr int B = W * 64, MR = 1 << MB;
    static_assert((size_t)W * MR * 2 <= sizeof(sm.cnt), "16-bit digit counters fit the counter space");
    const int lane = tid & 63, w = tid >> 6;
    uint64_t vor = 0, vand = ~0ull;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t e = striped_elem<IPT>(w, j, lane);
        if (e < len) {
            const uint64_t t = (uint64_t)KT<DT>::image(k[j]);
            vor |= t;
            vand &= t;
        }
    }
    uint64_t ror, rand_;
    block_or_and<W>(vor, vand, sm.red, ror, rand_, tid);
    const uint64_t diff = ror ^ rand_;
    int lo = 0, hi = -1;
    if (diff != 0) {
        lo = __builtin_ctzll(diff);
        hi = 63 - __builtin_clzll(diff);
    }
    // more than three digits vary: one pass and comparisons beat the LSD
    // passes (fewer varying bits: the LSD passes, which also suit chunks of
    // a few repeated values)
    if (hi - lo + 1 > 3 * RADIX_BITS) {
        const int shift = hi - (MB - 1);
        uint16_t *cnt16 = reinterpret_cast<uint16_t *>(sm.cnt);
        uint32_t rd[IPT];
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t e = striped_elem<IPT>(w, j, lane);
            rd[j] = e < len ? (uint32_t)((uint64_t)KT<DT>::image(k[j]) >> shift) & (MR - 1) : 0u;
        }
        rank_match_packed<MB, W, IPT, uint16_t>(rd, len, cnt16, mtot, tid);
        block_exscan<B, MR>(mtot, mstart, sm.wsum, tid);
        rank_finish_packed<MB, W, IPT, uint16_t>(rd, cnt16, mstart, tid);
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t e = striped_elem<IPT>(w, j, lane);
            if (e < len) sm.keys[rd[j] & 0xFFFFu] = k[j];
        }
        bool big = false;
        for (int d = tid; d < MR; d += B) big |= mtot[d] > (uint32_t)BMAX;
        grp_sync<W>();
        if (!__syncthreads_or(big)) {
#pragma unroll
            for (int j = 0; j < IPT; ++j) {
                const uint32_t e = striped_elem<IPT>(w, j, lane);
                if (e < len) {
                    const U key = sm.keys[e];
                    const I ti = KT<DT>::image(key);
                    const uint32_t d = (uint32_t)((uint64_t)ti >> shift) & (MR - 1);
                    const uint32_t b0 = mstart[d], b1 = b0 + mtot[d];
                    // one loop over the bucket (a wave runs as long as its
                    // largest bucket; two loops would each run that long)
                    uint32_t r = 0;
                    for (uint32_t q = b0; q < b1; ++q) {
                        const I tq = KT<DT>::image(sm.keys[q]);
                        r += (tq < ti || (tq == ti && q < e)) ? 1u : 0u;
                    }
                    out[b0 + r] = key;
                }
            }
            return;
        }
        // a large bucket: LSD passes over the chunk in its new order (the
        // pass was stable, so equal keys are still in input order)
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t e = striped_elem<IPT>(w, j, lane);
            k[j] = e < len ? sm.keys[e] : U(0);
        }
        grp_sync<W>();
    }
    lds_sort_regs<DT, false, W, IPT>(k, out, nullptr, len, sm, tid);
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
