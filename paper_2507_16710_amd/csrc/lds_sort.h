// On-chip sort of one tile by a group of waves (used for small inputs, for
// short segments and for the learned sort's chunks).
#pragma once

#include "radix_common.h"
#include "radix_kernels.h"

namespace ak {

// ------------------------------------------------ single-workgroup sort
// Stable LSD passes over the image bits [lo, hi] (8-bit digits from lo
// up) of a tile held in registers (wave-striped); afterwards the keys are in
// sm.keys[0..len) in their new order and k[j] holds element
// striped_elem(w, j, lane) of it.
template <int DT, bool VAL, int W, int IPT>
__device__ __forceinline__ void lsd_range(typename KT<DT>::U (&k)[IPT], uint32_t (&v)[IPT], uint32_t len,
                                          SmallSmem<typename KT<DT>::U, VAL, W, IPT> &sm, int tid, int lo, int hi) {
    constexpr int B = W * 64;
    uint32_t rd[IPT];  // digit, then rank | digit << 16
    for (int shift = lo; shift <= hi; shift += RADIX_BITS) {
        // per-thread indices re-derived every pass from an opaque copy of
        // the thread id: hoisted out of the loop they would hold one
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
    const int lane = tid & 63, w = tid >> 6;
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
        lsd_range<DT, VAL, W, IPT>(k, v, len, sm, tid, lo, hi);
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

// True in every thread of the group if `pred` holds in any of its threads
// (a group of one wave: a ballot; otherwise a block barrier).
template <int W>
__device__ __forceinline__ bool grp_any(bool pred) {
    if constexpr (W == 1) return ballot64(pred) != 0;
    else return __syncthreads_or(pred) != 0;
}

// Keys-only stable on-chip sort of a tile held in registers, same result as
// lds_sort_regs, with fewer ranking passes when the keys spread over many
// more bits than the tile needs to tell them apart.  If more than T + 8
// bits vary (T = 8 for tiles of at most 256 keys, else 16), stable LSD
// passes order the tile by its top T varying bits only; the keys sharing
// such a prefix then form small contiguous groups (about len / 2^T keys),
// in input order.  A key's final place is its place e in that order, less
// the keys before it in its group with a larger image, plus the keys after
// it with a smaller one (equal images keep their order, so the result is
// stable); each key walks its group in LDS and is stored there in `out`
// (every key is read before any is written, so `out` may be the input).
// A group longer than GMAX keys (many repeated keys) sends the tile to the
// LSD passes over all its varying bits instead.
template <int DT, int W, int IPT, int GMAX = 16>
__device__ __forceinline__ void lds_sort_top(typename KT<DT>::U (&k)[IPT], typename KT<DT>::U *out, uint32_t len,
                                             SmallSmem<typename KT<DT>::U, false, W, IPT> &sm, int tid) {
    using U = typename KT<DT>::U;
    if constexpr (key_bits(DT) > 64) {
        lds_sort_regs<DT, false, W, IPT>(k, out, nullptr, len, sm, tid);
    } else {
        using I = decltype(KT<DT>::image(k[0]));
        const int lane = tid & 63, w = tid >> 6;
        uint32_t v[IPT];  // no payload
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
        if (diff != 0) {
            const int lo = __builtin_ctzll(diff), hi = 63 - __builtin_clzll(diff);
            const int T = len <= 256u ? RADIX_BITS : 2 * RADIX_BITS;
            const bool top = hi - lo + 1 > T + RADIX_BITS;
            const int s0 = hi - T + 1;
            // one call site of the passes (a second copy would raise the
            // register count): the top bits first, and all varying bits if
            // a group is too long
            int first = top ? s0 : lo;
#pragma nounroll
            for (int round = 0; round < 2; ++round) {
                lsd_range<DT, false, W, IPT>(k, v, len, sm, tid, first, hi);
                if (first == lo) break;
                // (loops over a lane's items not unrolled: unrolled, their
                // loads would all be held in registers at once)
                bool big = false;
#pragma nounroll
                for (int j = 0; j < IPT; ++j) {
                    const uint32_t e = striped_elem<IPT>(w, j, lane);
                    if (e + GMAX < len)
                        big |= (KT<DT>::image(sm.keys[e]) >> s0) == (KT<DT>::image(sm.keys[e + GMAX]) >> s0);
                }
                if (!grp_any<W>(big)) {
#pragma nounroll
                    for (int j = 0; j < IPT; ++j) {
                        const uint32_t e = striped_elem<IPT>(w, j, lane);
                        if (e < len) {
                            // the key again from LDS (k[] stays dead here)
                            const U key = sm.keys[e];
                            const I ti = KT<DT>::image(key);
                            const I px = ti >> s0;
                            uint32_t gl = 0, sr = 0;
                            for (uint32_t q = e; q-- > 0;) {
                                const I tq = KT<DT>::image(sm.keys[q]);
                                if ((tq >> s0) != px) break;
                                gl += tq > ti ? 1u : 0u;
                            }
                            for (uint32_t q = e + 1; q < len; ++q) {
                                const I tq = KT<DT>::image(sm.keys[q]);
                                if ((tq >> s0) != px) break;
                                sr += tq < ti ? 1u : 0u;
                            }
                            out[e - gl + sr] = key;
                        }
                    }
                    return;
                }
                // long groups: LSD passes over every varying bit, from the
                // present order (equal keys are still in input order)
                first = lo;
            }
        }
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t e = striped_elem<IPT>(w, j, lane);
            if (e < len) out[e] = k[j];
        }
    }
}

// Loads up to W*64*IPT keys from `in` and sorts them on chip with
// lds_sort_top (`in` may equal `out`).
template <int DT, int W, int IPT>
__device__ __forceinline__ void lds_sort_tile_top(const typename KT<DT>::U *in, typename KT<DT>::U *out, uint32_t len,
                                                  SmallSmem<typename KT<DT>::U, false, W, IPT> &sm, int tid) {
    using U = typename KT<DT>::U;
    const int lane = tid & 63, w = tid >> 6;
    U k[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t e = striped_elem<IPT>(w, j, lane);
        k[j] = e < len ? in[e] : U(0);
    }
    lds_sort_top<DT, W, IPT>(k, out, len, sm, tid);
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
