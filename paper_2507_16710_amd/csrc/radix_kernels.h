// Kernel argument blocks and launch shapes of the radix kernels.
#pragma once

#include <type_traits>

#include "ak_internal.h"

namespace ak {

// What a radix run carries with the keys:
//   M_KEYS    nothing (sort in place);
//   M_PERM    uint32 indices: made in the first pass, the last pass writes
//             only them (sortperm);
//   M_PAIRS4  a 4-byte payload per key, moved with the keys through every
//             pass, both ending in the caller's buffers (sort by key);
//   M_PAIRS8  the same with an 8-byte payload;
//   M_LOWMEM  uint32 indices only: each pass gathers its keys through them
//             from the untouched key array, so no key scratch is needed
//             (sortperm with the smallest scratch).
enum : int { M_KEYS = 0, M_PERM = 1, M_PAIRS4 = 2, M_PAIRS8 = 3, M_LOWMEM = 4 };
template <int M>
struct ModeT {
    static constexpr bool VAL = M != M_KEYS;
    static constexpr bool PAIRS = M == M_PAIRS4 || M == M_PAIRS8;
    using V = typename std::conditional<M == M_PAIRS8, uint64_t, uint32_t>::type;
    // value class of the shape tables: 0 none, 1 four bytes, 2 eight bytes
    static constexpr int VCLASS = M == M_KEYS ? 0 : (M == M_PAIRS8 ? 2 : 1);
};
constexpr int mode_vclass(int m) { return m == M_KEYS ? 0 : (m == M_PAIRS8 ? 2 : 1); }

struct OnesweepArgs {
    void *keys;           // sort / pairs: keys (in/out); sortperm / lowmem: the const keys
    void *t0, *t1;        // key scratch buffers
    void *v0, *v1;        // value scratch buffers
    void *vals;           // sortperm / lowmem: the permutation output; pairs: the caller's payload
    uint64_t *lookback;   // tiles x RADIX look-back words, then groups x RADIX group words
    RunState *st;
    const float *model;   // learned model (code digits only)
    uint32_t n;
    int place;
    int cb;               // code bits (code digits only)
    int staged;           // code digits: model table staged in dynamic LDS
    // reduce-then-scan passes: digit counts, then offsets, per chunk of
    // chunk_tiles tiles, digit-major (ccnt[d * nchunks + c])
    uint32_t *ccnt;
    uint32_t nchunks, chunk_tiles;
};

// One-sweep tile shapes (W waves x IPT keys per lane).  A few shapes are
// compiled per (key width, with values); os_variant() picks one at run time
// (default from the tuning sweep; $AK_OS_VARIANT overrides it).
// Look-back words read per thread per round trip after the first.  One:
// most look-backs end within a round trip or two, and fewer words per round
// trip cost less than the rounds they save (2^31-key learned sort: 63.0 ms
// with 1, 63.8 with 2, 63.9-64.2 with 4, 66.6 with 8).
#ifndef AK_LB_M
#define AK_LB_M 1
#endif
constexpr int LB_M = AK_LB_M;
// Tiles per look-back group.  A tile looks back only inside its group (the
// group's first tile is inclusive by definition); every group's last tile
// publishes the group's digit totals, and the prefix of the groups before a
// tile comes from a second decoupled look-back over those group words.  The
// inclusive frontier then advances LB_GROUP times faster per round trip.
#ifndef AK_LB_GROUP
#define AK_LB_GROUP 16
#endif
constexpr int LB_GROUP = AK_LB_GROUP;
// look-back words of a pass over `tiles` tiles (tile words, then group words)
inline size_t lookback_words(size_t tiles) { return (tiles + (tiles + LB_GROUP - 1) / LB_GROUP) * 256; }

// A pass shape: W waves x IPT keys per lane per tile, and whether the pass
// runs on a persistent grid (a workgroup walks tiles and loads its next
// tile before it waits in the look-back) or one workgroup per tile.
struct OsShape {
    int w, ipt;
    bool pers;
};
constexpr int OS_NVAR = 4;
// [key class: 16/32-bit, 64-bit, 128-bit][value class: none, 4 bytes,
// 8 bytes][variant]
constexpr OsShape OS_SHAPES[3][3][OS_NVAR] = {
    // 16- and 32-bit keys
    {{{16, 8, false}, {16, 6, false}, {16, 12, false}, {16, 16, false}},
     {{8, 12, false}, {16, 8, false}, {16, 6, false}, {16, 12, true}},
     {{16, 4, false}, {16, 6, false}, {8, 8, false}, {16, 8, true}}},
    // 64-bit keys
    {{{16, 4, false}, {16, 8, false}, {16, 12, true}, {8, 24, true}},
     {{16, 4, false}, {8, 6, false}, {16, 8, true}, {8, 16, true}},
     {{16, 4, false}, {8, 6, false}, {16, 6, true}, {8, 12, true}}},
    // 128-bit keys (16 bytes staged per key)
    {{{16, 4, false}, {8, 4, false}, {16, 3, false}, {8, 8, true}},
     {{16, 2, false}, {8, 4, false}, {16, 4, false}, {8, 6, true}},
     {{16, 2, false}, {8, 4, false}, {16, 4, false}, {8, 6, true}}},
};
// Shapes of the code-digit passes (keys only; one persistent workgroup per
// CU next to the staged model table, so registers are not the limit and
// the tile is as large as the LDS left beside the table allows).
// os_code_variant() picks one ($AK_OS_CODE_VARIANT overrides it).
constexpr OsShape OS_CODE_SHAPES[2][OS_NVAR] = {
    {{16, 8, true}, {16, 6, true}, {16, 12, true}, {8, 12, true}},
    {{8, 20, true}, {16, 8, true}, {8, 16, true}, {16, 10, true}},
};
// default shape per (key class, value class): see radix.hip for the sweep
constexpr int OS_DEFAULT[3][3] = {{3, 3, 3}, {3, 2, 3}, {0, 1, 1}};
int os_variant(int dt, int mode, int64_t n);
int os_code_variant(int dt);
inline int os_tile(int dt, int mode, int64_t n) {
    const OsShape s = OS_SHAPES[key_class(dt)][mode_vclass(mode)][os_variant(dt, mode, n)];
    return s.w * 64 * s.ipt;
}
inline int os_code_tile(int dt) {
    const OsShape s = OS_CODE_SHAPES[key_bits(dt) == 64][os_code_variant(dt)];
    return s.w * 64 * s.ipt;
}
// Whether every variant of the table is compiled for (dtype, mode): the
// six original key types without payloads; the others compile their
// default variant (and, keys only, the small-input one).
constexpr bool os_all_variants(int dt, int mode) { return dt >= AK_I32 && dt <= AK_F64 && mode <= M_PERM; }

// Reduce-then-scan passes ($AK_OS_RTS=1) instead of one-sweep passes, and
// the tiles per reduce-then-scan chunk.
bool os_rts();
// Shape of the digit histogram of 16- to 64-bit keys: 0..2 the lane-private
// kernel (1024 x 8, 1024 x 16, 512 x 16 keys per batch), 3 the shared-
// counter one, also for code digits ($AK_HIST_VARIANT overrides the
// default).
int hist_variant();
uint32_t rts_chunk_tiles(uint32_t tiles);

// Radix runs of the modes and key types radix.hip does not instantiate:
// the six 32/64-bit key types with payloads or the low-memory sortperm
// (radix_pairs.hip), and the 16- and 128-bit key types (radix_wide.hip).
ak_status radix_sort_pairs_std(Workspace *ws, int dt, int mode, void *keys, void *vals, int64_t n, int slot);
ak_status radix_sort_wide(Workspace *ws, int dt, int mode, void *keys, void *vals, int64_t n, int slot);

template <typename U, bool VAL, int W, int IPT>
struct SmallSmem {
    U keys[W * 64 * IPT];
    uint32_t vals[VAL ? W * 64 * IPT : 1];
    uint32_t cnt[W * RADIX];
    uint32_t tot[RADIX];
    uint32_t start[RADIX];
    uint32_t wsum[W];
    uint64_t red[2 * W];
};

ak_status code_partition(Workspace *ws, int dt, void *keys, uint32_t n, const float *model, int L, int cb,
                         int slot);

}  // namespace ak
