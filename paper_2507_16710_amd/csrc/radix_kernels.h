// Kernel argument blocks and launch shapes of the radix kernels.
#pragma once

#include "ak_internal.h"

namespace ak {

struct OnesweepArgs {
    void *keys;           // sort: keys (in/out); sortperm: the const keys
    void *t0, *t1;        // key scratch buffers
    uint32_t *v0, *perm;  // value scratch, permutation output
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
constexpr int LB_M = 4;  // look-back words read per thread per round trip
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
constexpr OsShape OS_SHAPES[2][2][OS_NVAR] = {
    // 32-bit keys: keys only, with values
    {{{16, 8, false}, {16, 6, false}, {16, 12, false}, {16, 16, false}},
     {{8, 12, false}, {16, 8, false}, {16, 6, false}, {16, 12, true}}},
    // 64-bit keys: keys only, with values
    {{{16, 4, false}, {16, 8, false}, {16, 12, true}, {8, 24, true}},
     {{16, 4, false}, {8, 6, false}, {16, 8, true}, {8, 16, true}}},
};
// Shapes of the code-digit passes (keys only; one persistent workgroup per
// CU next to the staged model table, so registers are not the limit and
// the tile is as large as the LDS left beside the table allows).
// os_code_variant() picks one ($AK_OS_CODE_VARIANT overrides it).
constexpr OsShape OS_CODE_SHAPES[2][OS_NVAR] = {
    {{16, 8, true}, {16, 6, true}, {16, 12, true}, {8, 12, true}},
    {{8, 20, true}, {16, 8, true}, {8, 16, true}, {16, 10, true}},
};
int os_variant(int dt, bool val, int64_t n);
int os_code_variant(int dt);
inline int os_tile(int dt, bool val, int64_t n) {
    const OsShape s = OS_SHAPES[key_bits(dt) == 64][val][os_variant(dt, val, n)];
    return s.w * 64 * s.ipt;
}
inline int os_code_tile(int dt) {
    const OsShape s = OS_CODE_SHAPES[key_bits(dt) == 64][os_code_variant(dt)];
    return s.w * 64 * s.ipt;
}

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
