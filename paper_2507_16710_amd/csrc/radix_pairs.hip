// Radix runs that carry a payload (sort by key, 4- or 8-byte payloads) or
// only indices (the low-memory sortperm) for the six 32- and 64-bit key
// types; kernels in radix_impl.h.
#include "radix_impl.h"

namespace ak {

template <int DT>
static ak_status pairs_t(Workspace *ws, int mode, void *keys, void *vals, int64_t n, int slot) {
    switch (mode) {
    case M_PAIRS4: return radix_sort_t<DT, M_PAIRS4>(ws, keys, vals, n, slot);
    case M_PAIRS8: return radix_sort_t<DT, M_PAIRS8>(ws, keys, vals, n, slot);
    case M_LOWMEM: return radix_sort_t<DT, M_LOWMEM>(ws, keys, vals, n, slot);
    }
    set_error("radix_sort_pairs_std: bad mode");
    return AK_ERR_INTERNAL;
}

ak_status radix_sort_pairs_std(Workspace *ws, int dt, int mode, void *keys, void *vals, int64_t n, int slot) {
    switch (dt) {
    case AK_I32: return pairs_t<AK_I32>(ws, mode, keys, vals, n, slot);
    case AK_I64: return pairs_t<AK_I64>(ws, mode, keys, vals, n, slot);
    case AK_U32: return pairs_t<AK_U32>(ws, mode, keys, vals, n, slot);
    case AK_U64: return pairs_t<AK_U64>(ws, mode, keys, vals, n, slot);
    case AK_F32: return pairs_t<AK_F32>(ws, mode, keys, vals, n, slot);
    case AK_F64: return pairs_t<AK_F64>(ws, mode, keys, vals, n, slot);
    }
    set_error("radix_sort_pairs_std: unknown dtype");
    return AK_ERR_UNSUPPORTED_DTYPE;
}

}  // namespace ak
