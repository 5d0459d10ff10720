// Radix runs of the 16- and 128-bit integer keys (the other widths of the
// paper's sorting benchmarks, Sec. IV-C), in every mode: sort, sortperm,
// sort by key and the low-memory sortperm.  128-bit keys take 16 digit
// places; kernels in radix_impl.h.
#include "radix_impl.h"

namespace ak {

template <int DT>
static ak_status wide_t(Workspace *ws, int mode, void *keys, void *vals, int64_t n, int slot) {
    switch (mode) {
    case M_KEYS: return radix_sort_t<DT, M_KEYS>(ws, keys, nullptr, n, slot);
    case M_PERM: return radix_sort_t<DT, M_PERM>(ws, keys, vals, n, slot);
    case M_PAIRS4: return radix_sort_t<DT, M_PAIRS4>(ws, keys, vals, n, slot);
    case M_PAIRS8: return radix_sort_t<DT, M_PAIRS8>(ws, keys, vals, n, slot);
    case M_LOWMEM: return radix_sort_t<DT, M_LOWMEM>(ws, keys, vals, n, slot);
    }
    set_error("radix_sort_wide: bad mode");
    return AK_ERR_INTERNAL;
}

ak_status radix_sort_wide(Workspace *ws, int dt, int mode, void *keys, void *vals, int64_t n, int slot) {
    switch (dt) {
    case AK_I16: return wide_t<AK_I16>(ws, mode, keys, vals, n, slot);
    case AK_U16: return wide_t<AK_U16>(ws, mode, keys, vals, n, slot);
    case AK_I128: return wide_t<AK_I128>(ws, mode, keys, vals, n, slot);
    case AK_U128: return wide_t<AK_U128>(ws, mode, keys, vals, n, slot);
    }
    set_error("radix_sort_wide: unsupported dtype");
    return AK_ERR_UNSUPPORTED_DTYPE;
}

}  // namespace ak
