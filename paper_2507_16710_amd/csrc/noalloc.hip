// ak_sort_noalloc: the key sort of ak_sort for callers that cannot allocate
// device memory (code under graph capture, tight serving loops, harnesses
// that forbid allocation).  Its scratch is one file-scope device array per
// GPU, holding the run state, the look-back words and the key buffers of
// the largest admitted run; the kernels and their launch sequence are the
// ones ak_sort uses, launched directly (never through a graph).
#include <mutex>

#include "ak_internal.h"

namespace ak {

// Layout of the array: [run state | look-back words | arena for the key
// buffers and the per-tile counts].  The look-back region covers the most
// tiles an admitted run can have (2^21 64-bit keys in 4096-key tiles, or
// 2^22 32-bit keys in 8192- or 16384-key tiles: at most 512 tiles, 1.06
// MiB of words); the arena holds two key buffers of AK_NOALLOC_MAX_KEY_BYTES
// each plus the per-tile counts (512 KiB) and the prefix finish's state and
// run list (about 25 KiB at the largest admitted run).
constexpr size_t NA_STATE = (RUN_STATE_BYTES + 4095) & ~size_t(4095);
constexpr size_t NA_LOOKBACK = size_t(2) << 20;
constexpr size_t NA_ARENA = 2 * (size_t)AK_NOALLOC_MAX_KEY_BYTES + (size_t(2) << 20);
constexpr size_t NA_BYTES = NA_STATE + NA_LOOKBACK + NA_ARENA;

static __device__ __align__(256) uint8_t scratch[NA_BYTES];

namespace {
constexpr int NA_MAX_DEVICES = 64;
std::mutex g_na_mu;
// Per device: the array's device address (from hipGetSymbolAddress; the
// array's name in host code is only a stand-in) and the workspace view of
// it.  Set up once, on the device's first call.
void *g_na_ptr[NA_MAX_DEVICES] = {nullptr};
Workspace g_na_ws[NA_MAX_DEVICES];
}  // namespace

// Sets up the device's view of the array: the symbol's address on this
// device, the workspace fields pointing into it, and a zero fill of the run
// state and look-back words on `stream` (enqueued before this call's own
// kernels; later calls come after it in the caller's ordering).
static ak_status na_setup(int dev, hipStream_t stream, Workspace **out) {
    std::lock_guard<std::mutex> lk(g_na_mu);
    Workspace *ws = &g_na_ws[dev];
    if (!g_na_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
            set_error("hipGetSymbolAddress(scratch) returned NULL");
            return AK_ERR_HIP;
        }
        char *base = (char *)ptr;
        ws->device = dev;
        ws->state = (RunState *)base;
        ws->epoch_dev = reinterpret_cast<uint32_t *>(ws->state + RUN_SLOTS);
        ws->lookback = (uint64_t *)(base + NA_STATE);
        ws->lookback_bytes = NA_LOOKBACK;
        ws->arena = base + NA_STATE + NA_LOOKBACK;
        ws->arena_bytes = NA_ARENA;
        ws->fixed_lookback = true;
        ws->no_graph = true;
        ws->epoch = 0;
        ws->stream = stream;
        ak_status r = zero_fill(stream, base, NA_STATE + NA_LOOKBACK);
        if (r != AK_OK) return r;
        g_na_ptr[dev] = ptr;
    }
    ws->stream = stream;
    *out = ws;
    return AK_OK;
}

}  // namespace ak

using namespace ak;

extern "C" ak_status ak_sort_noalloc(void *keys, int64_t n, ak_dtype dtype, ak_stream_t stream) {
    set_error("");
    if (!dtype_ok(dtype)) {
        set_error("unknown dtype " + std::to_string((int)dtype));
        return AK_ERR_UNSUPPORTED_DTYPE;
    }
    if (n < 0 || (n > 0 && !keys)) {
        set_error("n < 0, or keys is NULL with n > 0");
        return AK_ERR_INVALID_ARG;
    }
    if ((uint64_t)n * (uint64_t)dtype_bytes(dtype) > (uint64_t)AK_NOALLOC_MAX_KEY_BYTES) {
        set_error("ak_sort_noalloc takes at most " + std::to_string(AK_NOALLOC_MAX_KEY_BYTES) +
                  " bytes of keys (" + std::to_string(n) + " keys given)");
        return AK_ERR_INVALID_ARG;
    }
    if (n == 0) return AK_OK;
    int dev = 0;
    AK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NA_MAX_DEVICES) {
        set_error("device index out of range");
        return AK_ERR_INVALID_ARG;
    }
    Workspace *ws = nullptr;
    ak_status r = na_setup(dev, (hipStream_t)stream, &ws);
    if (r != AK_OK) return r;
    std::lock_guard<std::mutex> lk(g_na_mu);
    ws_begin_call(ws);
    // what the run carves from the arena must fit (it always does for the
    // admitted sizes; checked before any launch all the same)
    const size_t need = radix_temp_bytes(dtype, n, false);
    if (need > NA_LOOKBACK + NA_ARENA) {
        set_error("internal: scratch of this run exceeds the static array");
        return AK_ERR_INTERNAL;
    }
    return radix_sort(ws, dtype, keys, nullptr, n, 0);
}
