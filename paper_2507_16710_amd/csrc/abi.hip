// The C ABI (include/ak.h): argument checks, per-(device, stream) workspace
// cache, error reporting, and dispatch into the drivers.
#include <algorithm>
#include <cstddef>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "ak_internal.h"
#include "radix_kernels.h"

namespace ak {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

ak_status hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return AK_ERR_HIP;
}

int num_cus() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
        cached[dev] = c;
    }
    return cached[dev];
}

// ------------------------------------------------------------- workspace
static std::mutex g_ws_mu;
static std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;

// Zeroes n 8-byte words at p, then `tail` (< 8) more bytes after them.
__global__ void k_zero_u64(uint64_t *p, size_t n, uint32_t tail) {
    const size_t t0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    for (size_t i = t0; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
    if (t0 < tail) reinterpret_cast<uint8_t *>(p + n)[t0] = 0;
}

ak_status zero_fill(hipStream_t s, void *p, size_t bytes) {
    if (!bytes) return AK_OK;
    const size_t n = bytes / 8;
    const unsigned grid = (unsigned)std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_zero_u64, dim3(grid), dim3(256), 0, s, (uint64_t *)p, n, (uint32_t)(bytes % 8));
    AK_LAUNCH_CHECK("k_zero_u64");
    return AK_OK;
}

Workspace *get_workspace(hipStream_t stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("hipGetDevice failed");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto key = std::make_pair(dev, stream);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) return it->second;
    Workspace *ws = new Workspace();
    ws->device = dev;
    ws->stream = stream;
    const size_t state_bytes = RUN_STATE_BYTES;
    if (hipMalloc((void **)&ws->state, state_bytes) != hipSuccess) {
        set_error("hipMalloc(run state) failed");
        delete ws;
        return nullptr;
    }
    ws->epoch_dev = reinterpret_cast<uint32_t *>(ws->state + RUN_SLOTS);
    if (zero_fill(stream, ws->state, state_bytes) != AK_OK ||
        hipStreamSynchronize(stream) != hipSuccess) {
        (void)hipFree(ws->state);
        delete ws;
        return nullptr;
    }
    g_ws[key] = ws;
    return ws;
}

// Grows *p to at least `need` bytes (rounded up by 1/8 to limit regrowth).
// The old buffer may still be read by queued work, so the stream is drained
// before it is freed.  With a caller arena bound, the buffer is carved from
// it instead (256-byte aligned, in request order; carving restarts at every
// entry point, so one call's buffers must fit together).
ak_status ws_reserve(Workspace *ws, void **p, size_t *have, size_t need) {
    if (need <= *have) return AK_OK;
    if (ws->arena) {
        const size_t off = (ws->arena_used + 255) & ~size_t(255);
        if (off > ws->arena_bytes || need > ws->arena_bytes - off) {
            set_error("workspace arena too small: this call needs at least " + std::to_string(off + need) +
                      " bytes, the arena has " + std::to_string(ws->arena_bytes));
            return AK_ERR_NO_MEMORY;
        }
        void *np = ws->arena + off;
        if (np != *p) ++ws->gen;
        *p = np;
        *have = need;
        ws->arena_used = off + need;
        // other data over the known look-back words
        if (off < ws->arena_lb_off + ws->arena_lb_ok && ws->arena_lb_off < off + need) ws->arena_lb_ok = 0;
        return AK_OK;
    }
    size_t sz = need + need / 8 + 4096;
    if (*p) {
        AK_HIP(hipStreamSynchronize(ws->stream));
        AK_HIP(hipFree(*p));
        *p = nullptr;
        *have = 0;
    }
    if (hipMalloc(p, sz) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error("workspace allocation of " + std::to_string(sz) + " bytes failed");
        return AK_ERR_NO_MEMORY;
    }
    *have = sz;
    ++ws->gen;
    return AK_OK;
}

ak_status ws_reserve_lookback(Workspace *ws, size_t need) {
    if (need <= ws->lookback_bytes) return AK_OK;
    if (ws->fixed_lookback) {
        set_error("look-back region too small for this run");
        return AK_ERR_INTERNAL;
    }
    if (ws->arena) {
        // carved like every arena buffer; zeroed only if these bytes held
        // other data since they last held look-back words
        const size_t off = (ws->arena_used + 255) & ~size_t(255);
        if (off > ws->arena_bytes || need > ws->arena_bytes - off) {
            set_error("workspace arena too small: this call needs at least " + std::to_string(off + need) +
                      " bytes, the arena has " + std::to_string(ws->arena_bytes));
            return AK_ERR_NO_MEMORY;
        }
        uint64_t *np = (uint64_t *)(ws->arena + off);
        if (np != ws->lookback) ++ws->gen;
        ws->lookback = np;
        ws->lookback_bytes = need;
        ws->arena_used = off + need;
        if (off == ws->arena_lb_off && need <= ws->arena_lb_ok) return AK_OK;
        ws->arena_lb_off = off;
        ws->arena_lb_ok = need;
        return zero_fill(ws->stream, ws->lookback, need);
    }
    void *p = ws->lookback;
    size_t have = ws->lookback_bytes;
    ak_status r = ws_reserve(ws, &p, &have, need);
    if (r != AK_OK) return r;
    ws->lookback = (uint64_t *)p;
    ws->lookback_bytes = have;
    return zero_fill(ws->stream, ws->lookback, ws->lookback_bytes);
}

// Each run takes 16 consecutive epochs (one per pass), handed out on the
// device by k_run_init from a counter this function mirrors.  Epochs are
// 30-bit; before they would wrap, the look-back words are cleared and both
// counters restart at 16, so a word left by an earlier run never matches.
ak_status ws_next_epoch(Workspace *ws, uint32_t *epoch) {
    uint32_t e = ws->epoch + 16;
    if (e + 16 >= (1u << 30)) {
        ak_status r = zero_fill(ws->stream, ws->lookback, ws->lookback_bytes);
        if (r != AK_OK) return r;
        e = 16;
    }
    ws->epoch = e;
    *epoch = e;
    return AK_OK;
}

bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st == hipStreamCaptureStatusActive;
}

uint32_t segmented_take_error(Workspace *ws);
void segmented_release(Workspace *ws);
void radix_release(Workspace *ws);

// Forgets every scratch buffer of the workspace, freeing the ones the
// library allocated (arena buffers belong to the caller).
static void drop_buffers(Workspace *ws) {
    void **bufs[] = {&ws->keys0, &ws->keys1, &ws->vals0, &ws->vals1, (void **)&ws->lookback, &ws->misc, &ws->misc2};
    size_t *sizes[] = {&ws->keys0_bytes, &ws->keys1_bytes, &ws->vals0_bytes, &ws->vals1_bytes, &ws->lookback_bytes,
                       &ws->misc_bytes, &ws->misc2_bytes};
    for (int i = 0; i < 7; ++i) {
        if (*bufs[i] && !ws->arena) (void)hipFree(*bufs[i]);
        *bufs[i] = nullptr;
        *sizes[i] = 0;
    }
    for (int i = 0; i < 6; ++i) {
        if (ws->aux[i] && !ws->arena) (void)hipFree(ws->aux[i]);
        ws->aux[i] = nullptr;
        ws->aux_bytes[i] = 0;
    }
    ++ws->gen;
}

// Start of an entry point: with an arena bound, carving restarts at its
// beginning (work queued by earlier calls on the stream runs first, so
// reusing the bytes is safe in stream order).  Pointers are kept so that a
// buffer carved at the same place again keeps its cached graphs.
void ws_begin_call(Workspace *ws) {
    ws->last_route = 0;
    if (!ws->arena) return;
    ws->arena_used = 0;
    ws->keys0_bytes = ws->keys1_bytes = ws->vals0_bytes = ws->vals1_bytes = 0;
    if (!ws->fixed_lookback) ws->lookback_bytes = 0;
    ws->misc_bytes = ws->misc2_bytes = 0;
    for (size_t &b : ws->aux_bytes) b = 0;
}

// With a caller arena bound, a call whose scratch cannot fit fails before
// it launches anything.
ak_status ws_arena_fits(Workspace *ws, size_t need) {
    if (!ws->arena || need <= ws->arena_bytes) return AK_OK;
    set_error("workspace arena too small: this call needs " + std::to_string(need) + " bytes, the arena has " +
              std::to_string(ws->arena_bytes));
    return AK_ERR_NO_MEMORY;
}

static void free_ws(Workspace *ws) {
    segmented_release(ws);
    radix_release(ws);
    drop_buffers(ws);
    if (ws->state) (void)hipFree(ws->state);
    delete ws;
}

}  // namespace ak

using namespace ak;

// ------------------------------------------------------------- checks
static bool overlaps(const void *a, size_t an, const void *b, size_t bn) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + bn && y < x + an;
}

// `wide`: the entry point takes the 16- and 128-bit key types too.
static ak_status check_keys(const void *keys, int64_t n, int dtype, bool wide = false) {
    if (wide ? !dtype_ok(dtype) : !dtype_std(dtype)) {
        set_error("unknown dtype " + std::to_string(dtype));
        return AK_ERR_UNSUPPORTED_DTYPE;
    }
    if (n < 0) {
        set_error("n < 0");
        return AK_ERR_INVALID_ARG;
    }
    if (n > AK_MAX_KEYS) {
        set_error("n > 2^31 keys is not supported (indices and grid-stride loops are 32-bit)");
        return AK_ERR_INVALID_ARG;
    }
    if (n > 0 && !keys) {
        set_error("keys is NULL");
        return AK_ERR_INVALID_ARG;
    }
    return AK_OK;
}

static Workspace *ws_or_error(ak_stream_t stream, ak_status *st) {
    Workspace *ws = get_workspace((hipStream_t)stream);
    *st = ws ? AK_OK : AK_ERR_HIP;
    if (ws) ws_begin_call(ws);
    return ws;
}

extern "C" {

const char *ak_status_string(ak_status s) {
    switch (s) {
    case AK_OK: return "ok";
    case AK_ERR_INVALID_ARG: return "invalid argument";
    case AK_ERR_UNSUPPORTED_DTYPE: return "unsupported dtype";
    case AK_ERR_NO_MEMORY: return "out of device memory";
    case AK_ERR_HIP: return "HIP runtime error";
    case AK_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char *ak_last_error(void) { return g_last_error.c_str(); }

ak_status ak_sort_route(int64_t *info, ak_stream_t stream) {
    g_last_error.clear();
    if (!info) {
        set_error("info is NULL");
        return AK_ERR_INVALID_ARG;
    }
    for (int i = 0; i < 5; ++i) info[i] = 0;
    Workspace *ws = get_workspace((hipStream_t)stream);
    if (!ws) return AK_ERR_HIP;
    AK_HIP(hipStreamSynchronize(ws->stream));
    if (ws->last_route == 0) return AK_OK;
    RunState st;   // the fields before the digit counts
    AK_HIP(hipMemcpy(&st, ws->state, offsetof(RunState, hist), hipMemcpyDeviceToHost));
    info[0] = st.pfx_active ? (int64_t)st.pfx_places : 0;
    info[1] = st.q;
    if (ws->last_route == 2 && st.pfx_active) return prefix_counts(ws, info + 2);
    return AK_OK;
}

ak_status ak_sort(void *keys, int64_t n, ak_dtype dtype, ak_stream_t stream) {
    g_last_error.clear();
    ak_status r = check_keys(keys, n, dtype, true);
    if (r != AK_OK || n == 0) return r;
    Workspace *ws = ws_or_error(stream, &r);
    if (!ws) return r;
    if ((r = ws_arena_fits(ws, radix_temp_bytes(dtype, n, false))) != AK_OK) return r;
    return radix_sort(ws, dtype, keys, nullptr, n, 0);
}

ak_status ak_sortperm(const void *keys, uint32_t *perm, int64_t n, ak_dtype dtype, ak_stream_t stream) {
    g_last_error.clear();
    ak_status r = check_keys(keys, n, dtype, true);
    if (r != AK_OK) return r;
    if (n > 0 && !perm) {
        set_error("perm is NULL");
        return AK_ERR_INVALID_ARG;
    }
    if (n == 0) return AK_OK;
    if (overlaps(keys, (size_t)n * dtype_bytes(dtype), perm, (size_t)n * 4)) {
        set_error("perm overlaps keys");
        return AK_ERR_INVALID_ARG;
    }
    Workspace *ws = ws_or_error(stream, &r);
    if (!ws) return r;
    if ((r = ws_arena_fits(ws, radix_temp_bytes(dtype, n, true))) != AK_OK) return r;
    return radix_sort(ws, dtype, const_cast<void *>(keys), perm, n, 0);
}

// Sortperm with the smallest scratch (indices only); same checks and result.
ak_status ak_sortperm_lowmem(const void *keys, uint32_t *perm, int64_t n, ak_dtype dtype, ak_stream_t stream) {
    g_last_error.clear();
    ak_status r = check_keys(keys, n, dtype, true);
    if (r != AK_OK) return r;
    if (n > 0 && !perm) {
        set_error("perm is NULL");
        return AK_ERR_INVALID_ARG;
    }
    if (n == 0) return AK_OK;
    if (overlaps(keys, (size_t)n * dtype_bytes(dtype), perm, (size_t)n * 4)) {
        set_error("perm overlaps keys");
        return AK_ERR_INVALID_ARG;
    }
    Workspace *ws = ws_or_error(stream, &r);
    if (!ws) return r;
    if ((r = ws_arena_fits(ws, radix_temp_bytes_mode(dtype, M_LOWMEM, n))) != AK_OK) return r;
    return radix_sort_mode(ws, dtype, M_LOWMEM, const_cast<void *>(keys), perm, n, 0);
}

ak_status ak_sort_by_key(void *keys, void *vals, int64_t n, ak_dtype dtype, int32_t val_bytes, ak_stream_t stream) {
    g_last_error.clear();
    ak_status r = check_keys(keys, n, dtype, true);
    if (r != AK_OK) return r;
    if (val_bytes != 4 && val_bytes != 8) {
        set_error("val_bytes must be 4 or 8");
        return AK_ERR_INVALID_ARG;
    }
    if (n > 0 && !vals) {
        set_error("vals is NULL");
        return AK_ERR_INVALID_ARG;
    }
    if (n == 0) return AK_OK;
    if (overlaps(keys, (size_t)n * dtype_bytes(dtype), vals, (size_t)n * (size_t)val_bytes)) {
        set_error("vals overlaps keys");
        return AK_ERR_INVALID_ARG;
    }
    const int mode = val_bytes == 8 ? M_PAIRS8 : M_PAIRS4;
    Workspace *ws = ws_or_error(stream, &r);
    if (!ws) return r;
    if ((r = ws_arena_fits(ws, radix_temp_bytes_mode(dtype, mode, n))) != AK_OK) return r;
    return radix_sort_mode(ws, dtype, mode, keys, vals, n, 0);
}

#define AK_PERM_T(SUF, T, DT)                                                              \
    ak_status ak_sortperm_##SUF(const T *keys, uint32_t *perm, int64_t n, ak_stream_t s) { \
        return ak_sortperm(keys, perm, n, DT, s);                                          \
    }
AK_PERM_T(i32, int32_t, AK_I32)
AK_PERM_T(i64, int64_t, AK_I64)
AK_PERM_T(u32, uint32_t, AK_U32)
AK_PERM_T(u64, uint64_t, AK_U64)
AK_PERM_T(f32, float, AK_F32)
AK_PERM_T(f64, double, AK_F64)

static ak_status search_entry(const void *v, int64_t n, const void *x, int64_t m, ak_dtype dtype, int64_t *out,
                              ak_stream_t stream, bool last) {
    g_last_error.clear();
    if (!dtype_std(dtype)) {
        set_error("unknown dtype " + std::to_string(dtype));
        return AK_ERR_UNSUPPORTED_DTYPE;
    }
    if (n < 0 || m < 0) {
        set_error("n < 0 or m < 0");
        return AK_ERR_INVALID_ARG;
    }
    if (n >= (int64_t(1) << 40)) {
        set_error("n >= 2^40 is not supported");
        return AK_ERR_INVALID_ARG;
    }
    if (m == 0) return AK_OK;
    if (!x || !out || (n > 0 && !v)) {
        set_error("sorted, keys or out is NULL");
        return AK_ERR_INVALID_ARG;
    }
    const size_t kb = (size_t)dtype_bytes(dtype);
    if (overlaps(out, (size_t)m * 8, x, (size_t)m * kb) || (n > 0 && overlaps(out, (size_t)m * 8, v, (size_t)n * kb))) {
        set_error("out overlaps sorted or keys");
        return AK_ERR_INVALID_ARG;
    }
    return search_sorted((hipStream_t)stream, dtype, v, n, x, m, last, out);
}

ak_status ak_accumulate(const void *in, void *out, int64_t n, ak_dtype dtype, int32_t inclusive,
                        ak_stream_t stream) {
    g_last_error.clear();
    ak_status r = check_keys(in, n, dtype);
    if (r != AK_OK || n == 0) return r;
    if (!out) {
        set_error("out is NULL");
        return AK_ERR_INVALID_ARG;
    }
    const size_t bytes = (size_t)n * dtype_bytes(dtype);
    if (out != in && overlaps(in, bytes, out, bytes)) {
        set_error("out overlaps in without being equal to it");
        return AK_ERR_INVALID_ARG;
    }
    Workspace *ws = ws_or_error(stream, &r);
    if (!ws) return r;
    if ((r = ws_arena_fits(ws, accumulate_temp_bytes(n))) != AK_OK) return r;
    return accumulate(ws, dtype, in, out, n, inclusive != 0);
}

ak_status ak_searchsortedfirst(const void *sorted, int64_t n, const void *keys, int64_t m, ak_dtype dtype,
                               int64_t *out, ak_stream_t stream) {
    return search_entry(sorted, n, keys, m, dtype, out, stream, false);
}

ak_status ak_searchsortedlast(const void *sorted, int64_t n, const void *keys, int64_t m, ak_dtype dtype,
                              int64_t *out, ak_stream_t stream) {
    return search_entry(sorted, n, keys, m, dtype, out, stream, true);
}

ak_status ak_segmented_sort(void *keys, const int64_t *offsets, int64_t nseg, ak_dtype dtype, ak_stream_t stream) {
    g_last_error.clear();
    if (!dtype_std(dtype)) {
        set_error("unknown dtype");
        return AK_ERR_UNSUPPORTED_DTYPE;
    }
    if (nseg < 0) {
        set_error("nseg < 0");
        return AK_ERR_INVALID_ARG;
    }
    if (nseg == 0) return AK_OK;
    if (!offsets || !keys) {
        set_error("keys or offsets is NULL");
        return AK_ERR_INVALID_ARG;
    }
    ak_status r;
    Workspace *ws = ws_or_error(stream, &r);
    if (!ws) return r;
    return segmented_sort(ws, dtype, keys, offsets, nseg);
}

ak_status ak_segmented_sort_n(void *keys, int64_t n, const int64_t *offsets, int64_t nseg, ak_dtype dtype,
                              ak_stream_t stream) {
    g_last_error.clear();
    if (!dtype_std(dtype)) {
        set_error("unknown dtype");
        return AK_ERR_UNSUPPORTED_DTYPE;
    }
    if (nseg < 0 || n < 0 || n > AK_MAX_KEYS) {
        set_error("nseg < 0, n < 0 or n > 2^31");
        return AK_ERR_INVALID_ARG;
    }
    if (nseg == 0 || n == 0) return AK_OK;
    if (!offsets || !keys) {
        set_error("keys or offsets is NULL");
        return AK_ERR_INVALID_ARG;
    }
    ak_status r;
    Workspace *ws = ws_or_error(stream, &r);
    if (!ws) return r;
    return segmented_sort_n(ws, dtype, keys, n, offsets, nseg);
}

#define AK_SEG_T(SUF, T, DT)                                                                  \
    ak_status ak_segmented_sort_##SUF(T *keys, const int64_t *off, int64_t nseg, ak_stream_t s) { \
        return ak_segmented_sort(keys, off, nseg, DT, s);                                     \
    }
AK_SEG_T(i32, int32_t, AK_I32)
AK_SEG_T(i64, int64_t, AK_I64)
AK_SEG_T(u32, uint32_t, AK_U32)
AK_SEG_T(u64, uint64_t, AK_U64)
AK_SEG_T(f32, float, AK_F32)
AK_SEG_T(f64, double, AK_F64)

ak_status ak_check_device_error(ak_stream_t stream) {
    g_last_error.clear();
    ak_status r;
    Workspace *ws = ws_or_error(stream, &r);
    if (!ws) return r;
    AK_HIP(hipStreamSynchronize(ws->stream));
    uint32_t flag = 0;
    for (int slot = 0; slot < RUN_SLOTS; ++slot) {
        uint32_t f = 0;
        AK_HIP(hipMemcpy(&f, &ws->state[slot].error, sizeof(f), hipMemcpyDeviceToHost));
        flag |= f;
    }
    flag |= segmented_take_error(ws);
    if (flag) {
        const uint32_t zero = 0;
        for (int slot = 0; slot < RUN_SLOTS; ++slot)
            AK_HIP(hipMemcpy(&ws->state[slot].error, &zero, sizeof(zero), hipMemcpyHostToDevice));
        set_error("a kernel found invalid input (decreasing segment offsets)");
        return AK_ERR_INVALID_ARG;
    }
    return AK_OK;
}

static ak_learned_cfg resolve_cfg(const ak_learned_cfg *cfg) {
    ak_learned_cfg c{};
    if (cfg) c = *cfg;
    if (c.leaves <= 0) c.leaves = 4096;
    if (c.buckets_log2 <= 0) c.buckets_log2 = 12;
    if (!(c.sample_frac > 0.f)) c.sample_frac = 0.01f;
    if (c.train_iters <= 0) c.train_iters = c.model == AK_MODEL_MLP ? 300 : 3;
    return c;
}

ak_status ak_sort_learned(void *keys, int64_t n, ak_dtype dtype, const ak_learned_cfg *cfg,
                          ak_learned_stats *stats, ak_stream_t stream) {
    g_last_error.clear();
    ak_status r = check_keys(keys, n, dtype);
    if (r != AK_OK) return r;
    ak_learned_cfg c = resolve_cfg(cfg);
    if (c.leaves > 65536 || (c.leaves & (c.leaves - 1)) || c.buckets_log2 > 14 || c.sample_frac > 1.f ||
        (c.model != AK_MODEL_RMI && c.model != AK_MODEL_MLP) ||
        (c.model == AK_MODEL_MLP && (c.leaves > 16384 || c.train_iters > 100000))) {
        set_error("bad learned config (leaves: power of two <= 65536, <= 16384 for the MLP; buckets_log2 <= 14; "
                  "sample_frac <= 1; model RMI or MLP; MLP steps <= 100000)");
        return AK_ERR_INVALID_ARG;
    }
    if (n == 0) {
        if (stats) *stats = ak_learned_stats{};
        return AK_OK;
    }
    Workspace *ws = ws_or_error(stream, &r);
    if (!ws) return r;
    if ((r = ws_arena_fits(ws, learned_temp_bytes(dtype, n, &c))) != AK_OK) return r;
    return learned_sort(ws, dtype, keys, n, &c, stats);
}

ak_status ak_mlp_loss_grad(const float *u, const float *y, int64_t K, const float *params, float *out,
                           ak_stream_t stream) {
    g_last_error.clear();
    if (K < 1 || K > (int64_t(1) << 20) || !u || !y || !params || !out) {
        set_error("bad arguments (1 <= K <= 2^20, non-NULL pointers)");
        return AK_ERR_INVALID_ARG;
    }
    ak_status r;
    Workspace *ws = ws_or_error(stream, &r);
    if (!ws) return r;
    return mlp_loss_grad(ws, u, y, K, params, out);
}

ak_status ak_mlp_fit(const void *sorted_sample, int64_t m, ak_dtype dtype, int32_t iters, int32_t leaves,
                     float *params, float *model, ak_stream_t stream) {
    g_last_error.clear();
    ak_status r = check_keys(sorted_sample, m, dtype);
    if (r != AK_OK) return r;
    if (m < 1 || !model || leaves < 1 || leaves > 16384 || (leaves & (leaves - 1)) || iters < 0 ||
        iters > 100000) {
        set_error("bad arguments (m >= 1, model non-NULL, leaves a power of two <= 16384, 0 <= iters <= 100000)");
        return AK_ERR_INVALID_ARG;
    }
    Workspace *ws = ws_or_error(stream, &r);
    if (!ws) return r;
    return mlp_fit(ws, dtype, sorted_sample, m, leaves, iters, model, params);
}

size_t ak_rmi_model_floats(int32_t leaves) { return leaves > 0 ? 8 + 4 * ((size_t)leaves + 1) : 0; }

ak_status ak_learned_sample(const void *keys, int64_t n, ak_dtype dtype, uint64_t seed, int64_t m, void *out,
                            ak_stream_t stream) {
    g_last_error.clear();
    ak_status r = check_keys(keys, n, dtype);
    if (r != AK_OK) return r;
    if (m < 0 || (m > 0 && (!out || n == 0)) || m > AK_MAX_KEYS) {
        set_error("bad sample size or output");
        return AK_ERR_INVALID_ARG;
    }
    if (m == 0) return AK_OK;
    return learned_sample((hipStream_t)stream, dtype, keys, n, seed, m, out);
}

ak_status ak_rmi_fit(const void *sorted_sample, int64_t m, ak_dtype dtype, int32_t leaves, int32_t iters,
                     float *model, ak_stream_t stream) {
    g_last_error.clear();
    ak_status r = check_keys(sorted_sample, m, dtype);
    if (r != AK_OK) return r;
    if (m == 0 || !model || leaves <= 0 || leaves > 65536 || (leaves & (leaves - 1)) || iters < 0) {
        set_error("bad model arguments (m > 0, leaves a power of two <= 65536, iters >= 0)");
        return AK_ERR_INVALID_ARG;
    }
    Workspace *ws = ws_or_error(stream, &r);
    if (!ws) return r;
    return rmi_fit(ws, dtype, sorted_sample, m, leaves, iters, model);
}

ak_status ak_rmi_leaf_grad(const void *sorted_sample, int64_t m, ak_dtype dtype, const float *model, float *out,
                           ak_stream_t stream) {
    g_last_error.clear();
    ak_status r = check_keys(sorted_sample, m, dtype);
    if (r != AK_OK) return r;
    if (m == 0 || !model || !out) {
        set_error("bad arguments");
        return AK_ERR_INVALID_ARG;
    }
    Workspace *ws = ws_or_error(stream, &r);
    if (!ws) return r;
    return rmi_leaf_grad(ws, dtype, sorted_sample, m, model, out);
}

ak_status ak_rmi_codes(const void *keys, int64_t n, ak_dtype dtype, const float *model, int32_t code_bits,
                       uint32_t *codes, ak_stream_t stream) {
    g_last_error.clear();
    ak_status r = check_keys(keys, n, dtype);
    if (r != AK_OK) return r;
    if (code_bits < 1 || code_bits > 24 || (n > 0 && (!model || !codes))) {
        set_error("bad arguments (1 <= code_bits <= 24)");
        return AK_ERR_INVALID_ARG;
    }
    if (n == 0) return AK_OK;
    return rmi_codes((hipStream_t)stream, dtype, keys, n, model, code_bits, codes);
}

size_t ak_temp_bytes(ak_op op, int64_t n, ak_dtype dtype) {
    if (!dtype_ok(dtype) || n <= 0) return 0;
    switch (op) {
    case AK_OP_SORT: return radix_temp_bytes(dtype, n, false);
    case AK_OP_SORTPERM: return radix_temp_bytes(dtype, n, true);
    case AK_OP_SORT_BY_KEY: return radix_temp_bytes_mode(dtype, M_PAIRS8, n);
    case AK_OP_SORTPERM_LOWMEM: return radix_temp_bytes_mode(dtype, M_LOWMEM, n);
    default: break;
    }
    if (!dtype_std(dtype)) return 0;
    switch (op) {
    case AK_OP_SEGMENTED: return segmented_temp_bytes(dtype, n, n);
    case AK_OP_LEARNED: {
        ak_learned_cfg c = resolve_cfg(nullptr);
        return learned_temp_bytes(dtype, n, &c);
    }
    case AK_OP_ACCUMULATE: return accumulate_temp_bytes(n);
    default: break;
    }
    return 0;
}

size_t ak_temp_bytes_segmented(int64_t n, int64_t nseg, ak_dtype dtype) {
    if (!dtype_std(dtype) || n <= 0 || nseg <= 0) return 0;
    return segmented_temp_bytes(dtype, n, nseg);
}

ak_status ak_set_workspace(void *dev_ptr, size_t bytes, ak_stream_t stream) {
    if (!dev_ptr && bytes) {
        set_error("dev_ptr is NULL but bytes > 0");
        return AK_ERR_INVALID_ARG;
    }
    if (dev_ptr && ((uintptr_t)dev_ptr & 255u)) {
        set_error("the workspace arena must be 256-byte aligned");
        return AK_ERR_INVALID_ARG;
    }
    if (dev_ptr && bytes < 4096) {
        set_error("the workspace arena must hold at least 4096 bytes");
        return AK_ERR_INVALID_ARG;
    }
    Workspace *ws = get_workspace((hipStream_t)stream);
    if (!ws) return AK_ERR_HIP;
    // queued work may still use the current buffers
    AK_HIP(hipStreamSynchronize(ws->stream));
    drop_buffers(ws);
    ws->arena = (char *)dev_ptr;
    ws->arena_bytes = dev_ptr ? bytes : 0;
    ws->arena_used = 0;
    ws->arena_lb_off = ws->arena_lb_ok = 0;
    return AK_OK;
}

ak_status ak_release_workspace(void) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    AK_HIP(hipDeviceSynchronize());
    for (auto &kv : g_ws) free_ws(kv.second);
    g_ws.clear();
    return AK_OK;
}

}  // extern "C"
