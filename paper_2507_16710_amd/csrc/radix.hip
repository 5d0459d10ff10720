// Driver of the LSD radix sort (kernels and launch sequences in
// radix_impl.h): shape choice, scratch sizes, the cached launch graphs of
// small runs, the sort / sortperm runs of the six 32- and 64-bit key types,
// and the code-digit passes of the learned sort.
#include <cstdlib>
#include <map>
#include <mutex>

#include "radix_impl.h"

namespace ak {

// Default pass shapes (OS_DEFAULT, radix_kernels.h) from the tuning sweep
// (per pass, same box): 32-bit keys 16 waves x 16 keys, one tile per
// workgroup (2^28 float32: 1.14 ms; no persistent shape was faster); 32-bit
// keys with indices 16 x 12 persistent (1.94 -> 1.60 ms); 64-bit keys 8 x 24
// persistent (2^30 int64: 7.43 -> 6.07 ms); 64-bit keys with indices 16 x 8
// persistent (2^28 int64: 3.21 -> 2.50 ms).  Large tiles amortise the
// per-tile work (digit scan, look-back, barriers) over more keys and make
// the digit runs of the scatter longer.  Payloads of 8 bytes and 128-bit
// keys take the largest tile whose staging buffer leaves room for a second
// workgroup or the persistent grid.
// Default shape of the code-digit passes per key width.  64-bit keys: a
// 10240-key tile, the largest whose staging buffer still fits the LDS beside
// the 64 KB model table, held by 8 waves x 20 keys (2^31 mixture keys, per
// pass: 16 x 6 keys 20.7 ms, 16 x 8 keys 18.0 ms, 16 x 10 keys 16.1 ms,
// 8 x 20 keys 15.6 ms)
static const int OS_CODE_DEFAULT[2] = {0, 0};

static int env_variant(const char *name) {
    const char *e = getenv(name);
    const int v = (e && *e) ? atoi(e) : -1;
    return v >= 0 && v < OS_NVAR ? v : -1;
}

// Key-only sorts of at most 2^21 keys are bound by launch latency: the
// first shape of the table (16 x 8 keys for 32-bit keys, 16 x 4 for 64-bit
// keys) gives more tiles per pass and was faster there (1M int64 keys: 233
// -> 205 us; 2^20 float32: 140 -> 128 us).  Sortperm keeps its shapes.
constexpr int64_t SMALL_SHAPE_MAX = int64_t(1) << 21;

int os_variant(int dt, int mode, int64_t n) {
    if (os_all_variants(dt, mode)) {
        static const int forced = env_variant("AK_OS_VARIANT");
        if (forced >= 0) return forced;
    }
    if (mode == M_KEYS && n <= SMALL_SHAPE_MAX) return 0;
    return OS_DEFAULT[key_class(dt)][mode_vclass(mode)];
}

int hist_variant() {
    static const int v = [] {
        const int e = env_variant("AK_HIST_VARIANT");
        return e >= 0 ? e : 0;
    }();
    return v;
}

int os_code_variant(int dt) {
    static const int forced = env_variant("AK_OS_CODE_VARIANT");
    return forced >= 0 ? forced : OS_CODE_DEFAULT[key_bits(dt) == 64];
}

int64_t small_sort_capacity(int) { return SMALL_W * 64 * SMALL_IPT; }

size_t radix_temp_bytes_mode(int dt, int mode, int64_t n) {
    if (n <= small_sort_capacity(dt)) return 0;
    const size_t kb = (size_t)dtype_bytes(dt);
    const int tile = os_tile(dt, mode, n);
    const size_t tiles = (size_t)((n + tile - 1) / tile);
    // the look-back words and per-tile counts; two key-sized ping-pong
    // buffers (sort: the second one lets an odd number of passes end in the
    // caller's buffer; sortperm: the const keys are never written), except
    // for the low-memory sortperm, which moves indices only; one index
    // buffer (sortperm) or two payload buffers (sort by key)
    size_t b = al256(lookback_words(tiles) * 8) + al256(rts_bytes(tiles));
    if (mode != M_LOWMEM) b += 2 * al256((size_t)n * kb);
    if (mode == M_PERM || mode == M_LOWMEM) b += al256((size_t)n * 4);
    if (mode == M_PAIRS4 || mode == M_PAIRS8) b += 2 * al256((size_t)n * (mode == M_PAIRS8 ? 8 : 4));
    if (mode == M_KEYS && prefix_dtype(dt) && n > PREFIX_MIN) b += prefix_finish_bytes(dt, n, n <= GRAPH_MAX);
    return b;
}

size_t radix_temp_bytes(int dt, int64_t n, bool perm) { return radix_temp_bytes_mode(dt, perm ? M_PERM : M_KEYS, n); }

size_t code_partition_bytes(int dt, int64_t n) {
    const size_t kb = (size_t)dtype_bytes(dt);
    const size_t tiles = (size_t)((n + os_code_tile(dt) - 1) / os_code_tile(dt));
    return 2 * al256((size_t)n * kb) + al256(lookback_words(tiles) * 8) + al256(rts_bytes(tiles));
}

bool os_rts() {
    static const bool p = [] {
        const char *e = getenv("AK_OS_RTS");
        return e && *e == '1';
    }();
    return p;
}

// Tiles per reduce-then-scan chunk: enough chunks for four workgroups per
// CU, at most 16 tiles each.
uint32_t rts_chunk_tiles(uint32_t tiles) {
    const uint32_t want = (uint32_t)num_cus() * 4;
    return std::max<uint32_t>(1, std::min<uint32_t>(16, (tiles + want - 1) / want));
}

// ------------------------------------------------------- graph replay
struct GraphCache {
    hipStream_t capture = nullptr;
    std::map<GraphKey, hipGraphExec_t> graphs;
};
static std::mutex g_graph_mu;
static std::map<Workspace *, GraphCache> g_graphs;
constexpr size_t GRAPH_CACHE_MAX = 64;

void radix_release(Workspace *ws) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(ws);
    if (it == g_graphs.end()) return;
    for (auto &kv : it->second.graphs) (void)hipGraphExecDestroy(kv.second);
    if (it->second.capture) (void)hipStreamDestroy(it->second.capture);
    g_graphs.erase(it);
}

ak_status graph_run(Workspace *ws, const GraphKey &key, const std::function<ak_status(hipStream_t)> &record) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    GraphCache &c = g_graphs[ws];
    if (!c.capture) AK_HIP(hipStreamCreateWithFlags(&c.capture, hipStreamNonBlocking));
    auto it = c.graphs.find(key);
    if (it == c.graphs.end()) {
        if (c.graphs.size() >= GRAPH_CACHE_MAX) {
            for (auto &kv : c.graphs) (void)hipGraphExecDestroy(kv.second);
            c.graphs.clear();
        }
        hipGraph_t g = nullptr;
        AK_HIP(hipStreamBeginCapture(c.capture, hipStreamCaptureModeRelaxed));
        ak_status lr = record(c.capture);
        hipError_t ce = hipStreamEndCapture(c.capture, &g);
        if (lr != AK_OK) {
            if (g) (void)hipGraphDestroy(g);
            return lr;
        }
        if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate");
        it = c.graphs.emplace(key, ex).first;
    }
    ProfScope ps("radix_graph", ws->stream);
    AK_HIP(hipGraphLaunch(it->second, ws->stream));
    return AK_OK;
}

// ------------------------------------------------------------ entries
template <int DT>
static ak_status std_t(Workspace *ws, void *keys, uint32_t *perm, int64_t n, int slot) {
    if (perm) return radix_sort_t<DT, M_PERM>(ws, keys, perm, n, slot);
    return radix_sort_t<DT, M_KEYS>(ws, keys, nullptr, n, slot);
}

ak_status radix_sort(Workspace *ws, int dt, void *keys, uint32_t *perm, int64_t n, int slot) {
    switch (dt) {
    case AK_I32: return std_t<AK_I32>(ws, keys, perm, n, slot);
    case AK_I64: return std_t<AK_I64>(ws, keys, perm, n, slot);
    case AK_U32: return std_t<AK_U32>(ws, keys, perm, n, slot);
    case AK_U64: return std_t<AK_U64>(ws, keys, perm, n, slot);
    case AK_F32: return std_t<AK_F32>(ws, keys, perm, n, slot);
    case AK_F64: return std_t<AK_F64>(ws, keys, perm, n, slot);
    }
    if (dtype_ok(dt)) return radix_sort_wide(ws, dt, perm ? M_PERM : M_KEYS, keys, perm, n, slot);
    set_error("radix_sort: unknown dtype");
    return AK_ERR_UNSUPPORTED_DTYPE;
}

ak_status radix_sort_mode(Workspace *ws, int dt, int mode, void *keys, void *vals, int64_t n, int slot) {
    if (mode == M_KEYS || mode == M_PERM) return radix_sort(ws, dt, keys, (uint32_t *)vals, n, slot);
    if (dtype_std(dt)) return radix_sort_pairs_std(ws, dt, mode, keys, vals, n, slot);
    return radix_sort_wide(ws, dt, mode, keys, vals, n, slot);
}

// ------------------------------------------- code-digit passes (learned)
// Stable LSD passes over the model code of every key instead of its bits:
// after ceil(cb/8) passes the keys are ordered by code, equal codes in
// input order.
template <int DT>
static ak_status code_partition_t(Workspace *ws, void *keys, uint32_t n, const float *model, int L, int cb,
                                  int slot) {
    using U = typename KT<DT>::U;
    ak_status r;
    if ((r = ws_reserve(ws, &ws->keys0, &ws->keys0_bytes, (size_t)n * sizeof(U))) != AK_OK) return r;
    if ((r = ws_reserve(ws, &ws->keys1, &ws->keys1_bytes, (size_t)n * sizeof(U))) != AK_OK) return r;
    const int TILE = os_code_tile(DT);
    const size_t tiles = (n + TILE - 1) / TILE;
    if ((r = ws_reserve_lookback(ws, lookback_words(tiles) * 8)) != AK_OK) return r;
    if ((r = ws_reserve(ws, &ws->aux[4], &ws->aux_bytes[4], rts_bytes(tiles))) != AK_OK) return r;
    uint32_t epoch;
    if ((r = ws_next_epoch(ws, &epoch)) != AK_OK) return r;
    const int nplaces = (cb + RADIX_BITS - 1) / RADIX_BITS;
    return launch_run<DT, M_KEYS, true>(ws->stream, ws, ws->state + slot, keys, nullptr, n, nplaces, model, cb,
                                        rmi_stage_bytes(L));
}

ak_status code_partition(Workspace *ws, int dt, void *keys, uint32_t n, const float *model, int L, int cb,
                         int slot) {
    switch (dt) {
    case AK_I32: return code_partition_t<AK_I32>(ws, keys, n, model, L, cb, slot);
    case AK_I64: return code_partition_t<AK_I64>(ws, keys, n, model, L, cb, slot);
    case AK_U32: return code_partition_t<AK_U32>(ws, keys, n, model, L, cb, slot);
    case AK_U64: return code_partition_t<AK_U64>(ws, keys, n, model, L, cb, slot);
    case AK_F32: return code_partition_t<AK_F32>(ws, keys, n, model, L, cb, slot);
    case AK_F64: return code_partition_t<AK_F64>(ws, keys, n, model, L, cb, slot);
    }
    return AK_ERR_UNSUPPORTED_DTYPE;
}

}  // namespace ak
