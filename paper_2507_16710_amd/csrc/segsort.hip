// Batched segmented sort: every segment [off[s], off[s+1]) sorted on its own,
// all segments in one persistent launch.
//
// Segments are binned by length into work buckets processed largest first:
//   long   (> b_max keys)         one workgroup, multi-pass LSD radix through
//                                 a scratch copy (one bucket per power of two,
//                                 longest first, so the tail is short ones)
//   medium (a_max < len <= b_max) one workgroup, on-chip sort
//   short  (2 <= len <= a_max)    one wave per segment, on-chip sort
// The tile shapes (keys per lane of the short and medium classes) are
// template variants chosen from a tuning table written by the autotuner;
// the class limits and the persistent grid are runtime knobs of the same
// table.  The launch sequence (reset, count, scan, place, sort) is captured
// once per (dtype, segment count, tuning) into a HIP graph and replayed; the
// kernels read every pointer from a device-side argument block that a tiny
// kernel rewrites before each replay.
#include <dlfcn.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "lds_sort.h"
#include "long_sort.h"

namespace ak {

constexpr int SEG_W = 4;              // waves of a persistent workgroup
constexpr int NB_LONG = 24;           // long buckets: 31 - floor(log2(len))
constexpr int B_MED = NB_LONG;        // medium bucket
constexpr int B_SHORT = NB_LONG + 1;  // short bucket
constexpr int NB = NB_LONG + 2;

struct SegArgs {
    void *keys;
    const int64_t *off;
    void *tmp;          // scratch, same layout as keys[off[0] ..)
    int32_t *list;      // segment ids, grouped by bucket
    int64_t nseg;
    int64_t base;       // off[0]
    int64_t end;        // off[nseg]
    uint32_t a_max, b_max;
};

struct SegState {
    uint32_t count[NB];
    uint32_t start[NB + 1];
    uint32_t cursor[NB];
    uint32_t next_item;
    uint32_t nitems;
    uint32_t error;
};

struct SegTune {
    int ipt_a = 4;      // short class: 64*ipt_a keys per wave
    int ipt_b = 16;     // medium class and long-class tiles: 256*ipt_b keys
    int grid_mult = 4;  // persistent workgroups per CU
    int b_max = 0;      // 0: the medium capacity
};

__device__ __forceinline__ int seg_bucket(uint32_t len, uint32_t a_max, uint32_t b_max) {
    if (len <= 1) return -1;
    if (len <= a_max) return B_SHORT;
    if (len <= b_max) return B_MED;
    const int lg = 31 - __builtin_clz(len);
    return 31 - lg < NB_LONG ? 31 - lg : NB_LONG - 1;
}

__global__ void k_seg_setargs(SegArgs *a, SegArgs v) { *a = v; }

__global__ void k_seg_reset(SegState *st) {
    const int t = threadIdx.x;
    if (t < NB) {
        st->count[t] = 0;
        st->cursor[t] = 0;
    }
    if (t == 0) {
        st->next_item = 0;
        st->nitems = 0;
    }
}

__global__ __launch_bounds__(256) void k_seg_count(const SegArgs *ap, SegState *st) {
    const SegArgs a = *ap;
    __shared__ uint32_t s_c[NB];
    if (threadIdx.x < NB) s_c[threadIdx.x] = 0;
    __syncthreads();
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s < a.nseg) {
        const int64_t lo = a.off[s], hi = a.off[s + 1];
        if (hi < lo || lo < a.base || hi > a.end) {
            atomicOr(&st->error, 1u);
        } else {
            const int b = seg_bucket((uint32_t)(hi - lo), a.a_max, a.b_max);
            if (b >= 0) atomicAdd(&s_c[b], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < NB && s_c[threadIdx.x]) atomicAdd(&st->count[threadIdx.x], s_c[threadIdx.x]);
}

__global__ void k_seg_scan(SegState *st) {
    if (threadIdx.x != 0) return;
    uint32_t run = 0;
    for (int b = 0; b < NB; ++b) {
        st->start[b] = run;
        run += st->count[b];
    }
    st->start[NB] = run;
    // short segments are taken SEG_W at a time (one per wave)
    st->nitems = st->start[B_SHORT] + (st->count[B_SHORT] + SEG_W - 1) / SEG_W;
}

__global__ __launch_bounds__(256) void k_seg_place(const SegArgs *ap, SegState *st) {
    const SegArgs a = *ap;
    __shared__ uint32_t s_c[NB], s_base[NB];
    if (threadIdx.x < NB) s_c[threadIdx.x] = 0;
    __syncthreads();
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int b = -1;
    uint32_t mine = 0;
    if (s < a.nseg) {
        const int64_t lo = a.off[s], hi = a.off[s + 1];
        if (hi >= lo && lo >= a.base && hi <= a.end) b = seg_bucket((uint32_t)(hi - lo), a.a_max, a.b_max);
        if (b >= 0) mine = atomicAdd(&s_c[b], 1u);
    }
    __syncthreads();
    if (threadIdx.x < NB && s_c[threadIdx.x])
        s_base[threadIdx.x] = atomicAdd(&st->cursor[threadIdx.x], s_c[threadIdx.x]);
    __syncthreads();
    if (b >= 0) a.list[st->start[b] + s_base[b] + mine] = (int32_t)s;
}

template <typename U, int IPT_A, int IPT_B>
union SegSmem {
    SmallSmem<U, false, SEG_W, IPT_B> med;
    SmallSmem<U, false, 1, IPT_A> shrt[SEG_W];
    LongSmem<U, SEG_W, IPT_B> lng;
};

template <int DT, int IPT_A, int IPT_B>
__global__ __launch_bounds__(SEG_W * 64) void k_seg_sort(const SegArgs *ap, SegState *st) {
    using U = typename KT<DT>::U;
    __shared__ SegSmem<U, IPT_A, IPT_B> sm;
    __shared__ uint32_t s_item;
    const SegArgs a = *ap;
    U *keys = (U *)a.keys;
    U *tmp = (U *)a.tmp;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t nitems = st->nitems;
    const uint32_t med0 = st->start[B_MED], short0 = st->start[B_SHORT], nshort = st->count[B_SHORT];
    while (true) {
        if (tid == 0) s_item = atomicAdd(&st->next_item, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= nitems) break;
        if (item < short0) {
            const int64_t s = a.list[item];
            const int64_t lo = a.off[s], len = a.off[s + 1] - lo;
            if (item < med0)
                sort_long<DT, SEG_W, IPT_B>(keys + lo, tmp + (lo - a.base), (uint32_t)len, sm.lng);
            else
                lds_sort_tile<DT, false, SEG_W, IPT_B>(keys + lo, keys + lo, nullptr, (uint32_t)len, sm.med, tid);
        } else {
            const uint32_t g = (item - short0) * SEG_W + w;
            if (g < nshort) {
                const int64_t s = a.list[short0 + g];
                const int64_t lo = a.off[s], len = a.off[s + 1] - lo;
                lds_sort_tile<DT, false, 1, IPT_A>(keys + lo, keys + lo, nullptr, (uint32_t)len, sm.shrt[w], lane);
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ tuning
static std::mutex g_tune_mu;
static SegTune g_tune[2];  // [0]: 32-bit keys, [1]: 64-bit keys
static bool g_tune_loaded = false;

static int json_int(const std::string &txt, const std::string &obj, const char *field, int dflt) {
    const size_t o = txt.find("\"" + obj + "\"");
    if (o == std::string::npos) return dflt;
    const size_t e = txt.find('}', o);
    const size_t f = txt.find(std::string("\"") + field + "\"", o);
    if (f == std::string::npos || f > e) return dflt;
    const size_t c = txt.find(':', f);
    if (c == std::string::npos) return dflt;
    return atoi(txt.c_str() + c + 1);
}

// Reads the tuning table: $AK_TUNE_TABLE, else tune_gfx950.json next to
// libak.so.  Missing file or fields keep the built-in defaults.
static void load_tune_table() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    std::string path;
    if (const char *env = getenv("AK_TUNE_TABLE")) path = env;
    if (path.empty()) {
        Dl_info info;
        if (dladdr((void *)&load_tune_table, &info) && info.dli_fname) {
            std::string so = info.dli_fname;
            path = so.substr(0, so.find_last_of('/') + 1) + "tune_gfx950.json";
        }
    }
    FILE *f = path.empty() ? nullptr : fopen(path.c_str(), "rb");
    if (!f) return;
    std::string txt;
    char buf[4096];
    size_t r;
    while ((r = fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, r);
    fclose(f);
    const char *names[2] = {"seg32", "seg64"};
    for (int i = 0; i < 2; ++i) {
        g_tune[i].ipt_a = json_int(txt, names[i], "ipt_a", g_tune[i].ipt_a);
        g_tune[i].ipt_b = json_int(txt, names[i], "ipt_b", g_tune[i].ipt_b);
        g_tune[i].grid_mult = json_int(txt, names[i], "grid_mult", g_tune[i].grid_mult);
        g_tune[i].b_max = json_int(txt, names[i], "b_max", g_tune[i].b_max);
    }
}

static bool tune_valid(int kb, const SegTune &t) {
    const bool a_ok = t.ipt_a == 2 || t.ipt_a == 4;
    const bool b_ok = t.ipt_b == 8 || t.ipt_b == 16 || (kb == 32 && t.ipt_b == 32);
    return a_ok && b_ok && t.grid_mult >= 1 && t.grid_mult <= 16 && t.b_max >= 0;
}

}  // namespace ak

// Sets the segmented-sort tuning for 32- or 64-bit keys (autotuner hook).
extern "C" ak_status ak_seg_set_tuning(int key_bits, int ipt_a, int ipt_b, int grid_mult, int b_max) {
    using namespace ak;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_table();
    SegTune t{ipt_a, ipt_b, grid_mult, b_max};
    if ((key_bits != 32 && key_bits != 64) || !tune_valid(key_bits, t)) {
        set_error("invalid segmented-sort tuning");
        return AK_ERR_INVALID_ARG;
    }
    g_tune[key_bits == 64] = t;
    return AK_OK;
}

namespace ak {

struct SegPlanKey {
    int dtype;
    int64_t nseg;
    int ipt_a, ipt_b, grid;
    bool operator<(const SegPlanKey &o) const {
        return std::tie(dtype, nseg, ipt_a, ipt_b, grid) < std::tie(o.dtype, o.nseg, o.ipt_a, o.ipt_b, o.grid);
    }
};

struct SegCache {
    SegArgs *args = nullptr;
    SegState *state = nullptr;
    hipStream_t capture = nullptr;
    std::map<SegPlanKey, hipGraphExec_t> graphs;
};
static std::mutex g_seg_mu;
static std::map<Workspace *, SegCache> g_seg;

template <int DT, int IA, int IB>
static void launch_sort_kernel(dim3 grid, hipStream_t s, const SegArgs *a, SegState *st) {
    hipLaunchKernelGGL((k_seg_sort<DT, IA, IB>), grid, dim3(SEG_W * 64), 0, s, a, st);
}

template <int DT>
static ak_status launch_seg_sort(const SegTune &t, dim3 grid, hipStream_t s, const SegArgs *a, SegState *st) {
    if (t.ipt_a == 2 && t.ipt_b == 8) launch_sort_kernel<DT, 2, 8>(grid, s, a, st);
    else if (t.ipt_a == 2 && t.ipt_b == 16) launch_sort_kernel<DT, 2, 16>(grid, s, a, st);
    else if (t.ipt_a == 4 && t.ipt_b == 8) launch_sort_kernel<DT, 4, 8>(grid, s, a, st);
    else if (t.ipt_a == 4 && t.ipt_b == 16) launch_sort_kernel<DT, 4, 16>(grid, s, a, st);
    else if constexpr (key_bits(DT) == 32) {
        if (t.ipt_a == 2 && t.ipt_b == 32) launch_sort_kernel<DT, 2, 32>(grid, s, a, st);
        else if (t.ipt_a == 4 && t.ipt_b == 32) launch_sort_kernel<DT, 4, 32>(grid, s, a, st);
        else return AK_ERR_INTERNAL;
    } else {
        return AK_ERR_INTERNAL;
    }
    AK_LAUNCH_CHECK("k_seg_sort");
    return AK_OK;
}

static ak_status seg_launch_all(int dt, const SegTune &t, int64_t nseg, int grid, hipStream_t s, SegArgs *a,
                                SegState *st) {
    const unsigned g = (unsigned)((nseg + 255) / 256);
    hipLaunchKernelGGL(k_seg_reset, dim3(1), dim3(64), 0, s, st);
    AK_LAUNCH_CHECK("k_seg_reset");
    hipLaunchKernelGGL(k_seg_count, dim3(g), dim3(256), 0, s, a, st);
    AK_LAUNCH_CHECK("k_seg_count");
    hipLaunchKernelGGL(k_seg_scan, dim3(1), dim3(64), 0, s, st);
    AK_LAUNCH_CHECK("k_seg_scan");
    hipLaunchKernelGGL(k_seg_place, dim3(g), dim3(256), 0, s, a, st);
    AK_LAUNCH_CHECK("k_seg_place");
    switch (dt) {
    case AK_I32: return launch_seg_sort<AK_I32>(t, dim3(grid), s, a, st);
    case AK_I64: return launch_seg_sort<AK_I64>(t, dim3(grid), s, a, st);
    case AK_U32: return launch_seg_sort<AK_U32>(t, dim3(grid), s, a, st);
    case AK_U64: return launch_seg_sort<AK_U64>(t, dim3(grid), s, a, st);
    case AK_F32: return launch_seg_sort<AK_F32>(t, dim3(grid), s, a, st);
    case AK_F64: return launch_seg_sort<AK_F64>(t, dim3(grid), s, a, st);
    }
    return AK_ERR_UNSUPPORTED_DTYPE;
}

size_t segmented_temp_bytes(int dt, int64_t n, int64_t nseg) {
    return (size_t)n * dtype_bytes(dt) + (size_t)(nseg > 0 ? nseg : 0) * 4 + sizeof(SegArgs) + sizeof(SegState);
}

ak_status segmented_sort(Workspace *ws, int dt, void *keys, const int64_t *offsets, int64_t nseg) {
    hipStream_t s = ws->stream;
    if (nseg >= (int64_t(1) << 31)) {
        set_error("nseg >= 2^31");
        return AK_ERR_INVALID_ARG;
    }
    int64_t ends[2] = {0, 0};
    AK_HIP(hipMemcpyAsync(&ends[0], offsets, 8, hipMemcpyDeviceToHost, s));
    AK_HIP(hipMemcpyAsync(&ends[1], offsets + nseg, 8, hipMemcpyDeviceToHost, s));
    AK_HIP(hipStreamSynchronize(s));
    const int64_t n = ends[1] - ends[0];
    if (ends[0] < 0 || n < 0 || n >= (int64_t(1) << 32)) {
        set_error("offsets[nseg] - offsets[0] must be in [0, 2^32) and offsets[0] >= 0");
        return AK_ERR_INVALID_ARG;
    }
    if (n == 0) return AK_OK;
    SegTune t;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_tune_table();
        t = g_tune[key_bits(dt) == 64];
    }
    if (!tune_valid(key_bits(dt), t)) t = SegTune{};
    const uint32_t a_max = 64u * (uint32_t)t.ipt_a;
    const uint32_t cap_b = 256u * (uint32_t)t.ipt_b;
    const uint32_t b_max = t.b_max > 0 ? std::min<uint32_t>((uint32_t)t.b_max, cap_b) : cap_b;
    const int grid = num_cus() * t.grid_mult;

    ak_status r;
    const size_t kb = (size_t)dtype_bytes(dt);
    if ((r = ws_reserve(ws, &ws->misc, &ws->misc_bytes, (size_t)n * kb)) != AK_OK) return r;
    if ((r = ws_reserve(ws, &ws->misc2, &ws->misc2_bytes, (size_t)nseg * 4)) != AK_OK) return r;

    std::lock_guard<std::mutex> lk(g_seg_mu);
    SegCache &c = g_seg[ws];
    if (!c.args) {
        AK_HIP(hipMalloc((void **)&c.args, sizeof(SegArgs)));
        AK_HIP(hipMalloc((void **)&c.state, sizeof(SegState)));
        AK_HIP(hipMemsetAsync(c.state, 0, sizeof(SegState), s));
        AK_HIP(hipStreamCreateWithFlags(&c.capture, hipStreamNonBlocking));
    }
    SegArgs v{};
    v.keys = keys;
    v.off = offsets;
    v.tmp = ws->misc;
    v.list = (int32_t *)ws->misc2;
    v.nseg = nseg;
    v.base = ends[0];
    v.end = ends[1];
    v.a_max = a_max;
    v.b_max = b_max;
    hipLaunchKernelGGL(k_seg_setargs, dim3(1), dim3(1), 0, s, c.args, v);
    AK_LAUNCH_CHECK("k_seg_setargs");

    SegPlanKey key{dt, nseg, t.ipt_a, t.ipt_b, grid};
    auto it = c.graphs.find(key);
    if (it == c.graphs.end()) {
        hipGraph_t g = nullptr;
        AK_HIP(hipStreamBeginCapture(c.capture, hipStreamCaptureModeRelaxed));
        ak_status lr = seg_launch_all(dt, t, nseg, grid, c.capture, c.args, c.state);
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
    AK_HIP(hipGraphLaunch(it->second, s));
    return AK_OK;
}

// Device error flag of the segmented sort on this workspace (cleared).
uint32_t segmented_take_error(Workspace *ws) {
    std::lock_guard<std::mutex> lk(g_seg_mu);
    auto it = g_seg.find(ws);
    if (it == g_seg.end() || !it->second.state) return 0;
    uint32_t f = 0;
    if (hipMemcpy(&f, &it->second.state->error, 4, hipMemcpyDeviceToHost) != hipSuccess) return 0;
    if (f) {
        const uint32_t z = 0;
        (void)hipMemcpy(&it->second.state->error, &z, 4, hipMemcpyHostToDevice);
    }
    return f;
}

void segmented_release(Workspace *ws) {
    std::lock_guard<std::mutex> lk(g_seg_mu);
    auto it = g_seg.find(ws);
    if (it == g_seg.end()) return;
    for (auto &kv : it->second.graphs) (void)hipGraphExecDestroy(kv.second);
    if (it->second.args) (void)hipFree(it->second.args);
    if (it->second.state) (void)hipFree(it->second.state);
    if (it->second.capture) (void)hipStreamDestroy(it->second.capture);
    g_seg.erase(it);
}

}  // namespace ak
