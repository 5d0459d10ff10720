// Internal definitions shared by the library's HIP sources (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/ak.h"

namespace ak {

// ----------------------------------------------------------------- keys
// Order-preserving unsigned image of a key's bits: unsigned order of the
// image equals the library's total order (Julia Base ordering: integers by
// value; floats -Inf < ... < -0.0 < +0.0 < ... < +Inf < NaN with all NaNs
// tied).  It is recomputed on every load and never stored: kernels move the
// original bits, so outputs are bit-identical to the inputs.
template <int DT> struct KT;
template <> struct KT<AK_U32> {
    using U = uint32_t;
    static __host__ __device__ __forceinline__ U image(U b) { return b; }
};
template <> struct KT<AK_I32> {
    using U = uint32_t;
    static __host__ __device__ __forceinline__ U image(U b) { return b ^ 0x80000000u; }
};
template <> struct KT<AK_F32> {
    using U = uint32_t;
    static __host__ __device__ __forceinline__ U image(U b) {
        if ((b & 0x7FFFFFFFu) > 0x7F800000u) return 0xFFFFFFFFu;  // any NaN
        return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    }
};
template <> struct KT<AK_U64> {
    using U = uint64_t;
    static __host__ __device__ __forceinline__ U image(U b) { return b; }
};
template <> struct KT<AK_I64> {
    using U = uint64_t;
    static __host__ __device__ __forceinline__ U image(U b) { return b ^ 0x8000000000000000ull; }
};
template <> struct KT<AK_F64> {
    using U = uint64_t;
    static __host__ __device__ __forceinline__ U image(U b) {
        if ((b & 0x7FFFFFFFFFFFFFFFull) > 0x7FF0000000000000ull) return ~0ull;
        return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
    }
};

// The paper's benchmarks also sort Int16 and Int128 keys (Sec. IV-C):
// 16-bit keys move as uint16_t, 128-bit keys as the compiler's unsigned
// 128-bit integer (two 64-bit words, little-endian, low word first).
using u128 = unsigned __int128;
template <> struct KT<AK_U16> {
    using U = uint16_t;
    static __host__ __device__ __forceinline__ U image(U b) { return b; }
};
template <> struct KT<AK_I16> {
    using U = uint16_t;
    static __host__ __device__ __forceinline__ U image(U b) { return (U)(b ^ 0x8000u); }
};
template <> struct KT<AK_U128> {
    using U = u128;
    static __host__ __device__ __forceinline__ U image(U b) { return b; }
};
template <> struct KT<AK_I128> {
    using U = u128;
    static __host__ __device__ __forceinline__ U image(U b) { return b ^ ((u128)1 << 127); }
};

constexpr int key_bits(int dt) {
    return (dt == AK_I64 || dt == AK_U64 || dt == AK_F64)   ? 64
           : (dt == AK_I16 || dt == AK_U16)                 ? 16
           : (dt == AK_I128 || dt == AK_U128)               ? 128
                                                            : 32;
}
// Shape class of a key width: 0 for 16- and 32-bit keys, 1 for 64, 2 for 128.
constexpr int key_class(int dt) { return key_bits(dt) <= 32 ? 0 : (key_bits(dt) == 64 ? 1 : 2); }
inline int dtype_bytes(int dt) { return key_bits(dt) / 8; }
// every key type (sort, sortperm, sort by key, sortperm_lowmem, no-alloc sort)
inline bool dtype_ok(int dt) { return dt >= AK_I32 && dt <= AK_U128; }
// the six 32- and 64-bit key types (every other entry point)
inline bool dtype_std(int dt) { return dt >= AK_I32 && dt <= AK_F64; }

// Low and high 64 bits of a key image (the high half is 0 below 128 bits).
__host__ __device__ __forceinline__ uint64_t img_lo(uint16_t t) { return t; }
__host__ __device__ __forceinline__ uint64_t img_hi(uint16_t) { return 0; }
__host__ __device__ __forceinline__ uint64_t img_lo(uint32_t t) { return t; }
__host__ __device__ __forceinline__ uint64_t img_hi(uint32_t) { return 0; }
__host__ __device__ __forceinline__ uint64_t img_lo(uint64_t t) { return t; }
__host__ __device__ __forceinline__ uint64_t img_hi(uint64_t) { return 0; }
__host__ __device__ __forceinline__ uint64_t img_lo(u128 t) { return (uint64_t)t; }
__host__ __device__ __forceinline__ uint64_t img_hi(u128 t) { return (uint64_t)(t >> 64); }

// ------------------------------------------------------------- wave64
__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// number of set bits of m in lanes below the calling lane
__device__ __forceinline__ uint32_t count_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// inclusive prefix sum across the 64 lanes of a wave
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(v, d, 64);
        if (lane >= (uint32_t)d) v += o;
    }
    return v;
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// ----------------------------------------------------- look-back words
// One 64-bit word per (tile, digit): count in bits 0..31, status in bits
// 32..33 (1 = this tile's own count, 2 = inclusive prefix through this
// tile), and the pass epoch in bits 34..63 so stale words from earlier
// passes never need clearing.
constexpr uint64_t LB_AGG = 1, LB_INC = 2;
__device__ __forceinline__ uint64_t lb_pack(uint32_t epoch, uint64_t flag, uint32_t cnt) {
    return (uint64_t)cnt | (flag << 32) | ((uint64_t)epoch << 34);
}
__device__ __forceinline__ void lb_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t lb_load(const uint64_t *p) {
    return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ----------------------------------------------------- radix run state
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int MAX_PLACES = 16;  // 8-bit digit places of a 128-bit key

struct PassDesc {
    int32_t active;  // 0: every key has the same digit here; the pass is skipped
    int32_t j;       // index of this pass among the active ones
    int32_t q;       // number of active passes
    int32_t shift;   // bit offset of the digit
};

// Copies of the digit counts that the histogram's workgroups add into
// (workgroup g into copy g % HIST_REP), so that fewer device-scope atomics
// queue on one address; the digit scan sums them.
constexpr int HIST_REP = 8;

// Device-resident state of one radix run.
struct RunState {
    uint32_t base[MAX_PLACES][RADIX];  // exclusive digit offsets per place
    uint32_t tile_ctr[MAX_PLACES];     // dynamic tile ids per pass
    PassDesc desc[MAX_PLACES];
    int32_t q;                         // number of active passes
    uint32_t error;                    // device-detected input error flag
    uint32_t epoch_base;               // look-back epoch of this run's first pass
    // prefix-partitioned sort (decided with the digit offsets): the passes
    // order the keys by the `pfx_places` top active places only, and the
    // chunk sort finishes every run of equal prefix on chip
    uint32_t pfx_active;
    int32_t pfx_shift;                 // bit offset of the prefix field
    uint32_t pfx_mask;                 // prefix field mask (after the shift)
    uint32_t pfx_places;               // digit places in the prefix field
    // digit counts per place, in HIST_REP copies; zero between runs (the
    // digit scan clears what it read)
    uint32_t hist[HIST_REP][MAX_PLACES][RADIX];
};

// ------------------------------------------------------------- errors
void set_error(const std::string &msg);
ak_status hip_fail(hipError_t e, const char *what);
#define AK_HIP(call)                                  \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)
#define AK_LAUNCH_CHECK(what)                                 \
    do {                                                      \
        hipError_t e_ = hipGetLastError();                    \
        if (e_ != hipSuccess) return hip_fail(e_, what);      \
    } while (0)

// ------------------------------------------------------------ profiling
// RAII bracket of one launch; records events only while profiling is on.
class ProfScope {
  public:
    ProfScope(const char *name, hipStream_t s);
    ~ProfScope();

  private:
    const char *name_;
    hipStream_t s_;
    void *a_ = nullptr, *b_ = nullptr;
};

// ------------------------------------------------------------ workspace
// Per (device, stream) scratch.  Regions are grown independently; the
// look-back region is zero-filled when (re)allocated and then relies on
// epochs, so it is never cleared between calls.
struct Workspace {
    int device = -1;
    hipStream_t stream = nullptr;
    void *keys0 = nullptr; size_t keys0_bytes = 0;
    void *keys1 = nullptr; size_t keys1_bytes = 0;
    void *vals0 = nullptr; size_t vals0_bytes = 0;
    void *vals1 = nullptr; size_t vals1_bytes = 0;   // second payload buffer (sort by key)
    uint64_t *lookback = nullptr; size_t lookback_bytes = 0;
    RunState *state = nullptr;      // several run states (sample sort, main run)
    uint32_t *epoch_dev = nullptr;  // device copy of `epoch` (advanced by k_run_init)
    uint32_t gen = 0;               // bumped whenever a buffer is reallocated
    void *misc = nullptr; size_t misc_bytes = 0;   // learned / segmented scratch
    void *misc2 = nullptr; size_t misc2_bytes = 0;
    void *aux[6] = {nullptr}; size_t aux_bytes[6] = {0};     // learned-sort scratch
    uint32_t epoch = 0;             // last epoch base handed out
    char *arena = nullptr;          // caller-owned scratch (ak_set_workspace), else null
    size_t arena_bytes = 0, arena_used = 0;
    // arena bytes [arena_lb_off, arena_lb_off + arena_lb_ok) hold nothing
    // but look-back words (zeroed once, then only words of earlier runs,
    // whose epochs never match a later run's), so a call that carves its
    // look-back region there again needs no zero fill
    size_t arena_lb_off = 0, arena_lb_ok = 0;
    // route of this call's radix run on state slot 0: 0 none or on chip,
    // 1 digit passes only, 2 passes with the prefix-partitioned finish
    int last_route = 0;
    // fixed_lookback: the look-back region is a fixed piece of memory that
    // outlives calls (sized for the largest run the owner admits), so an
    // arena carve never replaces or refills it; no_graph: launch directly,
    // never capture or instantiate a graph (both for the entry point that
    // allocates nothing)
    bool fixed_lookback = false;
    bool no_graph = false;
};

Workspace *get_workspace(hipStream_t stream);
ak_status ws_reserve(Workspace *ws, void **p, size_t *have, size_t need);
ak_status ws_reserve_lookback(Workspace *ws, size_t need);
// Called by every entry point before it reserves scratch.
void ws_begin_call(Workspace *ws);
// AK_OK unless a caller arena is bound and smaller than `need`.
ak_status ws_arena_fits(Workspace *ws, size_t need);
// Zeroes `bytes` at p with a fill kernel on s (no memset node in a graph).
ak_status zero_fill(hipStream_t s, void *p, size_t bytes);
// Mirrors the device's epoch advance of one run (16 epochs per run; both
// restart at 16 before 2^30) and clears the look-back words when it wraps.
ak_status ws_next_epoch(Workspace *ws, uint32_t *epoch);
// true while `s` is being captured into a graph
bool stream_capturing(hipStream_t s);

int num_cus();
// Run-state slots per workspace (several radix runs of one call) and the
// bytes of the state block: the slots, then the device epoch counter.
constexpr int RUN_SLOTS = 4;
constexpr size_t RUN_STATE_BYTES = sizeof(RunState) * RUN_SLOTS + 256;

// --------------------------------------------------------- radix driver
// Sorts keys (sort mode, in place) or writes perm (sortperm mode) on
// `stream`, using run state slot `slot` of the workspace.
ak_status radix_sort(Workspace *ws, int dtype, void *keys, uint32_t *perm, int64_t n, int slot);
// The same run carrying `vals` as `mode` says (radix_kernels.h: M_KEYS,
// M_PERM, M_PAIRS4, M_PAIRS8, M_LOWMEM), for every key type.
ak_status radix_sort_mode(Workspace *ws, int dtype, int mode, void *keys, void *vals, int64_t n, int slot);
// Scratch of radix_sort_mode.
size_t radix_temp_bytes_mode(int dtype, int mode, int64_t n);
// Binary search of keys x[0..m) in the sorted v[0..n) on stream s: out[i] =
// first index not below x[i] (n if none), or with `last` the last index not
// above x[i] (-1 if none).
ak_status search_sorted(hipStream_t s, int dtype, const void *v, int64_t n, const void *x, int64_t m, bool last,
                        int64_t *out);
// Prefix sums of in[0..n) into out (which may be in), inclusive or
// exclusive, on the workspace's stream; scratch: accumulate_temp_bytes(n).
ak_status accumulate(Workspace *ws, int dtype, const void *in, void *out, int64_t n, bool inclusive);
size_t accumulate_temp_bytes(int64_t n);
size_t radix_temp_bytes(int dtype, int64_t n, bool perm);

// Prefix-partitioned finish of a key-only radix run (learned.hip): scratch
// it needs beyond the radix passes, its reservation (before the run's
// launches), and its launches after the passes: the on-chip chunk sorts of
// the runs of equal prefix, then the segmented radix sort of the runs that
// exceed a chunk.  Every launch exits at once when the run took plain
// passes.
size_t prefix_finish_bytes(int dtype, int64_t n, bool small);
ak_status prefix_reserve(Workspace *ws, int dtype, int64_t n);
// Launches on s.  small: fixed launches only, so that the run can be
// captured (fallback runs sorted by one workgroup each instead of by the
// segmented sort); otherwise s must be the workspace's stream.
ak_status prefix_finish(Workspace *ws, hipStream_t s, int dtype, void *keys, int64_t n, const RunState *st,
                        bool small);
// Chunk capacity of the prefix finish; a run of equal prefix up to this
// length is sorted on chip.
int prefix_chunk_keys();
// Chunk sorts, fallback runs and fallback keys of the last prefix finish
// (waits for the stream).
ak_status prefix_counts(Workspace *ws, int64_t out[3]);

// Single-workgroup on-chip sort capacity (keys) for a dtype.
int64_t small_sort_capacity(int dtype);

// -------------------------------------------------------- segmented sort
ak_status segmented_sort(Workspace *ws, int dtype, void *keys, const int64_t *offsets, int64_t nseg);
// The same with the key count n given (scratch sized from n, the batch's
// ends read and checked on the device): never waits for the device.
ak_status segmented_sort_n(Workspace *ws, int dtype, void *keys, int64_t n, const int64_t *offsets, int64_t nseg);
// Sorts disjoint ranges keys[lo[s] .. hi[s]) within keys[0 .. end), with
// `tmp` as end keys of scratch (ranges with hi <= lo are skipped).
ak_status segmented_sort_ranges(Workspace *ws, int dtype, void *keys, const int64_t *lo, const int64_t *hi,
                                int64_t nseg, int64_t end, void *tmp);
size_t segmented_temp_bytes(int dtype, int64_t n, int64_t nseg);
size_t segmented_scratch_bytes(int dtype, int64_t n, int64_t nseg, bool with_tmp);
size_t code_partition_bytes(int dtype, int64_t n);

// ------------------------------------------------------------- learned
ak_status learned_sort(Workspace *ws, int dtype, void *keys, int64_t n, const ak_learned_cfg *cfg,
                       ak_learned_stats *stats);
size_t learned_temp_bytes(int dtype, int64_t n, const ak_learned_cfg *cfg);
ak_status learned_sample(hipStream_t s, int dtype, const void *keys, int64_t n, uint64_t seed, int64_t m,
                         void *out);
ak_status rmi_fit(Workspace *ws, int dtype, const void *sorted, int64_t m, int leaves, int iters,
                  float *model);
ak_status rmi_leaf_grad(Workspace *ws, int dtype, const void *sorted, int64_t m, const float *model,
                        float *out);
ak_status rmi_codes(hipStream_t s, int dtype, const void *keys, int64_t n, const float *model, int cb,
                    uint32_t *codes);
// Head of a model: root over the sorted sample's feature range in L equal
// widths (rc, ra, rb = 0, L).
ak_status rmi_root(hipStream_t s, int dtype, const void *sorted, uint32_t m, int L, float *model);
// MLP model (mlp.hip): fit + table (params_out optional), scratch bytes,
// and the forward/backward parity entry.
ak_status mlp_fit(Workspace *ws, int dtype, const void *sorted, int64_t m, int L, int iters, float *model,
                  float *params_out);
size_t mlp_scratch_bytes(int64_t m);
ak_status mlp_loss_grad(Workspace *ws, const float *u, const float *y, int64_t K, const float *params, float *out);

}  // namespace ak
