// Prefix sums (Sec. II-B accumulate with +), inclusive or exclusive, in
// place or out of place.  Integer keys sum with wrap-around in their width;
// float keys sum in their own precision.
//
// Reduce-then-scan over chunks of 4096 keys, three launches and no waiting
// between workgroups: every chunk's total (one coalesced read), an exclusive
// scan of the totals by one workgroup, then every chunk again: a striped
// coalesced load into LDS, a sequential scan of 16 consecutive keys per
// thread, a wave and workgroup scan of the thread totals, and a striped
// store.  Each chunk is read whole before any of it is written, so the
// output may alias the input.  One chunk needs only the last launch.
#include "ak_internal.h"

namespace ak {

constexpr int SCAN_B = 256, SCAN_IPT = 16, SCAN_W = SCAN_B / 64;
constexpr int SCAN_CHUNK = SCAN_B * SCAN_IPT;
constexpr int SCAN_PART_B = 1024;

// arithmetic type of a key type: unsigned integers of its width (wrap-around
// sums, the same bits for signed keys) or the float type itself
template <int DT> struct ScanType;
template <> struct ScanType<AK_I32> { using T = uint32_t; };
template <> struct ScanType<AK_U32> { using T = uint32_t; };
template <> struct ScanType<AK_I64> { using T = uint64_t; };
template <> struct ScanType<AK_U64> { using T = uint64_t; };
template <> struct ScanType<AK_F32> { using T = float; };
template <> struct ScanType<AK_F64> { using T = double; };

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T o = __shfl_up(v, d, 64);
        if (lane >= d) v = v + o;
    }
    return v;
}

// Exclusive scan of one value per thread over a workgroup of B threads;
// returns the workgroup total in *total.  s_w holds B/64 values.
template <int B, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *s_w, T *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const T incl = wave_incl_scan(v, lane);
    if (lane == 63) s_w[w] = incl;
    __syncthreads();
    T before = T(0), all = T(0);
#pragma unroll
    for (int i = 0; i < B / 64; ++i) {
        const T t = s_w[i];
        if (i < w) before = before + t;
        all = all + t;
    }
    *total = all;
    __syncthreads();  // s_w is reused by the caller's next scan
    return before + (incl - v);
}

// Total of every chunk (striped loads, then a workgroup reduction).
template <typename T>
__global__ __launch_bounds__(SCAN_B) void k_scan_reduce(const T *__restrict__ x, uint64_t n, T *__restrict__ part) {
    __shared__ T s_w[SCAN_W];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_CHUNK;
    T s = T(0);
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        const uint64_t i = base + (uint64_t)j * SCAN_B + threadIdx.x;
        if (i < n) s = s + x[i];
    }
    T total;
    (void)block_excl_scan<SCAN_B>(s, s_w, &total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// Exclusive scan of the chunk totals in place, by one workgroup: each thread
// takes a run of consecutive totals.
template <typename T>
__global__ __launch_bounds__(SCAN_PART_B) void k_scan_part(T *part, uint32_t nchunks) {
    __shared__ T s_w[SCAN_PART_B / 64];
    const uint32_t per = (nchunks + SCAN_PART_B - 1) / SCAN_PART_B;
    const uint32_t lo = min(nchunks, threadIdx.x * per), hi = min(nchunks, lo + per);
    // unrolled so that several loads of the run are in flight at once
    T s = T(0);
#pragma unroll 8
    for (uint32_t i = lo; i < hi; ++i) s = s + part[i];
    T total;
    T run = block_excl_scan<SCAN_PART_B>(s, s_w, &total);
#pragma unroll 8
    for (uint32_t i = lo; i < hi; ++i) {
        const T v = part[i];
        part[i] = run;
        run = run + v;
    }
}

// Every chunk's prefix sums, offset by the chunk's exclusive total (part =
// null: one chunk, offset 0).
// LDS slot of chunk element e: one pad slot after every 16, so that the
// threads' runs of 16 consecutive elements start in different banks
__device__ __forceinline__ uint32_t scan_slot(uint32_t e) { return e + (e >> 4); }

template <typename T, bool INCL>
__global__ __launch_bounds__(SCAN_B) void k_scan_down(const T *x, T *out, uint64_t n, const T *__restrict__ part) {
    __shared__ T s_v[SCAN_CHUNK + SCAN_CHUNK / 16];
    __shared__ T s_w[SCAN_W];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_CHUNK;
    const uint32_t len = (uint32_t)min((uint64_t)SCAN_CHUNK, n - base);
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        const uint32_t e = (uint32_t)(j * SCAN_B + tid);
        s_v[scan_slot(e)] = e < len ? x[base + e] : T(0);
    }
    __syncthreads();
    T v[SCAN_IPT];
    T s = T(0);
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        v[j] = s_v[scan_slot(tid * SCAN_IPT + j)];
        s = s + v[j];
    }
    T total;
    T run = block_excl_scan<SCAN_B>(s, s_w, &total);
    if (part) run = part[blockIdx.x] + run;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        if (INCL) run = run + v[j];
        s_v[scan_slot(tid * SCAN_IPT + j)] = run;
        if (!INCL) run = run + v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        const uint32_t e = (uint32_t)(j * SCAN_B + tid);
        if (e < len) out[base + e] = s_v[scan_slot(e)];
    }
}

size_t accumulate_temp_bytes(int64_t n) {
    const uint64_t nchunks = ((uint64_t)n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    return nchunks > 1 ? ((nchunks * 8 + 255) & ~uint64_t(255)) : 0;
}

template <int DT>
static ak_status accumulate_t(Workspace *ws, const void *in, void *out, int64_t n, bool inclusive) {
    using T = typename ScanType<DT>::T;
    hipStream_t s = ws->stream;
    const uint32_t nchunks = (uint32_t)(((uint64_t)n + SCAN_CHUNK - 1) / SCAN_CHUNK);
    T *part = nullptr;
    ProfScope ps("accumulate", s);
    if (nchunks > 1) {
        ak_status r;
        // the chunk totals live in the sortperm index scratch, which no
        // other call holds across calls (work on the stream runs in order)
        if ((r = ws_reserve(ws, &ws->vals0, &ws->vals0_bytes, (size_t)nchunks * sizeof(T))) != AK_OK) return r;
        part = (T *)ws->vals0;
        hipLaunchKernelGGL((k_scan_reduce<T>), dim3(nchunks), dim3(SCAN_B), 0, s, (const T *)in, (uint64_t)n, part);
        AK_LAUNCH_CHECK("k_scan_reduce");
        hipLaunchKernelGGL((k_scan_part<T>), dim3(1), dim3(SCAN_PART_B), 0, s, part, nchunks);
        AK_LAUNCH_CHECK("k_scan_part");
    }
    if (inclusive)
        hipLaunchKernelGGL((k_scan_down<T, true>), dim3(nchunks), dim3(SCAN_B), 0, s, (const T *)in, (T *)out,
                           (uint64_t)n, (const T *)part);
    else
        hipLaunchKernelGGL((k_scan_down<T, false>), dim3(nchunks), dim3(SCAN_B), 0, s, (const T *)in, (T *)out,
                           (uint64_t)n, (const T *)part);
    AK_LAUNCH_CHECK("k_scan_down");
    return AK_OK;
}

ak_status accumulate(Workspace *ws, int dt, const void *in, void *out, int64_t n, bool inclusive) {
    switch (dt) {
    case AK_I32: return accumulate_t<AK_I32>(ws, in, out, n, inclusive);
    case AK_I64: return accumulate_t<AK_I64>(ws, in, out, n, inclusive);
    case AK_U32: return accumulate_t<AK_U32>(ws, in, out, n, inclusive);
    case AK_U64: return accumulate_t<AK_U64>(ws, in, out, n, inclusive);
    case AK_F32: return accumulate_t<AK_F32>(ws, in, out, n, inclusive);
    case AK_F64: return accumulate_t<AK_F64>(ws, in, out, n, inclusive);
    }
    return AK_ERR_UNSUPPORTED_DTYPE;
}

}  // namespace ak
