// Binary search of many keys in one sorted array (Sec. II-B:
// searchsortedfirst / searchsortedlast), in the library's total order (the
// unsigned key image).
//
// One thread per key.  Every workgroup first copies the images of S evenly
// spaced elements of the sorted array into LDS; a key's search starts there
// (log2 S steps on chip) and ends with a bisection over the one gap of about
// n/S elements that holds its answer, read from global memory.
#include "ak_internal.h"

namespace ak {

constexpr int SEARCH_B = 256;
// staged images per workgroup: 64 KB (8192 64-bit or 16384 32-bit keys).
// 2^24 int64 keys in 2^28: 2048 staged elements 4.32 ms, 4096 3.91 ms, 8192
// 3.38 ms, 16384 3.35 ms; two such workgroups fit a CU.
constexpr size_t SEARCH_STAGE_BYTES = 65536;
constexpr int SEARCH_WG_PER_CU = 2;

// LAST = false: out[i] = number of elements whose image is below t(x[i])
// (the first index not below x[i]); LAST: that count for "not above", minus
// one (the last index not above x[i], -1 if none).  The elements that come
// before the answer are a prefix of v, so each step halves the range that
// holds the prefix length.
template <int DT, bool LAST>
__global__ __launch_bounds__(SEARCH_B) void k_search(const typename KT<DT>::U *__restrict__ v, uint64_t n,
                                                     const typename KT<DT>::U *__restrict__ x, uint64_t m,
                                                     int64_t *__restrict__ out) {
    using U = typename KT<DT>::U;
    constexpr uint32_t SEARCH_SPLIT = (uint32_t)(SEARCH_STAGE_BYTES / sizeof(U));
    __shared__ U s_sp[SEARCH_SPLIT];
    // staged element j is v[q_j] with q_j = j*n/S (S = min(SPLIT, n)): q_0 = 0
    // and the q_j strictly increase (n/S >= 1)
    const uint32_t S = (uint32_t)(n < SEARCH_SPLIT ? n : SEARCH_SPLIT);
    for (uint32_t j = threadIdx.x; j < S; j += SEARCH_B) s_sp[j] = KT<DT>::image(v[(uint64_t)j * n / S]);
    __syncthreads();
    for (uint64_t i = (uint64_t)blockIdx.x * SEARCH_B + threadIdx.x; i < m; i += (uint64_t)gridDim.x * SEARCH_B) {
        const U t = KT<DT>::image(x[i]);
        // c = staged elements that come before the answer
        uint32_t lo = 0, hi = S;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            const U a = s_sp[mid];
            if (LAST ? a <= t : a < t) lo = mid + 1;
            else hi = mid;
        }
        const uint32_t c = lo;
        // the prefix length lies in [q_{c-1} + 1, q_c] (0 when c = 0, n when
        // c = S)
        uint64_t a = c == 0 ? 0 : (uint64_t)(c - 1) * n / S + 1;
        uint64_t b = c == S ? n : (uint64_t)c * n / S;
        while (a < b) {
            const uint64_t mid = (a + b) >> 1;
            const U e = KT<DT>::image(v[mid]);
            if (LAST ? e <= t : e < t) a = mid + 1;
            else b = mid;
        }
        out[i] = LAST ? (int64_t)a - 1 : (int64_t)a;
    }
}

template <int DT>
static ak_status search_t(hipStream_t s, const void *v, int64_t n, const void *x, int64_t m, bool last,
                          int64_t *out) {
    using U = typename KT<DT>::U;
    const uint64_t want = ((uint64_t)m + SEARCH_B - 1) / SEARCH_B;
    const uint32_t grid = (uint32_t)std::min<uint64_t>(want, (uint64_t)num_cus() * SEARCH_WG_PER_CU);
    ProfScope ps("searchsorted", s);
    if (last)
        hipLaunchKernelGGL((k_search<DT, true>), dim3(grid), dim3(SEARCH_B), 0, s, (const U *)v, (uint64_t)n,
                           (const U *)x, (uint64_t)m, out);
    else
        hipLaunchKernelGGL((k_search<DT, false>), dim3(grid), dim3(SEARCH_B), 0, s, (const U *)v, (uint64_t)n,
                           (const U *)x, (uint64_t)m, out);
    AK_LAUNCH_CHECK("k_search");
    return AK_OK;
}

ak_status search_sorted(hipStream_t s, int dt, const void *v, int64_t n, const void *x, int64_t m, bool last,
                        int64_t *out) {
    if (m == 0) return AK_OK;
    switch (dt) {
    case AK_I32: return search_t<AK_I32>(s, v, n, x, m, last, out);
    case AK_I64: return search_t<AK_I64>(s, v, n, x, m, last, out);
    case AK_U32: return search_t<AK_U32>(s, v, n, x, m, last, out);
    case AK_U64: return search_t<AK_U64>(s, v, n, x, m, last, out);
    case AK_F32: return search_t<AK_F32>(s, v, n, x, m, last, out);
    case AK_F64: return search_t<AK_F64>(s, v, n, x, m, last, out);
    }
    return AK_ERR_UNSUPPORTED_DTYPE;
}

}  // namespace ak
