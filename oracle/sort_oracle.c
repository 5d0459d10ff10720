/*
 * Sort oracle: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of what the GPU sort
 * path computes.  Only the tests, the smoke check and the benchmark's CPU
 * baseline leg may load this library.  It shares no code, header, table or
 * helper with the HIP library.
 *
 * What it computes (paper Sec. II-B, "Algorithms Implemented"):
 *   - sort:      the keys of a collection in ascending order; the library's
 *                sorter is a merge sort, hence stable;
 *   - sortperm:  the index permutation that would sort the collection;
 *                ties (keys equal under the order) keep increasing index;
 *   - segmented: every segment [off[s], off[s+1]) sorted on its own.
 * Key types: 16-, 32-, 64- and 128-bit signed and unsigned integers (the
 * paper's benchmarks sort Int16 up to Int128, Sec. IV-C) and 32- and
 * 64-bit floats.  (sort_by_key, sortperm_lowmem: in oracle/__init__.py,
 * from sortperm.)
 * The order follows the Julia Base conventions the library adopts
 * (Sec. II, multiple dispatch onto the Base function names): integers by
 * value; floats by `isless`: -Inf < ... < -0.0 < +0.0 < ... < +Inf < NaN,
 * with every NaN equal to every other NaN (so NaNs keep input order).
 *
 * The comparator is the semantic definition, never a bit transform.  The
 * algorithm is a top-down stable merge sort: split in halves, sort each,
 * merge taking from the left run on ties.  The threaded variant sorts T
 * contiguous chunks with the same routine and then merges neighbouring
 * runs pairwise, again taking from the left run on ties, so its result is
 * the same stable order.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* dtype codes used by the oracle's own API (plain ints, not shared) */
enum { OR_I32 = 1, OR_I64 = 2, OR_U32 = 3, OR_U64 = 4, OR_F32 = 5, OR_F64 = 6,
       OR_I16 = 7, OR_U16 = 8, OR_I128 = 9, OR_U128 = 10 };

/* Julia's Int128 / UInt128 (Sec. IV: the sorting benchmarks run Int16 to
 * Int128 keys): the compiler's 128-bit integers, compared by value. */
typedef __int128 i128_t;
typedef unsigned __int128 u128_t;

/* ---- semantic "less than" for every supported key type ---- */
#define LESS_INT(a, b) ((a) < (b))
/* isless for floats: NaN is greater than everything else and ties with NaN;
 * -0.0 sorts before +0.0; otherwise numeric order. */
#define LESS_FLT(a, b)                                                      \
    (!isnan(a) && (isnan(b) || (a) < (b) ||                                 \
                   ((a) == (b) && signbit(a) && !signbit(b))))

/* ---- one stable merge sort per key type ----
 * msort_T(a, tmp, n): sorts a[0..n) stably; tmp has room for n elements.
 * merge_T(src, mid, n, dst): merges the sorted runs src[0..mid) and
 * src[mid..n) into dst, taking the left element on ties.            */
#define DEFINE_SORT(SUF, T, LESS)                                           \
    static void merge_##SUF(const T *src, int64_t mid, int64_t n, T *dst) { \
        int64_t i = 0, j = mid, k = 0;                                      \
        while (i < mid && j < n) {                                          \
            if (LESS(src[j], src[i])) dst[k++] = src[j++];                  \
            else dst[k++] = src[i++];                                       \
        }                                                                   \
        while (i < mid) dst[k++] = src[i++];                                \
        while (j < n) dst[k++] = src[j++];                                  \
    }                                                                       \
    static void msort_##SUF(T *a, T *tmp, int64_t n) {                      \
        if (n < 2) return;                                                  \
        int64_t mid = n / 2;                                                \
        msort_##SUF(a, tmp, mid);                                           \
        msort_##SUF(a + mid, tmp + mid, n - mid);                           \
        if (!LESS(a[mid], a[mid - 1])) return; /* already in order */      \
        merge_##SUF(a, mid, n, tmp);                                        \
        memcpy(a, tmp, (size_t)n * sizeof(T));                              \
    }

DEFINE_SORT(i32, int32_t, LESS_INT)
DEFINE_SORT(i64, int64_t, LESS_INT)
DEFINE_SORT(u32, uint32_t, LESS_INT)
DEFINE_SORT(u64, uint64_t, LESS_INT)
DEFINE_SORT(f32, float, LESS_FLT)
DEFINE_SORT(f64, double, LESS_FLT)
DEFINE_SORT(i16, int16_t, LESS_INT)
DEFINE_SORT(u16, uint16_t, LESS_INT)
DEFINE_SORT(i128, i128_t, LESS_INT)
DEFINE_SORT(u128, u128_t, LESS_INT)

/* ---- pairs (key, index) for sortperm: compare keys only ---- */
#define DEFINE_PAIR(SUF, T, LESS)                                           \
    typedef struct { T k; uint32_t i; } pair_##SUF;                         \
    static void pmerge_##SUF(const pair_##SUF *src, int64_t mid, int64_t n, \
                             pair_##SUF *dst) {                             \
        int64_t i = 0, j = mid, k = 0;                                      \
        while (i < mid && j < n) {                                          \
            if (LESS(src[j].k, src[i].k)) dst[k++] = src[j++];              \
            else dst[k++] = src[i++];                                       \
        }                                                                   \
        while (i < mid) dst[k++] = src[i++];                                \
        while (j < n) dst[k++] = src[j++];                                  \
    }                                                                       \
    static void psort_##SUF(pair_##SUF *a, pair_##SUF *tmp, int64_t n) {    \
        if (n < 2) return;                                                  \
        int64_t mid = n / 2;                                                \
        psort_##SUF(a, tmp, mid);                                           \
        psort_##SUF(a + mid, tmp + mid, n - mid);                           \
        if (!LESS(a[mid].k, a[mid - 1].k)) return;                          \
        pmerge_##SUF(a, mid, n, tmp);                                       \
        memcpy(a, tmp, (size_t)n * sizeof(pair_##SUF));                     \
    }                                                                       \
    static int sortperm_##SUF(const T *keys, uint32_t *perm, int64_t n) {   \
        pair_##SUF *p = (pair_##SUF *)malloc((size_t)n * sizeof(*p) + 1);   \
        pair_##SUF *t = (pair_##SUF *)malloc((size_t)n * sizeof(*t) + 1);   \
        if (!p || !t) { free(p); free(t); return -1; }                      \
        for (int64_t i = 0; i < n; i++) { p[i].k = keys[i]; p[i].i = (uint32_t)i; } \
        psort_##SUF(p, t, n);                                               \
        for (int64_t i = 0; i < n; i++) perm[i] = p[i].i;                   \
        free(p); free(t);                                                   \
        return 0;                                                           \
    }

DEFINE_PAIR(i32, int32_t, LESS_INT)
DEFINE_PAIR(i64, int64_t, LESS_INT)
DEFINE_PAIR(u32, uint32_t, LESS_INT)
DEFINE_PAIR(u64, uint64_t, LESS_INT)
DEFINE_PAIR(f32, float, LESS_FLT)
DEFINE_PAIR(f64, double, LESS_FLT)
DEFINE_PAIR(i16, int16_t, LESS_INT)
DEFINE_PAIR(u16, uint16_t, LESS_INT)
DEFINE_PAIR(i128, i128_t, LESS_INT)
DEFINE_PAIR(u128, u128_t, LESS_INT)

static size_t dtype_size(int dt) {
    switch (dt) {
    case OR_I32: case OR_U32: case OR_F32: return 4;
    case OR_I64: case OR_U64: case OR_F64: return 8;
    case OR_I16: case OR_U16: return 2;
    case OR_I128: case OR_U128: return 16;
    default: return 0;
    }
}

/* sort a[0..n) of dtype dt in place with scratch tmp */
static void sort_run(int dt, void *a, void *tmp, int64_t n) {
    switch (dt) {
    case OR_I32: msort_i32((int32_t *)a, (int32_t *)tmp, n); break;
    case OR_I64: msort_i64((int64_t *)a, (int64_t *)tmp, n); break;
    case OR_U32: msort_u32((uint32_t *)a, (uint32_t *)tmp, n); break;
    case OR_U64: msort_u64((uint64_t *)a, (uint64_t *)tmp, n); break;
    case OR_F32: msort_f32((float *)a, (float *)tmp, n); break;
    case OR_F64: msort_f64((double *)a, (double *)tmp, n); break;
    case OR_I16: msort_i16((int16_t *)a, (int16_t *)tmp, n); break;
    case OR_U16: msort_u16((uint16_t *)a, (uint16_t *)tmp, n); break;
    case OR_I128: msort_i128((i128_t *)a, (i128_t *)tmp, n); break;
    case OR_U128: msort_u128((u128_t *)a, (u128_t *)tmp, n); break;
    }
}

/* merge two adjacent sorted runs src[0..mid), src[mid..n) into dst */
static void merge_runs(int dt, const void *src, int64_t mid, int64_t n, void *dst) {
    switch (dt) {
    case OR_I32: merge_i32((const int32_t *)src, mid, n, (int32_t *)dst); break;
    case OR_I64: merge_i64((const int64_t *)src, mid, n, (int64_t *)dst); break;
    case OR_U32: merge_u32((const uint32_t *)src, mid, n, (uint32_t *)dst); break;
    case OR_U64: merge_u64((const uint64_t *)src, mid, n, (uint64_t *)dst); break;
    case OR_F32: merge_f32((const float *)src, mid, n, (float *)dst); break;
    case OR_F64: merge_f64((const double *)src, mid, n, (double *)dst); break;
    case OR_I16: merge_i16((const int16_t *)src, mid, n, (int16_t *)dst); break;
    case OR_U16: merge_u16((const uint16_t *)src, mid, n, (uint16_t *)dst); break;
    case OR_I128: merge_i128((const i128_t *)src, mid, n, (i128_t *)dst); break;
    case OR_U128: merge_u128((const u128_t *)src, mid, n, (u128_t *)dst); break;
    }
}

/* ---------------------------------------------------------------------
 * Exported API.  Return 0 on success, -1 on a bad argument or no memory.
 * ------------------------------------------------------------------- */

/* Stable ascending sort of keys[0..n) in place (single thread). */
int oracle_sort(int dt, void *keys, int64_t n) {
    size_t es = dtype_size(dt);
    if (!es || n < 0 || (n > 0 && !keys)) return -1;
    if (n < 2) return 0;
    void *tmp = malloc((size_t)n * es);
    if (!tmp) return -1;
    sort_run(dt, keys, tmp, n);
    free(tmp);
    return 0;
}

/* Stable sortperm: perm[i] = 0-based index of the i-th key in sorted order. */
int oracle_sortperm(int dt, const void *keys, uint32_t *perm, int64_t n) {
    if (!dtype_size(dt) || n < 0 || n > 4294967295LL || (n > 0 && (!keys || !perm)))
        return -1;
    if (n == 0) return 0;
    switch (dt) {
    case OR_I32: return sortperm_i32((const int32_t *)keys, perm, n);
    case OR_I64: return sortperm_i64((const int64_t *)keys, perm, n);
    case OR_U32: return sortperm_u32((const uint32_t *)keys, perm, n);
    case OR_U64: return sortperm_u64((const uint64_t *)keys, perm, n);
    case OR_F32: return sortperm_f32((const float *)keys, perm, n);
    case OR_F64: return sortperm_f64((const double *)keys, perm, n);
    case OR_I16: return sortperm_i16((const int16_t *)keys, perm, n);
    case OR_U16: return sortperm_u16((const uint16_t *)keys, perm, n);
    case OR_I128: return sortperm_i128((const i128_t *)keys, perm, n);
    case OR_U128: return sortperm_u128((const u128_t *)keys, perm, n);
    }
    return -1;
}

/* Segmented sort: each [off[s], off[s+1]) for s < nseg sorted on its own.
 * Offsets must be nondecreasing; keys outside [off[0], off[nseg]) untouched. */
int oracle_segsort(int dt, void *keys, const int64_t *off, int64_t nseg) {
    size_t es = dtype_size(dt);
    if (!es || nseg < 0 || (nseg > 0 && (!keys || !off))) return -1;
    int64_t maxlen = 0;
    for (int64_t s = 0; s < nseg; s++) {
        if (off[s + 1] < off[s] || off[s] < 0) return -1;
        if (off[s + 1] - off[s] > maxlen) maxlen = off[s + 1] - off[s];
    }
    if (maxlen < 2) return 0;
    void *tmp = malloc((size_t)maxlen * es);
    if (!tmp) return -1;
    for (int64_t s = 0; s < nseg; s++)
        sort_run(dt, (char *)keys + (size_t)off[s] * es, tmp, off[s + 1] - off[s]);
    free(tmp);
    return 0;
}

/* ---------------------------------------------------------------------
 * Binary search (Sec. II-B: searchsortedfirst / searchsortedlast, the
 * lower and upper bound of std::).  v[0..n) is sorted under the order above.
 * For every x[i]:
 *   last == 0: out[i] = smallest j in [0, n] with j == n or !less(v[j], x[i])
 *              (0-based index of the first element not below x[i]; n if none);
 *   last != 0: out[i] = largest j in [-1, n-1] with j == -1 or
 *              !less(x[i], v[j]) (0-based index of the last element not above
 *              x[i]; -1 if none).
 * "v[j] comes before the answer" holds for a prefix of v, so plain bisection
 * on that predicate finds the length of the prefix. */
#define DEFINE_SEARCH(SUF, T, LESS)                                                   \
    static void search_##SUF(const T *v, int64_t n, const T *x, int64_t m, int last, \
                             int64_t *out) {                                          \
        for (int64_t i = 0; i < m; ++i) {                                             \
            int64_t lo = 0, hi = n; /* prefix length lies in [lo, hi] */              \
            while (lo < hi) {                                                         \
                const int64_t mid = lo + (hi - lo) / 2;                               \
                const int before = last ? !LESS(x[i], v[mid]) : LESS(v[mid], x[i]);   \
                if (before) lo = mid + 1;                                             \
                else hi = mid;                                                        \
            }                                                                         \
            out[i] = last ? lo - 1 : lo;                                              \
        }                                                                             \
    }
DEFINE_SEARCH(i32, int32_t, LESS_INT)
DEFINE_SEARCH(i64, int64_t, LESS_INT)
DEFINE_SEARCH(u32, uint32_t, LESS_INT)
DEFINE_SEARCH(u64, uint64_t, LESS_INT)
DEFINE_SEARCH(f32, float, LESS_FLT)
DEFINE_SEARCH(f64, double, LESS_FLT)

int oracle_searchsorted(int dt, const void *v, int64_t n, const void *x, int64_t m, int last,
                        int64_t *out) {
    if (n < 0 || m < 0) return 1;
    switch (dt) {
    case OR_I32: search_i32((const int32_t *)v, n, (const int32_t *)x, m, last, out); break;
    case OR_I64: search_i64((const int64_t *)v, n, (const int64_t *)x, m, last, out); break;
    case OR_U32: search_u32((const uint32_t *)v, n, (const uint32_t *)x, m, last, out); break;
    case OR_U64: search_u64((const uint64_t *)v, n, (const uint64_t *)x, m, last, out); break;
    case OR_F32: search_f32((const float *)v, n, (const float *)x, m, last, out); break;
    case OR_F64: search_f64((const double *)v, n, (const double *)x, m, last, out); break;
    default: return 1;
    }
    return 0;
}

/* ---------------------------------------------------------------------
 * accumulate with + (Sec. II-B prefix scan), left to right:
 *   inclusive: out[i] = x[0] + ... + x[i];  exclusive: out[0] = 0,
 *   out[i] = x[0] + ... + x[i-1].
 * Integer keys: sums wrap around in the key's width (done in the unsigned
 * type of that width).  Float keys: the running sum is carried in a wider
 * type (double for float32, long double for float64) and each prefix is
 * returned as a double, so its error is far below one unit in the last
 * place of the key type: out is int32/int64/uint32/uint64 or double. */
#define DEFINE_ACC_INT(SUF, T, UT)                                                  \
    static void acc_##SUF(const T *x, int64_t n, int inclusive, T *out) {          \
        UT run = 0;                                                                 \
        for (int64_t i = 0; i < n; ++i) {                                           \
            const UT xi = (UT)x[i];                                                 \
            if (inclusive) run += xi;                                               \
            out[i] = (T)run;                                                        \
            if (!inclusive) run += xi;                                              \
        }                                                                           \
    }
DEFINE_ACC_INT(i32, int32_t, uint32_t)
DEFINE_ACC_INT(i64, int64_t, uint64_t)
DEFINE_ACC_INT(u32, uint32_t, uint32_t)
DEFINE_ACC_INT(u64, uint64_t, uint64_t)
#define DEFINE_ACC_FLT(SUF, T, W)                                                   \
    static void acc_##SUF(const T *x, int64_t n, int inclusive, double *out) {     \
        W run = 0;                                                                  \
        for (int64_t i = 0; i < n; ++i) {                                           \
            if (inclusive) run += (W)x[i];                                          \
            out[i] = (double)run;                                                   \
            if (!inclusive) run += (W)x[i];                                         \
        }                                                                           \
    }
DEFINE_ACC_FLT(f32, float, double)
DEFINE_ACC_FLT(f64, double, long double)

int oracle_accumulate(int dt, const void *x, int64_t n, int inclusive, void *out) {
    if (n < 0) return 1;
    switch (dt) {
    case OR_I32: acc_i32((const int32_t *)x, n, inclusive, (int32_t *)out); break;
    case OR_I64: acc_i64((const int64_t *)x, n, inclusive, (int64_t *)out); break;
    case OR_U32: acc_u32((const uint32_t *)x, n, inclusive, (uint32_t *)out); break;
    case OR_U64: acc_u64((const uint64_t *)x, n, inclusive, (uint64_t *)out); break;
    case OR_F32: acc_f32((const float *)x, n, inclusive, (double *)out); break;
    case OR_F64: acc_f64((const double *)x, n, inclusive, (double *)out); break;
    default: return 1;
    }
    return 0;
}

/* ---- threaded variant: T chunks sorted in parallel, then pairwise merges ---- */
typedef struct {
    int dt;
    char *a, *tmp;
    int64_t lo, mid, hi; /* sort job: [lo, hi); merge job: [lo,mid)+[mid,hi) */
    size_t es;
    int merge;
} job_t;

static void *run_job(void *arg) {
    job_t *j = (job_t *)arg;
    char *a = j->a + (size_t)j->lo * j->es;
    char *t = j->tmp + (size_t)j->lo * j->es;
    if (!j->merge) {
        sort_run(j->dt, a, t, j->hi - j->lo);
    } else {
        merge_runs(j->dt, a, j->mid - j->lo, j->hi - j->lo, t);
        memcpy(a, t, (size_t)(j->hi - j->lo) * j->es);
    }
    return NULL;
}

/* Same result as oracle_sort, using up to `threads` POSIX threads. */
int oracle_sort_mt(int dt, void *keys, int64_t n, int threads) {
    size_t es = dtype_size(dt);
    if (!es || n < 0 || (n > 0 && !keys)) return -1;
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    if (n < 2) return 0;
    if ((int64_t)threads > n / 2) threads = (int)(n / 2 > 0 ? n / 2 : 1);
    char *tmp = (char *)malloc((size_t)n * es);
    if (!tmp) return -1;
    /* chunk boundaries */
    int64_t bnd[257];
    for (int c = 0; c <= threads; c++) bnd[c] = n * c / threads;
    job_t jobs[256];
    pthread_t th[256];
    for (int c = 0; c < threads; c++) {
        jobs[c] = (job_t){dt, (char *)keys, tmp, bnd[c], bnd[c], bnd[c + 1], es, 0};
        pthread_create(&th[c], NULL, run_job, &jobs[c]);
    }
    for (int c = 0; c < threads; c++) pthread_join(th[c], NULL);
    /* merge neighbouring runs: width doubles every round */
    int runs = threads;
    int64_t rb[257];
    memcpy(rb, bnd, sizeof(int64_t) * (size_t)(threads + 1));
    while (runs > 1) {
        int nj = 0;
        for (int r = 0; r + 1 < runs; r += 2) {
            jobs[nj] = (job_t){dt, (char *)keys, tmp, rb[r], rb[r + 1], rb[r + 2], es, 1};
            pthread_create(&th[nj], NULL, run_job, &jobs[nj]);
            nj++;
        }
        for (int k = 0; k < nj; k++) pthread_join(th[k], NULL);
        int nr = 0;
        int64_t nb[257];
        for (int r = 0; r < runs; r += 2) nb[nr++] = rb[r];
        nb[nr] = rb[runs];
        memcpy(rb, nb, sizeof(int64_t) * (size_t)(nr + 1));
        runs = nr;
    }
    free(tmp);
    return 0;
}
