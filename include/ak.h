/*
 * ak.h -- C ABI of the MI355X (gfx950) sort library.
 *
 * What the calls compute follows the sorting primitives of the
 * AcceleratedKernels.jl paper (arXiv 2507.16710), Sec. II-B "Algorithms
 * Implemented":
 *   - sort a collection ascending (in place here); the paper's sorter is a
 *     merge sort, so results are those of a stable sort;
 *   - sortperm: the index permutation that would sort a collection;
 * with the Julia Base ordering the library adopts by dispatching onto the
 * Base function names (Sec. II): integers by value; floats with
 * -Inf < ... < -0.0 < +0.0 < ... < +Inf < NaN, all NaNs equal (so they keep
 * their input order).  The paper exposes every temporary buffer to the
 * caller and makes its size known from the input size ahead of the call
 * (Sec. II-B, end); here ak_temp_bytes reports it.  Device code cannot throw
 * (Sec. II), so every call returns a status code.
 *
 * Conventions for every call:
 *   - Array pointers are DEVICE pointers (hipMalloc / torch CUDA tensors) on
 *     the current HIP device; the caller owns them.  The library never keeps
 *     them after the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous on that stream unless stated otherwise.
 *   - Arguments are checked before anything is launched; on an error nothing
 *     is written and the status says why (detail in ak_last_error()).
 *   - n == 0 (or nseg == 0) returns AK_OK and launches nothing.
 *   - The library keeps one scratch workspace per (device, stream), grown on
 *     demand with hipMalloc (which synchronises the device) and freed by
 *     ak_release_workspace(), unless the caller binds its own device arena
 *     to the stream with ak_set_workspace().  Calls issued concurrently on
 *     DIFFERENT streams use different workspaces; calls on one stream are
 *     serialised by it.
 *   - Key counts are limited to n <= AK_MAX_KEYS = 2^31: indices, counters
 *     and grid-stride loops are 32-bit, and 2^31 keeps every index plus one
 *     stride below 2^32.  Larger n is rejected with AK_ERR_INVALID_ARG
 *     before anything is launched.
 */
#ifndef AK_H
#define AK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *ak_stream_t;

/* Largest key count any call accepts (see the conventions above). */
#define AK_MAX_KEYS ((int64_t)1 << 31)

typedef enum {
    AK_OK = 0,
    AK_ERR_INVALID_ARG = 1,       /* bad pointer, size, offsets or config   */
    AK_ERR_UNSUPPORTED_DTYPE = 2, /* dtype not handled by this entry point  */
    AK_ERR_NO_MEMORY = 3,         /* workspace could not be allocated        */
    AK_ERR_HIP = 4,               /* a HIP runtime call or launch failed     */
    AK_ERR_INTERNAL = 5           /* an internal consistency check failed    */
} ak_status;

/* Key types.  The 16- and 128-bit integers are the other widths the
 * paper's benchmarks sort (Sec. IV-C: Int16 up to Int128); a 128-bit key
 * is 16 bytes, little-endian (low 64-bit word first), signed ones in two's
 * complement.  ak_sort, ak_sortperm, ak_sort_by_key, ak_sortperm_lowmem
 * and ak_sort_noalloc take every type; the other calls take the six 32-
 * and 64-bit types and return AK_ERR_UNSUPPORTED_DTYPE for the rest. */
typedef enum {
    AK_I32 = 1, AK_I64 = 2, AK_U32 = 3, AK_U64 = 4, AK_F32 = 5, AK_F64 = 6,
    AK_I16 = 7, AK_U16 = 8, AK_I128 = 9, AK_U128 = 10
} ak_dtype;

/* ------------------------------------------------------------------ sort
 * Sec. II-B (merge_sort): sorts keys[0..n) ascending, in place.  Output keys
 * keep their original bit patterns (NaN payloads and signs included); NaNs
 * end up last, in input order.  LSD radix passes over the active digit
 * places; above 2^16 keys, when the digit counts show that the top places
 * spread the keys, only those places take passes and each run of equal
 * prefix is finished on chip (same result; ak_sort_route tells which).
 * Scratch: two key buffers, per-tile look-back words, and above 2^16 keys
 * the prefix finish's run lists, plus above 2^22 keys the segmented sort's
 * scratch for long runs (ak_temp_bytes gives the total).
 * Errors: AK_ERR_INVALID_ARG for n < 0, n > AK_MAX_KEYS or keys == NULL
 * with n > 0; AK_ERR_UNSUPPORTED_DTYPE for an unknown dtype. */
ak_status ak_sort(void *keys, int64_t n, ak_dtype dtype, ak_stream_t stream);

/* -------------------------------------------------------- sort, no alloc
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as ak_sort (bit for bit, same kernels), with all scratch in one
 * static device array per GPU (about 37 MiB, held by every GPU the library
 * runs on until the process ends) instead of a workspace.  The call
 * allocates nothing, captures no graph and never synchronises; the array's
 * run state is zeroed on the first call on a device, on that call's stream.
 * Limit: n * key bytes <= AK_NOALLOC_MAX_KEY_BYTES (2^21 64-bit or 2^22
 * 32-bit keys); larger n -> AK_ERR_INVALID_ARG before any launch.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (concurrent streams, or threads) race and must be ordered by the
 * caller.  Errors otherwise as ak_sort. */
#define AK_NOALLOC_MAX_KEY_BYTES ((int64_t)1 << 24)
ak_status ak_sort_noalloc(void *keys, int64_t n, ak_dtype dtype, ak_stream_t stream);

/* -------------------------------------------------------------- sortperm
 * Sec. II-B (sortperm): writes perm[0..n) (0-based uint32 indices) such that
 * keys[perm[0]] <= keys[perm[1]] <= ... under the order above, equal keys in
 * increasing index order (so the permutation is unique).  keys is not
 * modified.  keys and perm must not overlap.  Scratch: 2n keys + n indices.
 * Errors: as ak_sort, plus perm == NULL or perm overlapping keys. */
ak_status ak_sortperm(const void *keys, uint32_t *perm, int64_t n, ak_dtype dtype,
                      ak_stream_t stream);
ak_status ak_sortperm_i32(const int32_t *keys, uint32_t *perm, int64_t n, ak_stream_t stream);
ak_status ak_sortperm_i64(const int64_t *keys, uint32_t *perm, int64_t n, ak_stream_t stream);
ak_status ak_sortperm_u32(const uint32_t *keys, uint32_t *perm, int64_t n, ak_stream_t stream);
ak_status ak_sortperm_u64(const uint64_t *keys, uint32_t *perm, int64_t n, ak_stream_t stream);
ak_status ak_sortperm_f32(const float *keys, uint32_t *perm, int64_t n, ak_stream_t stream);
ak_status ak_sortperm_f64(const double *keys, uint32_t *perm, int64_t n, ak_stream_t stream);

/* ------------------------------------------------------- sort by key
 * Sec. II-B (merge_sort_by_key): sorts keys[0..n) ascending in place and
 * applies the same reordering to vals[0..n) (one payload of `val_bytes`
 * bytes per key, a separate DEVICE array, also in place).  Stable: keys
 * equal under the order keep their payloads in input order, so the result
 * is unique (the oracle: the payloads gathered through ak_sortperm's
 * permutation).  val_bytes is 4 or 8 (any 4- or 8-byte type, moved as
 * bits).  The payload travels with the keys through every digit pass.
 * Scratch: 2n keys + 2n payloads (ak_temp_bytes with AK_OP_SORT_BY_KEY is
 * the bound for 8-byte payloads).  Errors: as ak_sort, plus vals == NULL,
 * val_bytes not 4 or 8, or vals overlapping keys -> AK_ERR_INVALID_ARG. */
ak_status ak_sort_by_key(void *keys, void *vals, int64_t n, ak_dtype dtype, int32_t val_bytes,
                         ak_stream_t stream);

/* ----------------------------------------------------- sortperm, low memory
 * Sec. II-B (sortperm_lowmem): the permutation of ak_sortperm (identical
 * output) with less scratch: only n uint32 indices (plus the per-tile
 * counts), instead of 2n keys + n indices.  Every digit pass reads the
 * indices and fetches their keys from the untouched key array (random
 * reads after the first pass), so it is slower than ak_sortperm.
 * Errors: as ak_sortperm. */
ak_status ak_sortperm_lowmem(const void *keys, uint32_t *perm, int64_t n, ak_dtype dtype, ak_stream_t stream);

/* ------------------------------------------------------- segmented sort
 * Batched form of Sec. II-B's sort: for s in [0, nseg) the segment
 * keys[offsets[s] .. offsets[s+1]) is sorted ascending in place, on its own.
 * keys must hold at least offsets[nseg] elements (the library cannot check
 * the length of a raw pointer; the Python binding checks it).
 * offsets is a DEVICE array of nseg+1 nondecreasing int64 values >= 0; the
 * call reads offsets[0] and offsets[nseg] back to the host (one small
 * synchronous copy) to size its scratch.  Keys outside
 * [offsets[0], offsets[nseg]) are untouched.  Empty segments are allowed.
 * Scratch: offsets[nseg] - offsets[0] keys + per-segment work lists.
 * The launch sequence is captured once per (dtype, nseg, total) into a HIP
 * graph and replayed; pointers travel through a device-side argument block.
 * Errors: nseg < 0, NULL pointers, offsets[nseg] < offsets[0] or a total of
 * more than AK_MAX_KEYS keys -> AK_ERR_INVALID_ARG.  Offsets that decrease inside
 * the array are detected on the device and reported by
 * ak_check_device_error(). */
ak_status ak_segmented_sort(void *keys, const int64_t *offsets, int64_t nseg, ak_dtype dtype,
                            ak_stream_t stream);
/* The same segmented sort with the key count n of the keys array given:
 * scratch is sized from n (an upper bound of offsets[nseg]), and the
 * batch's ends offsets[0] and offsets[nseg] are read and checked on the
 * device, so the call never waits for the device (it synchronises only
 * when the workspace must first grow).  Ends outside [0, n] or decreasing
 * set the device error word (ak_check_device_error) and nothing is sorted;
 * decreasing offsets inside the array are reported the same way.
 * Errors (before any launch): n < 0, n > AK_MAX_KEYS, nseg < 0, NULL
 * pointers -> AK_ERR_INVALID_ARG; n == 0 or nseg == 0 launches nothing. */
ak_status ak_segmented_sort_n(void *keys, int64_t n, const int64_t *offsets, int64_t nseg, ak_dtype dtype,
                              ak_stream_t stream);
ak_status ak_segmented_sort_i32(int32_t *keys, const int64_t *offsets, int64_t nseg, ak_stream_t s);
ak_status ak_segmented_sort_i64(int64_t *keys, const int64_t *offsets, int64_t nseg, ak_stream_t s);
ak_status ak_segmented_sort_u32(uint32_t *keys, const int64_t *offsets, int64_t nseg, ak_stream_t s);
ak_status ak_segmented_sort_u64(uint64_t *keys, const int64_t *offsets, int64_t nseg, ak_stream_t s);
ak_status ak_segmented_sort_f32(float *keys, const int64_t *offsets, int64_t nseg, ak_stream_t s);
ak_status ak_segmented_sort_f64(double *keys, const int64_t *offsets, int64_t nseg, ak_stream_t s);

/* Tuning of the segmented sort for 32- or 64-bit keys (what the autotuner
 * writes to tune_gfx950.json next to libak.so, or $AK_TUNE_TABLE):
 *   ipt_a      keys per lane of the one-wave class (2 or 4: 128 / 256 keys)
 *   ipt_b      keys per lane of the one-workgroup class and of the long
 *              class's tiles (8 or 16; 32 too for 32-bit keys)
 *   grid_mult  persistent workgroups per compute unit (1..16)
 *   b_max      longest segment sorted on chip (0: the class capacity)
 *   xl_min     shortest segment sorted by many workgroups (>= 4096)
 * Takes effect for later calls (a new graph is captured).  AK_ERR_INVALID_ARG
 * for values outside those sets. */
ak_status ak_seg_set_tuning(int key_bits, int ipt_a, int ipt_b, int grid_mult, int b_max, int xl_min);

/* Synchronises `stream`, then returns AK_ERR_INVALID_ARG if a kernel on it
 * found invalid input (decreasing segment offsets) since the last check,
 * and clears the flag; otherwise AK_OK. */
ak_status ak_check_device_error(ak_stream_t stream);

/* ------------------------------------------------- learned-CDF partition sort
 * Same result as ak_sort (bit for bit), reached by partitioning the keys with
 * a learned model of their distribution (a two-level recursive model index:
 * a fixed log-feature root and `leaves` linear leaves trained on a sample the
 * sort draws itself), then sorting every partition on chip; runs of equal
 * model output longer than one workgroup can hold fall back to radix
 * passes.  Config fields (0 selects the default):
 *   leaves       number of linear leaves (default 4096; power of two <= 65536)
 *   buckets_log2 log2 of the number of top-level buckets reported in the
 *                statistics (default 12 = 4096, at most 14)
 *   sample_frac  fraction of keys sampled (default 0.01; at least 4096 keys)
 *   seed         SplitMix64 seed of the sample positions (default 0 is used
 *                as is)
 *   train_iters  Newton iterations of every leaf fit (default 3)
 *   untrained    1: skip training and use equal-width key ranges (the method
 *                without the model, for comparisons)
 *   model        AK_MODEL_RMI (default) or AK_MODEL_MLP (below)
 * `stats` may be NULL; if not, the call synchronises `stream` and fills it.
 * Integer and float dtypes are supported. */
typedef struct {
    int32_t leaves;
    int32_t buckets_log2;
    float sample_frac;
    int32_t train_iters;
    uint64_t seed;
    int32_t untrained;
    int32_t model;             /* AK_MODEL_RMI (0) or AK_MODEL_MLP (1)        */
    int32_t reserved[2];
} ak_learned_cfg;

/* The CDF model of ak_sort_learned (cfg->model):
 *   AK_MODEL_RMI  the two-level model above (train_iters: Newton steps of
 *                 every leaf fit, default 3);
 *   AK_MODEL_MLP  a 1-64-64-1 network (ak_mlp_fit; train_iters: Adam
 *                 steps, default 300), tabulated into the same leaf table,
 *                 so the per-key work of the sort is unchanged. */
#define AK_MODEL_RMI 0
#define AK_MODEL_MLP 1

typedef struct {
    int64_t n;
    int64_t sample_size;
    int32_t leaves;
    int32_t code_bits;
    int64_t max_bucket;        /* largest of the 2^buckets_log2 buckets        */
    double imbalance;          /* max_bucket / (n / 2^buckets_log2)           */
    int64_t fallback_keys;     /* keys in equal-code runs too long for LDS    */
    int64_t constant_keys;     /* of those, keys in runs of one repeated key   */
    int64_t fallback_runs;     /* number of such runs                          */
    int64_t chunks;            /* on-chip chunk sorts performed                */
} ak_learned_stats;

ak_status ak_sort_learned(void *keys, int64_t n, ak_dtype dtype, const ak_learned_cfg *cfg,
                          ak_learned_stats *stats, ak_stream_t stream);

/* -------------------------------------------- learned-model building blocks
 * Exposed so that every step can be checked on its own.  Model buffers are
 * DEVICE float arrays of ak_rmi_model_floats(leaves) = 8 + 4*(leaves+1)
 * floats laid out as [rc, ra, rb, leaves, 0, 0, 0, 0] followed by leaves+1
 * records [a, b, x0, lo] (record `leaves` is a sentinel with lo = 1).  For a
 * key with order-preserving unsigned image t: x = float(t) (round to
 * nearest even), r = float(bits of x);
 * leaf = clamp(floor(ra*(r - rc) + rb), 0, leaves-1);
 * F = clamp(a*(x - x0) + b, lo[leaf], lo[leaf+1]);
 * code = min(floor(F * 2^code_bits), 2^code_bits - 1).  The upper clamp of
 * a leaf is the lower clamp of the next, so with a >= 0 and nondecreasing lo
 * the code never decreases as the key grows.  Every float operation is
 * single precision, rounded to nearest even, multiply then add (never
 * fused). */
size_t ak_rmi_model_floats(int32_t leaves);

/* out[j] = keys[floor(splitmix64(seed, j) * n / 2^64)] for j < m, where
 * splitmix64(seed, j) is output j of SplitMix64 started at state `seed`. */
ak_status ak_learned_sample(const void *keys, int64_t n, ak_dtype dtype, uint64_t seed,
                            int64_t m, void *out, ak_stream_t stream);

/* Fits a model to an ascending sample of m keys: the root spans the
 * sample's feature range in `leaves` equal widths; every leaf is fitted to
 * the empirical CDF j/m of its samples by `iters` Newton steps that use the
 * forward (residual, loss) and backward (gradient, curvature) kernels, with
 * the slope kept >= 0 and the output clamped to [st/m, en/m]. */
ak_status ak_rmi_fit(const void *sorted_sample, int64_t m, ak_dtype dtype, int32_t leaves,
                     int32_t iters, float *model, ak_stream_t stream);

/* Forward + backward of every leaf for a given model (no update).  Each
 * leaf is evaluated in its scaled coordinate dx' = (x_j - x0_i) * s_i, with
 * s_i the power of two 2^-e, 2^e <= max |x - x0_i| over the leaf's samples
 * (1 for an empty or flat leaf), and slope a'_i = a_i / s_i, residual
 * r_j = a'_i*dx' + b_i - j/m.  out is a DEVICE array of 8*leaves floats:
 * out[8*i .. 8*i+7] = sum r^2, dL/da', dL/db, 2*sum dx'^2, 2*sum dx',
 * 2*count, s_i, 0 (float32 sums). */
ak_status ak_rmi_leaf_grad(const void *sorted_sample, int64_t m, ak_dtype dtype,
                           const float *model, float *out, ak_stream_t stream);

/* codes[i] = model code of keys[i] (see above), 1 <= code_bits <= 24. */
ak_status ak_rmi_codes(const void *keys, int64_t n, ak_dtype dtype, const float *model,
                       int32_t code_bits, uint32_t *codes, ak_stream_t stream);

/* -------------------------------------------------------- MLP CDF model
 * The alternative model of the learned sort: f(u) = w3 . tanh(W2 tanh(W1 u
 * + c1) + c2) + c3 with 64 + 64 hidden units, W1 = sp(A1), W2 = sp(A2), w3 =
 * sp(a3), sp = softplus (positive weights and increasing tanh: f increases
 * with u, a monotone CDF estimate).  u in [0, 1] is the root's log-like key
 * feature r (above) over the sample's range: u = (r - r_first) * s, s =
 * 1 / (r_last - r_first) in float32.  Parameters are AK_MLP_PARAMS raw
 * floats: A1[64] | c1[64] | A2[64][64] (row = layer-2 unit) | c2[64] |
 * a3[64] | c3.  Loss: mean over K points of (f(u_k) - y_k)^2. */
#define AK_MLP_PARAMS 4353

/* Forward and backward over K training points (DEVICE arrays u, y of K
 * floats) at `params` (DEVICE, AK_MLP_PARAMS floats): out (DEVICE,
 * AK_MLP_PARAMS + 1 floats) gets dL/dparams (raw parameters) and then L.
 * Float32 sums in a fixed order (64 points per workgroup, then the
 * workgroups in order).  Errors: K < 1, K > 2^20 or a NULL pointer ->
 * AK_ERR_INVALID_ARG. */
ak_status ak_mlp_loss_grad(const float *u, const float *y, int64_t K, const float *params, float *out,
                           ak_stream_t stream);

/* Fits the network to an ascending sample of m keys and tabulates it:
 *   training points: K = min(m, 4096) at ranks j_k = floor((2k+1) m / 2K),
 *   y_k = j_k / m; start at the quantiles of the u_k (layer-1 unit i steps
 *   at u[floor((2i+1) K / 128)]); `iters` Adam steps (lr 0.01, betas 0.9 /
 *   0.999, eps 1e-8);
 *   table: `model` (DEVICE, ak_rmi_model_floats(leaves) floats) gets the
 *   root of ak_rmi_fit (equal feature widths) and leaf records that
 *   interpolate f linearly in x = float32(image) between the knots u_i =
 *   i / leaves, lower clamps lo_i = running maximum of clamp(f(u_i), 0, 1),
 *   lo_0 = 0; `params` (DEVICE, AK_MLP_PARAMS floats, or NULL) gets the
 *   trained raw parameters.
 * Errors: m < 1, leaves not a power of two in [1, 16384], iters < 0 or
 * > 100000 -> AK_ERR_INVALID_ARG. */
ak_status ak_mlp_fit(const void *sorted_sample, int64_t m, ak_dtype dtype, int32_t iters, int32_t leaves,
                     float *params, float *model, ak_stream_t stream);

/* --------------------------------------------------------------- scratch */
typedef enum { AK_OP_SORT = 0, AK_OP_SORTPERM = 1, AK_OP_SEGMENTED = 2, AK_OP_LEARNED = 3,
               AK_OP_ACCUMULATE = 4, AK_OP_SORT_BY_KEY = 5, AK_OP_SORTPERM_LOWMEM = 6 } ak_op;

/* Bytes of device scratch one call of `op` on n keys needs (Sec. II-B: the
 * temporaries are known ahead of the call from the input size).  The value
 * is an upper bound, and a caller arena of this size (ak_set_workspace) is
 * enough for that call.  For AK_OP_SEGMENTED it assumes nseg <= n; use
 * ak_temp_bytes_segmented for the exact segment count.  Only the current
 * tuning table changes the segmented and learned figures.  Returns 0 for
 * n <= 0, an unknown dtype, or sizes sorted on chip without scratch. */
size_t ak_temp_bytes(ak_op op, int64_t n, ak_dtype dtype);
size_t ak_temp_bytes_segmented(int64_t n, int64_t nseg, ak_dtype dtype);

/* Binds a caller-owned device arena [dev_ptr, dev_ptr + bytes) as the
 * scratch of `stream` on the current device.  It waits for the stream, and
 * then frees the library's scratch buffers of that stream.  From then on,
 * every call on the stream carves its temporaries from the arena, 256-byte
 * aligned, starting again at its beginning in each call (earlier calls' work
 * runs first, in stream order), and allocates no scratch.  A call that needs
 * more than the arena holds returns AK_ERR_NO_MEMORY, launches nothing and
 * says how many bytes it needed; ak_temp_bytes gives the size.  The
 * per-stream run states (about 600 KB), segmented-sort argument blocks and
 * cached graphs stay library-owned.  The look-back words of the radix passes
 * are zero-filled when their piece of the arena last held other data (the
 * first call, or a call of another kind that carved its buffers there).
 *   dev_ptr: 256-byte aligned device memory of >= 4096 bytes, or NULL (with
 *            bytes == 0) to unbind and return to library-owned scratch.
 * The caller keeps the arena alive, and leaves it untouched, while it is
 * bound and until the stream's work on it has finished.  Calls on the
 * stream must not overlap (they never do when they share one stream).
 * Errors: misaligned or too small arena, NULL with bytes > 0 ->
 * AK_ERR_INVALID_ARG, nothing changed.  Synchronises the stream. */
ak_status ak_set_workspace(void *dev_ptr, size_t bytes, ak_stream_t stream);

/* Synchronises the device and frees every workspace and cached graph. */
ak_status ak_release_workspace(void);

/* ------------------------------------------------------------- prefix sums
 * Sec. II-B (accumulate with +, inclusive and exclusive; in place or not).
 * in and out hold n keys of `dtype` (DEVICE pointers); out may equal in
 * (in place) but must not overlap it otherwise.
 *   inclusive != 0: out[i] = in[0] + ... + in[i];
 *   inclusive == 0: out[0] = 0, out[i] = in[0] + ... + in[i-1].
 * Integer keys: sums wrap around in the key's width (two's complement for
 * signed keys), so results are exact.  Float keys: sums in the key's own
 * precision, associated as chunk totals of 4096 keys (16 consecutive keys
 * per thread, then wave and workgroup trees) plus a scan of those totals:
 * each result is within d x u x (sum of |in[j]| for j <= i) of the exact
 * sum, u the unit roundoff and d = 88 + 2 ceil(n / 2^22) the most roundings
 * a term passes through (first order).  Asynchronous on
 * `stream`; scratch: one value per 4096 keys (ak_temp_bytes with
 * AK_OP_ACCUMULATE).  Errors: n < 0, n > AK_MAX_KEYS, NULL pointers with n > 0,
 * partial overlap -> AK_ERR_INVALID_ARG; unknown dtype ->
 * AK_ERR_UNSUPPORTED_DTYPE; a bound arena too small -> AK_ERR_NO_MEMORY. */
ak_status ak_accumulate(const void *in, void *out, int64_t n, ak_dtype dtype, int32_t inclusive,
                        ak_stream_t stream);

/* ------------------------------------------------------------ binary search
 * Sec. II-B (searchsortedfirst / searchsortedlast, the lower and upper
 * bound of a sorted collection).  `sorted` holds n keys (DEVICE pointer)
 * in ascending order of this library's total order (the order ak_sort
 * produces: for floats -0.0 before +0.0 and every NaN last, all NaNs
 * equal); `keys` holds m query keys and `out` m int64 results (DEVICE
 * pointers; `out` must not overlap either input).  Indices are 0-based:
 *   ak_searchsortedfirst: out[i] = index of the first element that is not
 *       below keys[i] (n if none), i.e. keys[i] inserted there keeps the
 *       order and lands before its equals;
 *   ak_searchsortedlast:  out[i] = index of the last element that is not
 *       above keys[i] (-1 if none).
 * (The paper's 1-based results are out[i] + 1.)  If `sorted` is not in
 * that order the results are unspecified but in [0, n] / [-1, n-1].
 * Asynchronous on `stream`; no scratch memory.  Errors: n or m < 0, n >=
 * 2^40, a NULL pointer with m > 0 (or `sorted` NULL with n > 0), or `out`
 * overlapping an input -> AK_ERR_INVALID_ARG; unknown dtype ->
 * AK_ERR_UNSUPPORTED_DTYPE. */
ak_status ak_searchsortedfirst(const void *sorted, int64_t n, const void *keys, int64_t m, ak_dtype dtype,
                               int64_t *out, ak_stream_t stream);
ak_status ak_searchsortedlast(const void *sorted, int64_t n, const void *keys, int64_t m, ak_dtype dtype,
                              int64_t *out, ak_stream_t stream);

/* ----------------------------------------------------------- diagnostics
 * How the last call on `stream` ordered its keys, if that call was ak_sort
 * or ak_sortperm on more keys than one workgroup sorts on chip (all zeros
 * otherwise).  Waits for the stream.  info is a HOST array of 5:
 *   info[0] prefix places k: 0 if every active digit place took a pass;
 *           2..4 if the passes covered only the top k places (a key-only
 *           sort of more than 2^16 keys whose top places spread the keys)
 *           and each run of equal prefix was then sorted on chip;
 *   info[1] digit passes run;
 *   info[2] on-chip chunk sorts of the prefix finish;
 *   info[3] runs of equal prefix longer than a chunk, sorted instead by
 *           the segmented sort (above 2^22 keys) or by one workgroup each;
 *   info[4] keys in those runs.
 * Errors: info NULL -> AK_ERR_INVALID_ARG. */
ak_status ak_sort_route(int64_t *info, ak_stream_t stream);

/* ------------------------------------------------------------ profiling
 * While enabled, every library kernel launch is bracketed by HIP events
 * recorded on the stream it is launched on (a few microseconds per launch).
 * ak_profile_read waits for the recorded launches, writes one line
 * "kernel_name count total_ms" per kernel into buf (len bytes, always
 * NUL-terminated), clears the records and returns the bytes it needed. */
ak_status ak_profile_enable(int on);
size_t ak_profile_read(char *buf, size_t len);

const char *ak_status_string(ak_status s);
/* Detail of the last error on the calling thread ("" if none). */
const char *ak_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* AK_H */
