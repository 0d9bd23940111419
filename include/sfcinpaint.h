/*
 * sfcinpaint.h -- C ABI of the MI355X (gfx950) masked-L2 patch search for
 * exemplar-based inpainting, after Dahmen et al., "Space-Filling Curve
 * Indices as Acceleration Structure for Exemplar-Based Inpainting".
 *
 * The library answers the per-iteration question of exemplar-based inpainting
 * (Section I): which fully known patch of the image (the dictionary) best
 * matches the known pixels of a target patch under the masked L2 cost. It
 * does so either by a full scan of the dictionary (Section I) or through the
 * space-filling-curve multi-index of Section II (pixel subsets, PCA to D
 * dimensions, several shifted curves, binary search, a candidate window per
 * curve, exact rescoring of the candidates in image space).
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers (HIP device memory) unless the
 *    argument name ends in _host. All work is enqueued on the stream given in
 *    sfc_options (NULL = the default stream) or in a `stream` argument
 *    (a hipStream_t passed as void*). Outputs are valid once that stream has
 *    synchronised; functions that return a host value synchronise it.
 *  - Layouts: a volume is float32 [shape[0], ..., shape[ndim-1], channels],
 *    channel innermost, spatial dims slowest first. A mask is uint8
 *    [shape...], 1 = known, 0 = missing. A voxel id is the row-major linear
 *    index over the spatial dims. A patch has K^ndim pixels (K odd, centred
 *    on its voxel id); pixel rho is the row-major index in the K^ndim box;
 *    element e = rho*channels + ch. A target is float32 [Q, K^ndim, channels]
 *    and its mask uint8 [Q, K^ndim].
 *  - Every function returns an sfc_status (0 = success, negative = error),
 *    never throws, and leaves its outputs untouched on argument errors.
 *    sfc_last_error() gives a message for the calling thread's last error.
 *  - Results are deterministic: the same inputs give the same bits. The
 *    selected patch is the minimum of (cost, id), so ties go to the lowest id.
 */
#ifndef SFCINPAINT_H
#define SFCINPAINT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SFC_ABI_VERSION 2

typedef enum {
    SFC_OK = 0,
    SFC_EINVAL = -1,       /* invalid argument (null pointer, bad geometry, range) */
    SFC_ENOMEM = -2,       /* device allocation failed */
    SFC_EDEVICE = -3,      /* a HIP call or kernel launch failed */
    SFC_EEMPTY = -4,       /* the dictionary has no fully known patch */
    SFC_EUNSUPPORTED = -5  /* valid but outside what this build handles */
} sfc_status;

typedef enum { SFC_CURVE_MORTON = 0, SFC_CURVE_HILBERT = 1 } sfc_curve;

typedef enum {
    SFC_MODE_BRUTE_FP32 = 0,  /* full scan, float32 fixed-order cost */
    SFC_MODE_BRUTE_BF16 = 1,  /* full scan, bf16 MFMA filter + exact rescoring */
    SFC_MODE_BRUTE_FP8 = 2,   /* full scan, fp8 MFMA filter + exact rescoring */
    SFC_MODE_INDEX = 3        /* space-filling-curve multi-index */
} sfc_mode;

typedef enum { SFC_ORDER_CRIMINISI = 0, SFC_ORDER_RASTER = 1 } sfc_order;

/* The patch distance that ranks candidates: the masked squared L2 sum of
 * Section II, or the masked L1 sum of Section III.K's variant (the same
 * known elements in the same order, |t - v| added in float32). */
typedef enum { SFC_NORM_L2 = 0, SFC_NORM_L1 = 1 } sfc_norm;

typedef struct {
    int32_t ndim;       /* 2 or 3 */
    int32_t channels;   /* C >= 1 */
    int64_t shape[3];   /* spatial extent, slowest first; unused entries ignored */
} sfc_geometry;

typedef struct {
    uint32_t struct_size;  /* sizeof(sfc_options); older callers pass less */
    int32_t key_bits;      /* b, bits per principal coordinate (1..31), default 8 */
    int32_t window;        /* W, candidates taken from each curve, default 32 */
    int32_t curve;         /* sfc_curve, default SFC_CURVE_MORTON */
    int32_t query_block;   /* queries per float32-scan workgroup, 0 = library choice */
    int32_t scan_variant;  /* float32-scan tile shape: 0 = default or the one
                              sfc_autotune chose, k >= 1 = the k-th shape */
    void *stream;          /* hipStream_t; NULL = default stream */
    int32_t timing;        /* 1: record HIP events around the main kernels of
                              each sfc_query call (sfc_query_kernel_times);
                              default 0 */
    int32_t norm;          /* sfc_norm of the float32 scan and the index's
                              rescoring, default SFC_NORM_L2. With SFC_NORM_L1
                              the reduced-precision modes, batches, the fill
                              loop and sfc_autotune return SFC_EUNSUPPORTED, and
                              the float32 scan uses its default tile shape. */
} sfc_options;

typedef struct sfc_index sfc_index;  /* opaque */

typedef struct {
    int64_t n;             /* dictionary size */
    int64_t n_sub;         /* PCA subsample size (0 without an SFC index) */
    int32_t ndim, channels, K, P;
    int32_t has_sfc;       /* 0: dictionary only (full-scan modes) */
    int32_t n_subsets, reduced_dim, n_curves, key_bits, key_words, window, curve;
    float vmin, qscale;    /* byte-quantisation parameters */
} sfc_index_info;

typedef struct {
    int64_t cap;           /* entries the arrays hold */
    int64_t len;           /* entries written (<= cap) */
    int64_t *centre_host;  /* target centre of each iteration */
    int64_t *source_host;  /* chosen dictionary centre */
    float *cost_host;      /* its cost */
} sfc_fill_log;

/* Library ABI version (SFC_ABI_VERSION). */
int32_t sfc_abi_version(void);

/* Message for the calling thread's last error ("" if none). */
const char *sfc_last_error(void);

/* Fill the defaults documented in sfc_options. */
void sfc_options_default(sfc_options *opt);

/* Temporaries of the index build (and of the dictionary build) come from a
 * stream-ordered memory pool of the library, one per device, which keeps up
 * to 8 GiB of freed memory for reuse; freeing them never waits for work on
 * other streams. The environment variable SFC_TMP_POOL=0, read at the first
 * temporary on a device, makes them plain hipMalloc / hipFree allocations.
 *
 * Error-path testing: the n-th device allocation the library makes from now
 * on (any thread) fails with SFC_ENOMEM and the message "...: injected
 * allocation failure"; n <= 0 turns this off. Not for production use. */
void sfc_debug_fail_alloc(int64_t n);

/* Overflow-path testing: the candidate list of each query of the
 * reduced-precision scan holds `cap` entries (rounded down to a multiple of
 * 64, at least 64) instead of the automatic 2048..16384, so that lists
 * overflow and those queries take the float32 scan; cap <= 0 restores the
 * automatic size. Process-wide. Not for production use. */
void sfc_debug_list_capacity(int32_t cap);

/* Fill front (Fig. 1a: known pixels adjacent to unknown ones; adjacency =
 * shared face). Writes the front's voxel ids in ascending order to
 * centres[0 .. min(count, capacity)), and the total to *count_host.
 * mask: device uint8 [shape]. Synchronises `stream`. */
sfc_status sfc_fill_front(const uint8_t *mask, const sfc_geometry *g, int64_t *centres,
                          int64_t capacity, int64_t *count_host, void *stream);

/* Target patches (Fig. 1a: the search area is the known part of the patch
 * at a front voxel). For each centre: targets = volume value of in-bounds
 * known pixels, 0 elsewhere; target_masks = 1 where in bounds and known.
 * centres: device int64 [Q]; targets float32 [Q, K^ndim, C]; masks uint8
 * [Q, K^ndim]. Q = 0 is a no-op. */
sfc_status sfc_extract_targets(const float *volume, const uint8_t *mask,
                               const sfc_geometry *g, int32_t K, const int64_t *centres,
                               int64_t Q, float *targets, uint8_t *target_masks,
                               void *stream);

/* Dictionary only (Section I: every fully known K^ndim patch lying inside the
 * volume), for the full-scan modes. The handle BORROWS `volume`: it must stay
 * alive and its dictionary patches unchanged until sfc_index_free. The mask
 * is copied into the handle. Returns SFC_EEMPTY if no patch is fully known. */
sfc_status sfc_dictionary_build(const float *volume, const uint8_t *mask,
                                const sfc_geometry *g, int32_t K, const sfc_options *opt,
                                sfc_index **out);

/* Full SFC multi-index (Section II): byte quantisation, 3^ndim - 1 pixel
 * subsets of ceil(0.6 K^ndim) pixels each (Fig. 2), exact integer covariance,
 * float64 Jacobi eigendecomposition and an int8 basis of the first
 * reduced_dim components per subset (Section II.A), and n_curves shifted
 * curves per subset whose (key, id) arrays are sorted on the device
 * (Section II.C). Also usable for the full-scan modes. Same borrowing rule
 * as sfc_dictionary_build. Errors: SFC_EINVAL for K even, K > a side,
 * reduced_dim < 1 or > a subset's element count, n_curves < 1 or >
 * reduced_dim + 1, key_bits * reduced_dim > 256; SFC_EUNSUPPORTED for a
 * subset with more than 518 elements (the eigensolver's bound), n_curves *
 * window above 2048, or more than 2^32 voxels. */
sfc_status sfc_index_build(const float *volume, const uint8_t *mask, const sfc_geometry *g,
                           int32_t K, int32_t reduced_dim, int32_t n_curves,
                           const sfc_options *opt, sfc_index **out);

/* As sfc_index_build, but with the int8 bases given instead of computed:
 * bases_host holds, subset after subset, m_s x reduced_dim int8 row-major
 * (m_s = the subset's element count). */
sfc_status sfc_index_build_with_basis(const float *volume, const uint8_t *mask,
                                      const sfc_geometry *g, int32_t K, int32_t reduced_dim,
                                      int32_t n_curves, const sfc_options *opt,
                                      const int8_t *bases_host, sfc_index **out);

/* Best dictionary patch for each target (Fig. 1). cost = float32 sum over
 * known rho ascending, channel ascending, of d*d (d = target - patch value)
 * as a fused-multiply-add chain from +0; the answer minimises (cost, id).
 * SFC_MODE_BRUTE_* modes return the global minimum over the dictionary (the
 * reduced-precision ones certify it or fall back); SFC_MODE_INDEX returns the
 * minimum over the index's candidates. best_id int64 [Q], best_cost float32
 * [Q]. Q = 0 is a no-op. SFC_EINVAL for SFC_MODE_INDEX on a dictionary-only
 * handle. */
sfc_status sfc_query(sfc_index *idx, const float *targets, const uint8_t *target_masks,
                     int64_t Q, sfc_mode mode, int64_t *best_id, float *best_cost);

/* Size of the fixed device array that sfc_query_fp32_noalloc works in: one
 * copy per device, held until the process ends. */
#define SFC_NOALLOC_SCRATCH_BYTES (16u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * float32 full scan as sfc_query in SFC_MODE_BRUTE_FP32, with the same
 * answers bit for bit, but neither this call nor anything it calls allocates
 * device memory or creates events. Its row masks, padded targets and packed
 * per-query results live in the library's fixed array of
 * SFC_NOALLOC_SCRATCH_BYTES on the current device; sfc_noalloc_bytes(idx, Q)
 * gives what Q queries need: round256(qpad * K^(ndim-1) * 4) +
 * round256(qpad * K^ndim * channels * 4) + round256(qpad * 8), qpad = Q
 * rounded up to a multiple of 48 (about 16,500 queries of 9x9x3, 150,000 of
 * 9x9x1). The caller passes device inputs and outputs as for sfc_query;
 * the index's device must be the current device. Every call on a device
 * shares that device's array: two calls whose work overlaps on one device
 * (on different streams, or from different threads before the first has
 * finished on its stream) race and give wrong answers. The handle's own
 * growable buffers are not touched; the handle's timing switch is ignored.
 * Errors: SFC_EINVAL for a null pointer, Q < 0, Q above the array's
 * capacity (with the needed size in the message) or another device current;
 * SFC_EDEVICE if the array's address cannot be found. */
sfc_status sfc_query_fp32_noalloc(sfc_index *idx, const float *targets,
                                  const uint8_t *target_masks, int64_t Q, int64_t *best_id,
                                  float *best_cost);

/* Bytes of the fixed array that Q queries need in sfc_query_fp32_noalloc
 * (-1 for a NULL handle or Q < 0). */
int64_t sfc_noalloc_bytes(const sfc_index *idx, int64_t Q);

/* Exact k-NN query of Section II.D on an index built with Morton curves:
 * for each target, the chosen subset and grid cell as in SFC_MODE_INDEX, the
 * k dictionary patches whose cells on the unshifted curve (curve 0) are
 * nearest in squared Euclidean distance (ties: lower id), found by the
 * outside-in traversal of the curve (litmax/bigmin splits at the most
 * significant differing bit, searches restricted to the parent interval,
 * nearer part first, parts farther than the k-th distance skipped, regions
 * of at most mu entries scanned); the answer minimises (cost, id) over those
 * k, with the handle's norm. best_id int64 [Q], best_cost float32 [Q];
 * cand (nullable) int64 [Q, k] the k ids ascending, padded with -1 when the
 * dictionary has fewer; ncand (nullable) int32 [Q]. Q = 0 is a no-op.
 * SFC_EINVAL: no SFC index, k outside 1..256, mu < 1, null targets or
 * results; SFC_EUNSUPPORTED: Hilbert curves, reduced_dim above 16, or
 * 2*key_bits + ceil(log2(reduced_dim)) above 62 (the squared cell distances
 * are summed in int64). */
sfc_status sfc_query_knn(sfc_index *idx, const float *targets, const uint8_t *target_masks,
                         int64_t Q, int32_t k, int32_t mu, int64_t *best_id, float *best_cost,
                         int64_t *cand, int32_t *ncand);

/* Candidate sets of the index query: cand int64 [Q, n_curves*window], the
 * sorted unique dictionary ids per query padded with -1; ncand int32 [Q]. */
sfc_status sfc_query_candidates(sfc_index *idx, const float *targets,
                                const uint8_t *target_masks, int64_t Q, int64_t *cand,
                                int32_t *ncand);

/* Per-query subset choice and real principal coordinates (diagnostics):
 * subset int32 [Q], coords float64 [Q, reduced_dim]. */
sfc_status sfc_query_coords(sfc_index *idx, const float *targets,
                            const uint8_t *target_masks, int64_t Q, int32_t *subset,
                            double *coords);

/* Autotuner: times every float32-scan tile shape available for the handle's
 * (ndim, K, channels) on these targets (one warm-up and one timed run each,
 * HIP events on the handle's stream) and keeps the fastest for later
 * SFC_MODE_BRUTE_FP32 queries of this handle (unless options.scan_variant
 * forces one) and for handles of the same shape created later in the
 * process. *chosen_host receives the chosen shape (>= 1). Synchronises. */
sfc_status sfc_autotune(sfc_index *idx, const float *targets, const uint8_t *target_masks,
                        int64_t Q, int32_t *chosen_host);

/* One window width tried by sfc_autotune_window. */
typedef struct {
    int32_t window;        /* W */
    float recall;          /* fraction of targets whose index answer is the full scan's */
    float accel_error;     /* mean distance ratio index / scan - 1 over targets with a
                              nonzero scan cost (Section III.C's acceleration error):
                              sqrt(cost_index / cost_scan) - 1 for L2, cost_index /
                              cost_scan - 1 for L1 */
    float ms;              /* index query time on these targets (HIP events) */
} sfc_window_trial;

/* Window autotuner for SFC_MODE_INDEX: answers the targets with the float32
 * full scan, then with the index at W = 2, 4, 6, 8, 12, ..., 1024 (while
 * n_curves * W <= 2048), and keeps on the handle the smallest W whose recall
 * reaches target_recall (in [0, 1]) and whose acceleration error (Section
 * III.C, as in sfc_window_trial) is at most max_accel_error (a fraction, so
 * 0.01 for the paper's 1 %; a negative value drops this condition); the
 * largest W tried if none qualifies. *window_host receives it; the trials
 * (up to capacity) go to trials_host and their number to *count_host. The
 * window is a query-time parameter: the index itself is not rebuilt.
 * Synchronises. SFC_EINVAL for a NaN max_accel_error. */
sfc_status sfc_autotune_window(sfc_index *idx, const float *targets, const uint8_t *target_masks,
                               int64_t Q, float target_recall, float max_accel_error,
                               sfc_window_trial *trials_host, int32_t capacity,
                               int32_t *count_host, int32_t *window_host);

/* Statistics of the last sfc_query call on this handle (host values):
 * n_fallback = queries a reduced-precision scan could not certify. */
sfc_status sfc_query_stats(const sfc_index *idx, int64_t *n_fallback_host);

/* Work of the last SFC_MODE_BRUTE_BF16 query on this handle (host values):
 * *pass1_host = (query tile, candidate tile) pairs of the filter's first
 * pass (all of them), *pass2_host = pairs a second pass revisited (those
 * whose tile minimum can reach a query's threshold). On a handle with an SFC
 * index the index answer's exact cost seeds the threshold and there is no
 * second pass (*pass2_host = 0). Both 0 after other modes. */
sfc_status sfc_query_filter_tiles(const sfc_index *idx, int64_t *pass1_host, int64_t *pass2_host);

/* Duration of one kernel of the last sfc_query call. */
typedef struct {
    const char *kernel;    /* kernel name (static string owned by the library) */
    int32_t launches;      /* launches timed */
    float ms;              /* their total duration (HIP events on the handle's stream) */
} sfc_kernel_time;

/* Turns the recording of kernel durations (options.timing) on (1) or off
 * (0) for this handle's next queries; times already recorded and not yet
 * read are kept. SFC_EINVAL: NULL handle. */
sfc_status sfc_set_timing(sfc_index *idx, int32_t on);

/* Kernel durations of the sfc_query / sfc_query_knn calls made on this
 * handle since the times were last read, one entry per kernel (launches and
 * total milliseconds), recorded only while the handle's options.timing is 1
 * (else *count_host = 0); reading clears them, and at most 4096 launches
 * are kept between reads. The float32 scan records "scan_fp32_kernel", the
 * bf16 scan "filter_kernel<list>" and "list_rescore_kernel", plus
 * "filter_kernel<min>" on a dictionary-only handle (its first pass) and
 * "scan_fp32_kernel<fallback>" for the queries it could not settle, the
 * index query "prologue_kernel", "search_kernel" and "rescore_kernel", the
 * k-NN query "prologue_kernel", "knn_kernel" and "list_rescore_kernel".
 * Writes min(count, capacity) entries to times_host and the number of
 * kernels to *count_host. Waits for the timed launches to finish. */
sfc_status sfc_query_kernel_times(const sfc_index *idx, sfc_kernel_time *times_host,
                                  int32_t capacity, int32_t *count_host);

/* Handle description. */
sfc_status sfc_index_info_get(const sfc_index *idx, sfc_index_info *info_host);

/* Dictionary ids, ascending: device int64 [n]. */
sfc_status sfc_index_dictionary(const sfc_index *idx, int64_t *ids);

/* Byte-quantised volume: device uint8 [shape, C]. */
sfc_status sfc_index_quantized(const sfc_index *idx, uint8_t *xq);

/* A subset's int8 basis (host, m_s x reduced_dim) and element count. */
sfc_status sfc_index_get_basis(const sfc_index *idx, int32_t subset, int8_t *basis_host,
                               int32_t *rows_host);

/* A subset's grid parameters: lo_host int64 [reduced_dim], span_host. */
sfc_status sfc_index_get_params(const sfc_index *idx, int32_t subset, int64_t *lo_host,
                                int64_t *span_host);

/* Principal coordinates of every dictionary patch for one subset, exact
 * integers: device int64 [n, reduced_dim] in dictionary order. */
sfc_status sfc_index_projection(const sfc_index *idx, int32_t subset, int64_t *y);

/* One sorted curve: keys uint64 [n, key_words] (word 0 most significant)
 * and ids int64 [n], in (key, id) order. */
sfc_status sfc_index_export(const sfc_index *idx, int32_t subset, int32_t curve,
                            uint64_t *keys, int64_t *ids);

/* Release the handle and its device memory. NULL is a no-op. */
void sfc_index_free(sfc_index *idx);

/* Saved indices, for dictionaries used again (the paper precomputes and
 * stores its indices; Sections III and IV). sfc_index_save writes to the
 * host file `path` what defines an SFC index handle: a header (geometry,
 * K, reduced_dim, n_curves, key_bits, curve, window, dictionary size, a
 * hash of the dictionary ids and a checksum of the known voxels' byte
 * codes), the subsample statistics, the int8 bases and the grid origin and
 * span of every subset (a few KiB). sfc_index_load makes a handle from such
 * a file for the same volume and mask (borrowed and copied as in
 * sfc_index_build): the dictionary and byte codes are rebuilt and must
 * match the file's (size, hash, quantisation, checksum); the statistics and
 * bases are read, the curves rebuilt from them (projection, keys, sort: on
 * the GPU that is faster than reading sorted curves from host storage) and
 * the rebuilt grid must equal the saved one. reduced_dim, n_curves,
 * key_bits, curve and window come from the file, the other options from
 * `opt`. The loaded handle answers every query exactly as the saved one.
 * SFC_EINVAL: null pointer, a dictionary-only handle, an unreadable,
 * truncated or inconsistent file, or one made for another geometry, K,
 * volume or mask. */
sfc_status sfc_index_save(const sfc_index *idx, const char *path);
sfc_status sfc_index_load(const float *volume, const uint8_t *mask, const sfc_geometry *g,
                          int32_t K, const sfc_options *opt, const char *path, sfc_index **out);

/* The sort that orders every curve of an index (Section II.C: a curve's
 * entries by curve position), on caller arrays: each of `arrays`
 * consecutive arrays of n (key, id) pairs is sorted in place by key
 * ascending, stably (equal keys keep their input order; with ids ascending
 * on entry that is (key, id) order). keys: device uint64
 * [arrays][key_words][n], word 0 the most significant; ids: device uint32
 * [arrays][n]. An LSD radix sort over 8-bit digits that skips digit
 * positions constant over the arrays; its scratch (about 24 bytes per pair,
 * at most 8 GiB at a time) is allocated and freed inside the call, which
 * synchronizes `stream` (hipStream_t, NULL = default) before returning.
 * SFC_EINVAL: null pointer, n < 0, arrays < 1 or key_words outside 1..4;
 * SFC_EUNSUPPORTED: n >= 2^32. n <= 1 is a no-op. */
sfc_status sfc_sort_pairs(uint64_t *keys, uint32_t *ids, int64_t n, int32_t key_words,
                          int32_t arrays, void *stream);

/* Fill loop (Section I, Criminisi order): while a voxel is unknown, pick the
 * front voxel of highest (priority, confidence, -id) (SFC_ORDER_CRIMINISI)
 * or the lowest front id (SFC_ORDER_RASTER), query its target patch in
 * `mode`, copy the chosen patch into the unknown in-bounds pixels of the
 * target, mark them known. volume and mask are updated in place. The
 * dictionary is fixed at the start: `idx` if given (it must have been built
 * from this volume and mask), else a private one (with an SFC index when
 * mode == SFC_MODE_INDEX, using reduced_dim 8 and 4 curves). *n_iters_host
 * receives the iteration count; log (nullable, host arrays) the first cap
 * iterations. SFC_EINVAL if K < 3; SFC_EEMPTY if the dictionary is empty or
 * unknown voxels remain with an empty front. */
sfc_status sfc_inpaint(float *volume, uint8_t *mask, const sfc_geometry *g, int32_t K,
                       sfc_order order, sfc_mode mode, sfc_index *idx,
                       const sfc_options *opt, int64_t *n_iters_host, sfc_fill_log *log);

/* ---- Batches of images (many independent 2D images of uneven size, each
 * with its own dictionary: Section I's full scan per image), answered by one
 * persistent float32-scan launch over (image, query block, tile chunk) work
 * items. A query is captured once in a HIP graph on the batch's own stream
 * and replayed while its layout (per-image counts and the four buffer
 * pointers) stays the same; any change recaptures. Ordering with the
 * caller's stream (options.stream) uses events. */
typedef struct sfc_batch sfc_batch;  /* opaque */

/* volumes/masks: host arrays of n_images device pointers (each borrowed as
 * in sfc_dictionary_build); geoms: host array of n_images geometries, each
 * 2D with 1 to 3 channels. K in {5, 7, 9, 11}. SFC_EEMPTY if an image has no
 * fully known patch. */
sfc_status sfc_batch_create(int32_t n_images, const float *const *volumes_host,
                            const uint8_t *const *masks_host, const sfc_geometry *geoms_host,
                            int32_t K, const sfc_options *opt, sfc_batch **out);

/* Best patch of every target of every image. targets: the concatenation over
 * images of float32 [count_i, K*K, channels_i]; target_masks: uint8
 * [sum count_i, K*K]; best_id int64 / best_cost float32 [sum count_i], ids
 * local to each image (its voxel ids). counts_host: n_images counts (>= 0).
 * Same cost, order and tie rule as sfc_query in SFC_MODE_BRUTE_FP32. */
sfc_status sfc_batch_query(sfc_batch *b, const float *targets, const uint8_t *target_masks,
                           const int64_t *counts_host, int64_t *best_id, float *best_cost);

/* Autotuner for the batched scan: times each tile-shape set (one replay
 * after a warm-up run each) on these queries and keeps the fastest;
 * *chosen_host receives it (0..2). The outputs hold the last run's answers. */
sfc_status sfc_batch_autotune(sfc_batch *b, const float *targets, const uint8_t *target_masks,
                              const int64_t *counts_host, int64_t *best_id, float *best_cost,
                              int32_t *chosen_host);

/* Graph replays so far, work items of the current graph, tile-shape set. */
sfc_status sfc_batch_stats(const sfc_batch *b, int64_t *graph_replays_host,
                           int64_t *work_items_host, int32_t *shape_host);

/* Release the batch (NULL is a no-op). */
void sfc_batch_free(sfc_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* SFCINPAINT_H */
