/*
 * maskgs.h -- C ABI of the MI355X (gfx950) masked Gaussian rasterizer.
 *
 * Masked rasterization of 3D Gaussians, forward and backward, after
 * MaskGaussian (Liu et al., arXiv 2412.20522):
 *   - every Gaussian is splatted to a 2D Gaussian with a colour from
 *     view-dependent spherical harmonics and alpha_i = o_i * G2D_i(x)
 *     (Sec. 3.1), unaffected by its mask (Sec. 3.2-3.3);
 *   - per pixel, the Gaussians that intersect the pixel's tile and pass the
 *     alpha filter are composited front to back in depth order with the mask
 *     gating both colour accumulation and transmittance attenuation,
 *     Eq. (3)-(4), plus the final transmittance times the background colour
 *     (supplementary derivation of the mask gradient);
 *   - the backward pass returns dL/dM_i for every Gaussian that passed the
 *     alpha filter, whether its mask is 0 or 1, Eq. (6) with the colour
 *     behind read relative to T_{i+1} and the background term of the
 *     supplementary material, and the usual gradients of centres, conics,
 *     opacities and colours, which are zero for masked entries (Fig. 1).
 *   - masks come from two scores per Gaussian through a straight-through
 *     Gumbel-Softmax (Sec. 3.3); the mask-count loss is Eq. (7)-(8).
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers owned by the caller unless the
 *     parameter says "host".  The library never frees caller memory.
 *   - Every call is asynchronous on the caller's stream unless its comment
 *     says it synchronises.  A NULL stream is the null stream.
 *   - Arrays are dense, row-major, float32 unless stated; N = number of
 *     Gaussians, V = number of views, R = V * N projected records
 *     (record r = view * N + gaussian), K = number of (tile, Gaussian)
 *     instances, P = total pixels over all views.
 *   - Images are packed view after view, each view as [3, H_v, W_v];
 *     per-pixel arrays are packed view after view as [H_v, W_v].
 *   - Arguments are validated on the host.  A failing call returns a status
 *     other than MGS_OK, launches nothing, and sets the message returned by
 *     mgs_last_error.  No C++ exception crosses this boundary.
 *   - Conditions found on the device (capacity overflow, non-finite values)
 *     set device flags reported as MGS_ERR_CAPACITY / MGS_ERR_NONFINITE by the
 *     next call that synchronises (mgs_forward reads them when it reads K).
 */
#ifndef MASKGS_H
#define MASKGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MGS_API __attribute__((visibility("default")))
#define MGS_MAX_VIEWS 16
/* Side, in tiles, of the regions that list wide records. */
#define MGS_REGION_TILES 4

typedef struct ihipStream_t* mgs_stream; /* hipStream_t */

typedef enum {
    MGS_OK = 0,
    MGS_ERR_INVALID_ARG = 1,
    MGS_ERR_OOM = 2,
    MGS_ERR_CAPACITY = 3,
    MGS_ERR_NONFINITE = 4,
    MGS_ERR_HIP = 5,
    MGS_ERR_UNSUPPORTED = 6,
    MGS_ERR_STATE = 7
} mgs_status;

/* Pinhole camera.  viewmat maps world to camera, row-major 4x4, camera +z
 * forward, +y down, +x right; fx, fy, cx, cy in pixels; pixel (x, y) has its
 * centre at (x + 0.5, y + 0.5). */
typedef struct {
    float viewmat[16];
    float fx, fy, cx, cy;
    int32_t width, height;
} mgs_camera;

/* Rasterization constants (defaults from mgs_default_settings). */
typedef struct {
    int32_t tile_w, tile_h;  /* 8x8, 16x8, 16x16 or 32x8 pixels (16x16, Sec. 3.1) */
    int32_t batch_depth;     /* entries staged in LDS per batch: 32, 64, 128 or 256,
                                at most tile_w * tile_h */
    int32_t sh_degree;       /* 0..3 */
    float alpha_min;         /* alpha filter, 1/255 ("alpha > 0", Sec. 3.1) */
    float alpha_max;         /* alpha clamp, 0.99 */
    float t_min;             /* early termination: stop before T drops below 1e-4 */
    float q_max;             /* per-pixel cut on the Mahalanobis form, 9 (3 sigma) */
    float near_plane;        /* cull depth <= 0.2 */
    float dilation;          /* added to the 2D covariance diagonal, 0.3 */
    float jac_clamp;         /* lateral clamp of the EWA Jacobian, 1.3 * tan(fov/2) */
    float lambda_floor;      /* floor of the eigenvalue discriminant, 0.1 */
    float bg[3];             /* background colour */
    int32_t exact_mode;      /* 1: alpha_min = 0, t_min = 0, no Q cut, every valid
                                Gaussian in every tile (for calculus tests) */
    int32_t persistent;      /* 1: compositing pops tiles from a device queue */
    int32_t fwd_ppt;         /* pixels per thread in forward compositing: 1, 2 or 4
                                (tile_w * tile_h / ppt threads per workgroup, a
                                multiple of 64) */
    int32_t bwd_ppt;         /* pixels per thread in backward compositing */
    int32_t wide_tiles;      /* hybrid binning: a record covering more tiles than
                                this is listed once per region of
                                MGS_REGION_TILES^2 tiles it overlaps instead of
                                once per tile; the compositing merges a region's
                                list into each of its tiles' lists, so results
                                are those of plain binning.  0: 64 tiles;
                                < 0: off */
    int32_t stats;           /* 1: the forward writes per-pixel work counters
                                (mgs_frame_count_evals, exports STATS and EVALS);
                                0: it does not (slightly faster) */
    int32_t tile_cull;       /* 1: a record is listed only in the tiles (regions)
                                of its rectangle where it can pass the per-pixel
                                filters (Q <= q_max, alpha >= alpha_min) at some
                                pixel centre (a conservative exact test), and a
                                region entry joins a tile's list only if it
                                passes the same test for that tile, which leaves
                                every image and gradient unchanged;
                                0: every tile (region) of its rectangle, the
                                lists of Sec. 3.1 exactly (for list parity and
                                for counting entries examined on those lists) */
    int32_t mask_mode;       /* how M_i enters the rendering:
                                MGS_MASK_RASTER (0): masked rasterization,
                                Eq. 3-4, with dL/dM_i of Eq. 6 for every
                                Gaussian, sampled or not;
                                MGS_MASK_OPACITY (1): the prior-art product
                                of the ablation in Sec. 4.3 (Table 7): the
                                opacity becomes M_i * sigmoid(logit) before
                                the alpha clamp and filter, so an unsampled
                                Gaussian is filtered out and receives no
                                gradient at all; dL/dM_i is the chain rule
                                through that product */
} mgs_settings;

#define MGS_MASK_RASTER 0
#define MGS_MASK_OPACITY 1

/* Gaussian parameters (device pointers, float32). */
typedef struct {
    const float* means;          /* [N, 3] */
    const float* log_scales;     /* [N, 3] */
    const float* quats;          /* [N, 4] (w, x, y, z), need not be unit */
    const float* opacity_logits; /* [N], opacity = sigmoid(logit) */
    const float* sh;             /* [N, (d+1)^2, 3], index l*l + l + m */
    const float* masks;          /* [N], sampled mask M_i, normally 0 or 1;
                                    any value in [0, 1] is well defined */
    int64_t n;
} mgs_gaussians;

/* Gradient outputs (device pointers, float32).  Any pointer may be NULL to
 * skip that output.  With accumulate = 0 every output is overwritten; with
 * accumulate = 1 the parameter and mask gradients are added to what the
 * arrays hold (per-view calls summing a multi-view gradient), d_records is
 * still overwritten. */
typedef struct {
    float* d_means;          /* [N, 3] */
    float* d_log_scales;     /* [N, 3] */
    float* d_quats;          /* [N, 4] */
    float* d_opacity_logits; /* [N] */
    float* d_sh;             /* [N, (d+1)^2, 3] */
    float* d_masks;          /* [N], dL/dM_i, Eq. (6) plus background term */
    float* d_records;        /* [R = n_views N, 9] (mgs_backward only): the
                                per-record 2D gradients before the chain
                                rule, record v N + i for view v, Gaussian i:
                                dL/d(u, v), dL/d(a, b / a, c - b^2 / a) of the
                                stored conic, dL/dopacity (of M_i o_i under
                                MGS_MASK_OPACITY), dL/d(r, g, b); rows of
                                records without a valid projection are 0 */
    int32_t accumulate;      /* 0: overwrite, 1: add (see above) */
} mgs_gradients;

typedef struct {
    int64_t n_gaussians, n_views, n_records, n_pixels;
    int64_t n_instances;     /* K of the last forward: list entries (tile and
                                region) */
    int64_t total_tiles;
    int64_t instance_capacity;
    int64_t n_wide;          /* records listed per region (hybrid binning) */
    int32_t sort_passes;
    int32_t tile_bits;
} mgs_frame_stats;

typedef struct mgs_ctx mgs_ctx;
typedef struct mgs_frame mgs_frame;

/* ---------------------------------------------------------------------- */
/* lifecycle                                                               */
/* ---------------------------------------------------------------------- */

/* Library version (major * 10000 + minor * 100 + patch). */
MGS_API int mgs_version(void);

/* Fills *out with the defaults listed on mgs_settings. */
MGS_API mgs_status mgs_default_settings(mgs_settings* out);

/* Creates a context on HIP device `device` (checks it is a gfx950).  *out
 * (host) receives the handle; free it with mgs_destroy. */
MGS_API mgs_status mgs_create(int device, mgs_ctx** out);
MGS_API mgs_status mgs_destroy(mgs_ctx* ctx);

/* Message of the last failed call on ctx (or of the last failed mgs_create
 * when ctx is NULL).  The string belongs to the library and stays valid
 * until the next call on the same context. */
MGS_API const char* mgs_last_error(const mgs_ctx* ctx);

/* A frame holds what one forward saves for its backward (projected records,
 * sorted instance lists, tile ranges, per-pixel final transmittance and last
 * blended entry).  Its device buffers grow on demand and are reused by later
 * forwards.  One forward, then at most one backward, per frame at a time. */
MGS_API mgs_status mgs_frame_create(mgs_ctx* ctx, mgs_frame** out);
MGS_API mgs_status mgs_frame_destroy(mgs_frame* frame);
MGS_API mgs_status mgs_frame_get_stats(const mgs_frame* frame, mgs_frame_stats* out);

/* ---------------------------------------------------------------------- */
/* whole path                                                              */
/* ---------------------------------------------------------------------- */

/* Masked forward rendering of n_views cameras (host array cams[n_views],
 * 1 <= n_views <= MGS_MAX_VIEWS): projection, depth order of the records,
 * per-tile and per-region lists (key duplication, radix sort, ranges), masked
 * compositing (Eq. 3-4 with the background term).  images [3 * P], packed
 * per view and channel-planar, receives the rendering; t_final [P]
 * (optional, may be NULL) the final transmittance.  Synchronises the stream
 * once, to read the list entry counts and size the sort, unless the
 * frame has a fixed workspace (mgs_frame_reserve).  Limits: n_views * n
 * records and the pixels of all views each below 2^32.  Errors:
 * MGS_ERR_INVALID_ARG, MGS_ERR_NONFINITE (non-finite projected geometry),
 * MGS_ERR_CAPACITY, MGS_ERR_OOM, MGS_ERR_HIP. */
MGS_API mgs_status mgs_forward(mgs_frame* frame, mgs_stream stream, const mgs_gaussians* g, const mgs_camera* cams,
                               int n_views, const mgs_settings* st, float* images, float* t_final);

/* mgs_forward that also returns the importance by-products of the
 * compositing: the weight w = M_i alpha_i T_i with which Gaussian i enters a
 * pixel's colour (Eq. 3; the alpha_i T_i that score-based pruning ranks by,
 * Sec. 2, and that Eq. 6 contains, Sec. 3.4), summed (imp_sum [n]) and
 * maximised (imp_max [n]) over every pixel of every view where the Gaussian
 * is blended (after the alpha filter, before the early stop).  Both device,
 * caller-owned, float32, overwritten; the sums accumulate in FP64 and are
 * rounded once.  A masked Gaussian scores 0.  Per pixel the weights and the
 * final transmittance add up to 1.  The frame supports mgs_backward as after
 * mgs_forward, but keeps no work counters.  The first call on a frame with a
 * fixed workspace allocates an n-element FP64 accumulator. */
MGS_API mgs_status mgs_forward_importance(mgs_frame* frame, mgs_stream stream, const mgs_gaussians* g,
                                          const mgs_camera* cams, int n_views, const mgs_settings* st, float* images,
                                          float* t_final, float* imp_sum, float* imp_max);

/* Backward of the last mgs_forward on this frame (Eq. 6 with the
 * supplementary recursion and background term; reverse traversal with the
 * transmittance recovered by division).  dl_dimages [3 * P] is the gradient
 * of the loss w.r.t. the rendered images.  Writes every non-NULL field of
 * *grads (host struct of device pointers); d_masks receives dL/dM_i for
 * every Gaussian, masked or not, summed over views.  Per-record 2D gradients
 * and mask gradients are accumulated with FP64 atomics and rounded once.
 * The Gaussian parameters passed to the forward must be unchanged.
 * Asynchronous. */
MGS_API mgs_status mgs_backward(mgs_frame* frame, mgs_stream stream, const float* dl_dimages,
                                const mgs_gradients* grads);

/* Fixed workspace for stream capture (hipGraph): after a plain mgs_forward on
 * this frame, sizes the list-entry and batch-checkpoint buffers to
 * that forward's counts times `slack` (>= 1) and switches the frame to a mode
 * in which mgs_forward and mgs_backward neither allocate nor synchronise: the
 * live counts stay on the device, the sort and the compositing read them
 * there, and counts beyond the reservation raise a device flag instead of
 * growing buffers.  Records (N * views), tiles and pixels may not exceed the
 * forward the reservation was taken from (MGS_ERR_CAPACITY on the host).
 * slack <= 0 releases the fixed workspace.  Synchronises `stream` once.
 * Outputs of a forward whose counts overflowed are undefined; mgs_frame_check
 * reports it. */
MGS_API mgs_status mgs_frame_reserve(mgs_frame* frame, mgs_stream stream, double slack);

/* Synchronises `stream`, then reads the device flags and counts of the
 * frame's last forward: MGS_ERR_NONFINITE for non-finite projected geometry,
 * MGS_ERR_CAPACITY when a count exceeded a fixed workspace.  Updates the
 * frame statistics with the live counts. */
MGS_API mgs_status mgs_frame_check(mgs_frame* frame, mgs_stream stream);

/* Autotuner for the compositing configuration: times forward + backward
 * (one warm-up, best of four, HIP events on `stream`) for tile shapes 16x16,
 * 16x8, 32x8 and 8x8 with batch depths 32..256, then the pixels-per-thread
 * pairs with every batch depth at the best shape, then the wide-list
 * threshold, and returns the
 * fastest settings in *best (the other fields copied from *base) and their
 * time in *best_ms (may be NULL).  Images, tile lists and gradients agree
 * across these settings (tile-size invariance of the per-pixel cut), so the
 * choice affects time only.  Uses the plain path (frame without a fixed
 * workspace); overwrites images, the gradients and the frame state. */
MGS_API mgs_status mgs_autotune(mgs_frame* frame, mgs_stream stream, const mgs_gaussians* g, const mgs_camera* cams,
                                int n_views, const mgs_settings* base, float* images, const float* dl_dimages,
                                const mgs_gradients* grads, mgs_settings* best, double* best_ms);

/* Copies one array the last forward left in the frame into dst (device,
 * caller-owned, at least the reported size):
 *   MGS_EXPORT_RECORDS  [R, 12] f32 projected records (layout of mgs_project)
 *   MGS_EXPORT_DEPTH    [R] f32, MGS_EXPORT_RADIUS [R] f32, MGS_EXPORT_TILES [R] u32
 *   MGS_EXPORT_VALUES   [K] u32 list entries in (cell, depth, record) order,
 *                       as positions into ORDER
 *   MGS_EXPORT_RANGES   [total_tiles + total_regions, 2] u32 [start, end) into
 *                       VALUES: per tile (global tile ids, views in order,
 *                       row-major), then per region
 *   MGS_EXPORT_T_FINAL  [P] f32, MGS_EXPORT_LAST [P] i32
 *   MGS_EXPORT_STATS    [P, 4] i32 (examined, blended, blended with mask 0,
 *                       entries up to the last blended one)
 *   MGS_EXPORT_EVALS    [P, 4] i32 (evaluated, evaluated up to the last blended
 *                       entry, 0, 0)
 *   MGS_EXPORT_ORDER    [R] u32 record ids in (view, depth, record) order,
 *                       records without tiles last within their view
 * Records covering more tiles than the wide threshold are listed per region
 * (MGS_REGION_TILES x MGS_REGION_TILES tiles, row-major per view, views in
 * order) instead of per tile.  A tile's list is the merge, in (depth, record)
 * order, of its own entries with the entries of its region that belong to
 * it: with settings.tile_cull = 0 those whose square tile rectangle contains
 * the tile (the lists of Sec. 3.1), else those that pass the exact touch
 * test (as the tile's own entries then do).  LAST and STATS hold indices
 * into that merged list.
 * *bytes (host) receives the size; with dst NULL only the size is returned. */
typedef enum {
    MGS_EXPORT_RECORDS = 0,
    MGS_EXPORT_DEPTH,
    MGS_EXPORT_RADIUS,
    MGS_EXPORT_TILES,
    MGS_EXPORT_VALUES,
    MGS_EXPORT_RANGES,
    MGS_EXPORT_T_FINAL,
    MGS_EXPORT_LAST,
    MGS_EXPORT_STATS,
    MGS_EXPORT_ORDER,
    MGS_EXPORT_EVALS
} mgs_export;
MGS_API mgs_status mgs_frame_export(mgs_frame* frame, mgs_stream stream, int what, void* dst, size_t* bytes);

/* Gaussian-pixel work of the last forward on a frame, summed over pixels. */
typedef struct {
    int64_t examined;        /* entries examined in the forward, up to and including
                                each pixel's stop entry (the forward evaluations) */
    int64_t blended;         /* entries that passed the filters and were blended */
    int64_t blended_masked;  /* ... of which with mask 0 */
    int64_t bwd_examined;    /* entries the backward revisits: from the range start
                                to each pixel's last blended entry */
    int64_t evaluated;       /* entries actually evaluated in the forward: those of
                                the examined ones that can reach a pixel of their
                                tile (an exact per-tile test drops the others,
                                which cannot change any result) */
    int64_t bwd_evaluated;   /* ... of which up to each pixel's last blended entry
                                (the entries the backward evaluates) */
} mgs_eval_counts;

/* Sums the per-pixel counts of the last forward into *out (host).
 * Synchronises.  MGS_ERR_STATE if that forward ran with settings.stats = 0. */
MGS_API mgs_status mgs_frame_count_evals(mgs_frame* frame, mgs_stream stream, mgs_eval_counts* out);

/* ---------------------------------------------------------------------- */
/* per-stage timing with HIP events on the caller's stream                 */
/* ---------------------------------------------------------------------- */

typedef enum {
    MGS_STAGE_PROJECT = 0,
    MGS_STAGE_DEPTH_SORT,
    MGS_STAGE_SCAN,
    MGS_STAGE_DUPLICATE,
    MGS_STAGE_SORT,
    MGS_STAGE_RANGES,
    MGS_STAGE_COMPOSITE_FWD,
    MGS_STAGE_COMPOSITE_BWD,
    MGS_STAGE_PROJECT_BWD,
    MGS_STAGE_SAMPLE_MASKS,
    MGS_STAGE_MASK_GRAD,
    MGS_STAGE_LOSS,
    MGS_STAGE_ADAM,
    MGS_NUM_STAGES
} mgs_stage;

/* While enabled, every launch of a stage on ctx is bracketed by two HIP
 * events recorded on the launch stream.  Enabling clears earlier records. */
MGS_API mgs_status mgs_profile_enable(mgs_ctx* ctx, int on);

/* Waits for the recorded events, writes per stage the summed elapsed
 * milliseconds ms[MGS_NUM_STAGES] and launch counts launches[MGS_NUM_STAGES]
 * (host arrays), and clears the records.  Synchronises on the events. */
MGS_API mgs_status mgs_profile_read(mgs_ctx* ctx, double* ms, int64_t* launches);

/* ---------------------------------------------------------------------- */
/* stages, for stage-wise checking; all buffers caller-owned               */
/* ---------------------------------------------------------------------- */

/* EWA projection and SH colour (Sec. 3.1) of every Gaussian for every view.
 * rec [R, 12]: u, v, a, b / a, c - b^2 / a, opacity, mask, radius, r, g, b,
 *   tile count (u32 bits; the same values as radius[] and tiles[]);
 *   under MGS_MASK_OPACITY opacity is M_i * sigmoid(logit) and mask 1
 *   (conic (a, b, c) is the inverse 2D covariance, Q = a dx^2 + 2 b dx dy + c dy^2,
 *   stored in the form a (dx + (b / a) dy)^2 + (c - b^2 / a) dy^2, which FP32
 *   evaluates without cancellation for needle-shaped splats);
 * depth [R]: view-space z rounded to float32 from a double-precision
 *   transform (the sort key); radius [R]: ceil(3 sqrt(lambda_max));
 * tiles [R] (u32): number of tiles of the record's square footprint.
 * Culled records (depth <= near, singular covariance) have tiles = 0. */
MGS_API mgs_status mgs_project(mgs_ctx* ctx, mgs_stream stream, const mgs_gaussians* g, const mgs_camera* cams,
                               int n_views, const mgs_settings* st, float* rec, float* depth, float* radius,
                               uint32_t* tiles);

/* Scratch held by the library for mgs_scan_noalloc, per GPU (bytes). */
#define MGS_SCAN_NOALLOC_BYTES 65536
/* Largest n mgs_scan_noalloc accepts: ((65536 - 256) / 8 - 1) blocks of 4096. */
#define MGS_SCAN_NOALLOC_MAX_N 33419264

/* Binning stages.  Sec. 3.1 renders each pixel from the Gaussians that
 * intersect its 16x16 tile, in depth order; these four calls build those
 * per-tile lists: offsets of every record's entries (scan of the tile
 * counts), one (tile, depth) key per covered tile (duplication), the keys in
 * (tile, depth, record) order (stable radix sort) and each tile's slice of
 * the sorted list (ranges).
 *
 * Exclusive prefix sum of n u32 values; total_dev (device, one u64) gets
 * the sum.  scratch must hold mgs_scan_scratch_bytes(n) bytes. */
MGS_API size_t mgs_scan_scratch_bytes(int64_t n);
MGS_API mgs_status mgs_scan(mgs_ctx* ctx, mgs_stream stream, const uint32_t* in, int64_t n, uint32_t* out,
                            uint64_t* total_dev, void* scratch);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): mgs_scan
 * without the scratch argument.  Same result as mgs_scan.  Its scratch is a
 * library-owned device array of MGS_SCAN_NOALLOC_BYTES that every GPU holds
 * until the process ends (the address is taken per device by mgs_create);
 * nothing is allocated by this call.  n <= MGS_SCAN_NOALLOC_MAX_N, else
 * MGS_ERR_INVALID_ARG.  All calls on one GPU share the array: calls on one
 * stream are ordered, calls that overlap in time on one GPU (other streams,
 * other threads or contexts) race and give wrong results.  in, out
 * (device, caller-owned, n u32 each); total_dev (device, one u64,
 * optional).  Asynchronous. */
MGS_API mgs_status mgs_scan_noalloc(mgs_ctx* ctx, mgs_stream stream, const uint32_t* in, int64_t n, uint32_t* out,
                                    uint64_t* total_dev);

/* Tile lists of Sec. 3.1: writes, for every record r with tiles > 0 and
 * every tile t of its footprint, key = (global tile id << 32) | float bits
 * of depth and
 * value = r, starting at offsets[r].  Global tile ids number the tiles of
 * view 0 first, row-major.  Entries at or beyond capacity are not written
 * and raise the capacity flag. */
MGS_API mgs_status mgs_duplicate(mgs_ctx* ctx, mgs_stream stream, const float* rec, const float* depth,
                                 const float* radius, const uint32_t* tiles, const uint32_t* offsets, int64_t n,
                                 const mgs_camera* cams, int n_views, const mgs_settings* st, uint64_t* keys,
                                 uint32_t* vals, int64_t capacity);

/* Depth order within each tile (Sec. 3.1): stable LSD radix sort of K
 * (key, value) pairs on the low key_bits bits of the key (8 bits per pass).  Sorted pairs end in keys/vals; keys_alt and
 * vals_alt (K entries each) are scratch; scratch holds
 * mgs_sort_scratch_bytes(K) bytes. */
MGS_API size_t mgs_sort_scratch_bytes(int64_t K);
MGS_API mgs_status mgs_sort(mgs_ctx* ctx, mgs_stream stream, uint64_t* keys, uint32_t* vals, int64_t K,
                            int key_bits, uint64_t* keys_alt, uint32_t* vals_alt, void* scratch);

/* Each tile's list (Sec. 3.1): [start, end) of every global tile in the
 * sorted keys; tiles without entries get [0, 0).  ranges [total_tiles, 2]
 * (u32). */
MGS_API mgs_status mgs_tile_ranges(mgs_ctx* ctx, mgs_stream stream, const uint64_t* keys, int64_t K,
                                   int64_t total_tiles, uint32_t* ranges);

/* Chain rule from d_rec [R, 9] (the per-record 2D gradients: dL/du, dL/dv,
 * the conic gradient w.r.t. the three stored values (a, b / a, c - b^2 / a)
 * of the record, dL/dopacity, dL/d(r, g, b); the layout of
 * mgs_gradients.d_records) to the Gaussian parameters, summed over
 * views (no atomics: one thread per Gaussian), in double precision from the
 * 3D covariance to the conic.  grads->d_masks is ignored.  Under
 * MGS_MASK_OPACITY the d_rec opacity entry is dL/d(M_i opacity) and g->masks
 * is required (the logit gradient carries the factor M_i). */
MGS_API mgs_status mgs_project_backward(mgs_ctx* ctx, mgs_stream stream, const mgs_gaussians* g,
                                        const mgs_camera* cams, int n_views, const mgs_settings* st,
                                        const float* d_rec, const mgs_gradients* grads);

/* ---------------------------------------------------------------------- */
/* masks, loss, optimiser                                                  */
/* ---------------------------------------------------------------------- */

/* Straight-through Gumbel-Softmax over two scores per Gaussian (Sec. 3.3).
 * scores [n, 2] (column 0 = exists).  Philox4x32-10 with counter
 * (i lo, i hi, t lo, t hi) and key (seed lo, seed hi) gives uniforms
 * u = (bits >> 8 + 0.5) 2^-24 for the two scores, g = -log(-log u), computed
 * in double.  m_hard [n] = [s0 + g0 > s1 + g1]; y_soft [n] =
 * sigmoid((s0 + g0 - s1 - g1) / tau).  The counter step is
 * t = step + *step_offset when step_offset (device, one u64, optional) is
 * given: a captured training step then draws fresh masks at every replay
 * while mgs_step_advance moves the counter. */
MGS_API mgs_status mgs_sample_masks(mgs_ctx* ctx, mgs_stream stream, const float* scores, int64_t n, float tau,
                                    uint64_t seed, uint64_t step, const uint64_t* step_offset, float* m_hard,
                                    float* y_soft);

/* Deterministic masks with a straight-through estimator, the alternative to
 * Gumbel sampling in the ablation of Sec. 4.3 (Table 6): y = sigmoid(s0 - s1)
 * and m_hard = [y > threshold], both in double precision; y_soft = y.
 * mgs_mask_grad with tau = 1 then gives the straight-through gradient
 * (dL/dy taken as dL/dM).  threshold in (0, 1); the paper takes the value
 * of the method it compares with without printing it.  scores [n, 2]
 * (8-byte aligned); m_hard, y_soft [n] (device, caller-owned). */
MGS_API mgs_status mgs_threshold_masks(mgs_ctx* ctx, mgs_stream stream, const float* scores, int64_t n,
                                       float threshold, float* m_hard, float* y_soft);

/* The mask-count loss of Eq. (7), L_m = (mean M)^2 over the n hard masks,
 * into loss_m (device, one float; 0 for n = 0), summed in double.  scratch
 * holds mgs_reduce_scratch_bytes(n) bytes.  Asynchronous. */
MGS_API size_t mgs_reduce_scratch_bytes(int64_t n);
MGS_API mgs_status mgs_mask_loss(mgs_ctx* ctx, mgs_stream stream, const float* m_hard, int64_t n, float* loss_m,
                                 void* scratch);

/* Gradient to the scores through the straight-through mask, adding the
 * mask-count loss L_m = (mean M)^2 with weight w (Eq. 7-8):
 * d_scores[i, 0] = (d_masks[i] + w 2 sum(M) / n^2) y (1 - y) / tau,
 * d_scores[i, 1] = -d_scores[i, 0], where w = lambda_m, times *lambda_scale
 * when lambda_scale (device, one float, optional) is given -- under autograd
 * the incoming gradient of L_m, so that no value crosses to the host.
 * loss_m (device, one float, optional) receives L_m.  scratch holds
 * mgs_reduce_scratch_bytes(n) bytes.  d_scores 8-byte aligned. */
MGS_API mgs_status mgs_mask_grad(mgs_ctx* ctx, mgs_stream stream, const float* d_masks, const float* m_hard,
                                 const float* y_soft, int64_t n, float tau, float lambda_m, const float* lambda_scale,
                                 float* d_scores, float* loss_m, void* scratch);

/* Probabilistic pruning (Sec. 3.5, training and pruning): every Gaussian
 * draws n_draws (>= 1; 10 in the paper) hard masks with the rule of
 * mgs_sample_masks, at steps step0 .. step0 + n_draws - 1, and is kept iff at
 * least one draw is 1.  scores [n, 2] (8-byte aligned); keep [n] u32 (0/1,
 * device, caller-owned).  Asynchronous. */
MGS_API mgs_status mgs_prune_sample(mgs_ctx* ctx, mgs_stream stream, const float* scores, int64_t n, uint64_t seed,
                                    uint64_t step0, int n_draws, uint32_t* keep);

/* Removal of the pruned Gaussians from every per-Gaussian array (parameters,
 * scores, optimiser state; Sec. 3.5): stable compaction of the rows with
 * keep[i] != 0.  n_arrays arrays, host arrays of device pointers in[a] and
 * out[a] (distinct, caller-owned, out[a] holding at least as many rows as
 * are kept) with widths[a] (1 .. 2^20) floats per row; n < 2^31.  Rows past
 * the kept ones are left untouched.  n_kept (device, one u64, optional)
 * receives the number of kept rows.  scratch (device) holds
 * mgs_compact_scratch_bytes(n) bytes.  One launch per 32 arrays after the
 * scan.  Asynchronous, no allocation. */
MGS_API size_t mgs_compact_scratch_bytes(int64_t n);
MGS_API mgs_status mgs_compact_rows(mgs_ctx* ctx, mgs_stream stream, const uint32_t* keep, int64_t n, int n_arrays,
                                    const float* const* in, float* const* out, const int* widths, uint64_t* n_kept,
                                    void* scratch);

/* L1 rendering loss over m elements, the rendering loss L_render of Eq. (8)
 * (mean |image - target|, sign(0) = 0): d_images [m] (optional) =
 * sign(image - target) / m, times *grad_scale when grad_scale (device, one
 * float, optional) is given (the upstream gradient under autograd); loss
 * (device, one float, optional; 0 for m = 0).  At least one of d_images and
 * loss.  scratch holds mgs_reduce_scratch_bytes(m) bytes. */
MGS_API mgs_status mgs_l1_loss_grad(mgs_ctx* ctx, mgs_stream stream, const float* images, const float* targets,
                                    int64_t m, float* d_images, const float* grad_scale, float* loss, void* scratch);

/* One Adam step (Kingma and Ba) over n float32 parameters, in place on
 * params, m and v; step >= 1 is the bias-correction step count.  (The paper
 * trains every attribute and the mask scores with the optimiser of 3DGS,
 * Sec. 4.1, without restating it.) */
MGS_API mgs_status mgs_adam_step(mgs_ctx* ctx, mgs_stream stream, float* params, const float* grads, float* m,
                                 float* v, int64_t n, float lr, float beta1, float beta2, float eps, int64_t step);

/* One array of an Adam step over several arrays (device pointers, float32,
 * n elements each, updated in place; lr is this array's learning rate). */
typedef struct {
    float* params;
    const float* grads;
    float* m;
    float* v;
    int64_t n;
    float lr;
} mgs_adam_array;

/* The Adam step of mgs_adam_step over n_arrays arrays (host array of
 * descriptors; every attribute and the mask scores of a training step, each
 * with its own learning rate) in one launch per 16 arrays.  The
 * bias-correction step is t = step + *step_offset when step_offset (device,
 * one i64, optional) is given, else step; t must be >= 1 (with a device
 * offset this is not checked).  Arrays with n = 0 are skipped; n < 2^40.
 * Asynchronous, no allocation. */
MGS_API mgs_status mgs_adam_step_multi(mgs_ctx* ctx, mgs_stream stream, const mgs_adam_array* arrays, int n_arrays,
                                       float beta1, float beta2, float eps, int64_t step,
                                       const int64_t* step_offset);

/* counter[0] += delta on the device (one i64, caller-owned): advances the
 * step counter that mgs_sample_masks and mgs_adam_step_multi read, inside a
 * captured step.  Asynchronous. */
MGS_API mgs_status mgs_step_advance(mgs_ctx* ctx, mgs_stream stream, int64_t* counter, int64_t delta);

#ifdef __cplusplus
}
#endif

#endif /* MASKGS_H */
