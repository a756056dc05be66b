/*
 * qrender.h - C ABI of the Quantile Rendering library for AMD MI355X (gfx950).
 *
 * Renders per-Gaussian feature vectors (up to 512-D and beyond) of a set of
 * 3D Gaussians into [H, W, D] feature maps, either with the dense front-to-back
 * alpha blend of every Gaussian on each pixel's ray (Eq. 1 of Jeong et al.,
 * "Quantile Rendering: Efficiently Embedding High-dimensional Feature on 3D
 * Gaussian Splatting", Sec. 3) or with Quantile Rendering (Algorithm 1,
 * Sec. 4.2), which blends only the <= K Gaussians whose step in transmittance
 * crosses one of the thresholds t_m = 1 - m/(K+1) and normalises by 1 - T^Q.
 *
 * Pipeline (all calls asynchronous on the caller's HIP stream):
 *   qr_project -> qr_bin_sort -> qr_render_dense | qr_render_quantile
 *   (+ qr_render_*_backward for gradients).
 *
 * Conventions shared by every entry point:
 *  - Every array argument is a DEVICE pointer owned by the caller, unless
 *    marked "host". The library never allocates, frees or retains memory;
 *    scratch space is passed in as a caller-owned workspace.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Kernels are enqueued on it and the call returns without waiting, except
 *    where a call says it synchronises.
 *  - The return value is a qr_status. On QR_ERR_INVALID_ARG or
 *    QR_ERR_UNSUPPORTED nothing has been launched and no output is written.
 *    QR_ERR_HIP means a launch failed; outputs are then undefined.
 *    qr_last_error() returns a message describing the last failure of the
 *    calling thread.
 *  - Arrays are dense and row-major; "f32[N,4]" is N rows of 4 floats.
 *    Device arrays are expected to start on a 16-byte boundary (hipMalloc
 *    and torch allocations do): feature tables, maps and gradient maps are
 *    read and written with 16-byte vector accesses.
 *  - Screen tiles are 16 x 16 pixels, tile id = ty * tiles_x + tx with
 *    tiles_x = ceil(W / 16), tiles_y = ceil(H / 16). Pixel (px, py) is
 *    sampled at its centre (px + 0.5, py + 0.5). Feature maps are pixel-major
 *    [H, W, D] float32.
 *  - The library is stateless and thread-safe; calls on different streams
 *    may run concurrently when their outputs do not overlap.
 */
#ifndef QRENDER_H
#define QRENDER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QR_TILE 16
/* K (quantile Gaussians per ray) ranges over [1, QR_MAX_K] in every entry
 * point, backward passes included: the paper trains at K = 40 and sweeps K up
 * to 50. A workgroup keeps each pixel's <= K selections in LDS (8 bytes
 * each), so K above about 40 leaves room for one workgroup per CU. */
#define QR_MAX_K 64
/* Feature width D: a positive multiple of 16 (the column block of the matrix
 * core contractions of the dense blend and the backward passes) up to
 * QR_MAX_DIM. */
#define QR_MAX_DIM 4096
#define QR_BATCH_TILE_BITS 20  /* batched schedule item = (view << 20) | tile */

typedef enum qr_status {
  QR_OK = 0,
  QR_ERR_INVALID_ARG = -1, /* null pointer, non-positive size, bad range */
  QR_ERR_UNSUPPORTED = -2, /* dtype, D not a multiple of 16, K outside [1, QR_MAX_K] */
  QR_ERR_CAPACITY = -3,    /* workspace or pair capacity too small */
  QR_ERR_HIP = -4          /* a HIP runtime call or launch failed */
} qr_status;

/* Storage type of the feature table F [N, D]. Blending always accumulates in
 * float32; reduced types are decoded to float32 when loaded. */
typedef enum qr_dtype {
  QR_F32 = 0,      /* float32 */
  QR_BF16 = 1,     /* bfloat16 (upper half of a float32) */
  QR_FP8_E4M3 = 2  /* OCP FP8 e4m3 code times a per-Gaussian float32 scale */
} qr_dtype;

/* Reductions of qr_devoxelize. */
typedef enum {
  QR_REDUCE_MAX = 0,
  QR_REDUCE_MEAN = 1
} qr_reduce;

/* Selection rules of the Q-Render kernels (qr_params.selection). */
typedef enum {
  QR_SELECT_QUANTILE = 0,   /* Algorithm 1 */
  QR_SELECT_STRATIFIED = 1, /* Stratified-K (Appendix) */
  QR_SELECT_TOPK = 2        /* Top-K, the sampler compared with in Sec. 4.2 */
} qr_selection;

/* Pinhole camera, OpenCV axes (x right, y down, z forward). A world point X
 * maps to camera space as R_cw X + t (R_cw row-major). Gaussians whose
 * camera-space depth is <= z_near are culled. */
typedef struct qr_camera {
  float R_cw[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  float z_near;
} qr_camera;

/* Rasterisation constants (the 3D-GS conventions the paper renders with):
 *  alpha_min  a Gaussian is on a pixel's ray list only where alpha' >= alpha_min
 *             (typ. 1/255); it also defines the footprint ellipse.
 *  alpha_max  alpha' = min(alpha_max, o G) (typ. 0.99).
 *  T_eps      dense blend stops before transmittance falls below T_eps
 *             (typ. 1e-4; 0 blends every Gaussian on the ray).
 *  dilation   added to both diagonal entries of the 2D covariance, px^2
 *             (typ. 0.3).
 *  guard      x/z and y/z are clamped to guard x the half field of view when
 *             the projection Jacobian is formed (typ. 1.3). */
typedef struct qr_params {
  float alpha_min;
  float alpha_max;
  float T_eps;
  float dilation;
  float guard;
  /* Element type of the feature maps the Q-Render forward writes (`out` of
   * qr_render_quantile and of every qr_view of qr_render_quantile_batched):
   * QR_F32 (0, default) or QR_BF16 (round to nearest even from the float32
   * result; `out` then points to u16 codes). The dense blend writes
   * float32 only (QR_ERR_UNSUPPORTED otherwise); the backward passes ignore
   * it. */
  int32_t out_dtype;
  /* Thresholds of the Q-Render selection: QR_SELECT_QUANTILE (0, default,
   * Algorithm 1: t_m = 1 - m/(K+1)) or QR_SELECT_STRATIFIED (1, the
   * Stratified-K variant of the Appendix: per ray, a first pass estimates the
   * mean mu and population standard deviation sigma of T_0 = 1 and the
   * transmittance after every Gaussian the dense blend composites (with its
   * T_eps stop); then t_m = clip(mu + sigma Phi^-1(1 - m/(K+1)), 0, 1),
   * evaluated in double and rounded once to float, and Algorithm 1 runs with
   * these thresholds over the same Gaussians, ending at the dense stop or
   * once all K are consumed) or QR_SELECT_TOPK (2, the Top-K sampler that
   * Sec. 4.2 and its complexity table compare with: among the Gaussians the
   * dense blend composites, the K of largest dense weight T alpha' (equal
   * weights: the earlier list position), blended with those weights and
   * normalised by their sum; T_q reports 1 - that sum). The backward passes
   * support QR_SELECT_QUANTILE only. */
  int32_t selection;
} qr_params;

/* One view of a batched render (qr_render_quantile_batched). All pointers are
 * device pointers with the meaning of the same-named qr_render_quantile
 * arguments; T_q and n_sel may be NULL. Views may belong to different scenes
 * (different Gaussian sets and feature tables) and have different sizes. */
typedef struct qr_view {
  const uint32_t* tile_offsets;
  const uint32_t* sorted_gid;
  const float* means2d;
  const float* conic_opacity;
  const void* features;
  const float* feature_scale;
  float* out;
  float* T_q;
  int32_t* n_sel;
  int32_t width, height;
} qr_view;

/* Gradient buffers of one view of a batched backward
 * (qr_render_quantile_batched_backward); device pointers with the meaning of
 * the same-named qr_render_quantile_backward arguments. Views of one scene
 * may share (and so accumulate into) the same gradient arrays. */
typedef struct qr_view_grad {
  const float* grad_out;
  float* grad_features;
  float* grad_means2d;
  float* grad_conic_opacity;
} qr_view_grad;

/* Library version string (static storage). */
const char* qr_version(void);

/* Message for the last failed call on this thread ("" if none). */
const char* qr_last_error(void);

/*
 * qr_project - EWA splatting of N 3D Gaussians (Sec. 3: Sigma = R S S^T R^T
 * from scale s and quaternion r; a 2D Gaussian G(u) per pixel).
 *
 * Inputs (device): means3d f32[N,3]; scales f32[N,3] (linear, not log);
 * quats f32[N,4] as (w, x, y, z), normalised inside; opacity f32[N]
 * (activated, in [0,1]). cam, prm: host pointers.
 * Outputs (device): means2d f32[N,2] (u, v in pixels); conic_opacity f32[N,4]
 * = (a, b, c, o) with [[a, b], [b, c]] the inverse 2D covariance; depth f32[N]
 * (camera-space z); tile_rect i32[N,4] = (tx0, ty0, tx1, ty1), a half-open
 * tile rectangle covering every pixel where alpha' >= alpha_min (the bounding
 * box of the ellipse d^T conic d <= 2 ln(o / alpha_min)); tiles_touched
 * u32[N] = tile count of the rectangle. Culled Gaussians (behind z_near,
 * o < alpha_min, singular covariance, off screen, non-finite input) get
 * tiles_touched = 0 and an empty rectangle.
 * N = 0 is valid and launches nothing.
 */
int qr_project(void* stream, int64_t n,
               const float* means3d, const float* scales, const float* quats,
               const float* opacity, const qr_camera* cam, const qr_params* prm,
               float* means2d, float* conic_opacity, float* depth,
               int32_t* tile_rect, uint32_t* tiles_touched);

/*
 * qr_project_views - qr_project for a batch of n_views cameras of one image
 * size (Sec. 3, as above), in one launch per 32 cameras: record v*N + i of
 * every output is Gaussian i seen from cams[v], bit-identical to what
 * qr_project writes for that camera. cams: HOST array of n_views cameras
 * (copied into the launch arguments; the call keeps no pointer). Outputs are
 * device arrays of n_views*N records laid out as for qr_project.
 * Errors: QR_ERR_INVALID_ARG for n < 0, n_views <= 0, a camera with another
 * image size or a bad focal length, null pointers; QR_ERR_UNSUPPORTED for
 * n_views*N >= 2^40.
 */
int qr_project_views(void* stream, int64_t n,
                     const float* means3d, const float* scales, const float* quats,
                     const float* opacity, int32_t n_views, const qr_camera* cams,
                     const qr_params* prm, float* means2d, float* conic_opacity,
                     float* depth, int32_t* tile_rect, uint32_t* tiles_touched);

/*
 * qr_count_pairs - total number of (tile, Gaussian) pairs, sum of
 * tiles_touched. SYNCHRONISES the stream. `workspace` must hold at least
 * 8 bytes (device). Writes *total (host).
 */
int qr_count_pairs(void* stream, int64_t n, const uint32_t* tiles_touched,
                   void* workspace, size_t workspace_bytes, uint64_t* total);

/*
 * qr_bin_sort_workspace_size - bytes of device workspace qr_bin_sort needs for
 * n Gaussians, a tiles_x x tiles_y grid and room for `capacity` pairs.
 * Host-only; writes *bytes.
 */
int qr_bin_sort_workspace_size(int64_t n, int32_t tiles_x, int32_t tiles_y,
                               int64_t capacity, size_t* bytes);

/*
 * qr_bin_sort - per-tile, depth-ordered Gaussian lists (the ordered ray
 * sequence S_r of Eq. 1, built per tile as in 3D-GS).
 *
 * Emits one pair per tile in each tile_rect, keyed (tile id << 32) | bits of
 * the float32 depth: a bucket sort by tile (count, exclusive scan, scatter
 * into each tile's range) followed by an independent sort of each tile's
 * bucket by (depth bits << 32 | Gaussian index) - a bitonic sort in LDS for
 * buckets of up to 2,048 keys, a single-workgroup LSD radix sort through the
 * workspace for longer ones. The keys are unique, so each tile's list is
 * ordered by (depth, index) whatever order the scatter produced.
 * Inputs: tile_rect, tiles_touched, depth as written by qr_project.
 * Outputs: sorted_gid u32[capacity] (Gaussian index of each sorted pair);
 * sorted_keys u64[capacity] (nullable; the sorted keys); tile_offsets
 * u32[tiles_x*tiles_y + 1] with tile t's list at
 * [tile_offsets[t], tile_offsets[t+1]); total_pairs u32[1] = number of pairs.
 * If the pair count exceeds `capacity`, the call still succeeds
 * asynchronously but *total_pairs > capacity and the outputs are invalid:
 * callers check total_pairs and retry with a larger capacity.
 * The pair count must stay below 2^32 - 1.
 */
int qr_bin_sort(void* stream, int64_t n, int32_t tiles_x, int32_t tiles_y,
                const int32_t* tile_rect, const uint32_t* tiles_touched,
                const float* depth, int64_t capacity,
                void* workspace, size_t workspace_bytes,
                uint32_t* sorted_gid, uint64_t* sorted_keys,
                uint32_t* tile_offsets, uint32_t* total_pairs);

/*
 * qr_bin_sort_noalloc - qr_bin_sort with no workspace argument, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the workspace is a static
 * device array of QR_BIN_SORT_SCRATCH_BYTES, one copy per GPU, which each GPU
 * holds from the library's first use on it until the process ends. The call
 * itself allocates and frees nothing; the caller still passes inputs and
 * outputs as for qr_bin_sort, and the stream must belong to the current
 * device. Results are identical to qr_bin_sort's.
 * Every call on one GPU shares that GPU's array (the call clears what must
 * start at zero with a kernel on `stream`), so calls that overlap on one GPU
 * (different streams, or threads without ordering) race and must not be
 * made.
 * Errors: as qr_bin_sort, and QR_ERR_CAPACITY when the workspace that
 * qr_bin_sort_workspace_size gives for (n, tiles_x, tiles_y, capacity)
 * exceeds QR_BIN_SORT_SCRATCH_BYTES (nothing launched): about 4 million pairs
 * at frame-sized tile grids.
 */
#define QR_BIN_SORT_SCRATCH_BYTES 67108864 /* 64 MiB */
int qr_bin_sort_noalloc(void* stream, int64_t n, int32_t tiles_x, int32_t tiles_y,
                        const int32_t* tile_rect, const uint32_t* tiles_touched,
                        const float* depth, int64_t capacity,
                        uint32_t* sorted_gid, uint64_t* sorted_keys,
                        uint32_t* tile_offsets, uint32_t* total_pairs);

/*
 * qr_bin_sort_views - qr_bin_sort of a batch of views in one launch
 * sequence: the records are n_views blocks of n_per_view (as written by
 * qr_project_views), and view v's tiles_x x tiles_y grid takes tile ids
 * [v*T, (v+1)*T), T = tiles_x*tiles_y. For every tile of every view the list
 * is exactly the list qr_bin_sort builds for that view alone: VIEW-LOCAL
 * Gaussian ids in (depth, id) order. tile_offsets u32[n_views*T + 1] indexes
 * the one shared sorted_gid array (so view v's offsets start at
 * tile_offsets + v*T); sorted_keys (nullable) hold (stacked tile id << 32) |
 * depth bits. Workspace: qr_bin_sort_workspace_size(n_views*n_per_view,
 * tiles_x, n_views*tiles_y, capacity). Capacity semantics as qr_bin_sort.
 * Errors: as qr_bin_sort; also QR_ERR_INVALID_ARG for n_views <= 0.
 */
int qr_bin_sort_views(void* stream, int32_t n_views, int64_t n_per_view,
                      int32_t tiles_x, int32_t tiles_y,
                      const int32_t* tile_rect, const uint32_t* tiles_touched,
                      const float* depth, int64_t capacity,
                      void* workspace, size_t workspace_bytes,
                      uint32_t* sorted_gid, uint64_t* sorted_keys,
                      uint32_t* tile_offsets, uint32_t* total_pairs);

/*
 * qr_render_dense - dense alpha blend of Eq. 1 per pixel:
 *   alpha'_i = min(alpha_max, o_i exp(-(a dx^2 + 2 b dx dy + c dy^2)/2)),
 *   entries with alpha'_i < alpha_min are skipped, T_1 = 1,
 *   out = sum_i T_i alpha'_i f_i, T_{i+1} = T_i (1 - alpha'_i),
 * stopping before an entry that would take T below T_eps.
 * Inputs: the tile lists of qr_bin_sort, means2d / conic_opacity of
 * qr_project, features [N, dim] of type `dtype` (feature_scale f32[N] for
 * QR_FP8_E4M3, else ignored). dim must be a multiple of 16, <= QR_MAX_DIM.
 * Outputs: out f32[H,W,dim]; T_final f32[H,W] (nullable); n_contrib
 * i32[H,W] (nullable; tile-list position + 1 of the last blended entry).
 */
int qr_render_dense(void* stream, int32_t width, int32_t height,
                    const qr_params* prm, const uint32_t* tile_offsets,
                    const uint32_t* sorted_gid, const float* means2d,
                    const float* conic_opacity, const void* features,
                    int32_t dtype, const float* feature_scale, int32_t dim,
                    float* out, float* T_final, int32_t* n_contrib);

/*
 * qr_render_quantile - Quantile Rendering, Algorithm 1 per pixel:
 *   T = 1, T^Q = 1, f^Q = 0, k = 0; for each entry on the ray:
 *   T_test = T (1 - alpha'); if T_test < t_{k+1}: k += 1, w = T^Q alpha',
 *   f^Q += w f, T^Q *= 1 - alpha', and k advances past every further
 *   threshold T_test is below; the walk ends once k = K (equivalently
 *   T_test < 1/(K+1)); T = T_test. out = f^Q / (1 - T^Q), or 0 if nothing
 *   was selected. Thresholds t_m = 1 - m/(K+1) are rounded once to float32;
 *   the comparison is strict.
 * Inputs as qr_render_dense; 1 <= K <= QR_MAX_K.
 * Outputs: out f32[H,W,dim]; T_q f32[H,W] (nullable; T^Q); n_sel i32[H,W]
 * (nullable; number of selected Gaussians); T_final f32[H,W] (nullable;
 * Algorithm 1's full transmittance T when the walk ends: the stop test
 * breaks before T takes the stopping entry's T_test, so a stopped ray
 * reports T >= 1/(K+1)); last_pos i32[H,W] (nullable; tile-list position + 1
 * of the last entry on the ray that the walk examined, the stopping entry
 * included; 0 if none); sel_gid i32[H,W,K] and sel_w f32[H,W,K] (nullable;
 * selected Gaussian indices in ray order and their weights w^Q, padded with
 * -1 / 0). T_final and last_pos are defined for QR_SELECT_QUANTILE only
 * (QR_ERR_UNSUPPORTED if requested with another rule).
 */
int qr_render_quantile(void* stream, int32_t width, int32_t height,
                       const qr_params* prm, int32_t K,
                       const uint32_t* tile_offsets, const uint32_t* sorted_gid,
                       const float* means2d, const float* conic_opacity,
                       const void* features, int32_t dtype,
                       const float* feature_scale, int32_t dim,
                       float* out, float* T_q, int32_t* n_sel,
                       float* T_final, int32_t* last_pos,
                       int32_t* sel_gid, float* sel_w);

/*
 * qr_render_quantile_batched - Quantile Rendering of many views in one
 * launch (Algorithm 1, Sec. 4.2, applied to every (view, tile) work item of
 * `schedule`: device u32[n_items], item = (view << QR_BATCH_TILE_BITS) | tile,
 * views < 4096, tiles per view < 2^20, n_items < 2^31), each item rendered
 * exactly as qr_render_quantile renders that tile. `views` is a DEVICE array
 * of n_views qr_view records; all views share K, the feature dtype and dim.
 * Every (view, tile) to be rendered must appear once in the schedule.
 *   n_workgroups == 0: one workgroup per item; items are dealt to the XCDs
 *     in contiguous runs of the schedule, and workgroups retire as they
 *     finish (work on other streams can interleave). `workspace` is unused
 *     and may be NULL.
 *   n_workgroups > 0: that many persistent workgroups take items through
 *     atomic counters held in `workspace` (device, >= 32 bytes), which the
 *     call resets: the schedule is cut into eight contiguous ranges, one per
 *     XCD, each taken in order by the workgroups of its XCD first and by the
 *     others once their own range is used up.
 * Errors: QR_ERR_INVALID_ARG for null pointers, counts out of range or
 * n_workgroups < 0; QR_ERR_CAPACITY for a missing or short workspace in
 * persistent mode; QR_ERR_UNSUPPORTED for K, dtype or dim outside the limits.
 */
int qr_render_quantile_batched(void* stream, int32_t n_views, const qr_view* views,
                               const qr_params* prm, int32_t K, int32_t dtype,
                               int32_t dim, const uint32_t* schedule,
                               int64_t n_items, int32_t n_workgroups,
                               void* workspace, size_t workspace_bytes);

/*
 * qr_render_dense_batched - the dense blend of Eq. 1 (as qr_render_dense) for
 * many views in one launch over the same (view, tile) items, schedules,
 * launch modes and workspace as qr_render_quantile_batched, so that the two
 * renderers differ only in which Gaussians of each ray they blend. In each
 * qr_view record, `T_q` receives T_final and `n_sel` receives n_contrib of
 * qr_render_dense (both nullable); K does not apply. Each item is rendered
 * exactly as qr_render_dense renders that tile (bit-identical).
 * Errors: as qr_render_quantile_batched; QR_ERR_UNSUPPORTED for a bfloat16
 * output type.
 */
int qr_render_dense_batched(void* stream, int32_t n_views, const qr_view* views,
                            const qr_params* prm, int32_t dtype, int32_t dim,
                            const uint32_t* schedule, int64_t n_items,
                            int32_t n_workgroups, void* workspace, size_t workspace_bytes);

/*
 * qr_batch_schedule - builds a schedule for qr_render_quantile_batched on the
 * device, without a host round trip: every (view, tile) item, ordered by the
 * length of its tile list, longest first, in power-of-two length classes
 * (order inside a class is unspecified). `view_first` (device i32[n_views+1])
 * holds each view's first item index (prefix sums of its tile counts), so
 * item i belongs to the view v with view_first[v] <= i < view_first[v+1] and
 * is its tile i - view_first[v]. `views` is the device qr_view array whose
 * tile_offsets have been filled by qr_bin_sort. Writes schedule u32[n_items].
 * `workspace`: device, >= 256 bytes.
 */
int qr_batch_schedule(void* stream, int32_t n_views, const qr_view* views,
                      const int32_t* view_first, int64_t n_items, uint32_t* schedule,
                      void* workspace, size_t workspace_bytes);

/*
 * qr_render_dense_backward / qr_render_quantile_backward - gradients of the
 * two renderers given dL/d(out) = grad_out f32[H,W,dim]: the paper trains
 * its feature network through the renderer (Sec. 4.2 and Sec. 4.3: the
 * image-space contrastive loss of Eq. 2 is back-propagated through the
 * rendered feature map to the per-Gaussian features), and the same chain
 * gives the gradients of the 2D means, conics and opacities. The
 * derivatives are those of Eq. 1 (dense) and of Algorithm 1 (quantile) with
 * the discrete decisions held fixed. The forward walk is
 * recomputed (same float32 arithmetic, so the same entries are blended or
 * selected) and transmittance is recovered in a reverse sweep. Discrete
 * decisions pass no gradient; a clamped alpha' passes none to o or geometry.
 * Gradients are ACCUMULATED (atomic adds; the caller zeroes them first):
 * grad_features f32[N,dim] (w.r.t. the decoded float32 features),
 * grad_means2d f32[N,2], grad_conic_opacity f32[N,4] = d/d(a, b, c, o) with
 * b the single off-diagonal conic entry. Any gradient pointer may be NULL
 * to skip it. The dense call also takes its forward output `out`
 * f32[H,W,dim]: <grad_out, out> per pixel is the sum over the whole ray of
 * w_i <grad_out, f_i>, from which the tail sums of the gradient are formed in
 * one front-to-back pass. Other arguments as in the forward calls.
 */
int qr_render_dense_backward(void* stream, int32_t width, int32_t height,
                             const qr_params* prm, const uint32_t* tile_offsets,
                             const uint32_t* sorted_gid, const float* means2d,
                             const float* conic_opacity, const void* features,
                             int32_t dtype, const float* feature_scale,
                             int32_t dim, const float* out,
                             const float* grad_out, float* grad_features,
                             float* grad_means2d, float* grad_conic_opacity);

int qr_render_quantile_backward(void* stream, int32_t width, int32_t height,
                                const qr_params* prm, int32_t K,
                                const uint32_t* tile_offsets,
                                const uint32_t* sorted_gid,
                                const float* means2d, const float* conic_opacity,
                                const void* features, int32_t dtype,
                                const float* feature_scale, int32_t dim,
                                const float* grad_out, float* grad_features,
                                float* grad_means2d, float* grad_conic_opacity);

/*
 * qr_autotune_batched - the launch-shape autotuner of
 * qr_render_quantile_batched: for every candidate (schedule i of the host
 * array `schedules` of n_sched device schedules, each u32[n_items]; j of the
 * host array wg_per_cu[n_wg], 0 = one workgroup per item, w > 0 = w
 * persistent workgroups per CU of the current device), one warm-up launch and
 * `reps` timed launches on `stream` (HIP events; the call synchronises on
 * them). Writes the mean launch time to timings_ms[i * n_wg + j] (host) and
 * the fastest candidate to *best_schedule, *best_wg_per_cu (host). The
 * rendered outputs are those of the last launch. Other arguments as for
 * qr_render_quantile_batched; workspace >= 32 bytes if any w > 0. K = 0
 * times qr_render_dense_batched over the same candidates instead.
 * Errors: QR_ERR_INVALID_ARG for null host pointers, counts < 1 or w outside
 * [0, 64]; any error of the timed launch; QR_ERR_HIP for event failures.
 */
int qr_autotune_batched(void* stream, int32_t n_views, const qr_view* views,
                        const qr_params* prm, int32_t K, int32_t dtype, int32_t dim,
                        const uint32_t* const* schedules, int32_t n_sched, int64_t n_items,
                        const int32_t* wg_per_cu, int32_t n_wg, int32_t reps, void* workspace,
                        size_t workspace_bytes, float* timings_ms, int32_t* best_schedule,
                        int32_t* best_wg_per_cu);

/*
 * qr_render_quantile_batched_backward - qr_render_quantile_backward (the
 * gradients of Algorithm 1 that training through the renderer needs,
 * Sec. 4.2) for many views in one launch over the (view, tile) items of
 * `schedule`, the same
 * schedule format and launch modes as qr_render_quantile_batched (n_workgroups
 * = 0: one workgroup per item; > 0: persistent workgroups on per-XCD work
 * queues held in `workspace`, device, >= 32 bytes). `views` (device
 * qr_view[n_views]; out, T_q and n_sel are not used) and `grads` (device
 * qr_view_grad[n_views]) describe view v of every item (v << QR_BATCH_TILE_BITS)
 * | tile. Gradients are accumulated with atomic adds, so views of one scene
 * may share gradient arrays (their sum is the scene's gradient); the order of
 * the additions is unspecified.
 * Errors: as qr_render_quantile_batched.
 */
int qr_render_quantile_batched_backward(void* stream, int32_t n_views, const qr_view* views,
                                        const qr_view_grad* grads, const qr_params* prm,
                                        int32_t K, int32_t dtype, int32_t dim,
                                        const uint32_t* schedule, int64_t n_items,
                                        int32_t n_workgroups, void* workspace,
                                        size_t workspace_bytes);

/*
 * qr_sh_to_rgb - view-dependent colours of 3D-GS Gaussians for the RGB use of
 * Q-Render (Appendix, "Rendering RGB"): per Gaussian, with d the unit vector
 * from the camera centre (-R_cw^T t) to the mean, colour_ch = 1/2 +
 * sum over the first (degree+1)^2 real orthonormal spherical harmonics
 * Y_lm(d) (m = -l..l, index l^2+l+m, with the Condon-Shortley phase
 * (-1)^m: the sign convention of 3D-GS coefficients; d = 0 for a mean at
 * the camera centre) of
 * sh[i, l^2+l+m, ch], clipped below at 0. means3d: device f32[n,3]; sh:
 * device f32[n, coef_stride, 3], coef_stride >= (degree+1)^2; cam: host.
 * Writes out (device f32[n, out_dim], out_dim >= 3): the colour in columns
 * 0..2, zeros in the rest (a feature table for the renderers, whose dim must
 * be a multiple of 16). degree in [0, 3]. The caller owns every buffer; the
 * call only enqueues work on `stream`. Errors: QR_ERR_INVALID_ARG for n < 0,
 * coef_stride < (degree+1)^2, out_dim < 3, a null camera or (n > 0) a null
 * array; QR_ERR_UNSUPPORTED for a degree outside [0, 3] or n >= 2^39;
 * QR_ERR_HIP for a failed launch. n = 0 does nothing.
 */
int qr_sh_to_rgb(void* stream, int64_t n, int32_t degree, const float* means3d, const float* sh,
                 int32_t coef_stride, const qr_camera* cam, float* out, int32_t out_dim);

/*
 * qr_sh_to_rgb_views - qr_sh_to_rgb for a batch of n_views cameras (the same
 * colour model, Appendix "Rendering RGB"), each Gaussian's coefficients read
 * once for every camera of a launch (one launch per 32 cameras). cams: HOST
 * array of n_views cameras (their centres are copied into the launch
 * arguments; the call keeps no pointer). out: device f32[n_views, n,
 * out_dim]; view v's table starts at out + v*n*out_dim, out_dim a positive
 * multiple of 4 (16-byte rows; out 16-byte aligned). Errors: as
 * qr_sh_to_rgb, QR_ERR_INVALID_ARG for n_views <= 0, QR_ERR_UNSUPPORTED for
 * out_dim not a multiple of 4 or n*out_dim/4 >= 2^39.
 */
int qr_sh_to_rgb_views(void* stream, int64_t n, int32_t degree, const float* means3d,
                       const float* sh, int32_t coef_stride, const qr_camera* cams,
                       int32_t n_views, float* out, int32_t out_dim);

/*
 * qr_devoxelize - per-Gaussian features from voxel predictions (the step that
 * produces the feature table the renderer reads; Appendix, de-voxelisation):
 * out[g, c] = reduce over slots m in [offsets[g], offsets[g+1]) of
 * unique_pred[voxel_unique[m], c], reduce = QR_REDUCE_MAX (ties: the first
 * slot) or QR_REDUCE_MEAN. offsets: device i64[n_gauss+1]; voxel_unique:
 * device i32[n_slots]; unique_pred: device f32[n_unique, dim]; out: device
 * f32[n_gauss, dim]; argmax (max only, may be NULL): device i32[n_gauss, dim],
 * the slot that gave each maximum (for the backward). A Gaussian with no
 * (valid) slot gets the zero row and argmax -1. Slot indices outside
 * [0, n_unique) and offsets outside [0, n_slots] are ignored (checked in the
 * kernel). dim: a positive multiple of 4, <= QR_MAX_DIM.
 * qr_devoxelize_backward - ACCUMULATES dL/d(unique_pred) into grad_unique
 * (device f32[n_unique, dim]; the caller zeroes it) from grad_out (device
 * f32[n_gauss, dim]): max routes each element to its argmax slot's row, mean
 * spreads grad / count over the segment. Float atomics: the order of the
 * additions is unspecified.
 */
int qr_devoxelize(void* stream, int64_t n_gauss, int32_t dim, const int64_t* offsets,
                  const int32_t* voxel_unique, int64_t n_slots, int64_t n_unique,
                  const float* unique_pred, int32_t reduce, float* out, int32_t* argmax);

int qr_devoxelize_backward(void* stream, int64_t n_gauss, int32_t dim, const int64_t* offsets,
                           const int32_t* voxel_unique, int64_t n_slots, int64_t n_unique,
                           int32_t reduce, const float* grad_out, const int32_t* argmax,
                           float* grad_unique);

/*
 * qr_quantize_features - encodes a float32 feature table f32[N,dim] for
 * storage: QR_BF16 writes u16[N,dim] (round to nearest even); QR_FP8_E4M3
 * writes u8[N,dim] OCP e4m3 codes of f / s_i (nearest, ties to even,
 * |value| <= 448) and scale f32[N] with s_i = max_d |f_id| / 448 (1 for an
 * all-zero row). `scale` is ignored for QR_BF16.
 */
int qr_quantize_features(void* stream, int64_t n, int32_t dim,
                         const float* features, int32_t dtype, void* out,
                         float* scale);

#ifdef __cplusplus
}
#endif

#endif /* QRENDER_H */
