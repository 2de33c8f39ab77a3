/*
 * dbs.h — C ABI of the MI355X (gfx950) differentiable tile rasterizer for
 * Deformable Beta Splatting (arXiv 2501.18630).
 *
 * The library renders ellipsoidal Beta primitives (Sec. 3.2, Eq. 4) with
 * Spherical Beta colour (Sec. 3.3, Eq. 8) by depth-ordered front-to-back
 * compositing (Sec. 3.2, Eq. 6), and differentiates the result with respect
 * to every primitive parameter.  A render is four calls on one stream:
 *
 *   dbs_preprocess   project every (view, splat), Spherical Beta colour,
 *                    pixel box, tile count, depth key; count visible
 *                    records and tile pairs
 *   dbs_bin_sort     list, for every tile of every view, the splats whose
 *                    box overlaps it, ordered by (depth, splat id)
 *   dbs_render_fwd   composite every pixel front to back
 *   dbs_render_bwd   reverse pass: gradients of every splat parameter
 *
 * Conventions shared by every call:
 *   - All pointers are DEVICE pointers unless marked [host].  The caller owns
 *     all memory; no call allocates, frees or synchronises the device.  Calls
 *     only enqueue work on `stream` (a hipStream_t; NULL = legacy default
 *     stream), so a sequence of calls can be captured in a hipGraph.
 *   - A status is returned synchronously after argument validation and
 *     launch; DBS_ERR_HIP means a launch failed (hipGetLastError).  Errors
 *     found on the device (pair capacity exceeded) are reported through a
 *     device flag, never by aborting.
 *   - Views are rendered in one batch: view v's image occupies pixels
 *     [pixel_offset(v), pixel_offset(v) + W_v H_v) of the flat pixel index,
 *     with pixel_offset(v) = sum_{u<v} W_u H_u.  `image` is planar per view:
 *     channel c of pixel (x, y) of view v is image[3 pixel_offset(v) +
 *     c W_v H_v + y W_v + x].  `final_T` and `last_index` hold one value per
 *     flat pixel.
 *   - Camera: world->camera x_c = R x_w + t with OpenCV axes (x right, y down,
 *     z forward); pinhole u = fx x/z + cx, v = fy y/z + cy; the centre of
 *     pixel (x, y) is (x + 0.5, y + 0.5).  Splats with z <= near_plane, or
 *     with a non-positive projected-covariance determinant, are culled.
 *   - Every buffer that `dbs_*_bytes` sizes must stay untouched by the caller
 *     between the calls that use it.
 *   - The splat count n, the views and the tile shape (cfg->tile_w, tile_h)
 *     given to dbs_bin_sort, dbs_render_fwd, dbs_render_bwd, dbs_raster_bwd,
 *     dbs_project_bwd and dbs_render_stats must be the ones the last
 *     dbs_preprocess on the same `projected` used (and, for the raster calls,
 *     the last dbs_bin_sort on the same `bins`).  The buffers record what
 *     they were built for: dbs_bin_sort reports a mismatch with *overflow = 2
 *     and lists nothing, and the other calls then do nothing on the device
 *     (their outputs keep their previous contents) instead of reading the
 *     buffers with another layout.
 */
#ifndef DBS_H
#define DBS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DBS_OK = 0,
    DBS_ERR_INVALID_ARGUMENT = 1, /* null pointer, size out of range, bad camera */
    DBS_ERR_CAPACITY = 2,         /* a buffer size argument is below what the call needs */
    DBS_ERR_HIP = 3,              /* a kernel launch failed */
    DBS_ERR_UNSUPPORTED = 4       /* lobe count, tile shape or batch depth not built */
} dbs_status;

#define DBS_MAX_LOBES 8
#define DBS_MAX_VIEWS 1024
#define DBS_MAX_PAIRS ((int64_t)0x7fffffff)

/* Primitive parameters, Sec. 3.2 Eq. (4) and Sec. 3.3 Eq. (8).  FP32,
 * row-major, n splats, m Spherical Beta lobes (0..DBS_MAX_LOBES).
 *   means        [n,3]  centre mu
 *   scales       [n,3]  s, already activated (> 0)
 *   quats        [n,4]  q = (w,x,y,z), any non-zero norm; normalised inside
 *   opacities    [n]    o in [0,1], already activated
 *   betas        [n]    raw b; the kernel exponent is 4 e^b (Sec. 3.1, Eq. 3)
 *   diffuse      [n,3]  base colour c0
 *   lobe_angles  [n,m,2] (theta, phi): R_m = (sin th cos ph, sin th sin ph, cos th)
 *   lobe_colors  [n,m,3] c_m
 *   lobe_betas   [n,m]  raw b_m; the lobe exponent is 4 e^{b_m}
 * Lobe pointers may be NULL when m = 0.
 * The primitive is defined for real parameters: a splat with a NaN or
 * infinite value in any of its parameters is culled in every view (it
 * contributes to no pixel and receives zero gradient).  The exponents
 * 4 e^b and 4 e^{b_m} are evaluated in FP32 and held at the largest finite
 * float (b above about 87.3), so the kernel stays 1 at r^2 = 0 and 0 inside
 * the rest of the support. */
typedef struct {
    const float *means, *scales, *quats, *opacities, *betas, *diffuse;
    const float *lobe_angles, *lobe_colors, *lobe_betas;
    int64_t n;
    int32_t m;
} dbs_splats;

/* Gradients with the same shapes as dbs_splats, FP32.  dbs_render_bwd ADDS
 * into them (+=), so gradients accumulate across calls and views; the caller
 * zeroes them when it wants a fresh gradient, or sets DBS_FLAG_GRAD_STORE to
 * have them overwritten. */
typedef struct {
    float *means, *scales, *quats, *opacities, *betas, *diffuse;
    float *lobe_angles, *lobe_colors, *lobe_betas;
} dbs_splat_grads;

/* [host] One pinhole view. */
typedef struct {
    float viewmat[12];     /* row-major 3x4 [R | t], world -> camera */
    float fx, fy, cx, cy;  /* pixels */
    int32_t width, height; /* 1..16384 */
    float near_plane;      /* > 0 */
    float background[3];   /* fixed background colour, composited with T_final */
} dbs_camera;

/* Rasterisation settings.  The built tile shapes are 16x16, 16x8, 8x8, 32x8
 * and 32x16 pixels; batch is the number of splats the forward pass stages
 * in LDS at a time (64, 128 or 256; the reverse pass stages min(batch, 128)).
 * A splat contributes alpha = min(alpha_max, o B(r^2; b)) where r^2 < 1; a
 * pixel stops after the splat that takes its transmittance below t_eps. */
typedef struct {
    int32_t tile_w, tile_h;
    int32_t batch;
    float t_eps;           /* default 1e-4 */
    float alpha_max;       /* default 0.99; must lie in (0, 1) */
    uint32_t flags;        /* DBS_FLAG_* */
    float b_split;         /* threshold of DBS_FLAG_B_BELOW / DBS_FLAG_B_ABOVE, default 0 */
} dbs_raster_cfg;

/* Raster kernels run persistently: a fixed grid drains a device-side queue
 * of (view, tile) work items ordered heaviest first.  Without this flag one
 * workgroup is launched per work item. */
#define DBS_FLAG_PERSISTENT 1u

/* Decomposition render modes (Beta Decomposition section of the paper),
 * applied by dbs_preprocess; forward rendering only (the reverse calls
 * reject them with DBS_ERR_UNSUPPORTED).
 *   DIFFUSE_ONLY:  colour = c0 (the base colour; lighting decomposition)
 *   SPECULAR_ONLY: colour = the Spherical Beta lobes without c0
 *   B_BELOW / B_ABOVE: only primitives with b < b_split / b >= b_split
 *                  (geometry decomposition by the kernel shape b).
 * DIFFUSE_ONLY with SPECULAR_ONLY, or B_BELOW with B_ABOVE, is invalid. */
#define DBS_FLAG_DIFFUSE_ONLY 2u
#define DBS_FLAG_SPECULAR_ONLY 4u
#define DBS_FLAG_B_BELOW 8u
#define DBS_FLAG_B_ABOVE 16u

/* Gaussian-kernel + spherical-harmonics comparison mode: the baseline the
 * paper compares against (3D Gaussian Splatting's kernel and degree-3 SH
 * colour, Sec. 3.3 and Sec. 4), rendered by the same pipeline.  The records
 * are written by dbs_preprocess_gaussian_sh; dbs_render_fwd then takes
 * alpha = min(alpha_max, o exp(-m^2 / 2)) for Mahalanobis distance m < 3
 * (the 3-sigma ellipse is the support).  Forward only: dbs_preprocess and
 * the reverse calls reject the flag, and it cannot be combined with the
 * decomposition flags. */
#define DBS_FLAG_GAUSSIAN_SH 32u

/* Gradient store: dbs_project_bwd (and so dbs_render_bwd) writes the
 * gradients into `grads` instead of adding them, so the caller need not
 * clear the buffers first (every element of every splat is written; zero for
 * a splat no view sees).  Without it the gradients accumulate (+=).  The
 * other calls ignore it. */
#define DBS_FLAG_GRAD_STORE 64u

/* Fills *cfg with the defaults above (16x16 tiles, batch 256, persistent, no
 * decomposition). */
void dbs_default_cfg(dbs_raster_cfg *cfg);

/* ---- buffer sizes (bytes) ---------------------------------------------- */

/* `projected`: per (view, splat) records, the view table, counters and the
 * per-record screen-space gradient accumulator of the reverse pass.  The
 * buffer must be zero-filled once before its first use; the library keeps
 * the accumulator zero between calls (dbs_render_bwd clears what it
 * consumes). */
size_t dbs_projected_bytes(int64_t n, int32_t n_views);

/* `bins`: sorted tile lists for up to `pair_capacity` (tile, splat) pairs,
 * tile ranges and the work queue. */
size_t dbs_bins_bytes(int64_t pair_capacity, const dbs_camera *cams /*[host]*/, int32_t n_views,
                      const dbs_raster_cfg *cfg /*[host]*/);

/* `workspace`: scratch for dbs_bin_sort. */
size_t dbs_workspace_bytes(int64_t n, int32_t n_views, int64_t pair_capacity,
                           const dbs_camera *cams /*[host]*/, const dbs_raster_cfg *cfg /*[host]*/);

/* ---- the four calls ----------------------------------------------------- */

/* Projection of every (view, splat) record (Sec. 3.2: Sigma = R S S^T R^T,
 * Sigma' = J W Sigma W^T J^T, mu', conic Sigma'^{-1}, exact support box of
 * r^2 <= 1) and its Spherical Beta colour (Sec. 3.3, Eq. 8).  Geometry is
 * evaluated in FP64; the centre and conic are kept in FP64 for the raster
 * passes, the pixel box and depth key are rounded once.  Writes `projected` and, if `counts`
 * is not NULL, counts[0] = visible records (at least one tile),
 * counts[1] = (tile, splat) pairs.  cams: [host] n_views cameras. */
dbs_status dbs_preprocess(const dbs_splats *splats /*[host] struct of device pointers*/,
                          const dbs_camera *cams /*[host]*/, int32_t n_views,
                          const dbs_raster_cfg *cfg /*[host]*/,
                          void *projected, size_t projected_bytes,
                          int64_t *counts /* device int64[2] or NULL */, void *stream);

/* Projection for DBS_FLAG_GAUSSIAN_SH (cfg->flags must hold it): the same
 * records as dbs_preprocess, with the 3-sigma ellipse as the support (conic
 * Sigma'^{-1} / 9, pixel box mu' +- 3 (sqrt Sigma'00, sqrt Sigma'11)) and the
 * colour max(0, sum_k sh_k Y_k(V) + 1/2) from the 16 real spherical
 * harmonics Y_k of degree <= 3 (order l = 0..3, m = -l..l, Condon-Shortley
 * phase) at the view direction V = (mu - camera centre) / |mu - camera
 * centre|.  Reads means, scales, quats and opacities of `splats` (m, betas,
 * diffuse and lobes are ignored) and sh: device [n, 16, 3] FP32, coefficient
 * k of channel c at sh[(i * 16 + k) * 3 + c].  Other arguments and errors as
 * dbs_preprocess; sh == NULL with n > 0 is DBS_ERR_INVALID_ARGUMENT. */
dbs_status dbs_preprocess_gaussian_sh(const dbs_splats *splats /*[host] struct of device pointers*/,
                                      const float *sh, const dbs_camera *cams /*[host]*/, int32_t n_views,
                                      const dbs_raster_cfg *cfg /*[host]*/, void *projected,
                                      size_t projected_bytes, int64_t *counts /* device int64[2] or NULL */,
                                      void *stream);

/* Tile lists (Sec. 3.2, sorting by depth before Eq. 6): every visible record
 * is listed in each tile its pixel box overlaps; each list is ordered by the
 * fp32 bits of the camera-space depth, ties by splat index.  *overflow
 * (device int32) is set to 1 if the number of pairs exceeds pair_capacity,
 * to 2 if `projected` was written by a dbs_preprocess with another n,
 * n_views or tile shape (its pair count does not hold for this call), and
 * to 0 otherwise; in both error cases every tile list is left empty. */
dbs_status dbs_bin_sort(const void *projected, const dbs_camera *cams /*[host]*/, int32_t n_views,
                        const dbs_raster_cfg *cfg /*[host]*/, int64_t n,
                        int64_t pair_capacity, void *bins, size_t bins_bytes,
                        void *workspace, size_t workspace_bytes,
                        int32_t *overflow /* device int32 or NULL */, void *stream);

/* dbs_bin_sort for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same tile lists, bit for bit, with the scratch taken from a fixed
 * device array of DBS_NOALLOC_SCRATCH_BYTES that the library holds on each
 * GPU it runs on until the process ends, instead of a caller workspace.
 * Allocates nothing (no hipMalloc, no allocating library call).  Returns
 * DBS_ERR_CAPACITY when the scratch the call needs, dbs_workspace_bytes(n,
 * n_views, pair_capacity, cams, cfg), exceeds DBS_NOALLOC_SCRATCH_BYTES.
 * All calls on one GPU share that GPU's array, which keeps the last call's
 * contents (nothing in it needs to start at zero): calls that overlap on one
 * GPU (other streams, other threads) race and must be serialised by the
 * caller.  Other arguments, results and errors as dbs_bin_sort. */
#define DBS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
dbs_status dbs_bin_sort_noalloc(const void *projected, const dbs_camera *cams /*[host]*/, int32_t n_views,
                                const dbs_raster_cfg *cfg /*[host]*/, int64_t n, int64_t pair_capacity,
                                void *bins, size_t bins_bytes, int32_t *overflow /* device int32 or NULL */,
                                void *stream);

/* Front-to-back compositing, Sec. 3.2 Eq. (6), of every pixel of every view:
 *   image      [3 * sum(W H)] FP32, planar per view (see above);
 *               colour = sum_i c_i alpha_i T_i + T_final * background
 *   final_T    [sum(W H)] FP32 transmittance after the last processed splat
 *   last_index [sum(W H)] int32: position in the pair list of the last splat
 *               with r^2 < 1 that the pixel composited, -1 if none. */
dbs_status dbs_render_fwd(const void *projected, const void *bins, const dbs_camera *cams /*[host]*/,
                          int32_t n_views, const dbs_raster_cfg *cfg /*[host]*/, int64_t n,
                          float *image, float *final_T, int32_t *last_index, void *stream);

/* Reverse pass of dbs_render_fwd and dbs_preprocess: given dL/dimage (same
 * layout as image) it ADDS dL/dparameter to *grads for every parameter of
 * Sec. 3.2 Eq. (4) and Sec. 3.3 Eq. (8), including b and b_m through
 * beta = 4 e^b.  Transmittance is recomputed back to front from final_T and
 * last_index; a clamped alpha passes no gradient to o, b or the geometry.
 * `projected` is read and its gradient accumulator used (and left zero); it
 * may be called again on the same projected/bins with another dL_dimage. */
dbs_status dbs_render_bwd(const dbs_splats *splats /*[host] struct of device pointers*/,
                          const void *projected, const void *bins,
                          const dbs_camera *cams /*[host]*/, int32_t n_views,
                          const dbs_raster_cfg *cfg /*[host]*/,
                          const float *final_T, const int32_t *last_index, const float *dL_dimage,
                          dbs_splat_grads *grads /*[host] struct of device pointers*/, void *stream);

/* The two stages of dbs_render_bwd, callable on their own (same arguments):
 * dbs_raster_bwd walks the tile lists back to front and accumulates, per
 * record, the gradient of the screen-space quantities of Eq. (5)-(6)
 * (mu', conic, o, b, colour) inside `projected`; dbs_project_bwd chains them
 * to the parameters (Sec. 3.2 projection, Sec. 3.3 Eq. 8), ADDS into *grads
 * and clears the accumulator.  dbs_render_bwd = dbs_raster_bwd, then
 * dbs_project_bwd.  dbs_raster_bwd also marks, in a per-record bit mask kept
 * beside the accumulator, every record it sends gradient to; dbs_project_bwd
 * reads only the marked records' accumulators and clears them with their
 * marks.  It chains them through the projection of the last dbs_preprocess,
 * so it must follow dbs_raster_bwd without a dbs_preprocess on the same
 * `projected` in between. */
dbs_status dbs_raster_bwd(const void *projected, const void *bins, const dbs_camera *cams /*[host]*/,
                          int32_t n_views, const dbs_raster_cfg *cfg /*[host]*/, int64_t n,
                          const float *final_T, const int32_t *last_index, const float *dL_dimage,
                          void *stream);
dbs_status dbs_project_bwd(const dbs_splats *splats /*[host] struct of device pointers*/,
                           const void *projected, const dbs_camera *cams /*[host]*/, int32_t n_views,
                           const dbs_raster_cfg *cfg /*[host]*/,
                           dbs_splat_grads *grads /*[host] struct of device pointers*/, void *stream);

/* Work counts of a finished forward (profiling; not for the timed path).
 * out[0] += (pixel, pair) evaluations of the support test r^2 < 1 that the
 *           reverse pass makes: for each pixel, the list positions from its
 *           tile's start to its last_index;
 * out[1] += those with r^2 < 1 (the pairs composited by Eq. 6);
 * out[2] += evaluations of the forward: list positions from the start to the
 *           pixel's last_index, or to the list end if it never stopped;
 * out[3] += wavefront steps of the reverse pass: each wavefront covers an
 *           8x8 pixel block, each of its four 16-lane rows a 4x4 quadrant
 *           that walks its own culled list, and a step takes one entry of
 *           every row's list;
 * out[4] += those steps in which at least one pixel has r^2 < 1.
 * out: device int64[5], accumulated. */
dbs_status dbs_render_stats(const void *projected, const void *bins, const dbs_camera *cams /*[host]*/,
                            int32_t n_views, const dbs_raster_cfg *cfg /*[host]*/, int64_t n,
                            const float *final_T, const int32_t *last_index, int64_t *out, void *stream);

/* ---- loss glue ----------------------------------------------------------- */

/* L1 loss L = scale * sum_k |image_k - target_k| over k < count, and its
 * gradient dL/dimage_k = scale * sign(image_k - target_k) (sign(0) = 0).
 * loss (device float, may be NULL) is OVERWRITTEN with L. */
dbs_status dbs_l1_loss(const float *image, const float *target, int64_t count, float scale,
                       float *dL_dimage, float *loss, void *stream);

/* ---- training loss (Sec. 3.4, composite loss equation) ------------------ */

/* Photometric term of the composite loss, summed over the views of a batch:
 *   L = sum_v [ (1 - lambda) mean|x - y| + lambda (1 - mean SSIM(x, y)) ],
 * means over the 3 H_v W_v channel-pixels of view v.  SSIM per colour channel
 * over an 11x11 Gaussian window (sigma 1.5) with zero padding outside the
 * image, C1 = 0.01^2, C2 = 0.03^2 (the standard constants for [0, 1] images;
 * the paper names SSIM without them).  image, target: [3 sum H W] floats in
 * the dbs_render_fwd layout.  dL_dimage (same layout) is OVERWRITTEN with
 * dL/dimage; loss (device float, may be NULL) is OVERWRITTEN with L.
 * lambda_ssim in [0, 1] (the paper trains with 0.2).  cams: [host], only the
 * sizes are read.  Allocates nothing; one work item per (view, channel,
 * 32x16 tile). */
dbs_status dbs_photometric_loss(const float *image, const float *target, const dbs_camera *cams /*[host]*/,
                                int32_t n_views, float lambda_ssim, float *dL_dimage, float *loss, void *stream);

/* Regularisers of the composite loss: lambda_o sum_i |o_i| and
 * lambda_s sum_i sum_j |sqrt(eig_j(Sigma_i))| = lambda_s sum_i sum_j |s_ij|
 * (Sigma = R diag(s^2) R^T).  ADDS lambda_o sign(o) to grads->opacities and
 * lambda_s sign(s) to grads->scales (the other gradient pointers are not
 * touched); loss (device float, may be NULL) is INCREMENTED by the value.
 * The paper trains with lambda_o = lambda_s = 0.01. */
dbs_status dbs_regularizer(const dbs_splats *splats /*[host] struct of device pointers*/, float lambda_o,
                           float lambda_s, dbs_splat_grads *grads /*[host] struct of device pointers*/,
                           float *loss, void *stream);

/* ---- kernel-agnostic MCMC step (Sec. 3.4) -------------------------------- */

/* Splat parameters updated in place: the fields of dbs_splats, writable. */
typedef struct {
    float *means, *scales, *quats, *opacities, *betas, *diffuse;
    float *lobe_angles, *lobe_colors, *lobe_betas;
    int64_t n;
    int32_t m;
} dbs_splats_mut;

/* Scratch for dbs_mcmc_relocate (about 20 bytes per splat). */
size_t dbs_mcmc_workspace_bytes(int64_t n);

/* Relocation of dead primitives (Densification paragraph of Sec. 3.4 and
 * its appendix): a primitive with opacity <= dead_opacity is dead; each dead
 * primitive i becomes a copy (every parameter) of a live primitive j drawn
 * with probability proportional to its opacity, using rand[i] (uniform
 * 32-bit, caller-supplied, [n]): with w_j = floor(o_j 2^24) and inclusive
 * prefix sums P_j, j is the first index with P_j > floor(rand[i] W / 2^32),
 * W = sum_j w_j.  A live primitive drawn N - 1 times and its N - 1 copies all
 * get opacity 1 - (1 - o)^(1/N); no other parameter is adjusted.  Nothing
 * moves when no primitive is live.  n_relocated (device int32, may be NULL)
 * is OVERWRITTEN with the number of dead primitives moved.  Parameters are
 * updated in place; the caller resets any optimiser state it keeps. */
dbs_status dbs_mcmc_relocate(const dbs_splats_mut *splats /*[host] struct of device pointers*/,
                             float dead_opacity, const uint32_t *rand, void *workspace, size_t workspace_bytes,
                             int32_t *n_relocated, void *stream);

/* Positional noise of the Optimization paragraph of Sec. 3.4:
 *   mu += lambda_eps lr B(o; b') R diag(s) z,   B(o; b') = (1 - o)^(4 e^b'),
 * z: [n,3] standard normals supplied by the caller (R diag(s) z is then a
 * sample of N(0, Sigma)); the paper uses b' = ln 25.  Updates means in
 * place; the other parameters are read. */
dbs_status dbs_mcmc_noise(const dbs_splats_mut *splats /*[host] struct of device pointers*/, const float *z,
                          float lr, float lambda_eps, float b_prime, void *stream);

/* ---- introspection (tests, profiling) ------------------------------------ */

/* dbs_raster_bwd that also ADDS the number of global float atomics it issues
 * (one per non-zero (tile, splat, value) sum sent to the accumulator) to
 * *atomics (device int64), for atomic-throughput measurement.  Same
 * arguments and effect as dbs_raster_bwd otherwise; a separate, slightly
 * slower kernel build.  DBS_ERR_INVALID_ARGUMENT if atomics is NULL. */
dbs_status dbs_raster_bwd_count(const void *projected, const void *bins, const dbs_camera *cams /*[host]*/,
                                int32_t n_views, const dbs_raster_cfg *cfg /*[host]*/, int64_t n,
                                const float *final_T, const int32_t *last_index, const float *dL_dimage,
                                int64_t *atomics /*[device]*/, void *stream);

/* Device pointers into `projected` for n splats and n_views views:
 * per record r = v n + i (view-major):
 *   record [R] 64-byte line: double cx, cy (mu' in pixels); double A00, A01,
 *              A11 (conic); float o, 4 e^b; float r, g, b (colour); float pad
 *   bbox   [R] int16x4 (x_lo, x_hi, y_lo, y_hi) inclusive pixel box
 *   depth  [R] uint32 fp32 bits of the camera-space depth
 *   ntiles [R] uint32 number of tiles the box overlaps (0: culled/empty)
 *   counts     int64[2] (visible records, pairs)
 * The record is written for records with ntiles > 0 only.  Any output
 * pointer may be NULL. */
dbs_status dbs_projected_layout(void *projected, int64_t n, int32_t n_views, void **record, void **bbox,
                                void **depth, void **ntiles, void **counts);

/* Device pointers into `projected` to the state the calls keep between them
 * (inspection and tests):
 *   visbits  [n_views][S] uint32, S = 128 ceil(n / 4096): bit i % 32 of word
 *            i / 32 of row v is ntiles > 0 of record (v, i) (written by the
 *            preprocess; bits past n are zero)
 *   gradmask [ceil(n_views / 64)][n] uint64: bit v % 64 of word (v / 64, i)
 *            marks record (v, i) as holding gradient in its accumulator line
 *            (set by dbs_raster_bwd, cleared by dbs_project_bwd)
 *   sgrad    [R] 64-byte accumulator line per record: float dL/dmu' (2),
 *            dL/dA00, dL/dA01, dL/dA11, dL/do, dL/db, dL/dcolour (3), 6 unused
 * Between a dbs_project_bwd and the next dbs_raster_bwd, gradmask and sgrad
 * are all zero.  The preprocess also keeps, for dbs_bin_sort, each record's
 * tile rectangle packed in 32 bits (not exposed).  Any output pointer may be
 * NULL. */
dbs_status dbs_projected_state(void *projected, int64_t n, int32_t n_views, void **visbits, void **gradmask,
                               void **sgrad);

/* Device pointers into `bins`:
 *   pair_rec   [pair_capacity] uint32 record r = v n + i per pair, sorted
 *   tile_range [n_tiles] uint32x2 (start, end) into pair_rec per global tile
 *              (view tiles are numbered consecutively, view-major, row-major)
 *   tile_order [n_tiles] uint32 work order of global tiles, heaviest pair
 *              count class first (a class per count below 16, then 16 per
 *              octave), ties in tile order
 * *n_tiles receives the total tile count of all views. */
dbs_status dbs_bins_layout(void *bins, int64_t pair_capacity, const dbs_camera *cams /*[host]*/,
                           int32_t n_views, const dbs_raster_cfg *cfg /*[host]*/,
                           void **pair_rec, void **tile_range, void **tile_order,
                           int64_t *n_tiles);

const char *dbs_status_string(dbs_status s);

/* Library version, e.g. "dbs 0.2 gfx950". */
const char *dbs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DBS_H */
