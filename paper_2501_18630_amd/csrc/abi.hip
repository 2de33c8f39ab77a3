// C ABI of libdbs (include/dbs.h): argument validation, buffer layout and the
// launch sequence of each call.  Nothing here allocates or synchronises.
#include <math.h>
#include <string.h>

#include "dbs_internal.h"

namespace dbs {

int64_t total_tiles(const dbs_camera *cams, int32_t n_views, int tile_w, int tile_h)
{
    int64_t t = 0;
    for (int32_t v = 0; v < n_views; ++v)
        t += (int64_t)((cams[v].width + tile_w - 1) / tile_w) * ((cams[v].height + tile_h - 1) / tile_h);
    return t;
}

static bool finite(float x) { return isfinite(x); }

static dbs_status check_cams(const dbs_camera *cams, int32_t n_views)
{
    if (!cams || n_views < 1 || n_views > DBS_MAX_VIEWS) return DBS_ERR_INVALID_ARGUMENT;
    for (int32_t v = 0; v < n_views; ++v) {
        const dbs_camera &c = cams[v];
        if (c.width < 1 || c.height < 1 || c.width > 16384 || c.height > 16384) return DBS_ERR_INVALID_ARGUMENT;
        if (!(c.near_plane > 0.0f) || !finite(c.near_plane)) return DBS_ERR_INVALID_ARGUMENT;
        if (!finite(c.fx) || !finite(c.fy) || !finite(c.cx) || !finite(c.cy) || c.fx == 0.0f || c.fy == 0.0f)
            return DBS_ERR_INVALID_ARGUMENT;
        for (int k = 0; k < 12; ++k)
            if (!finite(c.viewmat[k])) return DBS_ERR_INVALID_ARGUMENT;
        for (int k = 0; k < 3; ++k)
            if (!finite(c.background[k])) return DBS_ERR_INVALID_ARGUMENT;
    }
    return DBS_OK;
}

static dbs_status check_cfg(const dbs_raster_cfg *cfg)
{
    if (!cfg) return DBS_ERR_INVALID_ARGUMENT;
    if (!(cfg->alpha_max > 0.0f && cfg->alpha_max < 1.0f)) return DBS_ERR_INVALID_ARGUMENT;
    if (!(cfg->t_eps >= 0.0f && cfg->t_eps < 1.0f)) return DBS_ERR_INVALID_ARGUMENT;
    const uint32_t known = DBS_FLAG_PERSISTENT | DBS_FLAG_DIFFUSE_ONLY | DBS_FLAG_SPECULAR_ONLY | DBS_FLAG_B_BELOW |
                           DBS_FLAG_B_ABOVE | DBS_FLAG_GAUSSIAN_SH | DBS_FLAG_GRAD_STORE;
    if ((cfg->flags & ~known) != 0) return DBS_ERR_INVALID_ARGUMENT;
    if ((cfg->flags & DBS_FLAG_GAUSSIAN_SH) &&
        (cfg->flags & ~(DBS_FLAG_GAUSSIAN_SH | DBS_FLAG_PERSISTENT | DBS_FLAG_GRAD_STORE)))
        return DBS_ERR_INVALID_ARGUMENT;
    if ((cfg->flags & DBS_FLAG_DIFFUSE_ONLY) && (cfg->flags & DBS_FLAG_SPECULAR_ONLY)) return DBS_ERR_INVALID_ARGUMENT;
    if ((cfg->flags & DBS_FLAG_B_BELOW) && (cfg->flags & DBS_FLAG_B_ABOVE)) return DBS_ERR_INVALID_ARGUMENT;
    if (!finite(cfg->b_split)) return DBS_ERR_INVALID_ARGUMENT;
    if (!raster_supported(cfg->tile_w, cfg->tile_h, cfg->batch)) return DBS_ERR_UNSUPPORTED;
    return DBS_OK;
}

static dbs_status check_sizes(int64_t n, int32_t n_views)
{
    if (n < 0) return DBS_ERR_INVALID_ARGUMENT;
    if ((uint64_t)n * (uint64_t)n_views >= 0xffffffffull) return DBS_ERR_UNSUPPORTED;
    return DBS_OK;
}

static dbs_status check_splats(const dbs_splats *s)
{
    if (!s) return DBS_ERR_INVALID_ARGUMENT;
    if (s->n < 0) return DBS_ERR_INVALID_ARGUMENT;
    if (s->m < 0 || s->m > DBS_MAX_LOBES) return DBS_ERR_UNSUPPORTED;
    if (s->n > 0) {
        if (!s->means || !s->scales || !s->quats || !s->opacities || !s->betas || !s->diffuse)
            return DBS_ERR_INVALID_ARGUMENT;
        if (s->m > 0 && (!s->lobe_angles || !s->lobe_colors || !s->lobe_betas)) return DBS_ERR_INVALID_ARGUMENT;
    }
    return DBS_OK;
}

static SplatPtrs splat_ptrs(const dbs_splats *s)
{
    SplatPtrs p;
    p.means = s->means; p.scales = s->scales; p.quats = s->quats; p.opacities = s->opacities;
    p.betas = s->betas; p.diffuse = s->diffuse; p.lobe_angles = s->lobe_angles;
    p.lobe_colors = s->lobe_colors; p.lobe_betas = s->lobe_betas;
    p.n = s->n; p.m = s->m;
    return p;
}

// render modes without a reverse pass
constexpr uint32_t kDecompositionFlags = DBS_FLAG_DIFFUSE_ONLY | DBS_FLAG_SPECULAR_ONLY | DBS_FLAG_B_BELOW |
                                         DBS_FLAG_B_ABOVE | DBS_FLAG_GAUSSIAN_SH;

static dbs_status hip_status(hipError_t e) { return e == hipSuccess ? DBS_OK : DBS_ERR_HIP; }

#define DBS_TRY(x)                      \
    do {                                \
        dbs_status st_ = (x);           \
        if (st_ != DBS_OK) return st_;  \
    } while (0)

}  // namespace dbs

using namespace dbs;

extern "C" {

void dbs_default_cfg(dbs_raster_cfg *cfg)
{
    if (!cfg) return;
    cfg->tile_w = 16;
    cfg->tile_h = 16;
    cfg->batch = 256;
    cfg->t_eps = 1e-4f;
    cfg->alpha_max = 0.99f;
    cfg->flags = DBS_FLAG_PERSISTENT;
    cfg->b_split = 0.0f;
}

size_t dbs_projected_bytes(int64_t n, int32_t n_views)
{
    if (n < 0 || n_views < 1 || n_views > DBS_MAX_VIEWS) return 0;
    return proj_layout(n, n_views).total;
}

size_t dbs_bins_bytes(int64_t pair_capacity, const dbs_camera *cams, int32_t n_views, const dbs_raster_cfg *cfg)
{
    if (pair_capacity < 0 || check_cams(cams, n_views) != DBS_OK || check_cfg(cfg) != DBS_OK) return 0;
    return bins_layout(pair_capacity, total_tiles(cams, n_views, cfg->tile_w, cfg->tile_h)).total;
}

size_t dbs_workspace_bytes(int64_t n, int32_t n_views, int64_t pair_capacity, const dbs_camera *cams,
                           const dbs_raster_cfg *cfg)
{
    if (n < 0 || pair_capacity < 0 || check_cams(cams, n_views) != DBS_OK || check_cfg(cfg) != DBS_OK) return 0;
    return work_layout(n, n_views, pair_capacity, total_tiles(cams, n_views, cfg->tile_w, cfg->tile_h)).total;
}

dbs_status dbs_preprocess(const dbs_splats *splats, const dbs_camera *cams, int32_t n_views,
                          const dbs_raster_cfg *cfg, void *projected, size_t projected_bytes, int64_t *counts,
                          void *stream)
{
    DBS_TRY(check_splats(splats));
    DBS_TRY(check_cams(cams, n_views));
    DBS_TRY(check_cfg(cfg));
    if (cfg->flags & DBS_FLAG_GAUSSIAN_SH) return DBS_ERR_INVALID_ARGUMENT;  // needs the SH coefficients
    DBS_TRY(check_sizes(splats->n, n_views));
    if (!projected) return DBS_ERR_INVALID_ARGUMENT;
    if (projected_bytes < proj_layout(splats->n, n_views).total) return DBS_ERR_CAPACITY;
    hipStream_t s = (hipStream_t)stream;
    ProjPtrs P = proj_ptrs(projected, splats->n, n_views);
    DBS_TRY(hip_status(launch_upload_views(cams, n_views, cfg->tile_w, cfg->tile_h, P, splats->n, splats->m, s)));
    return hip_status(launch_preprocess(splat_ptrs(splats), nullptr, P, n_views, cfg->tile_w, cfg->tile_h,
                                        cfg->flags, cfg->b_split, counts, s));
}

dbs_status dbs_preprocess_gaussian_sh(const dbs_splats *splats, const float *sh, const dbs_camera *cams,
                                      int32_t n_views, const dbs_raster_cfg *cfg, void *projected,
                                      size_t projected_bytes, int64_t *counts, void *stream)
{
    if (!splats) return DBS_ERR_INVALID_ARGUMENT;
    if (splats->n < 0) return DBS_ERR_INVALID_ARGUMENT;
    if (splats->n > 0 && (!splats->means || !splats->scales || !splats->quats || !splats->opacities || !sh))
        return DBS_ERR_INVALID_ARGUMENT;
    DBS_TRY(check_cams(cams, n_views));
    DBS_TRY(check_cfg(cfg));
    if (!(cfg->flags & DBS_FLAG_GAUSSIAN_SH)) return DBS_ERR_INVALID_ARGUMENT;
    DBS_TRY(check_sizes(splats->n, n_views));
    if (!projected) return DBS_ERR_INVALID_ARGUMENT;
    if (projected_bytes < proj_layout(splats->n, n_views).total) return DBS_ERR_CAPACITY;
    hipStream_t s = (hipStream_t)stream;
    ProjPtrs P = proj_ptrs(projected, splats->n, n_views);
    SplatPtrs sp = splat_ptrs(splats);
    sp.m = 0;
    DBS_TRY(hip_status(launch_upload_views(cams, n_views, cfg->tile_w, cfg->tile_h, P, splats->n, 0, s)));
    return hip_status(launch_preprocess(sp, sh, P, n_views, cfg->tile_w, cfg->tile_h, cfg->flags, cfg->b_split,
                                        counts, s));
}

dbs_status dbs_bin_sort(const void *projected, const dbs_camera *cams, int32_t n_views, const dbs_raster_cfg *cfg,
                        int64_t n, int64_t pair_capacity, void *bins, size_t bins_bytes, void *workspace,
                        size_t workspace_bytes, int32_t *overflow, void *stream)
{
    DBS_TRY(check_cams(cams, n_views));
    DBS_TRY(check_cfg(cfg));
    DBS_TRY(check_sizes(n, n_views));
    if (!projected || !bins || !workspace) return DBS_ERR_INVALID_ARGUMENT;
    if (pair_capacity < 0) return DBS_ERR_INVALID_ARGUMENT;
    if (pair_capacity > DBS_MAX_PAIRS) return DBS_ERR_UNSUPPORTED;
    const int64_t n_tiles = total_tiles(cams, n_views, cfg->tile_w, cfg->tile_h);
    if (n_tiles >= 0xffffffffll) return DBS_ERR_UNSUPPORTED;
    if (bins_bytes < bins_layout(pair_capacity, n_tiles).total) return DBS_ERR_CAPACITY;
    if (workspace_bytes < work_layout(n, n_views, pair_capacity, n_tiles).total) return DBS_ERR_CAPACITY;
    ProjPtrs P = proj_ptrs((void *)projected, n, n_views);
    BinsPtrs B = bins_ptrs(bins, n_tiles);
    return hip_status(launch_bin_sort(P, B, workspace, n, n_views, pair_capacity, n_tiles, cfg->tile_w,
                                      cfg->tile_h, overflow, (hipStream_t)stream));
}

dbs_status dbs_bin_sort_noalloc(const void *projected, const dbs_camera *cams, int32_t n_views,
                                const dbs_raster_cfg *cfg, int64_t n, int64_t pair_capacity, void *bins,
                                size_t bins_bytes, int32_t *overflow, void *stream)
{
    DBS_TRY(check_cams(cams, n_views));
    DBS_TRY(check_cfg(cfg));
    DBS_TRY(check_sizes(n, n_views));
    if (!projected || !bins) return DBS_ERR_INVALID_ARGUMENT;
    if (pair_capacity < 0) return DBS_ERR_INVALID_ARGUMENT;
    if (pair_capacity > DBS_MAX_PAIRS) return DBS_ERR_UNSUPPORTED;
    const int64_t n_tiles = total_tiles(cams, n_views, cfg->tile_w, cfg->tile_h);
    if (n_tiles >= 0xffffffffll) return DBS_ERR_UNSUPPORTED;
    if (bins_bytes < bins_layout(pair_capacity, n_tiles).total) return DBS_ERR_CAPACITY;
    if (work_layout(n, n_views, pair_capacity, n_tiles).total > (size_t)DBS_NOALLOC_SCRATCH_BYTES)
        return DBS_ERR_CAPACITY;
    void *work = nullptr;
    DBS_TRY(hip_status(noalloc_scratch(&work)));
    ProjPtrs P = proj_ptrs((void *)projected, n, n_views);
    BinsPtrs B = bins_ptrs(bins, n_tiles);
    return hip_status(launch_bin_sort(P, B, work, n, n_views, pair_capacity, n_tiles, cfg->tile_w, cfg->tile_h,
                                      overflow, (hipStream_t)stream));
}

dbs_status dbs_render_fwd(const void *projected, const void *bins, const dbs_camera *cams, int32_t n_views,
                          const dbs_raster_cfg *cfg, int64_t n, float *image, float *final_T, int32_t *last_index,
                          void *stream)
{
    DBS_TRY(check_cams(cams, n_views));
    DBS_TRY(check_cfg(cfg));
    DBS_TRY(check_sizes(n, n_views));
    if (!projected || !bins || !image || !final_T || !last_index) return DBS_ERR_INVALID_ARGUMENT;
    const int64_t n_tiles = total_tiles(cams, n_views, cfg->tile_w, cfg->tile_h);
    ProjPtrs P = proj_ptrs((void *)projected, n, n_views);
    BinsPtrs B = bins_ptrs((void *)bins, n_tiles);
    return hip_status(launch_raster_fwd(P, B, n, n_views, n_tiles, *cfg, image, final_T, last_index,
                                        (hipStream_t)stream));
}

static dbs_status check_grads(const dbs_splats *splats, const dbs_splat_grads *grads)
{
    if (!grads) return DBS_ERR_INVALID_ARGUMENT;
    if (splats->n > 0) {
        if (!grads->means || !grads->scales || !grads->quats || !grads->opacities || !grads->betas || !grads->diffuse)
            return DBS_ERR_INVALID_ARGUMENT;
        if (splats->m > 0 && (!grads->lobe_angles || !grads->lobe_colors || !grads->lobe_betas))
            return DBS_ERR_INVALID_ARGUMENT;
    }
    return DBS_OK;
}

static dbs_status raster_bwd(const void *projected, const void *bins, const dbs_camera *cams, int32_t n_views,
                             const dbs_raster_cfg *cfg, int64_t n, const float *final_T, const int32_t *last_index,
                             const float *dL_dimage, int64_t *atomics, void *stream)
{
    DBS_TRY(check_cams(cams, n_views));
    DBS_TRY(check_cfg(cfg));
    if (cfg->flags & kDecompositionFlags) return DBS_ERR_UNSUPPORTED;
    DBS_TRY(check_sizes(n, n_views));
    if (!projected || !bins || !final_T || !last_index || !dL_dimage) return DBS_ERR_INVALID_ARGUMENT;
    const int64_t n_tiles = total_tiles(cams, n_views, cfg->tile_w, cfg->tile_h);
    ProjPtrs P = proj_ptrs((void *)projected, n, n_views);
    BinsPtrs B = bins_ptrs((void *)bins, n_tiles);
    return hip_status(launch_raster_bwd(P, B, n, n_views, n_tiles, *cfg, final_T, last_index, dL_dimage,
                                        (float *)P.sgrad, atomics, (hipStream_t)stream));
}

dbs_status dbs_raster_bwd(const void *projected, const void *bins, const dbs_camera *cams, int32_t n_views,
                          const dbs_raster_cfg *cfg, int64_t n, const float *final_T, const int32_t *last_index,
                          const float *dL_dimage, void *stream)
{
    return raster_bwd(projected, bins, cams, n_views, cfg, n, final_T, last_index, dL_dimage, nullptr, stream);
}

dbs_status dbs_raster_bwd_count(const void *projected, const void *bins, const dbs_camera *cams, int32_t n_views,
                                const dbs_raster_cfg *cfg, int64_t n, const float *final_T,
                                const int32_t *last_index, const float *dL_dimage, int64_t *atomics, void *stream)
{
    if (!atomics) return DBS_ERR_INVALID_ARGUMENT;
    return raster_bwd(projected, bins, cams, n_views, cfg, n, final_T, last_index, dL_dimage, atomics, stream);
}

dbs_status dbs_project_bwd(const dbs_splats *splats, const void *projected, const dbs_camera *cams, int32_t n_views,
                           const dbs_raster_cfg *cfg, dbs_splat_grads *grads, void *stream)
{
    DBS_TRY(check_splats(splats));
    DBS_TRY(check_cams(cams, n_views));
    DBS_TRY(check_cfg(cfg));
    if (cfg->flags & kDecompositionFlags) return DBS_ERR_UNSUPPORTED;
    DBS_TRY(check_sizes(splats->n, n_views));
    if (!projected) return DBS_ERR_INVALID_ARGUMENT;
    DBS_TRY(check_grads(splats, grads));
    ProjPtrs P = proj_ptrs((void *)projected, splats->n, n_views);
    GradPtrs g;
    g.means = grads->means; g.scales = grads->scales; g.quats = grads->quats; g.opacities = grads->opacities;
    g.betas = grads->betas; g.diffuse = grads->diffuse; g.lobe_angles = grads->lobe_angles;
    g.lobe_colors = grads->lobe_colors; g.lobe_betas = grads->lobe_betas;
    return hip_status(launch_project_bwd(splat_ptrs(splats), P, n_views, g, (cfg->flags & DBS_FLAG_GRAD_STORE) != 0,
                                         (hipStream_t)stream));
}

dbs_status dbs_render_bwd(const dbs_splats *splats, const void *projected, const void *bins, const dbs_camera *cams,
                          int32_t n_views, const dbs_raster_cfg *cfg, const float *final_T, const int32_t *last_index,
                          const float *dL_dimage, dbs_splat_grads *grads, void *stream)
{
    DBS_TRY(check_splats(splats));
    DBS_TRY(check_grads(splats, grads));
    DBS_TRY(dbs_raster_bwd(projected, bins, cams, n_views, cfg, splats->n, final_T, last_index, dL_dimage, stream));
    return dbs_project_bwd(splats, projected, cams, n_views, cfg, grads, stream);
}

dbs_status dbs_render_stats(const void *projected, const void *bins, const dbs_camera *cams, int32_t n_views,
                            const dbs_raster_cfg *cfg, int64_t n, const float *final_T, const int32_t *last_index,
                            int64_t *out, void *stream)
{
    DBS_TRY(check_cams(cams, n_views));
    DBS_TRY(check_cfg(cfg));
    if (cfg->flags & DBS_FLAG_GAUSSIAN_SH) return DBS_ERR_UNSUPPORTED;
    DBS_TRY(check_sizes(n, n_views));
    if (!projected || !bins || !final_T || !last_index || !out) return DBS_ERR_INVALID_ARGUMENT;
    const int64_t n_tiles = total_tiles(cams, n_views, cfg->tile_w, cfg->tile_h);
    ProjPtrs P = proj_ptrs((void *)projected, n, n_views);
    BinsPtrs B = bins_ptrs((void *)bins, n_tiles);
    return hip_status(launch_raster_stats(P, B, n, n_views, n_tiles, *cfg, final_T, last_index, out,
                                          (hipStream_t)stream));
}

dbs_status dbs_l1_loss(const float *image, const float *target, int64_t count, float scale, float *dL_dimage,
                       float *loss, void *stream)
{
    if (count < 0) return DBS_ERR_INVALID_ARGUMENT;
    if (count > 0 && (!image || !target || !dL_dimage)) return DBS_ERR_INVALID_ARGUMENT;
    return hip_status(launch_l1_loss(image, target, count, scale, dL_dimage, loss, (hipStream_t)stream));
}

dbs_status dbs_photometric_loss(const float *image, const float *target, const dbs_camera *cams, int32_t n_views,
                                float lambda_ssim, float *dL_dimage, float *loss, void *stream)
{
    DBS_TRY(check_cams(cams, n_views));
    if (!image || !target || !dL_dimage) return DBS_ERR_INVALID_ARGUMENT;
    if (!(lambda_ssim >= 0.0f && lambda_ssim <= 1.0f)) return DBS_ERR_INVALID_ARGUMENT;
    return hip_status(launch_photometric_loss(image, target, cams, n_views, lambda_ssim, dL_dimage, loss,
                                              (hipStream_t)stream));
}

dbs_status dbs_regularizer(const dbs_splats *splats, float lambda_o, float lambda_s, dbs_splat_grads *grads,
                           float *loss, void *stream)
{
    DBS_TRY(check_splats(splats));
    DBS_TRY(check_grads(splats, grads));
    if (!finite(lambda_o) || !finite(lambda_s)) return DBS_ERR_INVALID_ARGUMENT;
    GradPtrs g{};
    g.opacities = grads->opacities;
    g.scales = grads->scales;
    return hip_status(launch_regularizer(splat_ptrs(splats), lambda_o, lambda_s, g, loss, (hipStream_t)stream));
}

static dbs_status check_splats_mut(const dbs_splats_mut *s, SplatMut *out)
{
    if (!s || s->n < 0) return DBS_ERR_INVALID_ARGUMENT;
    if (s->m < 0 || s->m > DBS_MAX_LOBES) return DBS_ERR_UNSUPPORTED;
    if (s->n > 0) {
        if (!s->means || !s->scales || !s->quats || !s->opacities || !s->betas || !s->diffuse)
            return DBS_ERR_INVALID_ARGUMENT;
        if (s->m > 0 && (!s->lobe_angles || !s->lobe_colors || !s->lobe_betas)) return DBS_ERR_INVALID_ARGUMENT;
    }
    out->means = s->means; out->scales = s->scales; out->quats = s->quats; out->opacities = s->opacities;
    out->betas = s->betas; out->diffuse = s->diffuse; out->lobe_angles = s->lobe_angles;
    out->lobe_colors = s->lobe_colors; out->lobe_betas = s->lobe_betas;
    out->n = s->n; out->m = s->m;
    return DBS_OK;
}

size_t dbs_mcmc_workspace_bytes(int64_t n)
{
    if (n < 0 || n > 0xffffffffll) return 0;
    return mcmc_layout(n).total;
}

dbs_status dbs_mcmc_relocate(const dbs_splats_mut *splats, float dead_opacity, const uint32_t *rand, void *workspace,
                             size_t workspace_bytes, int32_t *n_relocated, void *stream)
{
    SplatMut p;
    DBS_TRY(check_splats_mut(splats, &p));
    if (p.n >= 0xffffffffll) return DBS_ERR_UNSUPPORTED;
    if (!finite(dead_opacity)) return DBS_ERR_INVALID_ARGUMENT;
    if (p.n > 0 && (!rand || !workspace)) return DBS_ERR_INVALID_ARGUMENT;
    if (p.n > 0 && workspace_bytes < mcmc_layout(p.n).total) return DBS_ERR_CAPACITY;
    return hip_status(launch_mcmc_relocate(p, dead_opacity, rand, workspace, n_relocated, (hipStream_t)stream));
}

dbs_status dbs_mcmc_noise(const dbs_splats_mut *splats, const float *z, float lr, float lambda_eps, float b_prime,
                          void *stream)
{
    SplatMut p;
    DBS_TRY(check_splats_mut(splats, &p));
    if (p.n > 0 && !z) return DBS_ERR_INVALID_ARGUMENT;
    if (!finite(lr) || !finite(lambda_eps) || !finite(b_prime)) return DBS_ERR_INVALID_ARGUMENT;
    return hip_status(launch_mcmc_noise(p, z, lr, lambda_eps, b_prime, (hipStream_t)stream));
}

dbs_status dbs_projected_layout(void *projected, int64_t n, int32_t n_views, void **record, void **bbox,
                                void **depth, void **ntiles, void **counts)
{
    if (!projected || n < 0 || n_views < 1 || n_views > DBS_MAX_VIEWS) return DBS_ERR_INVALID_ARGUMENT;
    ProjPtrs P = proj_ptrs(projected, n, n_views);
    if (record) *record = P.rec;
    if (bbox) *bbox = P.bbox;
    if (depth) *depth = P.depth;
    if (ntiles) *ntiles = P.ntiles;
    if (counts) *counts = P.hdr->counts;
    return DBS_OK;
}

dbs_status dbs_projected_state(void *projected, int64_t n, int32_t n_views, void **visbits, void **gradmask,
                               void **sgrad)
{
    if (!projected || n < 0 || n_views < 1 || n_views > DBS_MAX_VIEWS) return DBS_ERR_INVALID_ARGUMENT;
    ProjPtrs P = proj_ptrs(projected, n, n_views);
    if (visbits) *visbits = P.visbits;
    if (gradmask) *gradmask = P.gradmask;
    if (sgrad) *sgrad = P.sgrad;
    return DBS_OK;
}

dbs_status dbs_bins_layout(void *bins, int64_t pair_capacity, const dbs_camera *cams, int32_t n_views,
                           const dbs_raster_cfg *cfg, void **pair_rec, void **tile_range, void **tile_order,
                           int64_t *n_tiles)
{
    if (!bins || pair_capacity < 0) return DBS_ERR_INVALID_ARGUMENT;
    DBS_TRY(check_cams(cams, n_views));
    DBS_TRY(check_cfg(cfg));
    const int64_t nt = total_tiles(cams, n_views, cfg->tile_w, cfg->tile_h);
    BinsPtrs B = bins_ptrs(bins, nt);
    if (pair_rec) *pair_rec = B.pair_rec;
    if (tile_range) *tile_range = B.tile_range;
    if (tile_order) *tile_order = B.tile_order;
    if (n_tiles) *n_tiles = nt;
    return DBS_OK;
}

const char *dbs_status_string(dbs_status s)
{
    switch (s) {
        case DBS_OK: return "ok";
        case DBS_ERR_INVALID_ARGUMENT: return "invalid argument";
        case DBS_ERR_CAPACITY: return "buffer too small";
        case DBS_ERR_HIP: return "HIP launch failure";
        case DBS_ERR_UNSUPPORTED: return "unsupported configuration";
    }
    return "unknown status";
}

const char *dbs_version(void) { return "dbs 0.2 gfx950"; }

}  // extern "C"
