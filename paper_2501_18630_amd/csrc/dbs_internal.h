// Internal declarations shared by the HIP sources of libdbs (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dbs.h"

namespace dbs {

constexpr int kWave = 64;

// One view as the kernels see it (written into `projected` by the preprocess).
struct alignas(16) ViewDesc {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    float near_plane;
    float bg[3];
    int32_t width, height;
    int32_t tiles_x, tiles_y;
    int32_t tile_offset;   // first global tile id of the view
    int32_t pad0;
    int64_t pixel_offset;  // first flat pixel of the view
    float campos[3];       // camera centre -R^T t (rounded from FP64)
    int32_t pad1;
};
static_assert(sizeof(ViewDesc) == 128, "ViewDesc layout");

// The view table is written before the kernels that read it and stays
// unchanged while they run.  Read through the constant address space, a view
// picked by a wave-uniform index is fetched with scalar loads into SGPRs,
// instead of vector loads that the compiler must wait for at every view.
typedef const __attribute__((address_space(4))) ViewDesc ConstViewDesc;
__device__ __forceinline__ ConstViewDesc &const_view(const ViewDesc *views, int32_t v)
{
    return ((ConstViewDesc *)views)[v];
}

// Header at the start of `projected`.
struct ProjHeader {
    int64_t counts[2];     // visible records, pairs
    int64_t n;
    int32_t n_views, m;
    int32_t tile_w, tile_h;
    int32_t pad[22];
};
static_assert(sizeof(ProjHeader) == 128, "ProjHeader layout");

// Header at the start of `bins`.
// overflow: 0 = binned, 1 = pair capacity exceeded, 2 = `projected` was
// written for another splat count, view count or tile shape (every list is
// left empty in both error cases).
struct BinsHeader {
    int32_t overflow;
    uint32_t n_vis;        // visible records
    uint32_t n_pairs;      // pairs actually binned (0 on overflow)
    uint32_t n_tiles;
    uint32_t queue[4];     // persistent work queues: fwd head, fwd done, bwd head, bwd done
    uint32_t n_rec;        // records the depth sort's first pass reads: n * n_views, 0 on a mismatch
    int32_t n_views, tile_w, tile_h;
    int64_t n;             // what the lists were built for
    uint32_t pad[18];
};
static_assert(sizeof(BinsHeader) == 128, "BinsHeader layout");

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// One 64-byte, line-aligned raster record per (view, splat): everything a
// raster pass gathers for a pair comes in one cache line.
struct alignas(64) RasterRec {
    double cx, cy;          // mu' in pixels (FP64)
    double a00, a01, a11;   // conic Sigma'^{-1} (FP64)
    float opacity, beta;    // o, 4 e^b
    float r, g, b;          // Spherical Beta colour of this view
    float pad;
};
static_assert(sizeof(RasterRec) == 64, "RasterRec layout");

// Words per view of the visibility bits: whole blocks of 4096 splats.
__host__ __device__ inline int64_t visbits_stride(int64_t n) { return (n + 4095) / 4096 * 128; }

// A record's tile rectangle in 32 bits, written by the preprocess and
// carried through the depth sort beside each record: first column tx0 in
// bits 0-9, first row ty0 in 10-19, w - 1 in 20-25, h - 1 in 26-31.  A
// rectangle that reaches past column or row 1023 or spans more than 64 tiles
// is stored as kRectEscape (no packed rectangle has that value: tx0 = 1023
// with w = 64 would reach column 1086), and its consumers take it from the
// record's pixel box instead.
constexpr uint32_t kRectEscape = 0xffffffffu;
__device__ __forceinline__ uint32_t pack_tile_rect(int tx0, int ty0, int w, int h)
{
    const bool fits = (uint32_t)tx0 + (uint32_t)w <= 1024u && (uint32_t)ty0 + (uint32_t)h <= 1024u &&
                      (uint32_t)(w - 1) < 64u && (uint32_t)(h - 1) < 64u;
    return fits ? (uint32_t)tx0 | (uint32_t)ty0 << 10 | (uint32_t)(w - 1) << 20 | (uint32_t)(h - 1) << 26
                : kRectEscape;
}

struct ProjLayout {
    size_t header, views, rec, bbox, depth, ntiles, rect, visbits, gradmask, sgrad, blockcnt, total;
};
inline ProjLayout proj_layout(int64_t n, int32_t n_views) {
    ProjLayout L;
    size_t R = (size_t)n * (size_t)n_views, o = 0;
    L.header = o; o = align_up(o + sizeof(ProjHeader));
    L.views = o;  o = align_up(o + sizeof(ViewDesc) * (size_t)n_views);
    L.rec = o;    o = align_up(o + 64 * R);
    L.bbox = o;   o = align_up(o + 8 * R);
    L.depth = o;  o = align_up(o + 4 * R);
    L.ntiles = o; o = align_up(o + 4 * R);
    L.rect = o;   o = align_up(o + 4 * R);
    L.visbits = o; o = align_up(o + 4 * (size_t)n_views * (size_t)visbits_stride(n));
    L.gradmask = o; o = align_up(o + 8 * (size_t)n * (size_t)((n_views + 63) / 64));
    L.sgrad = o;  o = align_up(o + 64 * R);   // screen-space gradient, one 64-byte line per record
    L.blockcnt = o; o = align_up(o + 16 * (size_t)((n + 255) / 256));  // per-workgroup counts of the preprocess
    L.total = o;
    return L;
}

// Capacity-independent parts first, so that the tile ranges and work order
// can be located from the tile count alone.
struct BinsLayout {
    size_t header, tile_range, tile_order, pair_rec, total;
};
inline BinsLayout bins_layout(int64_t cap, int64_t n_tiles) {
    BinsLayout L;
    size_t o = 0;
    L.header = o;     o = align_up(o + sizeof(BinsHeader));
    L.tile_range = o; o = align_up(o + 8 * (size_t)n_tiles);
    L.tile_order = o; o = align_up(o + 4 * (size_t)n_tiles);
    L.pair_rec = o;   o = align_up(o + 4 * (size_t)cap);
    L.total = o;
    return L;
}

// Radix sort / scan geometry.
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;   // elements per block
constexpr int kMaxRadixBits = 9;  // digits of 8 or 9 bits
constexpr int kMaxRadix = 1 << kMaxRadixBits;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
// Row stride of a radix pass's digit-major histogram over nblocks chunks.
inline int64_t hist_stride(int64_t nblocks) { return (nblocks + 3) / 4 * 4; }

struct WorkLayout {
    // bin/sort phase
    size_t keys_a, dvals_a, keys_b, dvals_b, block_sum, group_sum, pkeys_a, pkeys_b, pvals_b, hist, totals,
        tkeys_a, tvals_a, tkeys_b, sort_total;
    size_t total;
    int64_t hist_blocks;  // max sort blocks of any sort
};
inline WorkLayout work_layout(int64_t n, int32_t n_views, int64_t cap, int64_t n_tiles) {
    WorkLayout L;
    size_t R = (size_t)n * (size_t)n_views, o = 0;
    int64_t maxn = (int64_t)R;
    if (cap > maxn) maxn = cap;
    if (n_tiles > maxn) maxn = n_tiles;
    // the depth sort's first pass takes one chunk per 4096 splats of a view
    const int64_t nbc = (int64_t)n_views * ceil_div(n, kSortTile);
    L.hist_blocks = ceil_div(maxn > 0 ? maxn : 1, kSortTile);
    if (nbc > L.hist_blocks) L.hist_blocks = nbc;
    size_t hist_n = (size_t)hist_stride(L.hist_blocks) * kMaxRadix;
    // depth sort: keys and (record, packed tile rectangle) values, ping-pong
    L.keys_a = o;   o = align_up(o + 4 * R);
    L.dvals_a = o;  o = align_up(o + 8 * R);
    L.keys_b = o;   o = align_up(o + 4 * R);
    L.dvals_b = o;  o = align_up(o + 8 * R);
    // output offsets of blocks of 4096 records (pair counts) and the pair
    // counts of their groups of 256 records (pair emission)
    const int64_t nbs = ceil_div((int64_t)R > 0 ? (int64_t)R : 1, 4096);
    L.block_sum = o; o = align_up(o + 4 * (size_t)nbs);
    L.group_sum = o; o = align_up(o + 4 * (size_t)ceil_div((int64_t)R > 0 ? (int64_t)R : 1, 256));
    L.pkeys_a = o;  o = align_up(o + 4 * (size_t)cap);
    L.pkeys_b = o;  o = align_up(o + 4 * (size_t)cap);
    L.pvals_b = o;  o = align_up(o + 4 * (size_t)cap);
    L.hist = o;     o = align_up(o + 4 * hist_n);
    L.totals = o;   o = align_up(o + 4 * (size_t)kMaxRadix);  // digit totals of a radix pass
    L.tkeys_a = o;  o = align_up(o + 4 * (size_t)n_tiles);
    L.tvals_a = o;  o = align_up(o + 4 * (size_t)n_tiles);
    L.tkeys_b = o;  o = align_up(o + 4 * (size_t)n_tiles);
    L.sort_total = o;
    L.total = L.sort_total;
    return L;
}

// Device pointers of the splat parameters.
struct SplatPtrs {
    const float *means, *scales, *quats, *opacities, *betas, *diffuse;
    const float *lobe_angles, *lobe_colors, *lobe_betas;
    int64_t n;
    int32_t m;
};
struct GradPtrs {
    float *means, *scales, *quats, *opacities, *betas, *diffuse;
    float *lobe_angles, *lobe_colors, *lobe_betas;
};

// Splat parameters updated in place (MCMC step).
struct SplatMut {
    float *means, *scales, *quats, *opacities, *betas, *diffuse;
    float *lobe_angles, *lobe_colors, *lobe_betas;
    int64_t n;
    int32_t m;
};

// Workspace of the MCMC relocation: per-block weight sums (+ total), inclusive
// weight prefix sums, copy counts, draw targets, new opacities.
struct McmcLayout {
    int64_t nblocks;
    size_t bsum, prefix, count, target, onew, total;
};
McmcLayout mcmc_layout(int64_t n);

// Pointers into `projected`.
struct ProjPtrs {
    ProjHeader *hdr;
    ViewDesc *views;
    RasterRec *rec;
    short4 *bbox;
    uint32_t *depth, *ntiles;
    uint32_t *rect;  // [R] packed tile rectangle (pack_tile_rect), written where ntiles > 0
    // [V][visbits_stride(n)]: bit i % 32 of word i / 32 of row v set when record
    // (v, i) has ntiles > 0; a row covers whole blocks of 4096 splats (the
    // padding bits stay zero)
    uint32_t *visbits;
    // [(V+63)/64][n]: bit v%64 of word v/64 set when the raster reverse pass has
    // sent gradient to record (v, i)'s line of sgrad; cleared with the line
    uint64_t *gradmask;
    float4 *sgrad;  // [R][4]: dmu'(2), dA(3), do, db, dcolour(3), 6 unused
    // [ceil(n / 256)][2]: visible records and pairs of each preprocess
    // workgroup, summed into hdr->counts by one workgroup afterwards
    uint64_t *blockcnt;
};
inline ProjPtrs proj_ptrs(void *base, int64_t n, int32_t n_views) {
    ProjLayout L = proj_layout(n, n_views);
    char *b = (char *)base;
    ProjPtrs p;
    p.hdr = (ProjHeader *)(b + L.header);
    p.views = (ViewDesc *)(b + L.views);
    p.rec = (RasterRec *)(b + L.rec);
    p.bbox = (short4 *)(b + L.bbox);
    p.depth = (uint32_t *)(b + L.depth);
    p.ntiles = (uint32_t *)(b + L.ntiles);
    p.rect = (uint32_t *)(b + L.rect);
    p.visbits = (uint32_t *)(b + L.visbits);
    p.gradmask = (uint64_t *)(b + L.gradmask);
    p.sgrad = (float4 *)(b + L.sgrad);
    p.blockcnt = (uint64_t *)(b + L.blockcnt);
    return p;
}

struct BinsPtrs {
    BinsHeader *hdr;
    uint32_t *pair_rec;
    uint2 *tile_range;
    uint32_t *tile_order;
};
inline BinsPtrs bins_ptrs(void *base, int64_t n_tiles) {
    BinsLayout L = bins_layout(0, n_tiles);
    char *b = (char *)base;
    BinsPtrs p;
    p.hdr = (BinsHeader *)(b + L.header);
    p.pair_rec = (uint32_t *)(b + L.pair_rec);
    p.tile_range = (uint2 *)(b + L.tile_range);
    p.tile_order = (uint32_t *)(b + L.tile_order);
    return p;
}

// Host-side helpers (abi.hip).
int64_t total_tiles(const dbs_camera *cams, int32_t n_views, int tile_w, int tile_h);

// ---- launchers (one per source file) ----
// preprocess.hip
hipError_t launch_upload_views(const dbs_camera *cams, int32_t n_views, int tile_w, int tile_h,
                               ProjPtrs P, int64_t n, int32_t m, hipStream_t s);
// sh != nullptr selects the Gaussian-kernel + SH comparison mode ([n, 16, 3] coefficients)
hipError_t launch_preprocess(const SplatPtrs &sp, const float *sh, ProjPtrs P, int32_t n_views, int tile_w,
                             int tile_h, uint32_t flags, float b_split, int64_t *counts, hipStream_t s);
// sort.hip
// the device address of dbs_bin_sort_noalloc's scratch on the current device
// (DBS_NOALLOC_SCRATCH_BYTES), looked up once per device
hipError_t noalloc_scratch(void **out);
hipError_t launch_bin_sort(ProjPtrs P, BinsPtrs B, void *work, int64_t n, int32_t n_views,
                           int64_t cap, int64_t n_tiles, int tile_w, int tile_h,
                           int32_t *overflow_out, hipStream_t s);
// raster.hip
bool raster_supported(int tw, int th, int batch);
hipError_t launch_raster_fwd(ProjPtrs P, BinsPtrs B, int64_t n, int32_t n_views, int64_t n_tiles,
                             const dbs_raster_cfg &cfg, float *image, float *final_T,
                             int32_t *last_index, hipStream_t s);
hipError_t launch_raster_bwd(ProjPtrs P, BinsPtrs B, int64_t n, int32_t n_views, int64_t n_tiles,
                             const dbs_raster_cfg &cfg, const float *final_T,
                             const int32_t *last_index, const float *dL_dimage, float *sgrad, int64_t *atomics,
                             hipStream_t s);
hipError_t launch_raster_stats(ProjPtrs P, BinsPtrs B, int64_t n, int32_t n_views, int64_t n_tiles,
                               const dbs_raster_cfg &cfg, const float *final_T, const int32_t *last_index,
                               int64_t *out, hipStream_t s);
// project_bwd.hip (also the L1 loss)
// store: write the gradients instead of adding them to the buffers
hipError_t launch_project_bwd(const SplatPtrs &sp, ProjPtrs P, int32_t n_views, const GradPtrs &g, bool store,
                              hipStream_t s);
hipError_t launch_l1_loss(const float *image, const float *target, int64_t count, float scale,
                          float *grad, float *loss, hipStream_t s);
// mcmc.hip
hipError_t launch_mcmc_relocate(const SplatMut &p, float tau, const uint32_t *rand, void *work, int32_t *n_relocated,
                                hipStream_t s);
hipError_t launch_mcmc_noise(const SplatMut &p, const float *z, float lr, float lambda_eps, float b_prime,
                             hipStream_t s);
// loss.hip
hipError_t launch_photometric_loss(const float *image, const float *target, const dbs_camera *cams,
                                   int32_t n_views, float lam, float *grad, float *loss, hipStream_t s);
hipError_t launch_regularizer(const SplatPtrs &sp, float lam_o, float lam_s, const GradPtrs &g, float *loss,
                              hipStream_t s);

}  // namespace dbs
