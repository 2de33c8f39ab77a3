// Tile rasterizer: forward compositing and its reverse pass.
//
// Forward, Sec. 3.2 Eq. (6): each pixel walks its tile's list front to back,
// r^2 = d^T A d (Eq. 5, A = Sigma'^{-1}), alpha = min(alpha_max, o (1 - r^2)^beta)
// where r^2 < 1 (the Beta kernel of Sec. 3.1 is exactly zero elsewhere),
// C += c alpha T, T *= 1 - alpha, and stops after the splat that takes T
// below t_eps.  Output C + T bg, the final T and the last list position used.
//
// Reverse: each pixel walks the same list back to front from its last
// position.  Instead of storing per-pixel lists, the transmittance in front
// of splat i is recovered as T_i = T_{i+1} / (1 - alpha_i) (alpha <= alpha_max
// < 1), and the colour behind it, S_i = sum_{k>i} c_k alpha_k T_k + T_N bg, is
// accumulated on the way.  Then
//   dL/dc_i     = alpha_i T_i g
//   dL/dalpha_i = T_i (g . c_i) - (g . S_i) / (1 - alpha_i)
// and through alpha = o B, B = (1 - r^2)^beta, beta = 4 e^b (Sec. 3.1, Eq. 3):
//   dL/do = dL/dalpha B,  dL/db = dL/dalpha o B ln(1 - r^2) beta,
//   dL/dr^2 = -dL/dalpha o beta B / (1 - r^2)  (all zero when alpha is clamped),
//   dL/dmu' = -2 dL/dr^2 A d,   dL/dA = dL/dr^2 d d^T.
// Every record that is sent a non-zero sum also gets its bit in gradmask, so
// that the projection's reverse pass reads only the lines that hold gradient.
// The per-pixel terms are summed without their per-splat factors (o, beta,
// A), which are applied once per (tile, splat) before the global atomics.
// The ten per-(pixel, splat) values are summed over each 16-lane row with a
// DPP halving butterfly (wave_reduce.h), added into per-wavefront LDS slots
// (plain read-add-write: LDS float atomics cost about a cycle per lane), summed
// over the wavefronts once per batch, and added once per (tile, splat) to the
// per-record screen-space gradient with a global float atomic.
//
// Each wavefront owns an 8x8 pixel block, each 16-lane row of it a 4x4
// quadrant, and every row walks only the splats whose support can reach its
// quadrant (see `stage`).
//
// Work items are (view, tile) pairs.  A persistent grid drains a device
// queue ordered heaviest tile first; the last workgroup to finish resets the
// queue so that the next launch (or graph replay) starts from zero.
#include "dbs_internal.h"
#include "wave_reduce.h"

namespace dbs {

namespace {

struct RasterArgs {
    const ProjHeader *ph;
    const BinsHeader *bh;
    int64_t n;
    const ViewDesc *views;
    int32_t n_views;
    uint32_t n_tiles;
    const RasterRec *rec;
    const uint32_t *pair_rec;
    const uint2 *ranges;
    const uint32_t *order;
    uint32_t *queue;  // [head, done]
    float *image;
    float *final_T;
    int32_t *last_index;
    const float *dL_dimage;
    float *sgrad;     // [R][16] screen-space gradient per record
    uint64_t *gradmask;  // [(V+63)/64][n]: records whose sgrad line was sent gradient
    float t_eps, alpha_max;
    int32_t persistent;
    unsigned long long *atomics;  // counting reverse pass only: global float atomics issued (added to)
};

// r^2 = A00 dx^2 + 2 A01 dx dy + A11 dy^2 in FP64 with a fixed rounding
// sequence, so that the forward and reverse kernels take identical support
// decisions.  FP64 keeps 1 - r^2 accurate at the support edge, where the Beta
// kernel's slope beta (1 - r^2)^(beta - 1) is unbounded for beta < 1.
__device__ __forceinline__ double eval_r2(double dx, double dy, double a00, double a01x2, double a11)
{
    const double t = fma(a01x2, dy, __dmul_rn(a00, dx));
    return fma(dx, t, __dmul_rn(__dmul_rn(a11, dy), dy));
}

// B = (1 - r^2)^beta via exp2(beta log2(1 - r^2)); omr = 1 - r^2 > 0.
__device__ __forceinline__ float eval_kernel(float omr, float beta, float *lg)
{
    *lg = __builtin_amdgcn_logf(omr);
    return __builtin_amdgcn_exp2f(__fmul_rn(beta, *lg));
}

// alpha = min(alpha_max, o B), with the same clamp decision in both passes:
// a product that is not at most alpha_max (NaN included) is clamped, takes
// alpha_max and passes no gradient to o, b or the geometry.
__device__ __forceinline__ float clamp_alpha(float araw, float alpha_max, bool *clamped)
{
    *clamped = !(araw <= alpha_max);
    return *clamped ? alpha_max : araw;
}

__device__ __forceinline__ float2 unpack2(double d) { return __builtin_bit_cast(float2, d); }
__device__ __forceinline__ double pack2(float a, float b) { return __builtin_bit_cast(double, make_float2(a, b)); }

__device__ __forceinline__ int find_view(const ViewDesc *views, int32_t n_views, uint32_t g)
{
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((uint32_t)views[mid].tile_offset <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The buffers were built for this splat count, view count and tile shape:
// otherwise the pointers derived from them would not match the buffers'
// layout, and the raster calls leave everything untouched.
template <int TW, int TH>
__device__ __forceinline__ bool buffers_match(const RasterArgs &a)
{
    const BinsHeader *bh = a.bh;
    return bh->n == a.n && bh->n_views == a.n_views && bh->tile_w == TW && bh->tile_h == TH &&
           bh->n_tiles == a.n_tiles && a.ph->n == a.n && a.ph->n_views == a.n_views;
}

struct Item {
    uint32_t g;
    int32_t v;
    int32_t ox, oy;
    uint32_t start, end;
};

template <int TW, int TH>
__device__ __forceinline__ bool fetch_item(const RasterArgs &a, uint32_t *head, Item *s_item, int iter)
{
    if (threadIdx.x == 0) {
        uint32_t k;
        if (iter == 0 && !buffers_match<TW, TH>(a)) k = a.n_tiles;
        else if (a.persistent) k = atomicAdd(head, 1u);
        else k = iter == 0 ? blockIdx.x : a.n_tiles;
        Item it;
        it.g = 0xffffffffu;
        if (k < a.n_tiles) {
            it.g = a.order[k];
            it.v = find_view(a.views, a.n_views, it.g);
            const ViewDesc &V = a.views[it.v];
            const uint32_t lt = it.g - (uint32_t)V.tile_offset;
            it.ox = (int32_t)(lt % (uint32_t)V.tiles_x) * TW;
            it.oy = (int32_t)(lt / (uint32_t)V.tiles_x) * TH;
            const uint2 r = a.ranges[it.g];
            it.start = r.x;
            it.end = r.y;
        }
        *s_item = it;
    }
    __syncthreads();
    return s_item->g != 0xffffffffu;
}

__device__ __forceinline__ void finish_persistent(const RasterArgs &a, uint32_t *head, uint32_t *done)
{
    if (a.persistent && threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(done, 1u) == gridDim.x - 1) {
            atomicExch(head, 0u);
            atomicExch(done, 0u);
        }
    }
}

// ---------------------------------------------------------------- staging
//
// Each wavefront covers one 8x8 block of the tile (block w at
// ((w % (TW/8)) * 8, (w / (TW/8)) * 8)); each 16-lane row of a wavefront covers
// one 4x4 quadrant of its block (row r at ((r & 1) * 4, (r >> 1) * 4)), and
// lane i of a row the pixel (i & 3, i >> 2) of its quadrant.
//
// Culling in two levels.  When a batch of splats is staged in LDS, the staging
// thread tests every block's pixel-centre rectangle: exactly (the minimum of
// r^2 over it, as for quadrants below) in the reverse pass, against the
// axis-aligned box of the splat's r^2 < 1 ellipse (cheap, conservative) in the
// forward pass, where staging is a larger share of the work.  Each wavefront
// then compacts the splats that reach its block and tests its four quadrants
// exactly: the minimum of r^2 over the quadrant's pixel-centre rectangle.  A
// rectangle whose minimum is at least 1 + 1e-4 (+ a term for elongated
// splats, cull_threshold) cannot hold a pixel with r^2 < 1: the FP32 error of
// the minimum is below that margin, so the splat is left out of that row's
// list.  Each row walks its own list; the four rows of a wavefront
// step through their lists together.  The lists change which (pixel, splat)
// pairs are evaluated, never a result.

template <int TW, int TH>
struct Geo {
    static constexpr int NT = TW * TH;
    static constexpr int NW = NT / kWave;  // waves = 8x8 blocks
    static constexpr int BX = TW / 8;
    static_assert(TW % 8 == 0 && TH % 8 == 0, "tiles are made of 8x8 blocks");
};

// Tile-local pixel of a lane: block of wave w, quadrant of row lane/16.
template <int TW, int TH>
struct LanePixel {
    int bx, by, row, lx, ly;
    __device__ LanePixel(int w, int lane)
    {
        bx = (w % Geo<TW, TH>::BX) * 8;
        by = (w / Geo<TW, TH>::BX) * 8;
        row = lane >> 4;
        lx = bx + (row & 1) * 4 + (lane & 3);
        ly = by + (row >> 1) * 4 + ((lane >> 2) & 3);
    }
};

// min over p in [x0,x1] x [y0,y1] of (p - c)^T A (p - c), A positive definite.
// 0 when c lies in the rectangle.  Otherwise the minimum lies on an edge that
// faces c: on a vertical edge the minimiser over y has dq/dx = 2 dx det A / A11,
// which points into the rectangle (q falls inwards) unless c is beyond that
// edge, and likewise for horizontal edges.  So only the vertical edge on c's
// side (when c is outside the x range) and the horizontal edge on c's side
// (outside the y range) are evaluated, each at its minimiser clamped to the
// edge, which also covers the corners.
__device__ __forceinline__ float rect_min_r2(float cx, float cy, float a00, float a01, float a11, float x0,
                                             float x1, float y0, float y1)
{
    const float dx0 = x0 - cx, dx1 = x1 - cx, dy0 = y0 - cy, dy1 = y1 - cy;
    const bool inx = dx0 <= 0.0f && dx1 >= 0.0f, iny = dy0 <= 0.0f && dy1 >= 0.0f;
    const float r00 = __builtin_amdgcn_rcpf(a00), r11 = __builtin_amdgcn_rcpf(a11);
    const float dx = dx0 > 0.0f ? dx0 : dx1;  // the facing vertical edge
    const float dy = fminf(fmaxf(-a01 * dx * r11, dy0), dy1);
    const float qv = a00 * dx * dx + 2.0f * a01 * dx * dy + a11 * dy * dy;
    const float ey = dy0 > 0.0f ? dy0 : dy1;  // the facing horizontal edge
    const float ex = fminf(fmaxf(-a01 * ey * r00, dx0), dx1);
    const float qh = a00 * ex * ex + 2.0f * a01 * ex * ey + a11 * ey * ey;
    return inx ? (iny ? 0.0f : qh) : (iny ? qv : fminf(qv, qh));
}

// Culling threshold for the FP32 minimum of r^2 over a rectangle.  Rounding
// the conic to FP32 and evaluating the form perturb r^2 by a few ulp of the
// unsigned form |A00| dx^2 + 2 |A01 dx dy| + |A11| dy^2, which is at most about
// 2 kappa r^2 for the condition number kappa = l_max / l_min of A (the square
// of the footprint's aspect ratio).  The threshold adds 1e-6 kappa (over 16
// ulp of that) to the 1e-4 margin, so that no splat, however elongated, is
// culled from a rectangle holding a pixel with r^2 < 1.  kappa =
// (tr + sqrt(tr^2 - 4 det))^2 / (4 det), det in FP64.
__device__ __forceinline__ float cull_threshold(double a00, double a01, double a11)
{
    const float fdet = (float)(a00 * a11 - a01 * a01);
    if (!(fdet > 0.0f)) return 3.0e38f;  // not a valid projection: never cull
    const float tr = (float)(a00 + a11);
    const float r = __builtin_amdgcn_sqrtf(fmaxf(tr * tr - 4.0f * fdet, 0.0f));
    const float kappa = (tr + r) * (tr + r) * __builtin_amdgcn_rcpf(4.0f * fdet);
    return 1.0001f + 1e-6f * kappa;
}

// LDS image of a staged splat: tile-local centre and conic in FP64, (o, beta)
// packed in the second half of s_b, colour and the block mask in s_col.
struct Staged {
    double2 *c;    // (cx, cy) relative to the tile origin
    double2 *a;    // (A00, 2 A01)
    double2 *b;    // (A11, pack(o, beta))
    float4 *col;   // (r, g, b, block mask bits)
    uint32_t *rec; // record index (reverse pass only)
};

// Stage records [lo, lo + nb) of the pair list into LDS slot k = j - lo.
template <int TW, int TH, bool BOX_BLOCKS>
__device__ __forceinline__ void stage(const RasterArgs &a, uint32_t lo, int nb, double dox, double doy,
                                      const Staged &S, int tid)
{
    using G = Geo<TW, TH>;
    for (int k = tid; k < nb; k += G::NT) {
        const uint32_t rec = a.pair_rec[lo + (uint32_t)k];
        const RasterRec r = a.rec[rec];
        const double cx = r.cx - dox, cy = r.cy - doy;
        uint32_t mask = (1u << G::NW) - 1u;
        const double det = BOX_BLOCKS ? r.a00 * r.a11 - r.a01 * r.a01 : 0.0;
        if (!BOX_BLOCKS) {
            // exact: the minimum of r^2 over the block's pixel-centre rectangle
            const float fcx = (float)cx, fcy = (float)cy, f00 = (float)r.a00, f01 = (float)r.a01,
                        f11 = (float)r.a11;
            const float thr = cull_threshold(r.a00, r.a01, r.a11);
            mask = 0;
#pragma unroll
            for (int w = 0; w < G::NW; ++w) {
                const float bx = (float)((w % G::BX) * 8), by = (float)((w / G::BX) * 8);
                const float m = rect_min_r2(fcx, fcy, f00, f01, f11, bx + 0.5f, bx + 7.5f, by + 0.5f, by + 7.5f);
                if (!(m >= thr)) mask |= 1u << w;
            }
        } else if (det > 0.0) {
            // the axis-aligned box of the r^2 < 1 ellipse, half extents
            // sqrt(Sigma'_xx) = sqrt(A11 / det A) and sqrt(Sigma'_yy), det A in FP64
            // (no cancellation for elongated splats), widened by a relative 1e-4;
            // det A <= 0 (not from a valid projection) keeps every block
            const float fcx = (float)cx, fcy = (float)cy;
            const float idet = __builtin_amdgcn_rcpf((float)det);
            const float ex = __builtin_amdgcn_sqrtf((float)r.a11 * idet) * 1.0001f + 1e-4f;
            const float ey = __builtin_amdgcn_sqrtf((float)r.a00 * idet) * 1.0001f + 1e-4f;
            mask = 0;
#pragma unroll
            for (int w = 0; w < G::NW; ++w) {
                const float bx = (float)((w % G::BX) * 8), by = (float)((w / G::BX) * 8);
                if (fcx + ex >= bx + 0.5f && fcx - ex <= bx + 7.5f && fcy + ey >= by + 0.5f && fcy - ey <= by + 7.5f)
                    mask |= 1u << w;
            }
        }
        S.c[k] = make_double2(cx, cy);
        S.a[k] = make_double2(r.a00, 2.0 * r.a01);
        S.b[k] = make_double2(r.a11, pack2(r.opacity, r.beta));
        S.col[k] = make_float4(r.r, r.g, r.b, __uint_as_float(mask));
        if (S.rec) S.rec[k] = rec;
    }
}

__device__ __forceinline__ uint64_t lanes_below(int lane) { return lane ? (~0ull >> (64 - lane)) : 0ull; }

// Wave `w` collects, in order, the slots [0, nb) whose block mask has bit w.
__device__ __forceinline__ int build_list(const float4 *s_col, int nb, int w, uint8_t *list, int lane)
{
    int cnt = 0;
    for (int base = 0; base < nb; base += kWave) {
        const int k = base + lane;
        const bool in = k < nb && ((__float_as_uint(s_col[k].w) >> w) & 1u);
        const uint64_t bal = __ballot(in);
        if (in) list[cnt + __popcll(bal & lanes_below(lane))] = (uint8_t)k;
        cnt += __popcll(bal);
    }
    return cnt;
}

// Splits a wave's block list into the lists of its four rows (quadrants), in
// order: slot k goes to row r if its support reaches the quadrant and its list
// position lo + k is at most lim[r].  Row r's list starts at rows[r * RS + PAD];
// counts returned in cnt.
template <int RS, int PAD>
__device__ __forceinline__ void build_rows(const Staged &S, const uint8_t *blist, int cnt_b, int bx, int by,
                                           int64_t lo, const int32_t lim[4], uint8_t *rows, int cnt[4], int lane)
{
    cnt[0] = cnt[1] = cnt[2] = cnt[3] = 0;
    for (int base = 0; base < cnt_b; base += kWave) {
        const int e = base + lane;
        const bool valid = e < cnt_b;
        const int k = valid ? blist[e] : 0;
        const double2 c = S.c[k], aa = S.a[k], bb = S.b[k];
        const float fcx = (float)c.x, fcy = (float)c.y;
        const float f00 = (float)aa.x, f01 = (float)(0.5 * aa.y), f11 = (float)bb.x;
        const float thr = cull_threshold(aa.x, 0.5 * aa.y, bb.x);
        const int32_t j = (int32_t)(lo + k);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float x0 = (float)(bx + (r & 1) * 4) + 0.5f, y0 = (float)(by + (r >> 1) * 4) + 0.5f;
            const bool in = valid && j <= lim[r] &&
                            !(rect_min_r2(fcx, fcy, f00, f01, f11, x0, x0 + 3.0f, y0, y0 + 3.0f) >= thr);
            const uint64_t bal = __ballot(in);
            if (in) rows[r * RS + PAD + cnt[r] + __popcll(bal & lanes_below(lane))] = (uint8_t)k;
            cnt[r] += __popcll(bal);
        }
    }
}

__device__ __forceinline__ int pick4(const int v[4], int r)
{
    return r == 0 ? v[0] : (r == 1 ? v[1] : (r == 2 ? v[2] : v[3]));
}

__device__ __forceinline__ int max4(const int v[4]) { return max(max(v[0], v[1]), max(v[2], v[3])); }

// Reverse walk: at step s row r takes entry cnt[r] - 1 - s of its list.  Rows
// that take the same splat at the same step would add to the same LDS slot, so
// their sums are merged first and only the lowest such row stores.  Bit
// 4e + r of share[s], e = 0/1/2: row r's splat is also that of row r^(e+1);
// bit 12 + r: another, lower row stores for row r.  Zero: no two rows share.
template <int RS, int PAD>
__device__ __forceinline__ void mark_shared_steps(const uint8_t *rows, const int cnt[4], int steps, uint16_t *share,
                                                  int lane)
{
    for (int s0 = 0; s0 < steps; s0 += kWave) {
        const int st = s0 + lane;
        int kk[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int t = cnt[r] - 1 - st;
            kk[r] = (st < steps && t >= 0) ? (int)rows[r * RS + PAD + t] : -1 - r;
        }
        uint32_t word = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const bool e1 = kk[r] == kk[r ^ 1], e2 = kk[r] == kk[r ^ 2], e3 = kk[r] == kk[r ^ 3];
            const bool below = (e1 && (r ^ 1) < r) || (e2 && (r ^ 2) < r) || (e3 && (r ^ 3) < r);
            word |= ((uint32_t)e1 << r) | ((uint32_t)e2 << (4 + r)) | ((uint32_t)e3 << (8 + r)) |
                    ((uint32_t)below << (12 + r));
        }
        if (st < steps) share[st] = (uint16_t)word;
    }
}

// ---------------------------------------------------------------- forward

// GAUSS: the Gaussian-kernel comparison mode.  Its records carry the conic
// of the 3-sigma ellipse (Sigma'^{-1} / 9), so r^2 < 1 is the support and
// the kernel is exp(-m^2 / 2) = exp(-4.5 r^2) = exp2(-4.5 log2(e) r^2).
template <int TW, int TH, int BATCH, bool GAUSS = false>
__global__ __launch_bounds__(TW *TH) void raster_fwd_kernel(RasterArgs a)
{
    using G = Geo<TW, TH>;
    static_assert(BATCH <= 256, "list entries are 8-bit");
    __shared__ double2 s_c[BATCH], s_a[BATCH], s_b[BATCH];
    __shared__ float4 s_col[BATCH];
    __shared__ uint8_t s_blist[G::NW][BATCH];
    __shared__ uint8_t s_rows[G::NW][4 * BATCH];
    __shared__ Item s_item;
    const Staged S{s_c, s_a, s_b, s_col, nullptr};
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const LanePixel<TW, TH> P(w, lane);
    const double fpx = (double)P.lx + 0.5, fpy = (double)P.ly + 0.5;
    const uint8_t *my_row = &s_rows[w][P.row * BATCH];
    // A row's entries past its count are read too (and masked): every entry
    // ever read is then a slot index below BATCH.
    for (int i = lane; i < 4 * BATCH; i += kWave) s_rows[w][i] = 0;
    float amax = a.alpha_max;
    asm volatile("" : "+v"(amax));  // held in a VGPR: the clamp's select then needs no copy per step
    const float teps = a.t_eps;

    for (int iter = 0;; ++iter) {
        if (!fetch_item<TW, TH>(a, &a.queue[0], &s_item, iter)) break;
        const Item it = s_item;
        const ViewDesc &V = a.views[it.v];
        const int px = it.ox + P.lx, py = it.oy + P.ly;
        const bool inside = px < V.width && py < V.height;
        // a pixel has stopped once T < t_eps (t_eps >= 0): one outside the view
        // starts stopped at T = -1, and T only changes while a pixel runs
        float T = inside ? 1.0f : -1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
        int32_t last = -1;

        for (uint32_t start = it.start; start < it.end; start += BATCH) {
            if (__syncthreads_count(!(T < teps)) == 0) break;
            const int nb = (int)min((uint32_t)BATCH, it.end - start);
            stage<TW, TH, true>(a, start, nb, (double)it.ox, (double)it.oy, S, tid);
            __syncthreads();
            // rows whose pixels have all stopped take no entries
            const uint64_t live = __ballot(!(T < teps));
            int32_t lim[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) lim[r] = ((live >> (16 * r)) & 0xffffull) ? INT32_MAX : -1;
            const int cnt_b = live ? build_list(s_col, nb, w, s_blist[w], lane) : 0;
            int cnt[4];
            build_rows<BATCH, 0>(S, s_blist[w], cnt_b, P.bx, P.by, (int64_t)start, lim, s_rows[w], cnt, lane);
            // wave-uniform step bound (a scalar loop counter); the row's list
            // address is kept in one register (one add per step)
            const int my_cnt = pick4(cnt, P.row), steps = __builtin_amdgcn_readfirstlane(max4(cnt));
            int rbase = (w * 4 + P.row) * BATCH;  // my_row, as an index into s_rows
            asm volatile("" : "+v"(rbase));
            for (int t = 0; t < steps; ++t) {
                const bool on = t < my_cnt, running = !(T < teps), act = on && running;
                // two ballots of plain compares, combined on the scalar unit
                if (!(__ballot(on) & __ballot(running))) break;
                const int k = (&s_rows[0][0])[rbase + t];
                const double2 c = s_c[k], aa = s_a[k], bb = s_b[k];
                const double r2 = eval_r2(fpx - c.x, fpy - c.y, aa.x, aa.y, bb.x);
                if (act && r2 < 1.0) {
                    const float2 ob = unpack2(bb.y);
                    float lg;
                    const float B = GAUSS ? __builtin_amdgcn_exp2f(-6.4921276840003350f * (float)r2)
                                          : eval_kernel((float)(1.0 - r2), ob.y, &lg);
                    bool clamped;
                    const float alpha = clamp_alpha(__fmul_rn(ob.x, B), amax, &clamped);
                    const float wgt = alpha * T;
                    const float4 cc = s_col[k];
                    C0 = __fmaf_rn(cc.x, wgt, C0);
                    C1 = __fmaf_rn(cc.y, wgt, C1);
                    C2 = __fmaf_rn(cc.z, wgt, C2);
                    T = __fmul_rn(T, __fsub_rn(1.0f, alpha));
                    last = (int32_t)(start + (uint32_t)k);
                }
            }
        }
        if (inside) {
            const int64_t npx = (int64_t)V.width * V.height;
            const int64_t pl = (int64_t)py * V.width + px;
            float *img = a.image + 3 * V.pixel_offset + pl;
            img[0] = __fmaf_rn(T, V.bg[0], C0);
            img[npx] = __fmaf_rn(T, V.bg[1], C1);
            img[2 * npx] = __fmaf_rn(T, V.bg[2], C2);
            a.final_T[V.pixel_offset + pl] = T;
            a.last_index[V.pixel_offset + pl] = last;
        }
        __syncthreads();  // s_item and the LDS batch are reused by the next item
    }
    finish_persistent(a, &a.queue[0], &a.queue[1]);
}

// ---------------------------------------------------------------- reverse

__device__ __forceinline__ uint64_t wave_sum_u32(uint32_t v)
{
    uint64_t x = v;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

__device__ __forceinline__ int wave_max_i32(int v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
    return v;
}

// Per-row (16-lane) maxima of v, as four wave-uniform values.
__device__ __forceinline__ void row_max4_i32(int v, int out[4])
{
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 16));
#pragma unroll
    for (int r = 0; r < 4; ++r) out[r] = __builtin_amdgcn_readlane(v, 16 * r);
}

// At most 128 VGPRs below 512 threads (4 waves per SIMD, as many as the LDS
// allows): the register allocator otherwise drifts past 128 on small source
// changes.  32x16 tiles are held to 3 waves by their LDS anyway.  COUNT: the
// introspection variant that also counts the global float atomics it issues.
template <int TW, int TH, int BATCH, bool COUNT = false>
__global__ __launch_bounds__(TW *TH) __attribute__((amdgpu_waves_per_eu(TW * TH >= 512 ? 3 : 4))) void raster_bwd_kernel(RasterArgs a)
{
    using G = Geo<TW, TH>;
    constexpr int NT = G::NT;
    constexpr int NG = 10;
    static_assert(BATCH < 256, "list entries are 8-bit, slot BATCH is the sentinel");
    // Slot BATCH holds a sentinel splat that reaches no pixel.  PAD sentinel
    // entries precede each row's list, so that a row whose list is exhausted
    // keeps taking valid entries (and contributes nothing) while the other
    // rows of its wavefront step on: the step loop needs no per-lane bounds.
    constexpr int PAD = BATCH + 4, RS = PAD + BATCH;
    float amax = a.alpha_max;
    asm volatile("" : "+v"(amax));  // held in a VGPR: the clamp's select then needs no copy per step
    __shared__ double2 s_c[BATCH + 1], s_a[BATCH + 1], s_b[BATCH + 1];
    __shared__ float4 s_col[BATCH + 1];
    __shared__ uint32_t s_rec[BATCH];
    // per-wave sums (slot BATCH: the sentinel's; one more slot keeps the array a whole number of float4s);
    // wave 0's slot ends up with the total
    __shared__ __align__(16) float s_g[G::NW][BATCH + 2][NG];
    __shared__ uint8_t s_blist[G::NW][BATCH];
    __shared__ uint8_t s_rows[G::NW][4 * RS];
    __shared__ uint16_t s_share[G::NW][BATCH];
    __shared__ Item s_item;
    __shared__ int32_t s_maxlast;
    const Staged S{s_c, s_a, s_b, s_col, s_rec};
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const LanePixel<TW, TH> P(w, lane);
    const double fpx = (double)P.lx + 0.5, fpy = (double)P.ly + 0.5;
    const uint8_t *my_row = &s_rows[w][P.row * RS + PAD];
    // written once; the first work item's barrier orders them before any use
    if (tid == 0) {
        s_c[BATCH] = make_double2(1e30, 1e30);  // r^2 ~ 1e60 at every pixel
        s_a[BATCH] = make_double2(1.0, 0.0);
        s_b[BATCH] = make_double2(1.0, pack2(0.0f, 1.0f));
        s_col[BATCH] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    for (int i = lane; i < 4 * PAD; i += kWave) s_rows[w][(i / PAD) * RS + i % PAD] = (uint8_t)BATCH;
    const float kLn2 = 0.69314718055994531f;
    const int fld = row10_field(lane);  // value whose row total this lane stores
    uint32_t n_atomics = 0;  // COUNT only

    for (int iter = 0;; ++iter) {
        if (!fetch_item<TW, TH>(a, &a.queue[2], &s_item, iter)) break;
        const Item it = s_item;
        const ViewDesc &V = a.views[it.v];
        const int px = it.ox + P.lx, py = it.oy + P.ly;
        const bool inside = px < V.width && py < V.height;
        const int64_t npx = (int64_t)V.width * V.height;
        const int64_t pl = (int64_t)py * V.width + px;
        float T = 1.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
        int32_t last = -1;
        if (inside) {
            T = a.final_T[V.pixel_offset + pl];
            last = a.last_index[V.pixel_offset + pl];
            const float *gi = a.dL_dimage + 3 * V.pixel_offset + pl;
            g0 = gi[0];
            g1 = gi[npx];
            g2 = gi[2 * npx];
        }
        // last positions come from the forward over the same lists; keep them
        // inside this tile's range so that no pair outside it is ever read
        if (last >= (int32_t)it.end) last = (int32_t)it.end - 1;
        // g . S, S the colour composited behind the current splat (background included)
        float gS = g0 * (T * V.bg[0]) + g1 * (T * V.bg[1]) + g2 * (T * V.bg[2]);
        if (tid == 0) s_maxlast = -1;
        __syncthreads();
        const int32_t wave_last = wave_max_i32(last);
        int32_t row_last[4];
        row_max4_i32(last, row_last);
        if (lane == 0 && wave_last >= 0) atomicMax(&s_maxlast, wave_last);
        __syncthreads();
        const int64_t maxlast = s_maxlast;

        if (maxlast >= (int64_t)it.start) {
            for (int64_t hi = maxlast + 1; hi > (int64_t)it.start; hi -= BATCH) {
                const int64_t lo = hi - BATCH > (int64_t)it.start ? hi - BATCH : (int64_t)it.start;
                const int nb = (int)(hi - lo);
                stage<TW, TH, false>(a, (uint32_t)lo, nb, (double)it.ox, (double)it.oy, S, tid);
                static_assert(sizeof(s_g) % 16 == 0, "slots are cleared in float4s");
                for (int idx = tid; idx < (int)(sizeof(s_g) / 16); idx += NT)
                    reinterpret_cast<float4 *>(&s_g[0][0][0])[idx] = make_float4(0.f, 0.f, 0.f, 0.f);
                __syncthreads();
                // this wave only needs its own splats up to its last contributor
                const int64_t kmax64 = (int64_t)wave_last - lo;
                const int nbw = kmax64 < (int64_t)(nb - 1) ? (int)kmax64 + 1 : nb;
                // this pixel's last contributor as a slot of the batch (-1: none in it)
                const int64_t lk64 = (int64_t)last - lo;
                int last_k = lk64 < 0 ? -1 : (lk64 > (int64_t)BATCH ? BATCH : (int)lk64);
                asm volatile("" : "+v"(last_k));  // one compare per step for k <= last_k
                const int cnt_b = nbw > 0 ? build_list(s_col, nbw, w, s_blist[w], lane) : 0;
                int cnt[4];
                build_rows<RS, PAD>(S, s_blist[w], cnt_b, P.bx, P.by, lo, row_last, s_rows[w], cnt, lane);
                // wave-uniform (ballot counts): a scalar loop bound and counter
                const int my_cnt = pick4(cnt, P.row), steps = __builtin_amdgcn_readfirstlane(max4(cnt));
                mark_shared_steps<RS, PAD>(s_rows[w], cnt, steps, s_share[w], lane);
                // list entries are read one step ahead, back to front; past the
                // front (t < 0, down to -steps - 1 >= -PAD) they are the sentinel
                int kl_next = my_row[my_cnt - 1];
                for (int step = 0; step < steps; ++step) {
                    const int t = my_cnt - 1 - step;
                    const int k = kl_next;
                    __builtin_assume(k >= 0 && k <= BATCH);  // list entries are bytes
                    kl_next = my_row[t - 1];
                    const bool owner = fld >= 0;
                    float *dst = &s_g[w][k][owner ? fld : 0];
                    // read early: the slot's running sum, added to at the end of the step
                    const float prev = *dst;
                    const uint32_t share = __builtin_amdgcn_readfirstlane(s_share[w][step]);
                    const double2 c = s_c[k], aa = s_a[k];
                    double2 bb = s_b[k];
                    asm volatile("" : "+v"(bb.y));  // one 16-byte read of the slot's third pair
                    const double dxd = fpx - c.x, dyd = fpy - c.y;
                    const double r2 = eval_r2(dxd, dyd, aa.x, aa.y, bb.x);
                    const bool live = k <= last_k, in = r2 < 1.0, contrib = live && in;
                    // two ballots of plain compares, combined on the scalar unit
                    if (!(__ballot(live) & __ballot(in))) continue;
                    // Branch-free from here: a lane that does not take part uses
                    // r^2 = 0 (finite logs) and alpha = 0 (T, S unchanged), and
                    // its terms are multiplied by zero.
                    const float2 ob = unpack2(bb.y);
                    const float omr = contrib ? (float)(1.0 - r2) : 1.0f;
                    float lg;
                    const float B = eval_kernel(omr, ob.y, &lg);
                    const float araw = __fmul_rn(ob.x, B);
                    bool clamped;
                    const float alpha_c = clamp_alpha(araw, amax, &clamped);
                    const float alpha = contrib ? alpha_c : 0.0f;
                    const float inv = __builtin_amdgcn_rcpf(1.0f - alpha);
                    const float Ti = T * inv;
                    const float wgt = alpha * Ti;
                    const float4 cc = s_col[k];
                    const float gc = g0 * cc.x + g1 * cc.y + g2 * cc.z;
                    const float dLda = Ti * gc - inv * gS;
                    gS = __fmaf_rn(gc, wgt, gS);
                    T = Ti;  // a lane not taking part has alpha = 0, inv = 1 exactly
                    // per-splat factors (o, beta, A) are applied once after the sums
                    const float t1 = (contrib && !clamped) ? dLda * B : 0.0f;
                    const float gp = t1 * __builtin_amdgcn_rcpf(omr);
                    const float dx = (float)dxd, dy = (float)dyd;
                    const float u = gp * dx, wv = gp * dy;
                    float v[NG];
                    v[0] = u;
                    v[1] = wv;
                    v[2] = u * dx;
                    v[3] = u * dy;
                    v[4] = wv * dy;
                    v[5] = t1;
                    v[6] = t1 * lg;
                    v[7] = g0 * wgt;
                    v[8] = g1 * wgt;
                    v[9] = g2 * wgt;
                    float tot = row_reduce10(v, lane);
                    // A row holds a splat at most once in its list: only rows taking the
                    // same splat in this step share a slot.  Merge theirs, lowest stores.
                    bool store = owner;
                    if (share) {
                        const float x1 = from_lane(tot, lane ^ 16), x2 = from_lane(tot, lane ^ 32);
                        const float x3 = from_lane(tot, lane ^ 48);
                        tot += (lane_in(kRowLanes.m[share & 15u]) ? x1 : 0.0f) +
                               (lane_in(kRowLanes.m[(share >> 4) & 15u]) ? x2 : 0.0f) +
                               (lane_in(kRowLanes.m[(share >> 8) & 15u]) ? x3 : 0.0f);
                        store = store && !lane_in(kRowLanes.m[share >> 12]);
                    }
                    if (store) *dst = prev + tot;
                }
                __syncthreads();
                // per (tile, splat): apply the per-splat factors.
                // With gr2 = dL/dr^2 = -o beta g', d = p - mu':
                //   dL/dmu' = -2 gr2 A d  = 2 o beta A (sum g' d)
                //   dL/dA   = gr2 d d^T  = -o beta sum g' d d^T
                //   dL/db   = o beta ln2 sum dLda B log2(1 - r^2)
                for (int k = tid; k < nb; k += NT) {
                    float *sg = s_g[0][k];
#pragma unroll
                    for (int wv = 1; wv < G::NW; ++wv)
#pragma unroll
                        for (int f = 0; f < NG; ++f) sg[f] += s_g[wv][k][f];
                    const float2 ob = unpack2(s_b[k].y);
                    const float obt = ob.x * ob.y;
                    const float a00 = (float)s_a[k].x, a01 = (float)(0.5 * s_a[k].y), a11 = (float)s_b[k].x;
                    const float su = sg[0], sw = sg[1];
                    sg[0] = 2.0f * obt * (a00 * su + a01 * sw);
                    sg[1] = 2.0f * obt * (a01 * su + a11 * sw);
                    sg[2] *= -obt;
                    sg[3] *= -obt;
                    sg[4] *= -obt;
                    sg[6] *= obt * kLn2;
                    bool any = false;
#pragma unroll
                    for (int f = 0; f < NG; ++f) any = any || sg[f] != 0.0f;
                    if (any) {
                        const int64_t i = (int64_t)s_rec[k] - (int64_t)it.v * a.n;
                        atomicOr((unsigned long long *)&a.gradmask[(int64_t)(it.v >> 6) * a.n + i],
                                 1ull << (it.v & 63));
                    }
                }
                __syncthreads();
                // consecutive lanes take consecutive values of a record: each wave-wide
                // atomic touches a few 64-byte lines
                for (int idx = tid; idx < nb * NG; idx += NT) {
                    const int k = idx / NG, f = idx - k * NG;
                    const float sg = s_g[0][k][f];
                    if (sg != 0.0f) unsafeAtomicAdd(&a.sgrad[(int64_t)s_rec[k] * 16 + f], sg);
                    if (COUNT) n_atomics += sg != 0.0f;
                }
                __syncthreads();
            }
        }
        __syncthreads();
    }
    if (COUNT) {
        const uint64_t tot = wave_sum_u32(n_atomics);
        if (lane == 0 && tot) atomicAdd(a.atomics, (unsigned long long)tot);
    }
    finish_persistent(a, &a.queue[2], &a.queue[3]);
}

// ---------------------------------------------------------------- work counts

// One thread per pixel of a tile (tiles of TW x TH), plain loop over its list:
// counts support tests and contributors with the same eval_r2 as above.
template <int TW, int TH>
__global__ __launch_bounds__(TW *TH) void raster_stats_kernel(RasterArgs a, int64_t *out)
{
    if (!buffers_match<TW, TH>(a)) return;
    const uint32_t g = blockIdx.x;
    const int v = find_view(a.views, a.n_views, g);
    const ViewDesc &V = a.views[v];
    const uint32_t lt = g - (uint32_t)V.tile_offset;
    const int ox = (int)(lt % (uint32_t)V.tiles_x) * TW, oy = (int)(lt / (uint32_t)V.tiles_x) * TH;
    const int px = ox + (int)threadIdx.x % TW, py = oy + (int)threadIdx.x / TW;
    const uint2 r = a.ranges[g];
    uint64_t ev = 0, contrib = 0, ev_fwd = 0;
    if (px < V.width && py < V.height) {
        const int64_t pix = V.pixel_offset + (int64_t)py * V.width + px;
        int32_t last = a.last_index[pix];
        if (last >= (int32_t)r.y) last = (int32_t)r.y - 1;
        const bool stopped = a.final_T[pix] < a.t_eps;
        const double fpx = (double)(px - ox) + 0.5, fpy = (double)(py - oy) + 0.5;
        for (int32_t j = (int32_t)r.x; j <= last; ++j) {
            const RasterRec rr = a.rec[a.pair_rec[j]];
            const double r2 = eval_r2(fpx - (rr.cx - (double)ox), fpy - (rr.cy - (double)oy), rr.a00, 2.0 * rr.a01,
                                      rr.a11);
            contrib += r2 < 1.0;
        }
        ev = last >= (int32_t)r.x ? (uint64_t)(last - (int32_t)r.x + 1) : 0;
        ev_fwd = stopped ? ev : (uint64_t)(r.y - r.x);
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        ev += __shfl_xor(ev, off, kWave);
        contrib += __shfl_xor(contrib, off, kWave);
        ev_fwd += __shfl_xor(ev_fwd, off, kWave);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicAdd((unsigned long long *)&out[0], (unsigned long long)ev);
        atomicAdd((unsigned long long *)&out[1], (unsigned long long)contrib);
        atomicAdd((unsigned long long *)&out[2], (unsigned long long)ev_fwd);
    }
}

// Wavefront-level work of the reverse pass, with its exact traversal (staging,
// block and quadrant lists): out[3] += wavefront steps (each step the four rows
// take one entry of their lists), out[4] += steps with at least one pixel with
// r^2 < 1.  One workgroup per tile.
template <int TW, int TH, int BATCH>
__global__ __launch_bounds__(TW *TH) void raster_wave_stats_kernel(RasterArgs a, int64_t *out)
{
    using G = Geo<TW, TH>;
    __shared__ double2 s_c[BATCH], s_a[BATCH], s_b[BATCH];
    __shared__ float4 s_col[BATCH];
    __shared__ uint8_t s_blist[G::NW][BATCH];
    __shared__ uint8_t s_rows[G::NW][4 * BATCH];
    __shared__ int32_t s_maxlast;
    const Staged S{s_c, s_a, s_b, s_col, nullptr};
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const LanePixel<TW, TH> P(w, lane);
    const double fpx = (double)P.lx + 0.5, fpy = (double)P.ly + 0.5;
    const uint8_t *my_row = &s_rows[w][P.row * BATCH];
    if (!buffers_match<TW, TH>(a)) return;  // uniform
    const uint32_t g = blockIdx.x;
    const int v = find_view(a.views, a.n_views, g);
    const ViewDesc &V = a.views[v];
    const uint32_t lt = g - (uint32_t)V.tile_offset;
    const int ox = (int)(lt % (uint32_t)V.tiles_x) * TW, oy = (int)(lt / (uint32_t)V.tiles_x) * TH;
    const uint2 rg = a.ranges[g];
    const int px = ox + P.lx, py = oy + P.ly;
    int32_t last = -1;
    if (px < V.width && py < V.height) last = a.last_index[V.pixel_offset + (int64_t)py * V.width + px];
    if (last >= (int32_t)rg.y) last = (int32_t)rg.y - 1;
    if (tid == 0) s_maxlast = -1;
    __syncthreads();
    const int32_t wave_last = wave_max_i32(last);
    int32_t row_last[4];
    row_max4_i32(last, row_last);
    if (lane == 0 && wave_last >= 0) atomicMax(&s_maxlast, wave_last);
    __syncthreads();
    const int64_t maxlast = s_maxlast;
    uint64_t steps_n = 0, active = 0;
    for (int64_t hi = maxlast + 1; hi > (int64_t)rg.x; hi -= BATCH) {
        const int64_t lo = hi - BATCH > (int64_t)rg.x ? hi - BATCH : (int64_t)rg.x;
        const int nb = (int)(hi - lo);
        stage<TW, TH, false>(a, (uint32_t)lo, nb, (double)ox, (double)oy, S, tid);
        __syncthreads();
        const int64_t kmax64 = (int64_t)wave_last - lo;
        const int nbw = kmax64 < (int64_t)(nb - 1) ? (int)kmax64 + 1 : nb;
        const int cnt_b = nbw > 0 ? build_list(s_col, nbw, w, s_blist[w], lane) : 0;
        int cnt[4];
        build_rows<BATCH, 0>(S, s_blist[w], cnt_b, P.bx, P.by, lo, row_last, s_rows[w], cnt, lane);
        const int my_cnt = pick4(cnt, P.row), steps = max4(cnt);
        for (int step = 0; step < steps; ++step) {
            const int t = my_cnt - 1 - step;
            const bool has = t >= 0;
            const int k = has ? my_row[t] : 0;
            const double2 c = s_c[k], aa = s_a[k], bb = s_b[k];
            const double r2 = eval_r2(fpx - c.x, fpy - c.y, aa.x, aa.y, bb.x);
            const bool contrib = has && (int32_t)(lo + k) <= last && r2 < 1.0;
            steps_n += 1;
            active += __ballot(contrib) != 0;
        }
        __syncthreads();
    }
    if (lane == 0) {
        atomicAdd((unsigned long long *)&out[3], (unsigned long long)steps_n);
        atomicAdd((unsigned long long *)&out[4], (unsigned long long)active);
    }
}

// ---------------------------------------------------------------- dispatch

// The reverse pass keeps per-wavefront sums for every staged splat in LDS, so
// it stages at most 128 splats at a time (256 would halve its occupancy).
template <int TW, int TH, int BATCH>
struct Kern {
    static constexpr int BWD_BATCH = BATCH < 128 ? BATCH : 128;
    static void *fwd() { return (void *)raster_fwd_kernel<TW, TH, BATCH>; }
    static void *fwd_gauss() { return (void *)raster_fwd_kernel<TW, TH, BATCH, true>; }
    static void *bwd() { return (void *)raster_bwd_kernel<TW, TH, BWD_BATCH>; }
    static void *bwd_count() { return (void *)raster_bwd_kernel<TW, TH, BWD_BATCH, true>; }
};

struct Entry {
    int tw, th, batch;
    void *fwd, *bwd, *bwd_count, *fwd_gauss;
};

#define DBS_ENTRY(TW, TH, B)                                                                             \
    {TW, TH, B, Kern<TW, TH, B>::fwd(), Kern<TW, TH, B>::bwd(), Kern<TW, TH, B>::bwd_count(),           \
     Kern<TW, TH, B>::fwd_gauss()}
const Entry kEntries[] = {
    DBS_ENTRY(16, 16, 64),  DBS_ENTRY(16, 16, 128), DBS_ENTRY(16, 16, 256),
    DBS_ENTRY(16, 8, 64),   DBS_ENTRY(16, 8, 128),  DBS_ENTRY(16, 8, 256),
    DBS_ENTRY(8, 8, 64),    DBS_ENTRY(8, 8, 128),   DBS_ENTRY(8, 8, 256),
    DBS_ENTRY(32, 8, 64),   DBS_ENTRY(32, 8, 128),  DBS_ENTRY(32, 8, 256),
    DBS_ENTRY(32, 16, 64),  DBS_ENTRY(32, 16, 128), DBS_ENTRY(32, 16, 256),
};
#undef DBS_ENTRY

const Entry *find_entry(int tw, int th, int batch)
{
    for (const Entry &e : kEntries)
        if (e.tw == tw && e.th == th && e.batch == batch) return &e;
    return nullptr;
}

// Persistent grid: resident workgroups per CU x CUs (cached per device and kernel).
int persistent_grid(void *kernel, int threads)
{
    static int cached_dev = -1, cu = 0;
    static void *cached_k[64];
    static int cached_g[64];
    static int n_cached = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev != cached_dev) {
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        cached_dev = dev;
        n_cached = 0;
    }
    for (int k = 0; k < n_cached; ++k)
        if (cached_k[k] == kernel) return cached_g[k];
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const int g = per_cu * cu;
    if (n_cached < 64) {
        cached_k[n_cached] = kernel;
        cached_g[n_cached] = g;
        ++n_cached;
    }
    return g;
}

RasterArgs make_args(ProjPtrs P, BinsPtrs B, int64_t n, int32_t n_views, int64_t n_tiles,
                     const dbs_raster_cfg &cfg)
{
    RasterArgs a{};
    a.ph = P.hdr;
    a.bh = B.hdr;
    a.n = n;
    a.views = P.views;
    a.n_views = n_views;
    a.n_tiles = (uint32_t)n_tiles;
    a.rec = P.rec;
    a.pair_rec = B.pair_rec;
    a.ranges = B.tile_range;
    a.order = B.tile_order;
    a.queue = B.hdr->queue;
    a.t_eps = cfg.t_eps;
    a.alpha_max = cfg.alpha_max;
    a.persistent = (cfg.flags & DBS_FLAG_PERSISTENT) ? 1 : 0;
    return a;
}

hipError_t launch(void *kernel, int threads, RasterArgs &a, int64_t n_tiles, hipStream_t s)
{
    if (n_tiles <= 0) return hipSuccess;
    unsigned grid = (unsigned)n_tiles;
    if (a.persistent) {
        int g = persistent_grid(kernel, threads);
        if (g <= 0) return hipErrorInvalidValue;
        if ((int64_t)g < n_tiles) grid = (unsigned)g;
    }
    void *args[] = {&a};
    return hipLaunchKernel(kernel, dim3(grid), dim3(threads), args, 0, s);
}

}  // namespace

hipError_t launch_raster_fwd(ProjPtrs P, BinsPtrs B, int64_t n, int32_t n_views, int64_t n_tiles,
                             const dbs_raster_cfg &cfg, float *image, float *final_T, int32_t *last_index,
                             hipStream_t s)
{
    const Entry *e = find_entry(cfg.tile_w, cfg.tile_h, cfg.batch);
    if (!e) return hipErrorInvalidValue;
    RasterArgs a = make_args(P, B, n, n_views, n_tiles, cfg);
    a.image = image;
    a.final_T = final_T;
    a.last_index = last_index;
    return launch((cfg.flags & DBS_FLAG_GAUSSIAN_SH) ? e->fwd_gauss : e->fwd, cfg.tile_w * cfg.tile_h, a, n_tiles,
                  s);
}

hipError_t launch_raster_bwd(ProjPtrs P, BinsPtrs B, int64_t n, int32_t n_views, int64_t n_tiles,
                             const dbs_raster_cfg &cfg, const float *final_T, const int32_t *last_index,
                             const float *dL_dimage, float *sgrad, int64_t *atomics, hipStream_t s)
{
    const Entry *e = find_entry(cfg.tile_w, cfg.tile_h, cfg.batch);
    if (!e) return hipErrorInvalidValue;
    RasterArgs a = make_args(P, B, n, n_views, n_tiles, cfg);
    a.final_T = (float *)final_T;
    a.last_index = (int32_t *)last_index;
    a.dL_dimage = dL_dimage;
    a.sgrad = sgrad;
    a.gradmask = P.gradmask;
    a.atomics = (unsigned long long *)atomics;
    return launch(atomics ? e->bwd_count : e->bwd, cfg.tile_w * cfg.tile_h, a, n_tiles, s);
}

bool raster_supported(int tw, int th, int batch) { return find_entry(tw, th, batch) != nullptr; }

hipError_t launch_raster_stats(ProjPtrs P, BinsPtrs B, int64_t n, int32_t n_views, int64_t n_tiles,
                               const dbs_raster_cfg &cfg, const float *final_T, const int32_t *last_index,
                               int64_t *out, hipStream_t s)
{
    if (n_tiles <= 0) return hipSuccess;
    RasterArgs a = make_args(P, B, n, n_views, n_tiles, cfg);
    a.final_T = (float *)final_T;
    a.last_index = (int32_t *)last_index;
    const int tw = cfg.tile_w, th = cfg.tile_h;
    const dim3 grid((unsigned)n_tiles), block((unsigned)(tw * th));
#define DBS_STATS(TW, TH)                                                                     \
    if (tw == TW && th == TH) {                                                               \
        raster_stats_kernel<TW, TH><<<grid, block, 0, s>>>(a, out);                          \
        if (cfg.batch == 64) raster_wave_stats_kernel<TW, TH, 64><<<grid, block, 0, s>>>(a, out);   \
        else raster_wave_stats_kernel<TW, TH, 128><<<grid, block, 0, s>>>(a, out);            \
        return hipGetLastError();                                                             \
    }
    DBS_STATS(16, 16) DBS_STATS(16, 8) DBS_STATS(8, 8) DBS_STATS(32, 8) DBS_STATS(32, 16)
#undef DBS_STATS
    return hipErrorInvalidValue;
}

}  // namespace dbs
