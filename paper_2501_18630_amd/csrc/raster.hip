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
// The ten per-(pixel, splat) values are summed over each wavefront, then over
// the workgroup in LDS, then added once per (tile, splat) to the per-record
// screen-space gradient with a global float atomic.
//
// Work items are (view, tile) pairs.  A persistent grid drains a device
// queue ordered heaviest tile first; the last workgroup to finish resets the
// queue so that the next launch (or graph replay) starts from zero.
#include "dbs_internal.h"

namespace dbs {

namespace {

struct RasterArgs {
    const ViewDesc *views;
    int32_t n_views;
    uint32_t n_tiles;
    const float4 *centre, *conic, *color;
    const uint32_t *pair_rec;
    const uint2 *ranges;
    const uint32_t *order;
    uint32_t *queue;  // [head, done]
    float *image;
    float *final_T;
    int32_t *last_index;
    const float *dL_dimage;
    float *sgrad;     // [R][12]
    float t_eps, alpha_max;
    int32_t persistent;
};

// r^2 = A00 dx^2 + 2 A01 dx dy + A11 dy^2 with a fixed rounding sequence, so
// that the forward and reverse kernels take identical support decisions.
__device__ __forceinline__ float eval_r2(float dx, float dy, float a00, float a01x2, float a11)
{
    const float t = __fmaf_rn(a01x2, dy, __fmul_rn(a00, dx));
    return __fmaf_rn(dx, t, __fmul_rn(__fmul_rn(a11, dy), dy));
}

// alpha before the clamp: o (1 - r^2)^beta via exp2(beta log2(1 - r^2)).
__device__ __forceinline__ float eval_kernel(float r2, float beta, float *lg)
{
    const float omr = __fsub_rn(1.0f, r2);
    *lg = __builtin_amdgcn_logf(omr);
    return __builtin_amdgcn_exp2f(__fmul_rn(beta, *lg));
}

__device__ __forceinline__ int find_view(const ViewDesc *views, int32_t n_views, uint32_t g)
{
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((uint32_t)views[mid].tile_offset <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
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
        if (a.persistent) k = atomicAdd(head, 1u);
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

// ---------------------------------------------------------------- forward

template <int TW, int TH, int BATCH>
__global__ __launch_bounds__(TW *TH) void raster_fwd_kernel(RasterArgs a)
{
    constexpr int NT = TW * TH;
    __shared__ float4 s_p[BATCH];  // local centre x, y, A00, 2 A01
    __shared__ float4 s_q[BATCH];  // A11, o, beta, r
    __shared__ float2 s_c[BATCH];  // g, b
    __shared__ Item s_item;
    const int tid = threadIdx.x;
    const int lx = tid % TW, ly = tid / TW;
    const float fpx = (float)lx + 0.5f, fpy = (float)ly + 0.5f;

    for (int iter = 0;; ++iter) {
        if (!fetch_item<TW, TH>(a, &a.queue[0], &s_item, iter)) break;
        const Item it = s_item;
        const ViewDesc &V = a.views[it.v];
        const int px = it.ox + lx, py = it.oy + ly;
        const bool inside = px < V.width && py < V.height;
        bool done = !inside;
        float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
        int32_t last = -1;
        const float fox = (float)it.ox, foy = (float)it.oy;

        for (uint32_t start = it.start; start < it.end; start += BATCH) {
            if (__syncthreads_count(!done) == 0) break;
            for (int k = tid; k < BATCH; k += NT) {
                const uint32_t j = start + (uint32_t)k;
                if (j < it.end) {
                    const uint32_t rec = a.pair_rec[j];
                    const float4 c = a.centre[rec], q = a.conic[rec], col = a.color[rec];
                    s_p[k] = make_float4(__fadd_rn(__fsub_rn(c.x, fox), c.z), __fadd_rn(__fsub_rn(c.y, foy), c.w),
                                         q.x, 2.0f * q.y);
                    s_q[k] = make_float4(q.z, q.w, col.w, col.x);
                    s_c[k] = make_float2(col.y, col.z);
                }
            }
            __syncthreads();
            const int nb = (int)min((uint32_t)BATCH, it.end - start);
            if (!done) {
                for (int k = 0; k < nb; ++k) {
                    const float4 p = s_p[k];
                    const float dx = __fsub_rn(fpx, p.x), dy = __fsub_rn(fpy, p.y);
                    const float4 q = s_q[k];
                    const float r2 = eval_r2(dx, dy, p.z, p.w, q.x);
                    if (r2 < 1.0f) {
                        float lg;
                        const float B = eval_kernel(r2, q.z, &lg);
                        const float alpha = fminf(a.alpha_max, __fmul_rn(q.y, B));
                        const float w = alpha * T;
                        const float2 cc = s_c[k];
                        C0 = __fmaf_rn(q.w, w, C0);
                        C1 = __fmaf_rn(cc.x, w, C1);
                        C2 = __fmaf_rn(cc.y, w, C2);
                        T = __fmul_rn(T, __fsub_rn(1.0f, alpha));
                        last = (int32_t)(start + (uint32_t)k);
                        if (T < a.t_eps) {
                            done = true;
                            break;
                        }
                    }
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

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

template <int TW, int TH, int BATCH>
__global__ __launch_bounds__(TW *TH) void raster_bwd_kernel(RasterArgs a)
{
    constexpr int NT = TW * TH;
    constexpr int NG = 10;
    __shared__ float4 s_p[BATCH];
    __shared__ float4 s_q[BATCH];
    __shared__ float2 s_c[BATCH];
    __shared__ uint32_t s_rec[BATCH];
    __shared__ float s_g[BATCH][NG];
    __shared__ Item s_item;
    __shared__ int32_t s_maxlast;
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int lx = tid % TW, ly = tid / TW;
    const float fpx = (float)lx + 0.5f, fpy = (float)ly + 0.5f;
    const float kLn2 = 0.69314718055994531f;

    for (int iter = 0;; ++iter) {
        if (!fetch_item<TW, TH>(a, &a.queue[2], &s_item, iter)) break;
        const Item it = s_item;
        const ViewDesc &V = a.views[it.v];
        const int px = it.ox + lx, py = it.oy + ly;
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
        float S0 = T * V.bg[0], S1 = T * V.bg[1], S2 = T * V.bg[2];
        if (tid == 0) s_maxlast = -1;
        __syncthreads();
        if (last >= 0) atomicMax(&s_maxlast, last);
        __syncthreads();
        // last positions come from the forward over the same lists; clamp them to
        // this tile's range so that no pair outside it is ever read
        const int64_t maxlast = s_maxlast < (int64_t)it.end ? (int64_t)s_maxlast : (int64_t)it.end - 1;
        const float fox = (float)it.ox, foy = (float)it.oy;

        if (maxlast >= (int64_t)it.start) {
            for (int64_t hi = maxlast + 1; hi > (int64_t)it.start; hi -= BATCH) {
                const int64_t lo = hi - BATCH > (int64_t)it.start ? hi - BATCH : (int64_t)it.start;
                const int nb = (int)(hi - lo);
                for (int k = tid; k < nb; k += NT) {
                    const uint32_t j = (uint32_t)(lo + k);
                    const uint32_t rec = a.pair_rec[j];
                    const float4 c = a.centre[rec], q = a.conic[rec], col = a.color[rec];
                    s_p[k] = make_float4(__fadd_rn(__fsub_rn(c.x, fox), c.z), __fadd_rn(__fsub_rn(c.y, foy), c.w),
                                         q.x, 2.0f * q.y);
                    s_q[k] = make_float4(q.z, q.w, col.w, col.x);
                    s_c[k] = make_float2(col.y, col.z);
                    s_rec[k] = rec;
#pragma unroll
                    for (int f = 0; f < NG; ++f) s_g[k][f] = 0.0f;
                }
                __syncthreads();
                for (int k = nb - 1; k >= 0; --k) {
                    const int32_t j = (int32_t)(lo + k);
                    float v[NG];
#pragma unroll
                    for (int f = 0; f < NG; ++f) v[f] = 0.0f;
                    bool contrib = false;
                    if (j <= last) {
                        const float4 p = s_p[k];
                        const float dx = __fsub_rn(fpx, p.x), dy = __fsub_rn(fpy, p.y);
                        const float4 q = s_q[k];
                        const float r2 = eval_r2(dx, dy, p.z, p.w, q.x);
                        if (r2 < 1.0f) {
                            contrib = true;
                            float lg;
                            const float B = eval_kernel(r2, q.z, &lg);
                            const float araw = __fmul_rn(q.y, B);
                            const bool clamped = araw > a.alpha_max;
                            const float alpha = clamped ? a.alpha_max : araw;
                            const float inv = 1.0f / (1.0f - alpha);
                            const float Ti = T * inv;
                            const float w = alpha * Ti;
                            const float2 cc = s_c[k];
                            v[7] = g0 * w;
                            v[8] = g1 * w;
                            v[9] = g2 * w;
                            const float gc = g0 * q.w + g1 * cc.x + g2 * cc.y;
                            const float gS = g0 * S0 + g1 * S1 + g2 * S2;
                            const float dLda = Ti * gc - inv * gS;
                            S0 = __fmaf_rn(q.w, w, S0);
                            S1 = __fmaf_rn(cc.x, w, S1);
                            S2 = __fmaf_rn(cc.y, w, S2);
                            T = Ti;
                            if (!clamped) {
                                v[5] = dLda * B;
                                v[6] = dLda * araw * (lg * kLn2) * q.z;
                                const float gr2 = -dLda * q.z * araw / (1.0f - r2);
                                // d = p - mu': dr2/dmu' = -2 A d
                                v[0] = -gr2 * (2.0f * p.z * dx + p.w * dy);
                                v[1] = -gr2 * (p.w * dx + 2.0f * q.x * dy);
                                v[2] = gr2 * dx * dx;
                                v[3] = gr2 * dx * dy;
                                v[4] = gr2 * dy * dy;
                            }
                        }
                    }
                    if (__ballot(contrib)) {
#pragma unroll
                        for (int f = 0; f < NG; ++f) {
                            const float s = wave_sum(v[f]);
                            if (lane == 0 && s != 0.0f) atomicAdd(&s_g[k][f], s);
                        }
                    }
                }
                __syncthreads();
                for (int idx = tid; idx < nb * NG; idx += NT) {
                    const int k = idx / NG, f = idx - k * NG;
                    const float s = s_g[k][f];
                    if (s != 0.0f) unsafeAtomicAdd(&a.sgrad[(int64_t)s_rec[k] * 12 + f], s);
                }
                __syncthreads();
            }
        }
        __syncthreads();
    }
    finish_persistent(a, &a.queue[2], &a.queue[3]);
}

// ---------------------------------------------------------------- dispatch

template <int TW, int TH, int BATCH>
struct Kern {
    static void *fwd() { return (void *)raster_fwd_kernel<TW, TH, BATCH>; }
    static void *bwd() { return (void *)raster_bwd_kernel<TW, TH, BATCH>; }
};

struct Entry {
    int tw, th, batch;
    void *fwd, *bwd;
};

#define DBS_ENTRY(TW, TH, B) {TW, TH, B, Kern<TW, TH, B>::fwd(), Kern<TW, TH, B>::bwd()}
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

RasterArgs make_args(ProjPtrs P, BinsPtrs B, int32_t n_views, int64_t n_tiles, const dbs_raster_cfg &cfg)
{
    RasterArgs a{};
    a.views = P.views;
    a.n_views = n_views;
    a.n_tiles = (uint32_t)n_tiles;
    a.centre = P.centre;
    a.conic = P.conic;
    a.color = P.color;
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
    (void)n;
    const Entry *e = find_entry(cfg.tile_w, cfg.tile_h, cfg.batch);
    if (!e) return hipErrorInvalidValue;
    RasterArgs a = make_args(P, B, n_views, n_tiles, cfg);
    a.image = image;
    a.final_T = final_T;
    a.last_index = last_index;
    return launch(e->fwd, cfg.tile_w * cfg.tile_h, a, n_tiles, s);
}

hipError_t launch_raster_bwd(ProjPtrs P, BinsPtrs B, int64_t n, int32_t n_views, int64_t n_tiles,
                             const dbs_raster_cfg &cfg, const float *final_T, const int32_t *last_index,
                             const float *dL_dimage, float *sgrad, hipStream_t s)
{
    (void)n;
    const Entry *e = find_entry(cfg.tile_w, cfg.tile_h, cfg.batch);
    if (!e) return hipErrorInvalidValue;
    RasterArgs a = make_args(P, B, n_views, n_tiles, cfg);
    a.final_T = (float *)final_T;
    a.last_index = (int32_t *)last_index;
    a.dL_dimage = dL_dimage;
    a.sgrad = sgrad;
    return launch(e->bwd, cfg.tile_w * cfg.tile_h, a, n_tiles, s);
}

bool raster_supported(int tw, int th, int batch) { return find_entry(tw, th, batch) != nullptr; }

}  // namespace dbs
