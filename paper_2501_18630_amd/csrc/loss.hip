// Training loss of Sec. 3.4 (Optimization): the photometric term
// (1 - lambda) L1 + lambda (1 - SSIM) of the composite loss and its two
// regularisers, with their gradients.
//
// SSIM per colour channel over an 11 x 11 Gaussian window (sigma 1.5) with
// zero padding, C1 = 0.01^2, C2 = 0.03^2; means over the 3 H W channel-pixels
// of a view; the views of a batch add their losses.  With the five window
// means m1 = <x>, m2 = <y>, e11 = <x^2>, e22 = <y^2>, e12 = <xy> of pixel p,
//   S = a1 a2 / (b1 b2),  a1 = 2 m1 m2 + C1,  a2 = 2 (e12 - m1 m2) + C2,
//                         b1 = m1^2 + m2^2 + C1, b2 = e11 - m1^2 + e22 - m2^2 + C2,
// and dS/dx(q) = sum_p w(p - q) [dS/dm1(p) + 2 x(q) dS/de11(p) + y(q) dS/de12(p)],
// i.e. three more window sums of the per-pixel partials.
//
// One workgroup per (view, channel, 32 x 16 output tile) does all of it in
// LDS: the 52 x 36 input region (a 10-pixel apron: 5 for the statistics of
// the 42 x 26 partials region, 5 more for their window sums), separable
// window passes (row then column, the 2D window being g(a) g(b)), the SSIM
// map and its partials, their window sums and the gradient, which is written
// once.  The partials reuse the input region's LDS (x and y of the output
// pixels are read again from memory, a cache hit), so three workgroups fit
// on a CU instead of two.  HBM traffic is 12 bytes per channel-pixel.
#include "dbs_internal.h"

namespace dbs {

namespace {

constexpr int kTX = 32, kTY = 16, kR = 5;                    // output tile, window radius
constexpr int kIX = kTX + 4 * kR, kIY = kTY + 4 * kR;        // 52 x 36 input region
constexpr int kMX = kTX + 2 * kR, kMY = kTY + 2 * kR;        // 42 x 26 partials region
constexpr int kMaxLossViews = 32;
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct LossView {
    int32_t w, h;
    int64_t pix;      // first flat pixel of the view
    int32_t tiles_x;  // output tiles per row
    int32_t item0;    // first work item of the view (3 channels x tiles)
};

struct LossViews {
    LossView v[kMaxLossViews];
    float g[2 * kR + 1];  // normalised 1D Gaussian weights
    int32_t count;
    int32_t items;
};

__global__ __launch_bounds__(256) void photometric_loss_kernel(LossViews lv, const float *__restrict__ image,
                                                               const float *__restrict__ target, float lam,
                                                               float *__restrict__ grad, float *loss)
{
    // the input region is only needed for the row sums: the partials reuse its space
    constexpr int kXYD = 2 * kIY * kIX > 3 * kMY * kMX ? 2 * kIY * kIX : 3 * kMY * kMX;
    __shared__ float s_xyd[kXYD];
    __shared__ float s_h[5][kIY][kMX];   // row sums of x, y, xx, yy, xy; later the row sums of the partials
    float(*s_x)[kIX] = reinterpret_cast<float(*)[kIX]>(s_xyd);
    float(*s_y)[kIX] = reinterpret_cast<float(*)[kIX]>(s_xyd + kIY * kIX);
    float(*s_d)[kMY][kMX] = reinterpret_cast<float(*)[kMY][kMX]>(s_xyd);  // dS/dm1, dS/de11, dS/de12
    __shared__ float s_red[2][256 / kWave];
    const int tid = threadIdx.x;
    const int item = blockIdx.x;
    int v = 0;
    while (v + 1 < lv.count && lv.v[v + 1].item0 <= item) ++v;
    const LossView V = lv.v[v];
    const int local = item - V.item0;
    const int ntile = ((V.w + kTX - 1) / kTX) * ((V.h + kTY - 1) / kTY);
    const int c = local / ntile, t = local - c * ntile;
    const int ox = (t % V.tiles_x) * kTX, oy = (t / V.tiles_x) * kTY;
    const int64_t plane = (int64_t)V.w * V.h;
    const float *xs = image + 3 * V.pix + c * plane;
    const float *ys = target + 3 * V.pix + c * plane;
    float *gs = grad + 3 * V.pix + c * plane;
    float g[2 * kR + 1];
#pragma unroll
    for (int k = 0; k <= 2 * kR; ++k) g[k] = lv.g[k];

    // 1. input region, zero outside the image
    for (int i = tid; i < kIY * kIX; i += 256) {
        const int r = i / kIX, q = i - r * kIX;
        const int gy = oy - 2 * kR + r, gx = ox - 2 * kR + q;
        const bool in = gy >= 0 && gy < V.h && gx >= 0 && gx < V.w;
        const int64_t o = (int64_t)gy * V.w + gx;
        s_x[r][q] = in ? xs[o] : 0.0f;
        s_y[r][q] = in ? ys[o] : 0.0f;
    }
    __syncthreads();
    // Every window pass below gives each thread a short strip of outputs and
    // slides the 11 taps over registers, so each LDS value is read once per
    // strip instead of once per tap.
    // 2. row sums of the five moments: 36 rows x 7 strips of 6 of the 42 columns
    if (tid < kIY * 7) {
        const int r = tid / 7, q0 = (tid - r * 7) * 6;
        float x[16], y[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            x[k] = s_x[r][q0 + k];
            y[k] = s_y[r][q0 + k];
        }
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
#pragma unroll
            for (int k = 0; k <= 2 * kR; ++k) {
                const float xv = x[j + k], yv = y[j + k];
                a = fmaf(g[k], xv, a);
                b = fmaf(g[k], yv, b);
                aa = fmaf(g[k], xv * xv, aa);
                bb = fmaf(g[k], yv * yv, bb);
                ab = fmaf(g[k], xv * yv, ab);
            }
            s_h[0][r][q0 + j] = a;
            s_h[1][r][q0 + j] = b;
            s_h[2][r][q0 + j] = aa;
            s_h[3][r][q0 + j] = bb;
            s_h[4][r][q0 + j] = ab;
        }
    }
    __syncthreads();
    // 3. column sums -> window means, SSIM and its partials (zero outside the
    //    image): 42 columns x 6 strips of (up to) 5 of the 26 rows
    float ssim_sum = 0.f, l1_sum = 0.f;
    if (tid < kMX * 6) {
        const int q = tid % kMX, r0 = (tid / kMX) * 5;
        const int nr = kMY - r0 < 5 ? kMY - r0 : 5;
        float col[5][15];
#pragma unroll
        for (int m = 0; m < 5; ++m)
#pragma unroll
            for (int k = 0; k < 15; ++k) col[m][k] = r0 + k < kIY ? s_h[m][r0 + k][q] : 0.f;
        const int gx = ox - kR + q;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            if (j >= nr) break;
            const int r = r0 + j, gy = oy - kR + r;
            float d1 = 0.f, d2 = 0.f, d3 = 0.f;
            if (gy >= 0 && gy < V.h && gx >= 0 && gx < V.w) {
                float mo[5];
#pragma unroll
                for (int m = 0; m < 5; ++m) {
                    float acc = 0.f;
#pragma unroll
                    for (int k = 0; k <= 2 * kR; ++k) acc = fmaf(g[k], col[m][j + k], acc);
                    mo[m] = acc;
                }
                const float m1 = mo[0], m2 = mo[1], e11 = mo[2], e22 = mo[3], e12 = mo[4];
                const float a1 = 2.f * m1 * m2 + kC1, a2 = 2.f * (e12 - m1 * m2) + kC2;
                const float b1 = m1 * m1 + m2 * m2 + kC1, b2 = (e11 - m1 * m1) + (e22 - m2 * m2) + kC2;
                const float ib1 = 1.f / b1, ib2 = 1.f / b2, inv = ib1 * ib2;
                const float sv = a1 * a2 * inv;
                d1 = 2.f * m2 * (a2 - a1) * inv - 2.f * m1 * sv * (ib1 - ib2);
                d2 = -sv * ib2;
                d3 = 2.f * a1 * inv;
                if (r >= kR && r < kR + kTY && q >= kR && q < kR + kTX) ssim_sum += sv;
            }
            s_d[0][r][q] = d1;
            s_d[1][r][q] = d2;
            s_d[2][r][q] = d3;
        }
    }
    __syncthreads();
    // 4. row sums of the partials over the 32 output columns (into s_h):
    //    26 rows x 8 strips of 4
    float(*s_b)[kMY][kTX] = reinterpret_cast<float(*)[kMY][kTX]>(&s_h[0][0][0]);
    if (tid < kMY * 8) {
        const int r = tid / 8, q0 = (tid - r * 8) * 4;
        float dv[3][14];
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int k = 0; k < 14; ++k) dv[m][k] = s_d[m][r][q0 + k];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                float acc = 0.f;
#pragma unroll
                for (int k = 0; k <= 2 * kR; ++k) acc = fmaf(g[k], dv[m][j + k], acc);
                s_b[m][r][q0 + j] = acc;
            }
    }
    __syncthreads();
    // 5. column sums and the gradient of the output tile: 32 columns x 8 strips of 2 rows
    const float inv_n = 1.0f / (3.0f * (float)plane);
    {
        const int q = tid % kTX, r0 = (tid / kTX) * 2;
        float bv[3][12];
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int k = 0; k < 12; ++k) bv[m][k] = s_b[m][r0 + k][q];
        const int gx = ox + q;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int r = r0 + j, gy = oy + r;
            if (gy < V.h && gx < V.w) {
                float w1 = 0.f, w2 = 0.f, w3 = 0.f;
#pragma unroll
                for (int k = 0; k <= 2 * kR; ++k) {
                    w1 = fmaf(g[k], bv[0][j + k], w1);
                    w2 = fmaf(g[k], bv[1][j + k], w2);
                    w3 = fmaf(g[k], bv[2][j + k], w3);
                }
                const int64_t o = (int64_t)gy * V.w + gx;
                const float x = xs[o], y = ys[o];
                const float d = x - y;
                const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
                l1_sum += fabsf(d);
                gs[(int64_t)gy * V.w + gx] = ((1.f - lam) * sg - lam * (w1 + 2.f * x * w2 + y * w3)) * inv_n;
            }
        }
    }
    if (loss) {
        for (int off = kWave / 2; off > 0; off >>= 1) {
            ssim_sum += __shfl_xor(ssim_sum, off, kWave);
            l1_sum += __shfl_xor(l1_sum, off, kWave);
        }
        if ((tid & (kWave - 1)) == 0) {
            s_red[0][tid / kWave] = ssim_sum;
            s_red[1][tid / kWave] = l1_sum;
        }
        __syncthreads();
        if (tid == 0) {
            float ss = 0.f, ll = 0.f;
            for (int w = 0; w < 256 / kWave; ++w) {
                ss += s_red[0][w];
                ll += s_red[1][w];
            }
            float part = ((1.f - lam) * ll - lam * ss) * inv_n;
            if (local == 0) part += lam;  // the "1 -" of (1 - mean SSIM), once per view
            atomicAdd(loss, part);
        }
    }
}

__global__ void zero_loss_kernel(float *p) { *p = 0.0f; }

// lambda_o sum |o| + lambda_s sum |s|: gradients added, value accumulated.
__global__ __launch_bounds__(256) void regularizer_kernel(SplatPtrs sp, float lam_o, float lam_s, GradPtrs g,
                                                          float *loss)
{
    __shared__ float s_red[256 / kWave];
    float acc = 0.f;
    // grid-stride: one loss atomic per workgroup of at most 2048 (atomics on one
    // address serialise at its L2 line: 0.16 -> 0.06 ms for 3 M splats)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < sp.n; i += (int64_t)gridDim.x * blockDim.x) {
        const float o = sp.opacities[i];
        g.opacities[i] += lam_o * (o > 0.f ? 1.f : (o < 0.f ? -1.f : 0.f));
        acc += lam_o * fabsf(o);
        for (int k = 0; k < 3; ++k) {
            const float s = sp.scales[3 * i + k];
            g.scales[3 * i + k] += lam_s * (s > 0.f ? 1.f : (s < 0.f ? -1.f : 0.f));
            acc += lam_s * fabsf(s);
        }
    }
    if (loss) {
        for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0) s_red[threadIdx.x / kWave] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            float t = 0.f;
            for (int w = 0; w < 256 / kWave; ++w) t += s_red[w];
            atomicAdd(loss, t);
        }
    }
}

}  // namespace

hipError_t launch_photometric_loss(const float *image, const float *target, const dbs_camera *cams,
                                   int32_t n_views, float lam, float *grad, float *loss, hipStream_t s)
{
    double gw[2 * kR + 1], sum = 0.0;
    for (int k = 0; k <= 2 * kR; ++k) {
        const double d = (double)(k - kR);
        gw[k] = exp(-d * d / (2.0 * 1.5 * 1.5));
        sum += gw[k];
    }
    if (loss) zero_loss_kernel<<<1, 1, 0, s>>>(loss);
    int64_t pix = 0;
    for (int32_t first = 0; first < n_views; first += kMaxLossViews) {
        LossViews lv{};
        for (int k = 0; k <= 2 * kR; ++k) lv.g[k] = (float)(gw[k] / sum);
        lv.count = n_views - first < kMaxLossViews ? n_views - first : kMaxLossViews;
        int32_t items = 0;
        for (int k = 0; k < lv.count; ++k) {
            const dbs_camera &c = cams[first + k];
            LossView &V = lv.v[k];
            V.w = c.width;
            V.h = c.height;
            V.pix = pix;
            V.tiles_x = (c.width + kTX - 1) / kTX;
            V.item0 = items;
            items += 3 * V.tiles_x * ((c.height + kTY - 1) / kTY);
            pix += (int64_t)c.width * c.height;
        }
        lv.items = items;
        photometric_loss_kernel<<<(unsigned)items, 256, 0, s>>>(lv, image, target, lam, grad, loss);
    }
    return hipGetLastError();
}

hipError_t launch_regularizer(const SplatPtrs &sp, float lam_o, float lam_s, const GradPtrs &g, float *loss,
                              hipStream_t s)
{
    if (sp.n <= 0) return hipSuccess;
    const int64_t nb = ceil_div(sp.n, 256);
    regularizer_kernel<<<(unsigned)(nb < 2048 ? nb : 2048), 256, 0, s>>>(sp, lam_o, lam_s, g, loss);
    return hipGetLastError();
}

}  // namespace dbs
