// Per-(view, splat) projection and Spherical Beta colour.
//
// Sec. 3.2: Sigma = R S S^T R^T from the quaternion and scale, projected
// covariance Sigma' = J W Sigma W^T J^T (J the Jacobian of the pinhole map at
// the splat centre), centre mu', and the conic Sigma'^{-1} that Eq. (5)
// evaluates.  The Beta kernel is exactly zero outside r^2 < 1 (Sec. 3.1,
// Eq. 2), so the support's bounding box is mu' +- (sqrt(Sigma'_00),
// sqrt(Sigma'_11)); the record lists the pixel centres inside it and the
// number of tiles it overlaps.  Sec. 3.3, Eq. (8): colour = c0 + sum_m
// B(1 - R_m . V; b_m) c_m with B(x; b) = (1 - x)^(4 e^b).
//
// One thread per splat loops over the views, so every parameter is read from
// HBM once per call however many views are rendered.  Geometry is computed in
// FP64 (exact products of the FP32 inputs, then rounded once): the pixel box
// and the depth key are integer decisions that must not depend on FP32
// rounding.  The record keeps the centre and the conic in FP64: the raster
// passes evaluate r^2 in FP64, because the Beta kernel's slope at the
// support edge, beta (1 - r^2)^(beta - 1), is unbounded for beta < 1 and an
// FP32 r^2 would carry a large relative error in 1 - r^2 there.
#include "dbs_internal.h"

namespace dbs {

namespace {

constexpr int kUploadViews = 8;
struct ViewUpload {
    ViewDesc v[kUploadViews];
    int32_t first, count;
};

__global__ void upload_views_kernel(ViewUpload up, ViewDesc *views, ProjHeader *hdr, int64_t n,
                                    int32_t n_views, int32_t m, int32_t tw, int32_t th, int32_t reset)
{
    int t = threadIdx.x;
    if (t < up.count) views[up.first + t] = up.v[t];
    if (reset && t == 0) {
        hdr->counts[0] = 0;
        hdr->counts[1] = 0;
        hdr->n = n;
        hdr->n_views = n_views;
        hdr->m = m;
        hdr->tile_w = tw;
        hdr->tile_h = th;
    }
}

__device__ __forceinline__ bool finite3(float a, float b, float c)
{
    return isfinite(a) && isfinite(b) && isfinite(c);
}

__device__ inline uint64_t wave_sum_u64(uint64_t v)
{
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Real spherical harmonics of degree <= 3 at the unit direction (x, y, z), in
// the order l = 0..3, m = -l..l, with the Condon-Shortley phase: each constant
// is the normalisation sqrt((2l + 1) / (4 pi) (l - |m|)! / (l + |m|)!) (times
// sqrt 2 for m != 0) with the associated Legendre polynomial's own factor
// folded in, and the polynomials in x, y, z are the Cartesian forms of
// r^l P_l^|m|(cos theta) cos(m phi) (m > 0) or sin(|m| phi) (m < 0).
__device__ __forceinline__ void sh_basis3(float x, float y, float z, float Y[16])
{
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[0] = 0.28209479177387814f;
    Y[1] = -0.48860251190291992f * y;
    Y[2] = 0.48860251190291992f * z;
    Y[3] = -0.48860251190291992f * x;
    Y[4] = 1.0925484305920792f * x * y;
    Y[5] = -1.0925484305920792f * y * z;
    Y[6] = 0.31539156525252005f * (2.0f * zz - xx - yy);
    Y[7] = -1.0925484305920792f * x * z;
    Y[8] = 0.54627421529603959f * (xx - yy);
    Y[9] = -0.59004358992664352f * y * (3.0f * xx - yy);
    Y[10] = 2.8906114426405538f * x * y * z;
    Y[11] = -0.45704579946446572f * y * (4.0f * zz - xx - yy);
    Y[12] = 0.37317633259011540f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -0.45704579946446572f * x * (4.0f * zz - xx - yy);
    Y[14] = 1.4453057213202769f * z * (xx - yy);
    Y[15] = -0.59004358992664352f * x * (xx - 3.0f * yy);
}

// GSH: the Gaussian-kernel + SH comparison mode.  The support is the 3-sigma
// ellipse, so the stored conic is Sigma'^{-1} / 9 (r^2 < 1 there, and the
// raster takes exp(-4.5 r^2)) and the pixel box is 3 times as wide; the colour
// is max(0, sum_k sh_k Y_k(V) + 1/2).
template <int M, bool GSH>
__global__ __launch_bounds__(256) void preprocess_kernel(SplatPtrs sp, const float *sh, ProjPtrs P, int32_t n_views,
                                                         int32_t lw, int32_t lh, uint32_t flags, float b_split)
{
    __shared__ RasterRec s_stage[256 / kWave][kWave];  // one view's records of each wavefront
    constexpr bool LOBES_IN_LDS = M > 0 && M <= 4;
    constexpr int LOBE_REGS = (M > 0 && !LOBES_IN_LDS) ? M : 1;
    __shared__ float s_lobe[LOBES_IN_LDS ? M : 1][7][256];  // per lobe: direction (3), colour (3), exponent
    (void)s_lobe;
    const int64_t n = sp.n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int64_t i0 = i - lane;                      // the wavefront's first splat
    const bool full_wave = i0 + kWave <= n;           // every lane holds a splat (uniform)
    uint64_t vis = 0, pairs = 0;
    if (i < n) {
        const double mu[3] = {sp.means[3 * i], sp.means[3 * i + 1], sp.means[3 * i + 2]};
        // rotation of the normalised quaternion (w, x, y, z)
        double q0 = sp.quats[4 * i], q1 = sp.quats[4 * i + 1], q2 = sp.quats[4 * i + 2],
               q3 = sp.quats[4 * i + 3];
        double qn = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
        // The primitive is defined for real-valued parameters: a splat with a
        // NaN or infinite parameter is absent from every view (culled here, so
        // it neither reaches the image nor receives a gradient).  The centre's
        // coordinates are tested through their FP64 sum, which no finite FP32
        // values can overflow.
        bool fin = isfinite(qn) && isfinite(mu[0] + mu[1] + mu[2]) &&
                   finite3(sp.scales[3 * i], sp.scales[3 * i + 1], sp.scales[3 * i + 2]) &&
                   isfinite(sp.opacities[i]);
        bool ok = qn > 0.0;
        // geometry decomposition: primitives outside the b range are culled in every view
        if (flags & DBS_FLAG_B_BELOW) ok = ok && sp.betas[i] < b_split;
        if (flags & DBS_FLAG_B_ABOVE) ok = ok && sp.betas[i] >= b_split;
        const bool diffuse_on = !(flags & DBS_FLAG_SPECULAR_ONLY), specular_on = !(flags & DBS_FLAG_DIFFUSE_ONLY);
        double w = q0 / qn, x = q1 / qn, y = q2 / qn, z = q3 / qn;
        double Rq[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
                        2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
                        2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)};
        double s2[3];
        for (int k = 0; k < 3; ++k) {
            double s = sp.scales[3 * i + k];
            s2[k] = s * s;
        }
        // Sigma = R diag(s^2) R^T (symmetric, 6 entries)
        double Sig[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b) {
                double acc = Rq[3 * a] * s2[0] * Rq[3 * b] + Rq[3 * a + 1] * s2[1] * Rq[3 * b + 1] +
                             Rq[3 * a + 2] * s2[2] * Rq[3 * b + 2];
                Sig[a][b] = acc;
                Sig[b][a] = acc;
            }
        const float opac = sp.opacities[i];
        // beta = 4 e^b, held below FP32 overflow so that (1 - r^2)^beta stays
        // defined (1 at r^2 = 0, 0 elsewhere) for very large b
        const float beta = GSH ? 0.0f : fminf(4.0f * expf(sp.betas[i]), 3.4028235e38f);
        const bool c0_on = diffuse_on && !GSH;
        float c0r = 0.0f, c0g = 0.0f, c0b = 0.0f;
        if (!GSH) {
            const float d0 = sp.diffuse[3 * i], d1 = sp.diffuse[3 * i + 1], d2 = sp.diffuse[3 * i + 2];
            fin = fin && isfinite(sp.betas[i]) && finite3(d0, d1, d2);
            if (c0_on) {
                c0r = d0;
                c0g = d1;
                c0b = d2;
            }
        }
        // Up to four lobes (direction, colour, exponent) are held in LDS across
        // the views rather than in registers: 28 fewer VGPRs, one more wave per SIMD.
        float lr_r[LOBE_REGS][3], lc_r[LOBE_REGS][3], lbeta_r[LOBE_REGS];
#pragma unroll
        for (int mm = 0; mm < M; ++mm) {
            const int64_t l = i * M + mm;
            float st, ct, sph, cph;
            sincosf(sp.lobe_angles[2 * l], &st, &ct);
            sincosf(sp.lobe_angles[2 * l + 1], &sph, &cph);
            const float r3[3] = {st * cph, st * sph, ct};
            float c3[3];
            for (int c = 0; c < 3; ++c) c3[c] = sp.lobe_colors[3 * l + c];
            const float bm = fminf(4.0f * expf(sp.lobe_betas[l]), 3.4028235e38f);
            fin = fin && finite3(sp.lobe_angles[2 * l], sp.lobe_angles[2 * l + 1], sp.lobe_betas[l]) &&
                  finite3(c3[0], c3[1], c3[2]);
            if (LOBES_IN_LDS) {
                for (int c = 0; c < 3; ++c) {
                    s_lobe[mm][c][threadIdx.x] = r3[c];
                    s_lobe[mm][3 + c][threadIdx.x] = c3[c];
                }
                s_lobe[mm][6][threadIdx.x] = bm;
            } else {
                for (int c = 0; c < 3; ++c) {
                    lr_r[mm][c] = r3[c];
                    lc_r[mm][c] = c3[c];
                }
                lbeta_r[mm] = bm;
            }
        }

        // SH coefficients held in registers across the views (read once per splat)
        float shc[GSH ? 48 : 1];
        if (GSH) {
#pragma unroll
            for (int k = 0; k < 48; ++k) shc[k] = sh[i * 48 + k];
            float acc = 0.0f;
#pragma unroll
            for (int k = 0; k < 48; ++k) acc += 0.0f * shc[k];  // NaN iff some coefficient is NaN or infinite
            fin = fin && acc == 0.0f;
        }
        ok = ok && fin;

        for (int32_t v = 0; v < n_views; ++v) {
            const ViewDesc &V = P.views[v];
            const int64_t rec = (int64_t)v * n + i;
            const double W[9] = {V.R[0], V.R[1], V.R[2], V.R[3], V.R[4], V.R[5], V.R[6], V.R[7], V.R[8]};
            double tc[3];
            for (int r = 0; r < 3; ++r)
                tc[r] = W[3 * r] * mu[0] + W[3 * r + 1] * mu[1] + W[3 * r + 2] * mu[2] + (double)V.t[r];
            const float depth_f = (float)tc[2];
            P.depth[rec] = __float_as_uint(depth_f);
            uint32_t ntiles = 0, rect = kRectEscape;
            short4 bb = make_short4(0, -1, 0, -1);
            if (ok && tc[2] > (double)V.near_plane) {
                const double tx = tc[0], ty = tc[1], tz = tc[2];
                const double fx = V.fx, fy = V.fy;
                const double iz = 1.0 / tz, iz2 = iz * iz;
                const double J00 = fx * iz, J02 = -fx * tx * iz2;
                const double J11 = fy * iz, J12 = -fy * ty * iz2;
                // M = J W (2x3)
                double Mm[2][3];
                for (int b = 0; b < 3; ++b) {
                    Mm[0][b] = J00 * W[b] + J02 * W[6 + b];
                    Mm[1][b] = J11 * W[3 + b] + J12 * W[6 + b];
                }
                // T = M Sigma (2x3), Sigma' = T M^T
                double Tm[2][3];
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 3; ++b)
                        Tm[a][b] = Mm[a][0] * Sig[0][b] + Mm[a][1] * Sig[1][b] + Mm[a][2] * Sig[2][b];
                const double c00 = Tm[0][0] * Mm[0][0] + Tm[0][1] * Mm[0][1] + Tm[0][2] * Mm[0][2];
                const double c01 = Tm[0][0] * Mm[1][0] + Tm[0][1] * Mm[1][1] + Tm[0][2] * Mm[1][2];
                const double c11 = Tm[1][0] * Mm[1][0] + Tm[1][1] * Mm[1][1] + Tm[1][2] * Mm[1][2];
                const double det = c00 * c11 - c01 * c01;
                if (det > 0.0) {
                    const double mx = fx * tx * iz + (double)V.cx;
                    const double my = fy * ty * iz + (double)V.cy;
                    const double ext = GSH ? 3.0 : 1.0;
                    const double ex = ext * sqrt(c00), ey = ext * sqrt(c11);
                    double xl = ceil(mx - ex - 0.5), xh = floor(mx + ex - 0.5);
                    double yl = ceil(my - ey - 0.5), yh = floor(my + ey - 0.5);
                    xl = fmax(xl, 0.0);
                    yl = fmax(yl, 0.0);
                    xh = fmin(xh, (double)(V.width - 1));
                    yh = fmin(yh, (double)(V.height - 1));
                    if (xl <= xh && yl <= yh) {
                        const int ixl = (int)xl, ixh = (int)xh, iyl = (int)yl, iyh = (int)yh;
                        bb = make_short4((short)ixl, (short)ixh, (short)iyl, (short)iyh);
                        const int tw_ = (ixh >> lw) - (ixl >> lw) + 1, th_ = (iyh >> lh) - (iyl >> lh) + 1;
                        ntiles = (uint32_t)(tw_ * th_);
                        rect = pack_tile_rect(ixl >> lw, iyl >> lh, tw_, th_);
                        const double idet = 1.0 / (GSH ? 9.0 * det : det);
                        RasterRec rr;
                        rr.cx = mx;
                        rr.cy = my;
                        rr.a00 = c11 * idet;
                        rr.a01 = -c01 * idet;
                        rr.a11 = c00 * idet;
                        rr.opacity = opac;
                        rr.beta = beta;
                        // Spherical Beta colour; V = (mu - camera centre) / |.|
                        double cp[3];
                        for (int k = 0; k < 3; ++k)
                            cp[k] = -(W[k] * (double)V.t[0] + W[3 + k] * (double)V.t[1] + W[6 + k] * (double)V.t[2]);
                        const double vx = mu[0] - cp[0], vy = mu[1] - cp[1], vz = mu[2] - cp[2];
                        const double ivl = 1.0 / sqrt(vx * vx + vy * vy + vz * vz);
                        const float dx = (float)(vx * ivl), dy = (float)(vy * ivl), dz = (float)(vz * ivl);
                        float cr = c0r, cg = c0g, cb = c0b;
                        if (GSH) {
                            float Y[16];
                            sh_basis3(dx, dy, dz, Y);
                            cr = cg = cb = 0.5f;
#pragma unroll
                            for (int k = 0; k < 16; ++k) {
                                cr = __fmaf_rn(Y[k], shc[3 * k], cr);
                                cg = __fmaf_rn(Y[k], shc[3 * k + 1], cg);
                                cb = __fmaf_rn(Y[k], shc[3 * k + 2], cb);
                            }
                            cr = fmaxf(cr, 0.0f);
                            cg = fmaxf(cg, 0.0f);
                            cb = fmaxf(cb, 0.0f);
                        }
#pragma unroll
                        for (int mm = 0; mm < M; ++mm) {
                            const int tl = threadIdx.x;
                            const float r0 = LOBES_IN_LDS ? s_lobe[mm][0][tl] : lr_r[mm][0];
                            const float r1 = LOBES_IN_LDS ? s_lobe[mm][1][tl] : lr_r[mm][1];
                            const float r2 = LOBES_IN_LDS ? s_lobe[mm][2][tl] : lr_r[mm][2];
                            const float d = r0 * dx + r1 * dy + r2 * dz;
                            if (specular_on && d > 0.0f) {
                                const float bm = LOBES_IN_LDS ? s_lobe[mm][6][tl] : lbeta_r[mm];
                                const float wgt = exp2f(bm * log2f(d));
                                cr += wgt * (LOBES_IN_LDS ? s_lobe[mm][3][tl] : lc_r[mm][0]);
                                cg += wgt * (LOBES_IN_LDS ? s_lobe[mm][4][tl] : lc_r[mm][1]);
                                cb += wgt * (LOBES_IN_LDS ? s_lobe[mm][5][tl] : lc_r[mm][2]);
                            }
                        }
                        rr.r = cr;
                        rr.g = cg;
                        rr.b = cb;
                        rr.pad = 0.0f;
                        if (full_wave) s_stage[wv][lane] = rr;
                        else P.rec[rec] = rr;
                        vis += 1;
                        pairs += ntiles;
                    }
                }
            }
            if (full_wave) {
                // the wavefront's records of this view are 64 consecutive 64-byte
                // slots: written from LDS as contiguous 1 KB stores (16 B per lane),
                // the visible ones only
                const uint64_t vb = __ballot(ntiles > 0);
                __builtin_amdgcn_wave_barrier();
                float4 *dst = reinterpret_cast<float4 *>(P.rec + ((int64_t)v * n + i0));
                const float4 *src = reinterpret_cast<const float4 *>(&s_stage[wv][0]);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int c = k * kWave + lane;
                    if ((vb >> (c >> 2)) & 1ull) dst[c] = src[c];
                }
                __builtin_amdgcn_wave_barrier();
            }
            P.bbox[rec] = bb;
            P.ntiles[rec] = ntiles;
            P.rect[rec] = rect;
            {   // the wavefront's 64 visibility bits of this view (i0 is a multiple of 64)
                const uint64_t vbits = __ballot(ntiles > 0);
                if (lane == 0)
                    *reinterpret_cast<uint2 *>(P.visbits + (int64_t)v * visbits_stride(n) + (i0 >> 5)) =
                        make_uint2((uint32_t)vbits, (uint32_t)(vbits >> 32));
            }
        }
    }
    // Per-workgroup totals, stored (not added): atomics from every wavefront
    // into the two counters serialise at their L2 line (47 k per counter on
    // config 3, ~0.17 ms of the kernel); sum_counts_kernel adds the totals.
    vis = wave_sum_u64(vis);
    pairs = wave_sum_u64(pairs);
    __shared__ uint64_t s_cnt[2][256 / kWave];
    if ((threadIdx.x & (kWave - 1)) == 0) {
        s_cnt[0][threadIdx.x / kWave] = vis;
        s_cnt[1][threadIdx.x / kWave] = pairs;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        uint64_t t = 0;
#pragma unroll
        for (int k = 0; k < 256 / kWave; ++k) t += s_cnt[threadIdx.x][k];
        P.blockcnt[2 * (int64_t)blockIdx.x + threadIdx.x] = t;
    }
}

// hdr->counts = the sums of the preprocess workgroups' totals (one workgroup
// of 1024 threads); also copied to out when given.
__global__ __launch_bounds__(1024) void sum_counts_kernel(const uint64_t *blockcnt, int64_t nblk, ProjHeader *hdr,
                                                          int64_t *out)
{
    __shared__ uint64_t s_red[2][1024 / kWave];
    uint64_t v = 0, p = 0;
    for (int64_t b = threadIdx.x; b < nblk; b += 1024) {
        v += blockcnt[2 * b];
        p += blockcnt[2 * b + 1];
    }
    v = wave_sum_u64(v);
    p = wave_sum_u64(p);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        s_red[0][threadIdx.x / kWave] = v;
        s_red[1][threadIdx.x / kWave] = p;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        uint64_t t = 0;
        for (int k = 0; k < 1024 / kWave; ++k) t += s_red[threadIdx.x][k];
        hdr->counts[threadIdx.x] = (int64_t)t;
        if (out) out[threadIdx.x] = (int64_t)t;
    }
}

}  // namespace

hipError_t launch_upload_views(const dbs_camera *cams, int32_t n_views, int tile_w, int tile_h,
                               ProjPtrs P, int64_t n, int32_t m, hipStream_t s)
{
    int32_t tile_off = 0;
    int64_t pix_off = 0;
    for (int32_t first = 0; first < n_views; first += kUploadViews) {
        ViewUpload up{};
        up.first = first;
        up.count = n_views - first < kUploadViews ? n_views - first : kUploadViews;
        for (int k = 0; k < up.count; ++k) {
            const dbs_camera &c = cams[first + k];
            ViewDesc &d = up.v[k];
            for (int r = 0; r < 3; ++r) {
                for (int col = 0; col < 3; ++col) d.R[3 * r + col] = c.viewmat[4 * r + col];
                d.t[r] = c.viewmat[4 * r + 3];
                d.bg[r] = c.background[r];
            }
            d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
            d.near_plane = c.near_plane;
            d.width = c.width; d.height = c.height;
            d.tiles_x = (c.width + tile_w - 1) / tile_w;
            d.tiles_y = (c.height + tile_h - 1) / tile_h;
            d.tile_offset = tile_off;
            d.pixel_offset = pix_off;
            for (int k = 0; k < 3; ++k)
                d.campos[k] = (float)-((double)c.viewmat[k] * c.viewmat[3] + (double)c.viewmat[4 + k] * c.viewmat[7] +
                                       (double)c.viewmat[8 + k] * c.viewmat[11]);
            tile_off += d.tiles_x * d.tiles_y;
            pix_off += (int64_t)c.width * c.height;
        }
        upload_views_kernel<<<1, 64, 0, s>>>(up, P.views, P.hdr, n, n_views, m, tile_w, tile_h,
                                             first == 0 ? 1 : 0);
    }
    return hipGetLastError();
}

hipError_t launch_preprocess(const SplatPtrs &sp, const float *sh, ProjPtrs P, int32_t n_views, int tile_w,
                             int tile_h, uint32_t flags, float b_split, int64_t *counts_out, hipStream_t s)
{
    if (sp.n > 0) {
        // tile sizes are powers of two: pixel -> tile is a shift
        int lw = 0, lh = 0;
        while ((1 << lw) < tile_w) ++lw;
        while ((1 << lh) < tile_h) ++lh;
        if ((1 << lw) != tile_w || (1 << lh) != tile_h) return hipErrorInvalidValue;
        dim3 grid((unsigned)ceil_div(sp.n, 256));
        if (sh) {
            preprocess_kernel<0, true><<<grid, 256, 0, s>>>(sp, sh, P, n_views, lw, lh, flags, b_split);
        } else {
        switch (sp.m) {
#define DBS_PRE(MM)                                                                                          \
    case MM: preprocess_kernel<MM, false><<<grid, 256, 0, s>>>(sp, nullptr, P, n_views, lw, lh, flags, b_split); \
        break;
            DBS_PRE(0) DBS_PRE(1) DBS_PRE(2) DBS_PRE(3) DBS_PRE(4)
            DBS_PRE(5) DBS_PRE(6) DBS_PRE(7) DBS_PRE(8)
#undef DBS_PRE
            default: return hipErrorInvalidValue;
        }
        }
    }
    sum_counts_kernel<<<1, 1024, 0, s>>>(P.blockcnt, sp.n > 0 ? ceil_div(sp.n, 256) : 0, P.hdr, counts_out);
    return hipGetLastError();
}

}  // namespace dbs
