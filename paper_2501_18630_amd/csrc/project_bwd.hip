// Reverse pass of the projection and Spherical Beta colour.
//
// Input: per-record screen-space gradients accumulated by the raster reverse
// pass, one 64-byte line per record: dL/dmu' (2), dL/dA for the symmetric
// conic (A00, A01, A11 as full-matrix entries), dL/do, dL/db, dL/dcolour (3).
// Only the lines the raster pass sent gradient to are read: their records'
// bits in gradmask (on a dense scene most visible records are occluded and
// receive none).  Each line read is cleared, and so are the mask bits, so
// the accumulator is zero again for the next reverse pass.  Output: dL/dparameter for every parameter of
// Sec. 3.2 Eq. (4) and Sec. 3.3 Eq. (8), added to the caller's buffers, or,
// in store mode (DBS_FLAG_GRAD_STORE), written over them: every element of
// every splat is then written, zero for a splat no view sees.  In store mode
// the geometry kernel stores the means' gradient and the colour kernel then
// adds its view-direction part to it, so the two launches must run in this
// order on one stream (they do: both are enqueued by one call).
//
// Chain (Sec. 3.2):  A = Sigma'^{-1}  ->  dSigma' = -A G A;
//   Sigma' = M Sigma M^T, M = J W  ->  dSigma = M^T dSigma' M, dM = 2 dSigma' M Sigma;
//   dJ = dM W^T, with J(t) the pinhole Jacobian; mu'(t);  t = W mu + t_v;
//   Sigma = R diag(s^2) R^T  ->  ds_j = 2 s_j (R^T dSigma R)_jj,
//   dR = 2 dSigma R diag(s^2), R(q/|q|)  ->  dq.
// Colour (Sec. 3.3, Eq. 8): c = c0 + sum_m max(R_m.V, 0)^{beta_m} c_m,
//   beta_m = 4 e^{b_m}, V = (mu - campos)/|mu - campos|.
//
// Each splat's per-view terms are summed over the views before the single
// chain to (q, s), and parameters are read and gradients written once.  The
// per-view terms are computed on packed work lists of the records with gradient
// (see below), each added into its splat's accumulators in LDS.  Two kernels
// with disjoint register needs: the geometric chain (FP64) and the colour
// chain (Spherical Beta lobes in FP32), which clears the lines.
#include "dbs_internal.h"

namespace dbs {

namespace {

// `projected` was laid out for this splat and view count (else its record
// pointers would not match, and the call leaves everything untouched).
__device__ __forceinline__ bool proj_matches(const ProjPtrs &P, int64_t n, int32_t n_views)
{
    return P.hdr->n == n && P.hdr->n_views == n_views;
}

__device__ __forceinline__ bool line_is_zero(const float4 a, const float4 b, const float4 c)
{
    return a.x == 0.f && a.y == 0.f && a.z == 0.f && a.w == 0.f && b.x == 0.f && b.y == 0.f && b.z == 0.f &&
           b.w == 0.f && c.x == 0.f && c.y == 0.f;
}

// Work lists.  Only some of a splat's records hold gradient, and a thread
// that loops over every view for its own splat idles in the others.
// Instead, each wavefront lists the (splat, view) records of its 64 splats
// whose gradmask bit is set -- view-major, a window of kItemViews views at a
// time -- and processes that list 64 records at a time, every lane busy.  A record's terms are added into its
// splat's accumulators in LDS; a splat appears at most once per view, and
// the list is view-major, so a splat's terms are added in view order.
// The per-splat parts (Sigma from q and s before, the chain to q and s after)
// are done by the splat's own lane.
constexpr int kPackWaves = 4;
constexpr int kItemViews = 16;  // divides 64: a window's mask bits share one word
static_assert(64 % kItemViews == 0, "item windows must not straddle mask words");

__device__ __forceinline__ uint64_t lanes_below(int lane) { return lane ? (~0ull >> (64 - lane)) : 0ull; }

// Lists the records (lane, v), v in [v0, v1), of the wavefront's splats whose
// bit v is set in vm, view-major; returns the count.  item = lane | v << 6.
__device__ __forceinline__ int list_items(uint64_t vm, bool live, int v0, int v1, uint16_t *items, int lane)
{
    int cnt = 0;
    for (int v = v0; v < v1; ++v) {
        const bool vis = live && ((vm >> (v & 63)) & 1u);
        const uint64_t b = __ballot(vis);
        if (vis) items[cnt + __popcll(b & lanes_below(lane))] = (uint16_t)(lane | (v << 6));
        cnt += __popcll(b);
    }
    return cnt;
}

// Geometry: dL/dmu' (2), dL/dA (3), dL/do, dL/db  ->  mu, s, q, o, b.  FP64.
// store: write the gradients instead of adding them (every splat is written,
// zeros for a splat that no view sees).
__global__ __launch_bounds__(64 * kPackWaves) void project_bwd_geometry_kernel(SplatPtrs sp, ProjPtrs P,
                                                                               int32_t n_views, GradPtrs g, int store)
{
    constexpr int NA = 11;  // accumulators: dL/dmu (3), dL/do, dL/db, adjoint of Sigma (xx xy xz yy yz zz)
    __shared__ double s_sig[kPackWaves][6][kWave];
    __shared__ double s_acc[kPackWaves][NA][kWave];
    __shared__ float s_mu[kPackWaves][3][kWave];
    __shared__ int s_any[kPackWaves][kWave];
    __shared__ uint16_t s_item[kPackWaves][kWave * kItemViews];
    const int64_t n = sp.n;
    if (!proj_matches(P, n, n_views)) return;  // the same for the whole grid
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + (int64_t)w * kWave;  // the wavefront's first splat
    const int64_t i = i0 + lane;
    const bool live = i < n;

    double qv[4] = {1.0, 0.0, 0.0, 0.0}, sc[3] = {0.0, 0.0, 0.0}, iqn = 1.0;
    if (live) {
        for (int k = 0; k < 4; ++k) qv[k] = sp.quats[4 * i + k];
        const double qn = sqrt(qv[0] * qv[0] + qv[1] * qv[1] + qv[2] * qv[2] + qv[3] * qv[3]);
        iqn = 1.0 / qn;
        for (int k = 0; k < 4; ++k) qv[k] *= iqn;
        for (int k = 0; k < 3; ++k) {
            sc[k] = sp.scales[3 * i + k];
            s_mu[w][k][lane] = sp.means[3 * i + k];
        }
        const double w_ = qv[0], x = qv[1], y = qv[2], z = qv[3];
        const double R[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w_ * z), 2.0 * (x * z + w_ * y),
                             2.0 * (x * y + w_ * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w_ * x),
                             2.0 * (x * z - w_ * y), 2.0 * (y * z + w_ * x), 1.0 - 2.0 * (x * x + y * y)};
        const double s2[3] = {sc[0] * sc[0], sc[1] * sc[1], sc[2] * sc[2]};
        int e = 0;
        for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b)
                s_sig[w][e++][lane] = R[3 * a] * s2[0] * R[3 * b] + R[3 * a + 1] * s2[1] * R[3 * b + 1] +
                                      R[3 * a + 2] * s2[2] * R[3 * b + 2];
    }
    for (int c = 0; c < NA; ++c) s_acc[w][c][lane] = 0.0;
    s_any[w][lane] = 0;

    for (int v0 = 0; v0 < n_views; v0 += kItemViews) {
        const int v1 = v0 + kItemViews < n_views ? v0 + kItemViews : n_views;
        const uint64_t vm = live ? P.gradmask[(int64_t)(v0 >> 6) * n + i] : 0ull;
        const int cnt = list_items(vm, live, v0, v1, s_item[w], lane);
        __syncthreads();
        // each group's accumulator lines are loaded while the previous group computes
        // ga = (dmu'x, dmu'y, G00, G01), gbv = (G11, do, db, -); lines the raster pass never touched are zero
        const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
        bool has_n = lane < cnt;
        int item_n = has_n ? s_item[w][lane] : 0;
        float4 ga_n = z4, gbv_n = z4;
        if (has_n) {
            const float4 *line = P.sgrad + 4 * ((int64_t)(item_n >> 6) * n + i0 + (item_n & (kWave - 1)));
            ga_n = line[0];
            gbv_n = line[1];
        }
        for (int base = 0; base < cnt; base += kWave) {
            const bool has = has_n;
            const int item = item_n;
            const float4 ga = ga_n, gbv = gbv_n;
            const int kn = base + kWave + lane;
            has_n = kn < cnt;
            item_n = has_n ? s_item[w][kn] : 0;
            ga_n = gbv_n = z4;
            if (has_n) {
                const float4 *line = P.sgrad + 4 * ((int64_t)(item_n >> 6) * n + i0 + (item_n & (kWave - 1)));
                ga_n = line[0];
                gbv_n = line[1];
            }
            if (!has) continue;
            if (ga.x == 0.f && ga.y == 0.f && ga.z == 0.f && ga.w == 0.f && gbv.x == 0.f && gbv.y == 0.f &&
                gbv.z == 0.f)
                continue;
            const int j = item & (kWave - 1), v = item >> 6;
            s_any[w][j] = 1;
            const ViewDesc &V = P.views[v];
            const double mu[3] = {s_mu[w][0][j], s_mu[w][1][j], s_mu[w][2][j]};
            double Sig[6];
            for (int e = 0; e < 6; ++e) Sig[e] = s_sig[w][e][j];
            const double W[9] = {V.R[0], V.R[1], V.R[2], V.R[3], V.R[4], V.R[5], V.R[6], V.R[7], V.R[8]};
            const double tx = W[0] * mu[0] + W[1] * mu[1] + W[2] * mu[2] + (double)V.t[0];
            const double ty = W[3] * mu[0] + W[4] * mu[1] + W[5] * mu[2] + (double)V.t[1];
            const double tz = W[6] * mu[0] + W[7] * mu[1] + W[8] * mu[2] + (double)V.t[2];
            const double fx = V.fx, fy = V.fy;
            const double iz = 1.0 / tz, iz2 = iz * iz;
            const double J00 = fx * iz, J02 = -fx * tx * iz2, J11 = fy * iz, J12 = -fy * ty * iz2;
            double Mm[2][3];
            for (int b = 0; b < 3; ++b) {
                Mm[0][b] = J00 * W[b] + J02 * W[6 + b];
                Mm[1][b] = J11 * W[3 + b] + J12 * W[6 + b];
            }
            double Tm[2][3];  // M Sigma
            for (int a = 0; a < 2; ++a) {
                Tm[a][0] = Mm[a][0] * Sig[0] + Mm[a][1] * Sig[1] + Mm[a][2] * Sig[2];
                Tm[a][1] = Mm[a][0] * Sig[1] + Mm[a][1] * Sig[3] + Mm[a][2] * Sig[4];
                Tm[a][2] = Mm[a][0] * Sig[2] + Mm[a][1] * Sig[4] + Mm[a][2] * Sig[5];
            }
            const double c00 = Tm[0][0] * Mm[0][0] + Tm[0][1] * Mm[0][1] + Tm[0][2] * Mm[0][2];
            const double c01 = Tm[0][0] * Mm[1][0] + Tm[0][1] * Mm[1][1] + Tm[0][2] * Mm[1][2];
            const double c11 = Tm[1][0] * Mm[1][0] + Tm[1][1] * Mm[1][1] + Tm[1][2] * Mm[1][2];
            const double idet = 1.0 / (c00 * c11 - c01 * c01);
            const double A00 = c11 * idet, A01 = -c01 * idet, A11 = c00 * idet;

            // conic -> Sigma':  dC = -A G A
            const double G00 = ga.z, G01 = ga.w, G11 = gbv.x;
            const double AG00 = A00 * G00 + A01 * G01, AG01 = A00 * G01 + A01 * G11;
            const double AG10 = A01 * G00 + A11 * G01, AG11 = A01 * G01 + A11 * G11;
            const double dC00 = -(AG00 * A00 + AG01 * A01);
            const double dC01 = -(AG00 * A01 + AG01 * A11);
            const double dC11 = -(AG10 * A01 + AG11 * A11);
            // dSigma += M^T dC M (symmetric)
            double dS[6];
            {
                double P0[3], P1[3];  // rows of dC M
                for (int b = 0; b < 3; ++b) {
                    P0[b] = dC00 * Mm[0][b] + dC01 * Mm[1][b];
                    P1[b] = dC01 * Mm[0][b] + dC11 * Mm[1][b];
                }
                int e = 0;
                for (int a = 0; a < 3; ++a)
                    for (int b = a; b < 3; ++b) dS[e++] = Mm[0][a] * P0[b] + Mm[1][a] * P1[b];
            }
            // dM = 2 dC M Sigma = 2 dC Tm ; dJ = dM W^T (the non-zero entries of J)
            double dM0[3], dM1[3];
            for (int b = 0; b < 3; ++b) {
                dM0[b] = 2.0 * (dC00 * Tm[0][b] + dC01 * Tm[1][b]);
                dM1[b] = 2.0 * (dC01 * Tm[0][b] + dC11 * Tm[1][b]);
            }
            const double dJ00 = dM0[0] * W[0] + dM0[1] * W[1] + dM0[2] * W[2];
            const double dJ02 = dM0[0] * W[6] + dM0[1] * W[7] + dM0[2] * W[8];
            const double dJ11 = dM1[0] * W[3] + dM1[1] * W[4] + dM1[2] * W[5];
            const double dJ12 = dM1[0] * W[6] + dM1[1] * W[7] + dM1[2] * W[8];
            const double iz3 = iz2 * iz;
            const double dt0 = dJ02 * (-fx * iz2) + ga.x * fx * iz;
            const double dt1 = dJ12 * (-fy * iz2) + ga.y * fy * iz;
            const double dt2 = dJ00 * (-fx * iz2) + dJ02 * (2.0 * fx * tx * iz3) + dJ11 * (-fy * iz2) +
                               dJ12 * (2.0 * fy * ty * iz3) - ga.x * fx * tx * iz2 - ga.y * fy * ty * iz2;
            // this record's terms into the splat's accumulators
            for (int k3 = 0; k3 < 3; ++k3)
                atomicAdd(&s_acc[w][k3][j], W[k3] * dt0 + W[3 + k3] * dt1 + W[6 + k3] * dt2);
            atomicAdd(&s_acc[w][3][j], (double)gbv.y);
            atomicAdd(&s_acc[w][4][j], (double)gbv.z);
            for (int e = 0; e < 6; ++e) atomicAdd(&s_acc[w][5 + e][j], dS[e]);
        }
        __syncthreads();  // the list is rebuilt for the next window
    }
    if (!live) return;
    if (!s_any[w][lane]) {
        if (store) {
            for (int k = 0; k < 3; ++k) {
                g.means[3 * i + k] = 0.0f;
                g.scales[3 * i + k] = 0.0f;
            }
            for (int k = 0; k < 4; ++k) g.quats[4 * i + k] = 0.0f;
            g.opacities[i] = 0.0f;
            g.betas[i] = 0.0f;
        }
        return;
    }
    const double gmu[3] = {s_acc[w][0][lane], s_acc[w][1][lane], s_acc[w][2][lane]};
    const double go = s_acc[w][3][lane], gb = s_acc[w][4][lane];
    double dS[6];
    for (int e = 0; e < 6; ++e) dS[e] = s_acc[w][5 + e][lane];

    // Sigma = R diag(s^2) R^T  ->  s and the normalised quaternion
    const double w_ = qv[0], x = qv[1], y = qv[2], z = qv[3];
    const double R[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w_ * z), 2.0 * (x * z + w_ * y),
                         2.0 * (x * y + w_ * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w_ * x),
                         2.0 * (x * z - w_ * y), 2.0 * (y * z + w_ * x), 1.0 - 2.0 * (x * x + y * y)};
    const double D[9] = {dS[0], dS[1], dS[2], dS[1], dS[3], dS[4], dS[2], dS[4], dS[5]};
    double dR[9], gs[3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += 2.0 * D[3 * r + k] * R[3 * k + c];
            dR[3 * r + c] = acc * sc[c] * sc[c];
        }
    for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k) acc += R[3 * r + c] * D[3 * r + k] * R[3 * k + c];
        gs[c] = 2.0 * sc[c] * acc;
    }
    double dq[4];
    dq[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w_ * dR[5] + z * dR[6] + w_ * dR[7] - 2.0 * x * dR[8]);
    dq[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w_ * dR[2] + x * dR[3] + z * dR[5] - w_ * dR[6] + z * dR[7] - 2.0 * y * dR[8]);
    dq[3] = 2.0 * (-2.0 * z * dR[0] - w_ * dR[1] + x * dR[2] + w_ * dR[3] - 2.0 * z * dR[4] + y * dR[5] + x * dR[6] + y * dR[7]);
    const double qd = w_ * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
    float out[12];
    for (int k = 0; k < 3; ++k) {
        out[k] = (float)gmu[k];
        out[3 + k] = (float)gs[k];
    }
    for (int k = 0; k < 4; ++k) out[6 + k] = (float)((dq[k] - qv[k] * qd) * iqn);
    out[10] = (float)go;
    out[11] = (float)gb;
    if (!store) {  // accumulate
        for (int k = 0; k < 3; ++k) {
            out[k] += g.means[3 * i + k];
            out[3 + k] += g.scales[3 * i + k];
        }
        for (int k = 0; k < 4; ++k) out[6 + k] += g.quats[4 * i + k];
        out[10] += g.opacities[i];
        out[11] += g.betas[i];
    }
    for (int k = 0; k < 3; ++k) {
        g.means[3 * i + k] = out[k];
        g.scales[3 * i + k] = out[3 + k];
    }
    for (int k = 0; k < 4; ++k) g.quats[4 * i + k] = out[6 + k];
    g.opacities[i] = out[10];
    g.betas[i] = out[11];
}

// Colour (Sec. 3.3, Eq. 8): dL/dcolour -> c0, lobes (theta, phi, c_m, b_m) and
// mu through the view direction.  Runs after the geometry kernel and clears
// every line it reads.
//
// The lobe factor d = R_m . V is evaluated in FP64 (directions from FP64
// sin/cos, V normalised in FP64): near alignment 1 - d, dd/dtheta, dd/dphi and
// the component of the lobe pull orthogonal to V are all O(angle) or smaller,
// and FP32 directions carry ~1e-7 absolute error that swamps them (log d, and
// with it dL/db_m, loses all relative accuracy as d -> 1).  log2 d is taken
// from whichever of d and d - 1 is exact (lobe_log2), then the powers run in
// FP32 on the hardware exp2.
// log2 d for a lobe factor d in (0, 1], to FP32 relative precision.  Below
// 1/2 the hardware log2 is well conditioned.  From 1/2 up, x = d - 1 is exact
// in FP64 and ln d = log1p x = 2 atanh u with u = x / (2 + x), |u| <= 1/3:
// the odd series of atanh in u^2 loses a factor 9 per term, seven terms
// leave < 2e-8.  Both are evaluated and one is selected (no divergence).
__device__ __forceinline__ float lobe_log2(double d)
{
    constexpr float kLog2e = 1.44269504088896341f;
    const float lo = __builtin_amdgcn_logf(fmaxf((float)d, 1e-30f));
    const float x = (float)(d - 1.0);
    const float den = 2.0f + x;
    float u = x * __builtin_amdgcn_rcpf(den);
    u = __fmaf_rn(__fmaf_rn(-u, den, x), __builtin_amdgcn_rcpf(den), u);  // one Newton step
    const float u2 = u * u;
    float sr = 1.0f / 13.0f;
    sr = __fmaf_rn(sr, u2, 1.0f / 11.0f);
    sr = __fmaf_rn(sr, u2, 1.0f / 9.0f);
    sr = __fmaf_rn(sr, u2, 1.0f / 7.0f);
    sr = __fmaf_rn(sr, u2, 1.0f / 5.0f);
    sr = __fmaf_rn(sr, u2, 1.0f / 3.0f);
    sr = __fmaf_rn(sr, u2, 1.0f);
    const float hi = 2.0f * kLog2e * u * sr;
    return d < 0.5 ? lo : hi;
}

// Store mode, a splat with no colour gradient: its colour gradients are zero
// (the geometry kernel has stored the means' zeros).
template <int M>
__device__ __forceinline__ void store_zero_color(const GradPtrs &g, int64_t i)
{
    for (int k = 0; k < 3; ++k) g.diffuse[3 * i + k] = 0.0f;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int64_t l = i * M + m;
        g.lobe_angles[2 * l] = 0.0f;
        g.lobe_angles[2 * l + 1] = 0.0f;
        for (int c = 0; c < 3; ++c) g.lobe_colors[3 * l + c] = 0.0f;
        g.lobe_betas[l] = 0.0f;
    }
}

template <int M>
__global__ __launch_bounds__(256) void project_bwd_color_kernel(SplatPtrs sp, ProjPtrs P, int32_t n_views,
                                                                GradPtrs g, int store)
{
    const int64_t n = sp.n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !proj_matches(P, n, n_views)) return;
    {   // a splat none of whose records has gradient reads no parameters
        uint64_t anyw = 0;
        for (int32_t k = 0; k < (n_views + 63) / 64; ++k) anyw |= P.gradmask[(int64_t)k * n + i];
        if (!anyw) {
            if (store) store_zero_color<M>(g, i);
            return;
        }
    }
    constexpr int MM = M > 0 ? M : 1;
    const double mu[3] = {sp.means[3 * i], sp.means[3 * i + 1], sp.means[3 * i + 2]};
    double st[MM], ct[MM], sph[MM], cph[MM];
    float lcol[MM][3], lbeta[MM];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int64_t l = i * M + m;
        sincos((double)sp.lobe_angles[2 * l], &st[m], &ct[m]);
        sincos((double)sp.lobe_angles[2 * l + 1], &sph[m], &cph[m]);
        for (int c = 0; c < 3; ++c) lcol[m][c] = sp.lobe_colors[3 * l + c];
        lbeta[m] = fminf(4.0f * expf(sp.lobe_betas[l]), 3.4028235e38f);  // as in the projection
    }
    float gmu[3] = {0.f, 0.f, 0.f}, gc0[3] = {0.f, 0.f, 0.f};
    float gth[MM], gph[MM], gcm[MM][3], gbm[MM];
#pragma unroll
    for (int m = 0; m < MM; ++m) {
        gth[m] = gph[m] = gbm[m] = 0.0f;
        gcm[m][0] = gcm[m][1] = gcm[m][2] = 0.0f;
    }
    bool any = false;
    // one record's colour gradient: dL/dcolour of view v from its line (ga, gbv, gcv)
    auto record = [&](int32_t v, float4 *line, const float4 ga, const float4 gbv, const float4 gcv) {
        if (line_is_zero(ga, gbv, gcv)) return;
        {
            const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
            line[0] = z; line[1] = z; line[2] = z; line[3] = z;
        }
        const float gcf[3] = {gbv.w, gcv.x, gcv.y};
        if (gcf[0] == 0.f && gcf[1] == 0.f && gcf[2] == 0.f) return;
        any = true;
        for (int c = 0; c < 3; ++c) gc0[c] += gcf[c];
        if (M == 0) return;
        ConstViewDesc &V = const_view(P.views, v);
        double vd3[3];
        for (int k = 0; k < 3; ++k)
            vd3[k] = mu[k] + ((double)V.R[k] * V.t[0] + (double)V.R[3 + k] * V.t[1] + (double)V.R[6 + k] * V.t[2]);
        const double ivl = 1.0 / sqrt(vd3[0] * vd3[0] + vd3[1] * vd3[1] + vd3[2] * vd3[2]);
        const double Vd[3] = {vd3[0] * ivl, vd3[1] * ivl, vd3[2] * ivl};
        double aV[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const double lr0 = st[m] * cph[m], lr1 = st[m] * sph[m], lr2 = ct[m];
            const double d = lr0 * Vd[0] + lr1 * Vd[1] + lr2 * Vd[2];
            if (d > 0.0) {
                const float l2 = lobe_log2(d);
                const float lnd = l2 * 0.69314718055994531f;
                const float pw = __builtin_amdgcn_exp2f((lbeta[m] - 1.0f) * l2);  // d^(beta-1)
                const float wgt = pw * (float)d;                             // d^beta
                const float adj_w = gcf[0] * lcol[m][0] + gcf[1] * lcol[m][1] + gcf[2] * lcol[m][2];
                for (int c = 0; c < 3; ++c) gcm[m][c] += wgt * gcf[c];
                gbm[m] += adj_w * wgt * lnd * lbeta[m];
                const float adj_d = adj_w * lbeta[m] * pw;
                // dR/dtheta = (ct cph, ct sph, -st), dR/dphi = (-st sph, st cph, 0)
                const double dth = ct[m] * (cph[m] * Vd[0] + sph[m] * Vd[1]) - st[m] * Vd[2];
                const double dph = lr0 * Vd[1] - lr1 * Vd[0];
                gth[m] += adj_d * (float)dth;
                gph[m] += adj_d * (float)dph;
                aV[0] += adj_d * lr0;
                aV[1] += adj_d * lr1;
                aV[2] += adj_d * lr2;
            }
        }
        const double vdot = aV[0] * Vd[0] + aV[1] * Vd[1] + aV[2] * Vd[2];
        for (int k = 0; k < 3; ++k) gmu[k] += (float)((aV[k] - Vd[k] * vdot) * ivl);
    };
    // Only the records the raster pass sent gradient to, one set mask bit after
    // another (a lane does as many steps as its splat has such records, not one
    // per view); the next record's line is loaded while one computes.  This
    // kernel runs last and clears the mask words and the lines it reads.
    for (int32_t w0 = 0; w0 < n_views; w0 += 64) {
        uint64_t *wd = &P.gradmask[(int64_t)(w0 >> 6) * n + i];
        uint64_t vm = *wd;
        if (!vm) continue;
        *wd = 0ull;
        int32_t v = w0 + __builtin_ctzll(vm);
        vm &= vm - 1;
        float4 *line = P.sgrad + 4 * ((int64_t)v * n + i);
        float4 na = line[0], nb = line[1], nc = line[2];
        for (;;) {
            const int32_t cv = v;
            float4 *cl = line;
            const float4 ga = na, gbv = nb, gcv = nc;
            const bool more = vm != 0;
            if (more) {
                v = w0 + __builtin_ctzll(vm);
                vm &= vm - 1;
                line = P.sgrad + 4 * ((int64_t)v * n + i);
                na = line[0];
                nb = line[1];
                nc = line[2];
            }
            record(cv, cl, ga, gbv, gcv);
            if (!more) break;
        }
    }
    if (!any) {
        if (store) store_zero_color<M>(g, i);
        return;
    }
    // the means always add: the geometry kernel has written its part
    for (int k = 0; k < 3; ++k) g.means[3 * i + k] += gmu[k];
    if (store) {
        for (int k = 0; k < 3; ++k) g.diffuse[3 * i + k] = gc0[k];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int64_t l = i * M + m;
            g.lobe_angles[2 * l] = gth[m];
            g.lobe_angles[2 * l + 1] = gph[m];
            for (int c = 0; c < 3; ++c) g.lobe_colors[3 * l + c] = gcm[m][c];
            g.lobe_betas[l] = gbm[m];
        }
    } else {
        for (int k = 0; k < 3; ++k) g.diffuse[3 * i + k] += gc0[k];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int64_t l = i * M + m;
            g.lobe_angles[2 * l] += gth[m];
            g.lobe_angles[2 * l + 1] += gph[m];
            for (int c = 0; c < 3; ++c) g.lobe_colors[3 * l + c] += gcm[m][c];
            g.lobe_betas[l] += gbm[m];
        }
    }
}

__global__ __launch_bounds__(256) void l1_loss_kernel(const float *__restrict__ img, const float *__restrict__ tgt,
                                                      int64_t count, float scale, float *__restrict__ grad,
                                                      float *loss)
{
    __shared__ float s_part[256 / kWave];
    float acc = 0.0f;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x) {
        const float d = img[k] - tgt[k];
        grad[k] = d > 0.0f ? scale : (d < 0.0f ? -scale : 0.0f);
        acc += fabsf(d);
    }
    if (loss) {
        for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0) s_part[threadIdx.x / kWave] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            float t = 0.0f;
            for (int w = 0; w < 256 / kWave; ++w) t += s_part[w];
            atomicAdd(loss, t * scale);
        }
    }
}

__global__ void zero_f32_kernel(float *p) { *p = 0.0f; }

}  // namespace

hipError_t launch_project_bwd(const SplatPtrs &sp, ProjPtrs P, int32_t n_views, const GradPtrs &g, bool store,
                              hipStream_t s)
{
    if (sp.n <= 0) return hipSuccess;
    const int st = store ? 1 : 0;
    project_bwd_geometry_kernel<<<(unsigned)ceil_div(sp.n, 64 * kPackWaves), 64 * kPackWaves, 0, s>>>(sp, P, n_views,
                                                                                                    g, st);
    switch (sp.m) {
#define DBS_PB(MM)                                                                                          \
    case MM: project_bwd_color_kernel<MM><<<(unsigned)ceil_div(sp.n, 256), 256, 0, s>>>(sp, P, n_views, g, st); \
        break;
        DBS_PB(0) DBS_PB(1) DBS_PB(2) DBS_PB(3) DBS_PB(4) DBS_PB(5) DBS_PB(6) DBS_PB(7) DBS_PB(8)
#undef DBS_PB
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_l1_loss(const float *image, const float *target, int64_t count, float scale, float *grad,
                          float *loss, hipStream_t s)
{
    if (loss) zero_f32_kernel<<<1, 1, 0, s>>>(loss);
    if (count > 0) {
        int64_t blocks = ceil_div(count, 256);
        if (blocks > 2048) blocks = 2048;
        l1_loss_kernel<<<(unsigned)blocks, 256, 0, s>>>(image, target, count, scale, grad, loss);
    }
    return hipGetLastError();
}

}  // namespace dbs
