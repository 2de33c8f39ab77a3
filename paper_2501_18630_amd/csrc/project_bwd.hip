// Reverse pass of the projection and Spherical Beta colour.
//
// Input: per-record screen-space gradients accumulated by the raster reverse
// pass, one 64-byte line per record: dL/dmu' (2), dL/dA for the symmetric
// conic (A00, A01, A11 as full-matrix entries), dL/do, dL/db, dL/dcolour (3).
// Each line is cleared after it is read, so the accumulator is zero again
// for the next reverse pass.  Output: dL/dparameter for every parameter of
// Sec. 3.2 Eq. (4) and Sec. 3.3 Eq. (8), ADDED to the caller's buffers.
//
// Chain (Sec. 3.2):  A = Sigma'^{-1}  ->  dSigma' = -A G A;
//   Sigma' = M Sigma M^T, M = J W  ->  dSigma = M^T dSigma' M, dM = 2 dSigma' M Sigma;
//   dJ = dM W^T, with J(t) the pinhole Jacobian; mu'(t);  t = W mu + t_v;
//   Sigma = R diag(s^2) R^T  ->  ds_j = 2 s_j (R^T dSigma R)_jj,
//   dR = 2 dSigma R diag(s^2), R(q/|q|)  ->  dq.
// Colour (Sec. 3.3, Eq. 8): c = c0 + sum_m max(R_m.V, 0)^{beta_m} c_m,
//   beta_m = 4 e^{b_m}, V = (mu - campos)/|mu - campos|.
//
// One thread per splat loops over the views: the per-splat gradient is summed
// in registers (no atomics), Sigma's adjoint is summed over views before the
// single chain to (q, s), and parameters are read and gradients written once.
// The geometric chain runs in FP64; the Spherical Beta lobes in FP32.
#include "dbs_internal.h"

namespace dbs {

namespace {

template <int M>
__global__ __launch_bounds__(256) void project_bwd_kernel(SplatPtrs sp, ProjPtrs P, int32_t n_views, GradPtrs g)
{
    const int64_t n = sp.n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int MM = M > 0 ? M : 1;

    const double mu[3] = {sp.means[3 * i], sp.means[3 * i + 1], sp.means[3 * i + 2]};
    const double q0 = sp.quats[4 * i], q1 = sp.quats[4 * i + 1], q2 = sp.quats[4 * i + 2], q3 = sp.quats[4 * i + 3];
    const double qn = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    const double w = q0 / qn, x = q1 / qn, y = q2 / qn, z = q3 / qn;
    const double Rq[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
                          2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
                          2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)};
    const double sc[3] = {sp.scales[3 * i], sp.scales[3 * i + 1], sp.scales[3 * i + 2]};
    double Sig[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = a; b < 3; ++b) {
            const double acc = Rq[3 * a] * sc[0] * sc[0] * Rq[3 * b] + Rq[3 * a + 1] * sc[1] * sc[1] * Rq[3 * b + 1] +
                               Rq[3 * a + 2] * sc[2] * sc[2] * Rq[3 * b + 2];
            Sig[a][b] = acc;
            Sig[b][a] = acc;
        }

    float lr[MM][3], dth[MM][3], dph[MM][3], lcol[MM][3], lbeta[MM];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int64_t l = i * M + m;
        float st, ct, sph, cph;
        sincosf(sp.lobe_angles[2 * l], &st, &ct);
        sincosf(sp.lobe_angles[2 * l + 1], &sph, &cph);
        lr[m][0] = st * cph; lr[m][1] = st * sph; lr[m][2] = ct;
        dth[m][0] = ct * cph; dth[m][1] = ct * sph; dth[m][2] = -st;
        dph[m][0] = -st * sph; dph[m][1] = st * cph; dph[m][2] = 0.0f;
        for (int c = 0; c < 3; ++c) lcol[m][c] = sp.lobe_colors[3 * l + c];
        lbeta[m] = 4.0f * expf(sp.lobe_betas[l]);
    }

    double gmu[3] = {0, 0, 0}, go = 0, gb = 0, gc0[3] = {0, 0, 0};
    double dSig[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    float gth[MM], gph[MM], gcm[MM][3], gbm[MM];
#pragma unroll
    for (int m = 0; m < MM; ++m) {
        gth[m] = gph[m] = gbm[m] = 0.0f;
        gcm[m][0] = gcm[m][1] = gcm[m][2] = 0.0f;
    }
    bool any = false;

    for (int32_t v = 0; v < n_views; ++v) {
        const int64_t rec = (int64_t)v * n + i;
        if (P.ntiles[rec] == 0) continue;
        float4 *line = P.sgrad + 4 * rec;
        const float4 ga = line[0], gbv = line[1], gcv = line[2];
        // ga = (dmu'x, dmu'y, G00, G01), gbv = (G11, do, db, dr), gcv = (dg, db_col, -, -)
        if (ga.x == 0.f && ga.y == 0.f && ga.z == 0.f && ga.w == 0.f && gbv.x == 0.f && gbv.y == 0.f &&
            gbv.z == 0.f && gbv.w == 0.f && gcv.x == 0.f && gcv.y == 0.f)
            continue;
        {
            const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
            line[0] = z; line[1] = z; line[2] = z; line[3] = z;
        }
        any = true;
        const ViewDesc &V = P.views[v];
        const double W[9] = {V.R[0], V.R[1], V.R[2], V.R[3], V.R[4], V.R[5], V.R[6], V.R[7], V.R[8]};
        double tc[3];
        for (int r = 0; r < 3; ++r)
            tc[r] = W[3 * r] * mu[0] + W[3 * r + 1] * mu[1] + W[3 * r + 2] * mu[2] + (double)V.t[r];
        const double tx = tc[0], ty = tc[1], tz = tc[2], fx = V.fx, fy = V.fy;
        const double J00 = fx / tz, J02 = -fx * tx / (tz * tz), J11 = fy / tz, J12 = -fy * ty / (tz * tz);
        double Mm[2][3];
        for (int b = 0; b < 3; ++b) {
            Mm[0][b] = J00 * W[b] + J02 * W[6 + b];
            Mm[1][b] = J11 * W[3 + b] + J12 * W[6 + b];
        }
        double Tm[2][3];  // M Sigma
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b)
                Tm[a][b] = Mm[a][0] * Sig[0][b] + Mm[a][1] * Sig[1][b] + Mm[a][2] * Sig[2][b];
        const double c00 = Tm[0][0] * Mm[0][0] + Tm[0][1] * Mm[0][1] + Tm[0][2] * Mm[0][2];
        const double c01 = Tm[0][0] * Mm[1][0] + Tm[0][1] * Mm[1][1] + Tm[0][2] * Mm[1][2];
        const double c11 = Tm[1][0] * Mm[1][0] + Tm[1][1] * Mm[1][1] + Tm[1][2] * Mm[1][2];
        const double det = c00 * c11 - c01 * c01;
        const double A00 = c11 / det, A01 = -c01 / det, A11 = c00 / det;

        go += gbv.y;
        gb += gbv.z;
        const double gcol[3] = {gbv.w, gcv.x, gcv.y};
        for (int c = 0; c < 3; ++c) gc0[c] += gcol[c];

        // colour: lobes and the view direction
        double cp[3];
        for (int k = 0; k < 3; ++k)
            cp[k] = -(W[k] * (double)V.t[0] + W[3 + k] * (double)V.t[1] + W[6 + k] * (double)V.t[2]);
        const double vv[3] = {mu[0] - cp[0], mu[1] - cp[1], mu[2] - cp[2]};
        const double vl = sqrt(vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2]);
        const double Vd[3] = {vv[0] / vl, vv[1] / vl, vv[2] / vl};
        double adjV[3] = {0, 0, 0};
        const float Vf[3] = {(float)Vd[0], (float)Vd[1], (float)Vd[2]};
        const float gcf[3] = {gbv.w, gcv.x, gcv.y};
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const float d = lr[m][0] * Vf[0] + lr[m][1] * Vf[1] + lr[m][2] * Vf[2];
            if (d > 0.0f) {
                const float lgd = __builtin_amdgcn_logf(d);                 // log2 d
                const float pw = __builtin_amdgcn_exp2f((lbeta[m] - 1.0f) * lgd);
                const float wgt = pw * d;
                const float adj_w = gcf[0] * lcol[m][0] + gcf[1] * lcol[m][1] + gcf[2] * lcol[m][2];
                for (int c = 0; c < 3; ++c) gcm[m][c] += wgt * gcf[c];
                gbm[m] += adj_w * wgt * (lgd * 0.69314718055994531f) * lbeta[m];
                const float adj_d = adj_w * lbeta[m] * pw;
                gth[m] += adj_d * (dth[m][0] * Vf[0] + dth[m][1] * Vf[1] + dth[m][2] * Vf[2]);
                gph[m] += adj_d * (dph[m][0] * Vf[0] + dph[m][1] * Vf[1] + dph[m][2] * Vf[2]);
                for (int k = 0; k < 3; ++k) adjV[k] += (double)(adj_d * lr[m][k]);
            }
        }
        const double vd = adjV[0] * Vd[0] + adjV[1] * Vd[1] + adjV[2] * Vd[2];
        for (int k = 0; k < 3; ++k) gmu[k] += (adjV[k] - Vd[k] * vd) / vl;

        // conic -> Sigma'
        const double G00 = ga.z, G01 = ga.w, G11 = gbv.x;
        const double AG00 = A00 * G00 + A01 * G01, AG01 = A00 * G01 + A01 * G11;
        const double AG10 = A01 * G00 + A11 * G01, AG11 = A01 * G01 + A11 * G11;
        const double dC00 = -(AG00 * A00 + AG01 * A01);
        const double dC01 = -(AG00 * A01 + AG01 * A11);
        const double dC11 = -(AG10 * A01 + AG11 * A11);
        const double dC[2][2] = {{dC00, dC01}, {dC01, dC11}};
        // dSigma += M^T dC M
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int r = 0; r < 2; ++r)
                    for (int c = 0; c < 2; ++c) acc += Mm[r][a] * dC[r][c] * Mm[c][b];
                dSig[a][b] += acc;
            }
        // dM = 2 dC M Sigma = 2 dC Tm ; dJ = dM W^T
        double dM[2][3];
        for (int r = 0; r < 2; ++r)
            for (int b = 0; b < 3; ++b) dM[r][b] = 2.0 * (dC[r][0] * Tm[0][b] + dC[r][1] * Tm[1][b]);
        const double dJ00 = dM[0][0] * W[0] + dM[0][1] * W[1] + dM[0][2] * W[2];
        const double dJ02 = dM[0][0] * W[6] + dM[0][1] * W[7] + dM[0][2] * W[8];
        const double dJ11 = dM[1][0] * W[3] + dM[1][1] * W[4] + dM[1][2] * W[5];
        const double dJ12 = dM[1][0] * W[6] + dM[1][1] * W[7] + dM[1][2] * W[8];
        const double iz2 = 1.0 / (tz * tz), iz3 = iz2 / tz;
        double dt[3];
        dt[0] = dJ02 * (-fx * iz2) + ga.x * fx / tz;
        dt[1] = dJ12 * (-fy * iz2) + ga.y * fy / tz;
        dt[2] = dJ00 * (-fx * iz2) + dJ02 * (2.0 * fx * tx * iz3) + dJ11 * (-fy * iz2) + dJ12 * (2.0 * fy * ty * iz3)
                - ga.x * fx * tx * iz2 - ga.y * fy * ty * iz2;
        for (int k = 0; k < 3; ++k) gmu[k] += W[k] * dt[0] + W[3 + k] * dt[1] + W[6 + k] * dt[2];
    }
    if (!any) return;

    // Sigma = R diag(s^2) R^T
    double dR[9], gs[3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += (dSig[r][k] + dSig[k][r]) * Rq[3 * k + c];
            dR[3 * r + c] = acc * sc[c] * sc[c];
        }
    for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k) acc += Rq[3 * r + c] * dSig[r][k] * Rq[3 * k + c];
        gs[c] = 2.0 * sc[c] * acc;
    }
    double dq[4];
    dq[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] - 2.0 * x * dR[8]);
    dq[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] - 2.0 * y * dR[8]);
    dq[3] = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * z * dR[4] + y * dR[5] + x * dR[6] + y * dR[7]);
    const double qd = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
    const double qv[4] = {w, x, y, z};

    for (int k = 0; k < 3; ++k) {
        g.means[3 * i + k] += (float)gmu[k];
        g.scales[3 * i + k] += (float)gs[k];
        g.diffuse[3 * i + k] += (float)gc0[k];
    }
    for (int k = 0; k < 4; ++k) g.quats[4 * i + k] += (float)((dq[k] - qv[k] * qd) / qn);
    g.opacities[i] += (float)go;
    g.betas[i] += (float)gb;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int64_t l = i * M + m;
        g.lobe_angles[2 * l] += gth[m];
        g.lobe_angles[2 * l + 1] += gph[m];
        for (int c = 0; c < 3; ++c) g.lobe_colors[3 * l + c] += gcm[m][c];
        g.lobe_betas[l] += gbm[m];
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

hipError_t launch_project_bwd(const SplatPtrs &sp, ProjPtrs P, int32_t n_views, const GradPtrs &g, hipStream_t s)
{
    if (sp.n <= 0) return hipSuccess;
    dim3 grid((unsigned)ceil_div(sp.n, 256));
    switch (sp.m) {
#define DBS_PB(MM) case MM: project_bwd_kernel<MM><<<grid, 256, 0, s>>>(sp, P, n_views, g); break;
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
