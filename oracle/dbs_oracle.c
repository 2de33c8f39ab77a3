/*
 * CPU FP64 oracle for the Deformable Beta Splatting rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py load this library.  The product path (the HIP
 * library and its Python binding) never links, loads or calls it, and this
 * file includes nothing from the product tree.
 *
 * Everything here is a plain, slow, brute-force statement of what the paper
 * defines, evaluated in double precision:
 *
 *   Beta kernel B(x; b) = (1 - x)^beta, beta = 4 e^b ........ Sec. 3.1, Eqs. (2)-(3)
 *   primitive {mu, o, q, s, b, f} ........................... Sec. 3.2, Eq. (4)
 *   Sigma = R S S^T R^T, Sigma' = J W Sigma W^T J^T ......... Sec. 3.2 (text before Eq. 5)
 *   r_i(x)^2 = (x - mu')^T Sigma'^{-1} (x - mu') ............ Sec. 3.2, Eq. (5)
 *   depth-ordered front-to-back compositing ................. Sec. 3.2, Eq. (6)
 *   Spherical Beta colour c0 + sum_m B(1 - R_m.V; b_m) c_m .. Sec. 3.3, Eq. (8)
 *   comparison mode: Gaussian kernel + degree-3 SH colour ... Sec. 3.3 (the
 *     spherical-harmonics colour it replaces), Sec. 4 (the 3DGS baseline)
 *
 * Conventions the paper leaves open (fixed identically on the GPU side):
 *   - camera: world->camera x_c = R x_w + t, OpenCV axes (x right, y down,
 *     z forward); pinhole u = fx x/z + cx, v = fy y/z + cy; the centre of
 *     pixel (u, v) is at (u + 0.5, v + 0.5);
 *   - J is the affine (EWA) Jacobian of the pinhole map at the splat centre;
 *   - quaternion order (w, x, y, z), normalised before use; scales and
 *     opacity are passed already activated; b and b_m are raw;
 *   - a splat is culled when t_z <= near or det(Sigma') <= 0, and in every
 *     view when any of its parameters is not finite (NaN or +-inf);
 *   - lobe direction R_m = (sin th cos ph, sin th sin ph, cos th) (parity
 *     unpinned: the paper prints no example that fixes this convention);
 *     V = (mu - camera centre)/|mu - camera centre|;
 *   - depth order: ascending fp32-rounded t_z, ties by splat index;
 *   - alpha = min(alpha_max, o B(r^2; b)); a splat takes part iff r^2 < 1;
 *     the pixel stops after the splat that brings T below t_eps;
 *   - output = sum_i c_i alpha_i T_i + T_final * background.
 *
 * The gradient is exact reverse mode over the stored per-pixel list of
 * (splat, alpha, T) — no recomputation of T by division.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

typedef struct {
    double R[9];       /* world->camera rotation, row-major */
    double t[3];       /* world->camera translation */
    double fx, fy, cx, cy;
    int32_t width, height;
    double near_plane;
    double bg[3];
} ob_camera;

typedef struct {
    int64_t n;
    int32_t m;                 /* Spherical Beta lobes per splat */
    const double *means;       /* [n,3] */
    const double *scales;      /* [n,3] activated, > 0 */
    const double *quats;       /* [n,4] (w,x,y,z), any non-zero norm */
    const double *opacities;   /* [n]   activated, in [0,1] */
    const double *betas;       /* [n]   raw b */
    const double *diffuse;     /* [n,3] c0 */
    const double *lobe_angles; /* [n,m,2] (theta, phi) */
    const double *lobe_colors; /* [n,m,3] c_m */
    const double *lobe_betas;  /* [n,m]  raw b_m */
    /* [n,16,3] degree-3 SH coefficients, or NULL.  Non-NULL selects the
     * Gaussian-kernel + SH comparison mode: kernel exp(-m^2/2) for
     * Mahalanobis distance m < 3, colour max(0, sum_k sh_k Y_k(V) + 1/2);
     * betas, diffuse and the lobes are not read. */
    const double *sh;
} ob_splats;

typedef struct {               /* gradients (or |contribution| sums); same shapes as ob_splats */
    double *means, *scales, *quats, *opacities, *betas, *diffuse,
           *lobe_angles, *lobe_colors, *lobe_betas;
} ob_grads;

/* ------------------------------------------------------------------------ */
/* Beta kernel, Sec. 3.1 Eqs. (2)-(3): (1 - x)^(4 e^b) on [0, 1], zero beyond. */
double ob_beta_kernel(double x, double b)
{
    if (!(x < 1.0)) return 0.0;
    if (x < 0.0) x = 0.0;
    return pow(1.0 - x, 4.0 * exp(b));
}

/* Real spherical harmonics of degree l <= 3 at the unit direction d, in the
 * order (l, m) = (0,0), (1,-1), (1,0), (1,1), (2,-2), ..., (3,3), written
 * from their definition: with cos(th) = d_z and ph = atan2(d_y, d_x),
 *   Y_l^0 = K_l^0 P_l^0(cos th),
 *   Y_l^m = sqrt(2) K_l^m cos(m ph) P_l^m(cos th)      (m > 0),
 *   Y_l^m = sqrt(2) K_l^|m| sin(|m| ph) P_l^|m|(cos th) (m < 0),
 *   K_l^m = sqrt((2l + 1) / (4 pi) (l - m)! / (l + m)!),
 * where the associated Legendre functions P_l^m carry the Condon-Shortley
 * phase (-1)^m. */
static double assoc_legendre(int l, int m, double x)
{
    double s = sqrt(1.0 - x * x);
    switch (10 * l + m) {
    case 0: return 1.0;
    case 10: return x;
    case 11: return -s;
    case 20: return 0.5 * (3.0 * x * x - 1.0);
    case 21: return -3.0 * x * s;
    case 22: return 3.0 * s * s;
    case 30: return 0.5 * (5.0 * x * x * x - 3.0 * x);
    case 31: return -1.5 * (5.0 * x * x - 1.0) * s;
    case 32: return 15.0 * x * s * s;
    case 33: return -15.0 * s * s * s;
    }
    return 0.0;
}

static double factorial(int k) { double f = 1.0; for (int i = 2; i <= k; ++i) f *= i; return f; }

void ob_sh_basis3(const double *d, double *Y)
{
    double ct = d[2], ph = atan2(d[1], d[0]);
    int k = 0;
    for (int l = 0; l <= 3; ++l)
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
            double P = assoc_legendre(l, am, ct);
            if (m == 0) Y[k] = K * P;
            else if (m > 0) Y[k] = sqrt(2.0) * K * cos(m * ph) * P;
            else Y[k] = sqrt(2.0) * K * sin(am * ph) * P;
            ++k;
        }
}

/* Unit-quaternion rotation matrix (w,x,y,z), row-major.  q is normalised here. */
void ob_quat_to_rot(const double *q_in, double *R)
{
    double n = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3]);
    double w = q_in[0] / n, x = q_in[1] / n, y = q_in[2] / n, z = q_in[3] / n;
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* Everything the forward model derives for one (splat, view). */
typedef struct {
    int valid;
    double tc[3];          /* camera-space centre */
    double Rq[9];          /* rotation from the normalised quaternion */
    double qn[4];          /* normalised quaternion */
    double qnorm;
    double Sig[9];         /* 3D covariance R diag(s^2) R^T */
    double Jm[6];          /* 2x3 Jacobian */
    double Mm[6];          /* J W */
    double cov[3];         /* Sigma'00, Sigma'01, Sigma'11 */
    double det;
    double conic[3];       /* A00, A01, A11 */
    double mean2d[2];
    double extent[2];
    double beta;
    double color[3];
    double vdir[3], vlen;  /* unit view direction and |mu - campos| */
    int32_t bbox[4];       /* x_lo, x_hi, y_lo, y_hi (inclusive) */
} ob_fwd;

/* 1 when every parameter of splat i is a finite number.  The paper defines
 * the primitive for real-valued parameters only; a splat with a NaN or
 * infinite parameter is treated as absent (culled in every view), so that
 * it neither poisons the image nor receives a gradient. */
static int params_finite(const ob_splats *s, int64_t i)
{
    for (int k = 0; k < 3; ++k)
        if (!isfinite(s->means[3 * i + k]) || !isfinite(s->scales[3 * i + k])) return 0;
    for (int k = 0; k < 4; ++k)
        if (!isfinite(s->quats[4 * i + k])) return 0;
    if (!isfinite(s->opacities[i])) return 0;
    if (s->sh) {
        for (int k = 0; k < 48; ++k)
            if (!isfinite(s->sh[48 * i + k])) return 0;
        return 1;
    }
    if (!isfinite(s->betas[i])) return 0;
    for (int k = 0; k < 3; ++k)
        if (!isfinite(s->diffuse[3 * i + k])) return 0;
    for (int64_t k = 0; k < s->m; ++k) {
        const int64_t l = i * s->m + k;
        if (!isfinite(s->lobe_angles[2 * l]) || !isfinite(s->lobe_angles[2 * l + 1])) return 0;
        if (!isfinite(s->lobe_colors[3 * l]) || !isfinite(s->lobe_colors[3 * l + 1]) ||
            !isfinite(s->lobe_colors[3 * l + 2]))
            return 0;
        if (!isfinite(s->lobe_betas[l])) return 0;
    }
    return 1;
}

static void project_one(const ob_splats *s, int64_t i, const ob_camera *cam, ob_fwd *f)
{
    memset(f, 0, sizeof(*f));
    if (!params_finite(s, i)) return;
    const double *mu = s->means + 3 * i;
    const double *W = cam->R;
    /* camera-space centre, summed left to right: ((W0 mu0 + W1 mu1) + W2 mu2) + t */
    for (int r = 0; r < 3; ++r)
        f->tc[r] = W[3 * r + 0] * mu[0] + W[3 * r + 1] * mu[1] + W[3 * r + 2] * mu[2] + cam->t[r];
    if (!(f->tc[2] > cam->near_plane)) return;

    const double *q = s->quats + 4 * i;
    f->qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(f->qnorm > 0.0)) return;
    for (int k = 0; k < 4; ++k) f->qn[k] = q[k] / f->qnorm;
    ob_quat_to_rot(q, f->Rq);

    const double *sc = s->scales + 3 * i;
    double s2[3] = {sc[0] * sc[0], sc[1] * sc[1], sc[2] * sc[2]};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += f->Rq[3 * a + k] * s2[k] * f->Rq[3 * b + k];
            f->Sig[3 * a + b] = acc;
        }

    double tx = f->tc[0], ty = f->tc[1], tz = f->tc[2];
    f->Jm[0] = cam->fx / tz; f->Jm[1] = 0.0;           f->Jm[2] = -cam->fx * tx / (tz * tz);
    f->Jm[3] = 0.0;          f->Jm[4] = cam->fy / tz;  f->Jm[5] = -cam->fy * ty / (tz * tz);
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += f->Jm[3 * a + k] * W[3 * k + b];
            f->Mm[3 * a + b] = acc;
        }
    double C2[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) acc += f->Mm[3 * a + k] * f->Sig[3 * k + l] * f->Mm[3 * b + l];
            C2[2 * a + b] = acc;
        }
    f->cov[0] = C2[0];
    f->cov[1] = 0.5 * (C2[1] + C2[2]);
    f->cov[2] = C2[3];
    f->det = f->cov[0] * f->cov[2] - f->cov[1] * f->cov[1];
    if (!(f->det > 0.0)) return;
    f->conic[0] = f->cov[2] / f->det;
    f->conic[1] = -f->cov[1] / f->det;
    f->conic[2] = f->cov[0] / f->det;

    f->mean2d[0] = cam->fx * tx / tz + cam->cx;
    f->mean2d[1] = cam->fy * ty / tz + cam->cy;
    /* the exact axis-aligned bounding box of {d : d^T Sigma'^{-1} d <= 1}
     * (of the 3-sigma ellipse, d^T Sigma'^{-1} d <= 9, in the comparison mode) */
    double ext = s->sh ? 3.0 : 1.0;
    f->extent[0] = ext * sqrt(f->cov[0]);
    f->extent[1] = ext * sqrt(f->cov[2]);

    /* pixel centres (u + 0.5) inside [mu' - e, mu' + e], clipped to the image */
    double xl = ceil(f->mean2d[0] - f->extent[0] - 0.5), xh = floor(f->mean2d[0] + f->extent[0] - 0.5);
    double yl = ceil(f->mean2d[1] - f->extent[1] - 0.5), yh = floor(f->mean2d[1] + f->extent[1] - 0.5);
    if (xl < 0.0) xl = 0.0;
    if (yl < 0.0) yl = 0.0;
    if (xh > cam->width - 1) xh = cam->width - 1;
    if (yh > cam->height - 1) yh = cam->height - 1;
    if (xl > xh || yl > yh) {      /* covers no pixel centre: empty box */
        f->bbox[0] = 0; f->bbox[1] = -1; f->bbox[2] = 0; f->bbox[3] = -1;
    } else {
        f->bbox[0] = (int32_t)xl; f->bbox[1] = (int32_t)xh;
        f->bbox[2] = (int32_t)yl; f->bbox[3] = (int32_t)yh;
    }

    f->beta = s->sh ? 0.0 : 4.0 * exp(s->betas[i]);

    /* Spherical Beta colour, Sec. 3.3 Eq. (8) */
    double campos[3];
    for (int k = 0; k < 3; ++k) campos[k] = -(W[k] * cam->t[0] + W[3 + k] * cam->t[1] + W[6 + k] * cam->t[2]);
    double v[3] = {mu[0] - campos[0], mu[1] - campos[1], mu[2] - campos[2]};
    f->vlen = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int k = 0; k < 3; ++k) f->vdir[k] = v[k] / f->vlen;
    if (s->sh) {  /* comparison mode: SH colour, offset by 1/2 and clamped at 0 */
        double Y[16];
        ob_sh_basis3(f->vdir, Y);
        for (int c = 0; c < 3; ++c) {
            double acc = 0.5;
            for (int k = 0; k < 16; ++k) acc += Y[k] * s->sh[(i * 16 + k) * 3 + c];
            f->color[c] = acc > 0.0 ? acc : 0.0;
        }
        f->valid = 1;
        return;
    }
    for (int c = 0; c < 3; ++c) f->color[c] = s->diffuse[3 * i + c];
    for (int m = 0; m < s->m; ++m) {
        double th = s->lobe_angles[2 * (i * s->m + m)], ph = s->lobe_angles[2 * (i * s->m + m) + 1];
        double Rm[3] = {sin(th) * cos(ph), sin(th) * sin(ph), cos(th)};
        double x = 1.0 - (Rm[0] * f->vdir[0] + Rm[1] * f->vdir[1] + Rm[2] * f->vdir[2]);
        double w = ob_beta_kernel(x, s->lobe_betas[i * s->m + m]);
        for (int c = 0; c < 3; ++c) f->color[c] += w * s->lobe_colors[3 * (i * s->m + m) + c];
    }
    f->valid = 1;
}

/* Per-splat projection for one view.  Output arrays may be NULL. */
int ob_project(const ob_splats *s, const ob_camera *cam,
               int32_t *valid, double *tcam, double *mean2d, double *cov2d, double *conic,
               double *extent, double *beta, double *color, uint32_t *depth_key, int32_t *bbox)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s->n; ++i) {
        ob_fwd f;
        project_one(s, i, cam, &f);
        if (valid) valid[i] = f.valid;
        if (tcam) for (int k = 0; k < 3; ++k) tcam[3 * i + k] = f.tc[k];
        if (mean2d) for (int k = 0; k < 2; ++k) mean2d[2 * i + k] = f.mean2d[k];
        if (cov2d) for (int k = 0; k < 3; ++k) cov2d[3 * i + k] = f.cov[k];
        if (conic) for (int k = 0; k < 3; ++k) conic[3 * i + k] = f.conic[k];
        if (extent) for (int k = 0; k < 2; ++k) extent[2 * i + k] = f.extent[k];
        if (beta) beta[i] = f.beta;
        if (color) for (int k = 0; k < 3; ++k) color[3 * i + k] = f.color[k];
        if (depth_key) {
            float z = (float)f.tc[2];
            uint32_t bits;
            memcpy(&bits, &z, 4);
            depth_key[i] = bits;
        }
        if (bbox) for (int k = 0; k < 4; ++k) bbox[4 * i + k] = f.bbox[k];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* depth order: ascending fp32 depth bits, ties by splat index */
typedef struct { uint32_t key; int64_t id; } ob_sortrec;

static int cmp_sortrec(const void *a, const void *b)
{
    const ob_sortrec *x = (const ob_sortrec *)a, *y = (const ob_sortrec *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

typedef struct {
    int64_t n_order;
    int64_t *order;     /* visible splats in depth order */
    ob_fwd *fw;         /* forward record per splat (index = splat id) */
} ob_scene;

static int scene_build(const ob_splats *s, const ob_camera *cam, ob_scene *sc)
{
    sc->fw = (ob_fwd *)malloc(sizeof(ob_fwd) * (size_t)(s->n > 0 ? s->n : 1));
    ob_sortrec *tmp = (ob_sortrec *)malloc(sizeof(ob_sortrec) * (size_t)(s->n > 0 ? s->n : 1));
    sc->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(s->n > 0 ? s->n : 1));
    if (!sc->fw || !tmp || !sc->order) { free(sc->fw); free(tmp); free(sc->order); return -1; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s->n; ++i) project_one(s, i, cam, &sc->fw[i]);
    int64_t k = 0;
    for (int64_t i = 0; i < s->n; ++i) {
        if (!sc->fw[i].valid) continue;
        float z = (float)sc->fw[i].tc[2];
        uint32_t bits;
        memcpy(&bits, &z, 4);
        tmp[k].key = bits;
        tmp[k].id = i;
        ++k;
    }
    qsort(tmp, (size_t)k, sizeof(ob_sortrec), cmp_sortrec);
    for (int64_t j = 0; j < k; ++j) sc->order[j] = tmp[j].id;
    sc->n_order = k;
    free(tmp);
    return 0;
}

static void scene_free(ob_scene *sc) { free(sc->fw); free(sc->order); }

/* one step of the per-pixel list kept for the reverse pass */
typedef struct {
    int64_t id;
    double alpha, T;        /* alpha_i and the transmittance in front of it */
    double dx, dy, r2, B;   /* offset p - mu', r^2, kernel value */
    int clamped;
} ob_step;

/* Composite one pixel front to back, Eq. (6).  Returns the number of steps;
 * fills steps[] if non-NULL (capacity n_order). */
static int64_t composite_pixel(const ob_splats *s, const ob_scene *sc, double px, double py,
                               double alpha_max, double t_eps, double *rgb, double *T_out,
                               double *T_prev_out, int64_t *last_out, ob_step *steps)
{
    double T = 1.0, C[3] = {0.0, 0.0, 0.0}, T_prev = 1.0;
    int64_t last = -1, n = 0;
    for (int64_t j = 0; j < sc->n_order; ++j) {
        int64_t i = sc->order[j];
        const ob_fwd *f = &sc->fw[i];
        double dx = px - f->mean2d[0], dy = py - f->mean2d[1];
        double r2 = f->conic[0] * dx * dx + 2.0 * f->conic[1] * dx * dy + f->conic[2] * dy * dy;
        double B;
        if (s->sh) {                               /* Gaussian, cut at 3 sigma */
            if (!(r2 < 9.0)) continue;
            B = exp(-0.5 * r2);
        } else {
            if (!(r2 < 1.0)) continue;             /* bounded support: exactly zero */
            B = pow(1.0 - r2, f->beta);
        }
        double a = s->opacities[i] * B;
        int clamped = 0;
        if (a > alpha_max) { a = alpha_max; clamped = 1; }
        if (steps) {
            steps[n].id = i; steps[n].alpha = a; steps[n].T = T;
            steps[n].dx = dx; steps[n].dy = dy; steps[n].r2 = r2; steps[n].B = B;
            steps[n].clamped = clamped;
        }
        ++n;
        for (int c = 0; c < 3; ++c) C[c] += f->color[c] * a * T;
        T_prev = T;
        T *= (1.0 - a);
        last = i;
        if (T < t_eps) break;
    }
    for (int c = 0; c < 3; ++c) rgb[c] = C[c];
    *T_out = T;
    if (T_prev_out) *T_prev_out = T_prev;
    *last_out = last;
    return n;
}

/* Render the listed pixels (pix_xy [npix,2] integer pixel indices).
 * out_rgb includes T_final * background.  Optional outputs may be NULL:
 *   out_T_prev: transmittance in front of the last processed splat,
 *   out_nsteps: number of splats that took part (r^2 < 1) up to termination. */
int ob_render(const ob_splats *s, const ob_camera *cam, double alpha_max, double t_eps,
              int64_t npix, const int32_t *pix_xy, double *out_rgb, double *out_T,
              double *out_T_prev, int64_t *out_last, int64_t *out_nsteps)
{
    ob_scene sc;
    if (scene_build(s, cam, &sc)) return -1;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t p = 0; p < npix; ++p) {
        double rgb[3], T, Tp;
        int64_t last;
        int64_t n = composite_pixel(s, &sc, pix_xy[2 * p] + 0.5, pix_xy[2 * p + 1] + 0.5,
                                    alpha_max, t_eps, rgb, &T, &Tp, &last, NULL);
        for (int c = 0; c < 3; ++c) out_rgb[3 * p + c] = rgb[c] + T * cam->bg[c];
        out_T[p] = T;
        if (out_T_prev) out_T_prev[p] = Tp;
        out_last[p] = last;
        if (out_nsteps) out_nsteps[p] = n;
    }
    scene_free(&sc);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Reverse mode of the projection and colour model for one (splat, view).
 * Inputs are the adjoints of the screen-space quantities the compositing
 * uses:  mean2d (2), the symmetric conic adjoint G (G00, G01, G11) with
 * dL/dA_ab = G_ab for the full 2x2 matrix A, opacity, raw b (already
 * through beta = 4 e^b) and colour (3).  The parameter adjoints are added
 * to g (and |.| of each one to a when a != NULL). */
typedef struct {
    double mean2d[2], G[3], opacity, b, color[3];
} ob_screen_adj;

static void add_grad(double *g, int64_t idx, double v) { g[idx] += v; }

static void chain_one(const ob_splats *s, int64_t i, const ob_camera *cam, const ob_fwd *f,
                      const ob_screen_adj *sa, ob_grads *g)
{
    const double *W = cam->R;
    const int m_l = s->m;
    add_grad(g->opacities, i, sa->opacity);
    add_grad(g->betas, i, sa->b);

    /* colour -> c0, lobes, and the view direction */
    double adjV[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < 3; ++c) add_grad(g->diffuse, 3 * i + c, sa->color[c]);
    for (int m = 0; m < m_l; ++m) {
        int64_t lm = i * m_l + m;
        double th = s->lobe_angles[2 * lm], ph = s->lobe_angles[2 * lm + 1];
        double Rm[3] = {sin(th) * cos(ph), sin(th) * sin(ph), cos(th)};
        double dR_dth[3] = {cos(th) * cos(ph), cos(th) * sin(ph), -sin(th)};
        double dR_dph[3] = {-sin(th) * sin(ph), sin(th) * cos(ph), 0.0};
        double x = Rm[0] * f->vdir[0] + Rm[1] * f->vdir[1] + Rm[2] * f->vdir[2];   /* R.V */
        double bm = 4.0 * exp(s->lobe_betas[lm]);
        double w = x > 0.0 ? pow(x, bm) : 0.0;
        double adj_w = 0.0;
        for (int c = 0; c < 3; ++c) {
            add_grad(g->lobe_colors, 3 * lm + c, w * sa->color[c]);
            adj_w += sa->color[c] * s->lobe_colors[3 * lm + c];
        }
        if (x > 0.0) {
            add_grad(g->lobe_betas, lm, adj_w * w * log(x) * bm);
            double adj_x = adj_w * bm * pow(x, bm - 1.0);
            add_grad(g->lobe_angles, 2 * lm,
                     adj_x * (dR_dth[0] * f->vdir[0] + dR_dth[1] * f->vdir[1] + dR_dth[2] * f->vdir[2]));
            add_grad(g->lobe_angles, 2 * lm + 1,
                     adj_x * (dR_dph[0] * f->vdir[0] + dR_dph[1] * f->vdir[1] + dR_dph[2] * f->vdir[2]));
            for (int k = 0; k < 3; ++k) adjV[k] += adj_x * Rm[k];
        } else {
            add_grad(g->lobe_betas, lm, 0.0);
        }
    }
    /* V = v/|v|, v = mu - campos */
    double vd = adjV[0] * f->vdir[0] + adjV[1] * f->vdir[1] + adjV[2] * f->vdir[2];
    double gmu[3];
    for (int k = 0; k < 3; ++k) gmu[k] = (adjV[k] - f->vdir[k] * vd) / f->vlen;

    /* conic A = Sigma'^{-1}:  dL/dSigma' = -A G A */
    double A[4] = {f->conic[0], f->conic[1], f->conic[1], f->conic[2]};
    double G[4] = {sa->G[0], sa->G[1], sa->G[1], sa->G[2]};
    double AG_[4], dC[4];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) AG_[2 * r + c] = A[2 * r] * G[c] + A[2 * r + 1] * G[2 + c];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) dC[2 * r + c] = -(AG_[2 * r] * A[c] + AG_[2 * r + 1] * A[2 + c]);

    /* Sigma' = M Sigma M^T, M = J W:  dSigma = M^T dC M ; dM = 2 dC M Sigma */
    double dSig[9], dM[6], dJ[6];
    for (int a3 = 0; a3 < 3; ++a3)
        for (int b3 = 0; b3 < 3; ++b3) {
            double acc = 0.0;
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c) acc += f->Mm[3 * r + a3] * dC[2 * r + c] * f->Mm[3 * c + b3];
            dSig[3 * a3 + b3] = acc;
        }
    for (int r = 0; r < 2; ++r)
        for (int b3 = 0; b3 < 3; ++b3) {
            double acc = 0.0;
            for (int c = 0; c < 2; ++c)
                for (int k = 0; k < 3; ++k) acc += dC[2 * r + c] * f->Mm[3 * c + k] * f->Sig[3 * k + b3];
            dM[3 * r + b3] = 2.0 * acc;
        }
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k) {
            double acc = 0.0;
            for (int b3 = 0; b3 < 3; ++b3) acc += dM[3 * r + b3] * W[3 * k + b3];
            dJ[3 * r + k] = acc;
        }

    /* J and mu' as functions of the camera-space centre t */
    double tx = f->tc[0], ty = f->tc[1], tz = f->tc[2];
    double fx = cam->fx, fy = cam->fy;
    double dt[3] = {0.0, 0.0, 0.0};
    dt[0] += dJ[2] * (-fx / (tz * tz));
    dt[1] += dJ[5] * (-fy / (tz * tz));
    dt[2] += dJ[0] * (-fx / (tz * tz)) + dJ[2] * (2.0 * fx * tx / (tz * tz * tz))
           + dJ[4] * (-fy / (tz * tz)) + dJ[5] * (2.0 * fy * ty / (tz * tz * tz));
    dt[0] += sa->mean2d[0] * fx / tz;
    dt[1] += sa->mean2d[1] * fy / tz;
    dt[2] += -sa->mean2d[0] * fx * tx / (tz * tz) - sa->mean2d[1] * fy * ty / (tz * tz);
    /* t = W mu + t_v */
    for (int k = 0; k < 3; ++k) gmu[k] += W[k] * dt[0] + W[3 + k] * dt[1] + W[6 + k] * dt[2];
    for (int k = 0; k < 3; ++k) add_grad(g->means, 3 * i + k, gmu[k]);

    /* Sigma = R diag(s^2) R^T */
    const double *sc = s->scales + 3 * i;
    const double *Rq = f->Rq;
    double dR[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += (dSig[3 * r + k] + dSig[3 * k + r]) * Rq[3 * k + c];
            dR[3 * r + c] = acc * sc[c] * sc[c];
        }
    for (int c = 0; c < 3; ++c) {
        double acc = 0.0;   /* (R^T dSig R)_cc */
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k) acc += Rq[3 * r + c] * dSig[3 * r + k] * Rq[3 * k + c];
        add_grad(g->scales, 3 * i + c, 2.0 * sc[c] * acc);
    }
    /* rotation matrix entries as functions of the normalised quaternion */
    double w = f->qn[0], x = f->qn[1], y = f->qn[2], z = f->qn[3];
    double dq[4];
    dq[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] - 2.0 * x * dR[8]);
    dq[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] - 2.0 * y * dR[8]);
    dq[3] = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * z * dR[4] + y * dR[5] + x * dR[6] + y * dR[7]);
    /* q_n = q/|q| */
    double qd = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
    for (int k = 0; k < 4; ++k) add_grad(g->quats, 4 * i + k, (dq[k] - f->qn[k] * qd) / f->qnorm);
}


/* Number of parameters of one splat, in the order means(3) scales(3)
 * quats(4) opacity beta diffuse(3) lobe_angles(2m) lobe_colors(3m)
 * lobe_betas(m). */
static int n_params(int m) { return 15 + 6 * m; }

static void splat_params_get(const ob_grads *g, int64_t i, int m, double *out)
{
    int k = 0;
    for (int c = 0; c < 3; ++c) out[k++] = g->means[3 * i + c];
    for (int c = 0; c < 3; ++c) out[k++] = g->scales[3 * i + c];
    for (int c = 0; c < 4; ++c) out[k++] = g->quats[4 * i + c];
    out[k++] = g->opacities[i];
    out[k++] = g->betas[i];
    for (int c = 0; c < 3; ++c) out[k++] = g->diffuse[3 * i + c];
    for (int c = 0; c < 2 * m; ++c) out[k++] = g->lobe_angles[2 * m * i + c];
    for (int c = 0; c < 3 * m; ++c) out[k++] = g->lobe_colors[3 * m * i + c];
    for (int c = 0; c < m; ++c) out[k++] = g->lobe_betas[m * i + c];
}

static void splat_params_add(ob_grads *g, int64_t i, int m, const double *v)
{
    int k = 0;
    for (int c = 0; c < 3; ++c) g->means[3 * i + c] += v[k++];
    for (int c = 0; c < 3; ++c) g->scales[3 * i + c] += v[k++];
    for (int c = 0; c < 4; ++c) g->quats[4 * i + c] += v[k++];
    g->opacities[i] += v[k++];
    g->betas[i] += v[k++];
    for (int c = 0; c < 3; ++c) g->diffuse[3 * i + c] += v[k++];
    for (int c = 0; c < 2 * m; ++c) g->lobe_angles[2 * m * i + c] += v[k++];
    for (int c = 0; c < 3 * m; ++c) g->lobe_colors[3 * m * i + c] += v[k++];
    for (int c = 0; c < m; ++c) g->lobe_betas[m * i + c] += v[k++];
}

/* Jacobian [n_params][10] of splat i's parameter adjoints with respect to its
 * ten screen-space adjoints (mean2d 2, G 3, opacity, b, colour 3), by running
 * the (linear) reverse chain on unit vectors.  `scratch` holds zeros for
 * splat i on entry and on exit. */
static void splat_jacobian(const ob_splats *s, int64_t i, const ob_camera *cam, const ob_fwd *f,
                           ob_grads *scratch, double *J)
{
    const int q = n_params(s->m);
    double *col = (double *)malloc(sizeof(double) * (size_t)q);
    for (int j = 0; j < 10; ++j) {
        ob_screen_adj e;
        memset(&e, 0, sizeof(e));
        ((double *)&e)[j] = 1.0;
        chain_one(s, i, cam, f, &e, scratch);
        splat_params_get(scratch, i, s->m, col);
        for (int p = 0; p < q; ++p) {
            J[p * 10 + j] = col[p];
            col[p] = -col[p];
        }
        splat_params_add(scratch, i, s->m, col);   /* x + (-x) = 0 exactly */
    }
    free(col);
}

/* Gradient of L = sum_p dL_drgb[p] . rgb[p] over the listed pixels.
 * grads are ACCUMULATED (+=).  abs_sum (may be NULL) receives, per parameter
 * p, the error scale sum over pixels and screen-space adjoints j of
 * |J_pj| |s_j(pixel)|, with J the Jacobian of the reverse chain from the ten
 * screen-space adjoints of the splat to its parameters: a computation that
 * sums the per-pixel screen-space adjoints in finite precision and then
 * applies the chain has an error bounded by a multiple of it.  abs_contrib
 * (may be NULL) receives the smaller scale sum over pixels of
 * |sum_j J_pj s_j(pixel)|, the magnitude of each pixel's own contribution to
 * the gradient of p. */
int ob_render_bwd(const ob_splats *s, const ob_camera *cam, double alpha_max, double t_eps,
                  int64_t npix, const int32_t *pix_xy, const double *dL_drgb,
                  ob_grads *grads, ob_grads *abs_sum, ob_grads *abs_contrib)
{
    ob_scene sc;
    if (s->sh) return -2;  /* the comparison mode is forward only */
    if (scene_build(s, cam, &sc)) return -1;
    int64_t cap = sc.n_order > 0 ? sc.n_order : 1;
    int64_t chunk = 256;
    const int q = n_params(s->m);
    double **jac = NULL;
    ob_grads scratch;
    memset(&scratch, 0, sizeof(scratch));
    const int want_j = abs_sum != NULL || abs_contrib != NULL;
    if (want_j) {
        size_t n1 = (size_t)(s->n > 0 ? s->n : 1);
        size_t m1 = (size_t)(s->m > 0 ? s->m : 1);
        jac = (double **)calloc(n1, sizeof(double *));
        scratch.means = (double *)calloc(3 * n1, sizeof(double));
        scratch.scales = (double *)calloc(3 * n1, sizeof(double));
        scratch.quats = (double *)calloc(4 * n1, sizeof(double));
        scratch.opacities = (double *)calloc(n1, sizeof(double));
        scratch.betas = (double *)calloc(n1, sizeof(double));
        scratch.diffuse = (double *)calloc(3 * n1, sizeof(double));
        scratch.lobe_angles = (double *)calloc(2 * n1 * m1, sizeof(double));
        scratch.lobe_colors = (double *)calloc(3 * n1 * m1, sizeof(double));
        scratch.lobe_betas = (double *)calloc(n1 * m1, sizeof(double));
    }
    double *absv = (double *)malloc(sizeof(double) * (size_t)q);
    double *absc = (double *)malloc(sizeof(double) * (size_t)q);
    ob_step *steps = (ob_step *)malloc(sizeof(ob_step) * (size_t)cap * (size_t)chunk);
    int64_t *nsteps = (int64_t *)malloc(sizeof(int64_t) * (size_t)chunk);
    double *Tfin = (double *)malloc(sizeof(double) * (size_t)chunk);
    if (!steps || !nsteps || !Tfin) { free(steps); free(nsteps); free(Tfin); scene_free(&sc); return -1; }

    for (int64_t p0 = 0; p0 < npix; p0 += chunk) {
        int64_t pc = npix - p0 < chunk ? npix - p0 : chunk;
        /* forward lists, in parallel */
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t pp = 0; pp < pc; ++pp) {
            int64_t p = p0 + pp;
            double rgb[3], T;
            int64_t last;
            nsteps[pp] = composite_pixel(s, &sc, pix_xy[2 * p] + 0.5, pix_xy[2 * p + 1] + 0.5,
                                         alpha_max, t_eps, rgb, &T, NULL, &last, steps + pp * cap);
            Tfin[pp] = T;
        }
        /* reverse mode, serial (parameter gradients are shared) */
        for (int64_t pp = 0; pp < pc; ++pp) {
            int64_t p = p0 + pp;
            const double *gp = dL_drgb + 3 * p;
            const ob_step *st = steps + pp * cap;
            /* out = C + T_final bg  ->  adjoint of the running transmittance */
            double adjT = gp[0] * cam->bg[0] + gp[1] * cam->bg[1] + gp[2] * cam->bg[2];
            for (int64_t k = nsteps[pp] - 1; k >= 0; --k) {
                const ob_step *e = &st[k];
                const ob_fwd *f = &sc.fw[e->id];
                double gc = gp[0] * f->color[0] + gp[1] * f->color[1] + gp[2] * f->color[2];
                ob_screen_adj sa;
                memset(&sa, 0, sizeof(sa));
                for (int c = 0; c < 3; ++c) sa.color[c] = gp[c] * e->alpha * e->T;
                /* C_{k+1} = C_k + c a T_k ;  T_{k+1} = T_k (1 - a) */
                double adj_a = gc * e->T - adjT * e->T;
                adjT = adjT * (1.0 - e->alpha) + gc * e->alpha;
                if (!e->clamped) {
                    double o = s->opacities[e->id];
                    sa.opacity = adj_a * e->B;
                    /* B = (1 - r2)^beta,  beta = 4 e^b */
                    sa.b = adj_a * o * e->B * log(1.0 - e->r2) * f->beta;
                    double adj_r2 = adj_a * o * (-f->beta) * pow(1.0 - e->r2, f->beta - 1.0);
                    /* r2 = d^T A d,  d = p - mu' */
                    sa.G[0] = adj_r2 * e->dx * e->dx;
                    sa.G[1] = adj_r2 * e->dx * e->dy;
                    sa.G[2] = adj_r2 * e->dy * e->dy;
                    sa.mean2d[0] = -adj_r2 * 2.0 * (f->conic[0] * e->dx + f->conic[1] * e->dy);
                    sa.mean2d[1] = -adj_r2 * 2.0 * (f->conic[1] * e->dx + f->conic[2] * e->dy);
                }
                chain_one(s, e->id, cam, f, &sa, grads);
                if (want_j) {
                    if (!jac[e->id]) {
                        jac[e->id] = (double *)malloc(sizeof(double) * (size_t)q * 10);
                        splat_jacobian(s, e->id, cam, f, &scratch, jac[e->id]);
                    }
                    const double *J = jac[e->id];
                    const double *sv = (const double *)&sa;
                    for (int pp2 = 0; pp2 < q; ++pp2) {
                        double acc = 0.0, con = 0.0;
                        for (int j = 0; j < 10; ++j) {
                            acc += fabs(J[pp2 * 10 + j]) * fabs(sv[j]);
                            con += J[pp2 * 10 + j] * sv[j];
                        }
                        absv[pp2] = acc;
                        absc[pp2] = fabs(con);
                    }
                    if (abs_sum) splat_params_add(abs_sum, e->id, s->m, absv);
                    if (abs_contrib) splat_params_add(abs_contrib, e->id, s->m, absc);
                }
            }
        }
    }
    if (want_j) {
        for (int64_t i = 0; i < s->n; ++i) free(jac[i]);
        free(jac);
        free(scratch.means); free(scratch.scales); free(scratch.quats); free(scratch.opacities);
        free(scratch.betas); free(scratch.diffuse); free(scratch.lobe_angles); free(scratch.lobe_colors);
        free(scratch.lobe_betas);
    }
    free(absv);
    free(absc);
    free(steps); free(nsteps); free(Tfin);
    scene_free(&sc);
    return 0;
}

/* Threads the OpenMP loops use (n >= 1); returns the resulting maximum.  For
 * timing the oracle on a chosen number of host cores. */
int ob_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Tile binning rule (integer).  A width x height image is cut into
 * tile_w x tile_h tiles with row-major tile ids.  A splat belongs to every
 * tile its inclusive pixel box (x_lo, x_hi, y_lo, y_hi) overlaps; culled
 * splats and empty boxes belong to none.  Each tile lists its splats by
 * ascending (depth_key, splat id). */
typedef struct { int64_t tile; uint32_t key; int64_t id; } ob_pair;

static int cmp_pair(const void *a, const void *b)
{
    const ob_pair *x = (const ob_pair *)a, *y = (const ob_pair *)b;
    if (x->tile != y->tile) return x->tile < y->tile ? -1 : 1;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* All tiles: emit every (tile, splat) pair, then sort lexicographically.
 * tile_start [n_tiles + 1] receives offsets into ids [capacity].
 * Returns the number of pairs, -1 on allocation failure, -2 if it exceeds
 * capacity (tile_start is still complete in that case). */
int64_t ob_bin(int64_t n, const int32_t *valid, const int32_t *bbox, const uint32_t *depth_key,
               int32_t width, int32_t height, int32_t tile_w, int32_t tile_h,
               int64_t capacity, int64_t *tile_start, int64_t *ids)
{
    int64_t tiles_x = (width + tile_w - 1) / tile_w, tiles_y = (height + tile_h - 1) / tile_h;
    int64_t n_tiles = tiles_x * tiles_y;
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *b = bbox + 4 * i;
        if (!valid[i] || b[0] > b[1] || b[2] > b[3]) continue;
        total += (int64_t)(b[1] / tile_w - b[0] / tile_w + 1) * (b[3] / tile_h - b[2] / tile_h + 1);
    }
    ob_pair *pairs = (ob_pair *)malloc(sizeof(ob_pair) * (size_t)(total > 0 ? total : 1));
    if (!pairs) return -1;
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *b = bbox + 4 * i;
        if (!valid[i] || b[0] > b[1] || b[2] > b[3]) continue;
        for (int64_t ty = b[2] / tile_h; ty <= b[3] / tile_h; ++ty)
            for (int64_t tx = b[0] / tile_w; tx <= b[1] / tile_w; ++tx) {
                pairs[k].tile = ty * tiles_x + tx;
                pairs[k].key = depth_key[i];
                pairs[k].id = i;
                ++k;
            }
    }
    qsort(pairs, (size_t)total, sizeof(ob_pair), cmp_pair);
    int64_t j = 0;
    for (int64_t t = 0; t < n_tiles; ++t) {
        tile_start[t] = j;
        while (j < total && pairs[j].tile == t) ++j;
    }
    tile_start[n_tiles] = total;
    for (int64_t q = 0; q < total && q < capacity; ++q) ids[q] = pairs[q].id;
    free(pairs);
    return total > capacity ? -2 : total;
}

/* Requested tiles only, by brute force over all splats for each tile (for
 * spot checks on large inputs).  list_start [n_req + 1], ids [capacity]. */
int64_t ob_bin_tiles(int64_t n, const int32_t *valid, const int32_t *bbox, const uint32_t *depth_key,
                     int32_t width, int32_t tile_w, int32_t tile_h,
                     int64_t n_req, const int64_t *tiles, int64_t capacity,
                     int64_t *list_start, int64_t *ids)
{
    int64_t tiles_x = (width + tile_w - 1) / tile_w;
    ob_sortrec *buf = (ob_sortrec *)malloc(sizeof(ob_sortrec) * (size_t)(n > 0 ? n : 1));
    if (!buf) return -1;
    int64_t total = 0;
    for (int64_t r = 0; r < n_req; ++r) {
        int64_t tx = tiles[r] % tiles_x, ty = tiles[r] / tiles_x;
        int64_t x0 = tx * tile_w, x1 = x0 + tile_w - 1, y0 = ty * tile_h, y1 = y0 + tile_h - 1;
        int64_t k = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int32_t *b = bbox + 4 * i;
            if (!valid[i] || b[0] > b[1] || b[2] > b[3]) continue;
            if (b[1] < x0 || b[0] > x1 || b[3] < y0 || b[2] > y1) continue;
            buf[k].key = depth_key[i];
            buf[k].id = i;
            ++k;
        }
        qsort(buf, (size_t)k, sizeof(ob_sortrec), cmp_sortrec);
        list_start[r] = total;
        for (int64_t j = 0; j < k; ++j)
            if (total + j < capacity) ids[total + j] = buf[j].id;
        total += k;
    }
    list_start[n_req] = total;
    free(buf);
    return total > capacity ? -2 : total;
}
