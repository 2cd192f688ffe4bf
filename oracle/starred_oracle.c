/*
 * starred_oracle.c -- plain FP64 CPU oracle for the STARRED loss and gradient.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call
 * this file: only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it. It shares no source with the HIP library.
 *
 * Every function is the direct definition of what the paper's method computes
 * (Millon et al., "Image deconvolution and PSF reconstruction with STARRED"),
 * written out in double precision with no blocking, fusion or FFT:
 *
 *   deconvolution mode, Sec. 2.2, Eqs. (8)-(11):
 *     f_i = Gamma_i + h + sum_k a_ki r_k                     (Eq. 9)
 *     m_i = D S_i f_i                                        (Eq. 8, 10)
 *     L   = 1/2 sum_i (d_i - m_i)^T C^-1 (d_i - m_i)          (Eq. 10, C diagonal)
 *         + lambda || W o Phi^T h ||_1                        (Eq. 11, first two terms)
 *   PSF mode, Sec. 2.1, Eqs. (2)-(7):
 *     s   = moffat(eta_M) + b                                (Eq. 2)
 *     m_k = D (s * a_k r_k)                                  (Eq. 3)
 *     L   = 1/2 sum_k (t_k - m_k)^T C^-1 (t_k - m_k) + lambda || W o Phi^T b ||_1   (Eqs. 4-6)
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - r: Gaussian of FWHM 2 fine pixels (Sec. 2.1, Eq. 1), point-sampled at pixel
 *     centres, unit integral, untruncated. Fine pixel (y,x) has centre (x,y).
 *   - S_i: linear 'same' convolution, zero padding, kernel centre floor(K/2).
 *   - D: block sum over s x s fine pixels (flux conserving).
 *   - Phi^T: isotropic undecimated a-trous starlet with the B3 spline filter
 *     [1,4,6,4,1]/16 at dilation 2^j, whole-sample mirror boundary; J planes
 *     counting the coarse one.  sgn(0) = 0 for the L1 subgradient.
 *   - Frame i of data side n_i sees the central window of h with offset
 *     o_i = (N - s n_i)/2.
 *   - Moffat: A (1 + (u/ax)^2 + (v/ay)^2)^-beta with (u,v) the offset from the grid
 *     centre floor(N/2) rotated by phi.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Target Gaussian r (Sec. 2.1, Eq. 1 and Eq. 3)                              */
/* ------------------------------------------------------------------------- */

double ora_sigma_from_fwhm(double fwhm) { return fwhm / (2.0 * sqrt(2.0 * log(2.0))); }

/* r(x - cx, y - cy): isotropic Gaussian, unit integral over the plane. */
static double gauss2(double dx, double dy, double sigma)
{
    return exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma)) / (2.0 * ORA_PI * sigma * sigma);
}

/* 1-D factor of r: r(dx,dy) = g(dx) g(dy). */
static double gauss1(double t, double sigma)
{
    return exp(-(t * t) / (2.0 * sigma * sigma)) / (sqrt(2.0 * ORA_PI) * sigma);
}

/* ------------------------------------------------------------------------- */
/* Frame layout                                                               */
/* ------------------------------------------------------------------------- */

/* Window offset of each frame inside h; returns -1 if a frame does not fit. */
int ora_frame_offsets(int E, const int *n, int s, int N, int *o)
{
    for (int i = 0; i < E; ++i) {
        int fine = s * n[i];
        if (fine > N || ((N - fine) % 2) != 0) return -1;
        o[i] = (N - fine) / 2;
    }
    return 0;
}

static long fine_offset(int E, const int *n, int s, int upto)
{
    long off = 0;
    for (int i = 0; i < upto && i < E; ++i) off += (long)(s * n[i]) * (s * n[i]);
    return off;
}

static long data_offset(const int *n, int upto)
{
    long off = 0;
    for (int i = 0; i < upto; ++i) off += (long)n[i] * n[i];
    return off;
}

static long kern_offset(const int *K, int upto)
{
    long off = 0;
    for (int i = 0; i < upto; ++i) off += (long)K[i] * K[i];
    return off;
}

/* ------------------------------------------------------------------------- */
/* Scene rendering (Sec. 2.2, Eq. 9)                                          */
/* params = [h N^2 | Gamma E | a E*M (epoch-major) | c M*2 (cx, cy)]          */
/* ------------------------------------------------------------------------- */

void ora_render_scene(int E, const int *n, int s, int N, int M, double fwhm,
                      const double *params, double *scene)
{
    const double *h = params;
    const double *Gam = params + (long)N * N;
    const double *a = Gam + E;
    const double *c = a + (long)E * M;
    double sigma = ora_sigma_from_fwhm(fwhm);
    int *o = (int *)malloc(sizeof(int) * (E > 0 ? E : 1));
    ora_frame_offsets(E, n, s, N, o);
    for (int i = 0; i < E; ++i) {
        int F = s * n[i];
        double *f = scene + fine_offset(E, n, s, i);
        for (int y = 0; y < F; ++y)
            for (int x = 0; x < F; ++x) {
                int Y = y + o[i], X = x + o[i];
                double v = Gam[i] + h[(long)Y * N + X];
                for (int k = 0; k < M; ++k)
                    v += a[(long)i * M + k] * gauss2(X - c[2 * k], Y - c[2 * k + 1], sigma);
                f[(long)y * F + x] = v;
            }
    }
    free(o);
}

/* ------------------------------------------------------------------------- */
/* S_i then D (Eq. 8): 'same' convolution with zero padding, centre floor(K/2), */
/* then block sum over s x s.                                                  */
/* ------------------------------------------------------------------------- */

/* u = k (*) f, both square, f of side F, k of side K. */
static void conv_same(const double *f, int F, const double *k, int K, double *u)
{
    int kap = K / 2;
    for (int y = 0; y < F; ++y)
        for (int x = 0; x < F; ++x) {
            double acc = 0.0;
            for (int v = 0; v < K; ++v) {
                int yy = y - v + kap;
                if (yy < 0 || yy >= F) continue;
                for (int uu = 0; uu < K; ++uu) {
                    int xx = x - uu + kap;
                    if (xx < 0 || xx >= F) continue;
                    acc += k[(long)v * K + uu] * f[(long)yy * F + xx];
                }
            }
            u[(long)y * F + x] = acc;
        }
}

/* transpose of conv_same: g(y,x) = sum_{v,u} k(v,u) gh(y + v - kap, x + u - kap) */
static void corr_same(const double *gh, int F, const double *k, int K, double *g)
{
    int kap = K / 2;
    for (int y = 0; y < F; ++y)
        for (int x = 0; x < F; ++x) {
            double acc = 0.0;
            for (int v = 0; v < K; ++v) {
                int yy = y + v - kap;
                if (yy < 0 || yy >= F) continue;
                for (int uu = 0; uu < K; ++uu) {
                    int xx = x + uu - kap;
                    if (xx < 0 || xx >= F) continue;
                    acc += k[(long)v * K + uu] * gh[(long)yy * F + xx];
                }
            }
            g[(long)y * F + x] = acc;
        }
}

/* D: data pixel (p,q) sums fine pixels [s p, s p + s) x [s q, s q + s). */
static void block_sum(const double *u, int n, int s, double *m)
{
    int F = s * n;
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) {
            double acc = 0.0;
            for (int aa = 0; aa < s; ++aa)
                for (int bb = 0; bb < s; ++bb) acc += u[(long)(s * p + aa) * F + s * q + bb];
            m[(long)p * n + q] = acc;
        }
}

/* D^T: every fine pixel of a block receives the data pixel's value. */
static void block_sum_adj(const double *r, int n, int s, double *gh)
{
    int F = s * n;
    for (int y = 0; y < F; ++y)
        for (int x = 0; x < F; ++x) gh[(long)y * F + x] = r[(long)(y / s) * n + (x / s)];
}

void ora_conv_sub(int E, const int *n, const int *K, int s, const double *kernels,
                  const double *scene, double *model)
{
    int i;
#pragma omp parallel for schedule(dynamic)
    for (i = 0; i < E; ++i) {
        int F = s * n[i];
        double *u = (double *)malloc(sizeof(double) * F * F);
        conv_same(scene + fine_offset(E, n, s, i), F, kernels + kern_offset(K, i), K[i], u);
        block_sum(u, n[i], s, model + data_offset(n, i));
        free(u);
    }
}

void ora_conv_sub_adj(int E, const int *n, const int *K, int s, const double *kernels,
                      const double *resid, double *grad_scene)
{
    int i;
#pragma omp parallel for schedule(dynamic)
    for (i = 0; i < E; ++i) {
        int F = s * n[i];
        double *gh = (double *)malloc(sizeof(double) * F * F);
        block_sum_adj(resid + data_offset(n, i), n[i], s, gh);
        corr_same(gh, F, kernels + kern_offset(K, i), K[i], grad_scene + fine_offset(E, n, s, i));
        free(gh);
    }
}

/* ------------------------------------------------------------------------- */
/* Starlet transform Phi^T and its adjoint Phi (Eqs. 6, 11; Starck et al.)    */
/* ------------------------------------------------------------------------- */

static int mirror(int i, int N)
{
    if (i < 0) i = -i;
    if (i > N - 1) i = 2 * (N - 1) - i;
    return i;
}

static const double B3[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};

/* out = H_j in: B3 taps at offsets {-2..2} * 2^j along rows, then along columns. */
static void starlet_smooth(const double *in, int N, int j, double *out, double *tmp)
{
    int d = 1 << j;
    for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x) {
            double acc = 0.0;
            for (int t = -2; t <= 2; ++t) acc += B3[t + 2] * in[(long)y * N + mirror(x + t * d, N)];
            tmp[(long)y * N + x] = acc;
        }
    for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x) {
            double acc = 0.0;
            for (int t = -2; t <= 2; ++t) acc += B3[t + 2] * tmp[(long)mirror(y + t * d, N) * N + x];
            out[(long)y * N + x] = acc;
        }
}

/* out = H_j^T in, written as the scatter of every tap of H_j (the literal transpose). */
static void starlet_smooth_T(const double *in, int N, int j, double *out, double *tmp)
{
    int d = 1 << j;
    long NN = (long)N * N;
    /* transpose of the column pass first */
    for (long p = 0; p < NN; ++p) tmp[p] = 0.0;
    for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x)
            for (int t = -2; t <= 2; ++t)
                tmp[(long)mirror(y + t * d, N) * N + x] += B3[t + 2] * in[(long)y * N + x];
    /* then the transpose of the row pass */
    for (long p = 0; p < NN; ++p) out[p] = 0.0;
    for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x)
            for (int t = -2; t <= 2; ++t)
                out[(long)y * N + mirror(x + t * d, N)] += B3[t + 2] * tmp[(long)y * N + x];
}

/* coeffs: J planes of N^2. alpha_j = c_j - c_{j+1} (j < J-1), alpha_{J-1} = c_{J-1},
 * with c_0 = img and c_{j+1} = H_j c_j. */
void ora_starlet_fwd(int N, int J, const double *img, double *coeffs)
{
    long NN = (long)N * N;
    double *c = (double *)malloc(sizeof(double) * NN);
    double *cn = (double *)malloc(sizeof(double) * NN);
    double *tmp = (double *)malloc(sizeof(double) * NN);
    memcpy(c, img, sizeof(double) * NN);
    for (int j = 0; j < J - 1; ++j) {
        starlet_smooth(c, N, j, cn, tmp);
        for (long p = 0; p < NN; ++p) coeffs[j * NN + p] = c[p] - cn[p];
        memcpy(c, cn, sizeof(double) * NN);
    }
    memcpy(coeffs + (long)(J - 1) * NN, c, sizeof(double) * NN);
    free(c);
    free(cn);
    free(tmp);
}

/* img = Phi z = sum_j A_j^T z_j, with A_j = P_j - P_{j+1} (j < J-1), A_{J-1} = P_{J-1},
 * P_j = H_{j-1} ... H_0 (P_0 = I).  P_j^T z = H_0^T ( ... H_{j-1}^T z). Each term is
 * computed on its own, the plain sum of transposes. */
void ora_starlet_adj(int N, int J, const double *coeffs, double *img)
{
    long NN = (long)N * N;
    double *acc = (double *)calloc(NN, sizeof(double));
    double *w = (double *)malloc(sizeof(double) * NN);
    double *w2 = (double *)malloc(sizeof(double) * NN);
    double *tmp = (double *)malloc(sizeof(double) * NN);
    for (int j = 0; j < J; ++j) {
        const double *z = coeffs + (long)j * NN;
        /* + P_j^T z_j */
        memcpy(w, z, sizeof(double) * NN);
        for (int l = j - 1; l >= 0; --l) {
            starlet_smooth_T(w, N, l, w2, tmp);
            memcpy(w, w2, sizeof(double) * NN);
        }
        for (long p = 0; p < NN; ++p) acc[p] += w[p];
        if (j < J - 1) {
            /* - P_{j+1}^T z_j */
            memcpy(w, z, sizeof(double) * NN);
            for (int l = j; l >= 0; --l) {
                starlet_smooth_T(w, N, l, w2, tmp);
                memcpy(w, w2, sizeof(double) * NN);
            }
            for (long p = 0; p < NN; ++p) acc[p] -= w[p];
        }
    }
    memcpy(img, acc, sizeof(double) * NN);
    free(acc);
    free(w);
    free(w2);
    free(tmp);
}

static double sgn(double v) { return (v > 0.0) - (v < 0.0); }

/* L1 prior lambda * sum W o |alpha| and its subgradient z = lambda W sgn(alpha)
 * (Eq. 6).  W has J entries (w_stride 0) or J*N*N (w_stride 1).  sgn_override,
 * if given, holds -1/0/+1 to use in place of sgn(alpha) or 2 to keep it. */
static double l1_prior(int N, int J, const double *alpha, const double *W, int w_stride,
                       double lambda, const signed char *sgn_override, double *z)
{
    long NN = (long)N * N;
    double L = 0.0;
    for (int j = 0; j < J; ++j)
        for (long p = 0; p < NN; ++p) {
            double wj = w_stride ? W[j * NN + p] : W[j];
            double a = alpha[j * NN + p];
            L += lambda * wj * fabs(a);
            if (z) {
                double sg = sgn(a);
                if (sgn_override && sgn_override[j * NN + p] != 2) sg = sgn_override[j * NN + p];
                z[j * NN + p] = lambda * wj * sg;
            }
        }
    return L;
}

/* ------------------------------------------------------------------------- */
/* Deconvolution loss and gradient (Eqs. 9-11)                                */
/* loss[0] = 1/2 chi^2, loss[1] = L1 term, loss[2] = total.  grad may be NULL. */
/* ------------------------------------------------------------------------- */

void ora_loss_grad(int E, const int *n, const int *K, int s, int N, int M, int J,
                   int w_stride, double lambda, double fwhm,
                   const double *data, const double *invvar, const double *kernels,
                   const double *W, const double *params, double *grad, double *loss,
                   const signed char *sgn_override)
{
    long NN = (long)N * N;
    long nfine = fine_offset(E, n, s, E);
    long ndata = data_offset(n, E);
    double sigma = ora_sigma_from_fwhm(fwhm);
    int *o = (int *)malloc(sizeof(int) * (E > 0 ? E : 1));
    ora_frame_offsets(E, n, s, N, o);

    double *scene = (double *)malloc(sizeof(double) * (nfine > 0 ? nfine : 1));
    double *model = (double *)malloc(sizeof(double) * (ndata > 0 ? ndata : 1));
    double *rho = (double *)malloc(sizeof(double) * (ndata > 0 ? ndata : 1));
    ora_render_scene(E, n, s, N, M, fwhm, params, scene);
    ora_conv_sub(E, n, K, s, kernels, scene, model);

    /* Eq. (10): 1/2 sum_i (d_i - m_i)^T C^-1 (d_i - m_i), C^-1 = diag(invvar) */
    double chi = 0.0;
    for (long p = 0; p < ndata; ++p) {
        double r = model[p] - data[p];
        rho[p] = invvar[p] * r;
        chi += 0.5 * invvar[p] * r * r;
    }

    double *alpha = (double *)malloc(sizeof(double) * J * NN);
    double *z = (double *)malloc(sizeof(double) * J * NN);
    ora_starlet_fwd(N, J, params, alpha);
    double l1 = l1_prior(N, J, alpha, W, w_stride, lambda, sgn_override, z);
    loss[0] = chi;
    loss[1] = l1;
    loss[2] = chi + l1;

    if (grad) {
        const double *a = params + NN + E;
        const double *c = a + (long)E * M;
        double *gh = grad;
        double *gG = grad + NN;
        double *ga = gG + E;
        double *gc = ga + (long)E * M;
        double *gscene = (double *)malloc(sizeof(double) * (nfine > 0 ? nfine : 1));
        ora_conv_sub_adj(E, n, K, s, kernels, rho, gscene);

        for (long p = 0; p < NN; ++p) gh[p] = 0.0;
        for (long q = 0; q < 2L * M; ++q) gc[q] = 0.0;
        for (int i = 0; i < E; ++i) {
            int F = s * n[i];
            const double *g = gscene + fine_offset(E, n, s, i);
            double sG = 0.0;
            for (int y = 0; y < F; ++y)
                for (int x = 0; x < F; ++x) {
                    gh[(long)(y + o[i]) * N + (x + o[i])] += g[(long)y * F + x];
                    sG += g[(long)y * F + x];
                }
            gG[i] = sG;
            for (int k = 0; k < M; ++k) {
                double sa = 0.0, scx = 0.0, scy = 0.0;
                for (int y = 0; y < F; ++y)
                    for (int x = 0; x < F; ++x) {
                        double X = x + o[i], Y = y + o[i];
                        double r = gauss2(X - c[2 * k], Y - c[2 * k + 1], sigma);
                        double gv = g[(long)y * F + x];
                        sa += gv * r;
                        scx += gv * r * (X - c[2 * k]) / (sigma * sigma);
                        scy += gv * r * (Y - c[2 * k + 1]) / (sigma * sigma);
                    }
                ga[(long)i * M + k] = sa;
                gc[2 * k] += a[(long)i * M + k] * scx;
                gc[2 * k + 1] += a[(long)i * M + k] * scy;
            }
        }
        /* prior gradient Phi z added to the h block */
        double *pz = (double *)malloc(sizeof(double) * NN);
        ora_starlet_adj(N, J, z, pz);
        for (long p = 0; p < NN; ++p) gh[p] += pz[p];
        free(pz);
        free(gscene);
    }
    free(alpha);
    free(z);
    free(scene);
    free(model);
    free(rho);
    free(o);
}

/* ------------------------------------------------------------------------- */
/* Eq. 11, third term, and its App. C estimate                               */
/* ------------------------------------------------------------------------- */

/* P = sum_k <a_k> r_k on the N x N grid, <a_k> the mean of a_ik over the epochs. */
static void pts_image(int E, int N, int M, double fwhm, const double *params, double *P, double *amean)
{
    const double *a = params + (long)N * N + E;
    const double *c = a + (long)E * M;
    const double sigma = ora_sigma_from_fwhm(fwhm);
    for (int k = 0; k < M; ++k) {
        double m = 0.0;
        for (int i = 0; i < E; ++i) m += a[(long)i * M + k];
        amean[k] = m / E;
    }
    for (int Y = 0; Y < N; ++Y)
        for (int X = 0; X < N; ++X) {
            double v = 0.0;
            for (int k = 0; k < M; ++k) v += amean[k] * gauss2(X - c[2 * k], Y - c[2 * k + 1], sigma);
            P[(long)Y * N + X] = v;
        }
}

/* lam_pts || W (.) Phi^T P ||_1 added to loss[1] and loss[2]; with grad, its
 * gradient: dL/da_ik = <Phi z, r_k> / E for every epoch i, dL/dc_k =
 * <a_k> <Phi z, dr_k/dc_k>, z = lam_pts W sgn(Phi^T P) (sgn_override as in the
 * h prior). */
void ora_pts_term(int E, int N, int M, int J, int w_stride, double lam_pts, double fwhm, const double *W,
                  const double *params, double *grad, double *loss, const signed char *sgn_override)
{
    long NN = (long)N * N;
    double *P = (double *)malloc(sizeof(double) * NN);
    double *amean = (double *)malloc(sizeof(double) * (M > 0 ? M : 1));
    double *alpha = (double *)malloc(sizeof(double) * J * NN);
    double *z = (double *)malloc(sizeof(double) * J * NN);
    pts_image(E, N, M, fwhm, params, P, amean);
    ora_starlet_fwd(N, J, P, alpha);
    const double L = l1_prior(N, J, alpha, W, w_stride, lam_pts, sgn_override, z);
    loss[1] += L;
    loss[2] += L;
    if (grad) {
        const double *c = params + NN + E + (long)E * M;
        const double sigma = ora_sigma_from_fwhm(fwhm);
        double *ga = grad + NN + E, *gc = ga + (long)E * M;
        double *q = (double *)malloc(sizeof(double) * NN);
        ora_starlet_adj(N, J, z, q);
        for (int k = 0; k < M; ++k) {
            double da = 0.0, dcx = 0.0, dcy = 0.0;
            for (int Y = 0; Y < N; ++Y)
                for (int X = 0; X < N; ++X) {
                    const double r = gauss2(X - c[2 * k], Y - c[2 * k + 1], sigma);
                    const double qv = q[(long)Y * N + X];
                    da += qv * r;
                    dcx += qv * r * (X - c[2 * k]) / (sigma * sigma);
                    dcy += qv * r * (Y - c[2 * k + 1]) / (sigma * sigma);
                }
            for (int i = 0; i < E; ++i) ga[(long)i * M + k] += da / E;
            gc[2 * k] += amean[k] * dcx;
            gc[2 * k + 1] += amean[k] * dcy;
        }
        free(q);
    }
    free(P);
    free(amean);
    free(alpha);
    free(z);
}

/* App. C: lambda_pts = lambda (||W (.) Phi^T f||_1 - ||W (.) Phi^T h||_1)
 *                      / sum_k <a_k> ||W (.) Phi^T r_k||_1,
 * f the epoch average of the scene on the N x N grid (<Gamma> + h + sum_k <a_k> r_k).
 * The printed formula also multiplies the h norm by lambda; the text describes the
 * difference of the two image norms, which is what is computed here. */
double ora_lambda_pts_estimate(int E, int N, int M, int J, int w_stride, double lambda, double fwhm,
                               const double *W, const double *params)
{
    long NN = (long)N * N;
    const double *h = params, *Gam = params + NN, *c = params + NN + E + (long)E * M;
    const double sigma = ora_sigma_from_fwhm(fwhm);
    double *img = (double *)malloc(sizeof(double) * NN);
    double *amean = (double *)malloc(sizeof(double) * (M > 0 ? M : 1));
    double *alpha = (double *)malloc(sizeof(double) * J * NN);
    double gm = 0.0;
    for (int i = 0; i < E; ++i) gm += Gam[i];
    gm /= E;
    pts_image(E, N, M, fwhm, params, img, amean);
    for (long p = 0; p < NN; ++p) img[p] += gm + h[p];
    ora_starlet_fwd(N, J, img, alpha);
    const double Lf = l1_prior(N, J, alpha, W, w_stride, 1.0, NULL, NULL);
    ora_starlet_fwd(N, J, h, alpha);
    const double Lh = l1_prior(N, J, alpha, W, w_stride, 1.0, NULL, NULL);
    double den = 0.0;
    for (int k = 0; k < M; ++k) {
        for (int Y = 0; Y < N; ++Y)
            for (int X = 0; X < N; ++X) img[(long)Y * N + X] = gauss2(X - c[2 * k], Y - c[2 * k + 1], sigma);
        ora_starlet_fwd(N, J, img, alpha);
        den += amean[k] * l1_prior(N, J, alpha, W, w_stride, 1.0, NULL, NULL);
    }
    free(img);
    free(amean);
    free(alpha);
    return lambda * (Lf - Lh) / den;
}

/* Model images only (for making noiseless data): model packed n_i^2. */
void ora_forward_model(int E, const int *n, const int *K, int s, int N, int M, double fwhm,
                       const double *kernels, const double *params, double *model)
{
    long nfine = fine_offset(E, n, s, E);
    double *scene = (double *)malloc(sizeof(double) * (nfine > 0 ? nfine : 1));
    ora_render_scene(E, n, s, N, M, fwhm, params, scene);
    ora_conv_sub(E, n, K, s, kernels, scene, model);
    free(scene);
}

/* ------------------------------------------------------------------------- */
/* PSF mode (Sec. 2.1, Eqs. 2-7)                                              */
/* params = [eta_M 5 = (A, alpha_x, alpha_y, phi, beta) | b N^2 | a S | c S*2] */
/* ------------------------------------------------------------------------- */

/* Moffat m(eta_M) on the N x N grid centred at floor(N/2); dm (5*N^2) optional:
 * dm/dA, dm/dalpha_x, dm/dalpha_y, dm/dphi, dm/dbeta. */
void ora_moffat(int N, const double *eta, double *m, double *dm)
{
    double A = eta[0], ax = eta[1], ay = eta[2], phi = eta[3], beta = eta[4];
    double cs = cos(phi), sn = sin(phi);
    int c0 = N / 2;
    long NN = (long)N * N;
    for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x) {
            double dx = x - c0, dy = y - c0;
            double u = cs * dx + sn * dy;
            double v = -sn * dx + cs * dy;
            double Q = (u / ax) * (u / ax) + (v / ay) * (v / ay);
            double base = pow(1.0 + Q, -beta);
            double val = A * base;
            long p = (long)y * N + x;
            m[p] = val;
            if (dm) {
                double dQ = -beta * val / (1.0 + Q); /* dm/dQ */
                dm[0 * NN + p] = base;
                dm[1 * NN + p] = dQ * (-2.0 * u * u / (ax * ax * ax));
                dm[2 * NN + p] = dQ * (-2.0 * v * v / (ay * ay * ay));
                dm[3 * NN + p] = dQ * (2.0 * u * v * (1.0 / (ax * ax) - 1.0 / (ay * ay)));
                dm[4 * NN + p] = -val * log(1.0 + Q);
            }
        }
}

/* 1-D factor tables of the shifted Gaussian: G[x*N + x'] = g(x - x' - c) and
 * Gd[x*N + x'] = g(x - x' - c) (x - x' - c)/sigma^2, the derivative of g(x - x' - c)
 * with respect to c. */
static void gauss_tables(int N, double c, double sigma, double *G, double *Gd)
{
    for (int x = 0; x < N; ++x)
        for (int xp = 0; xp < N; ++xp) {
            double t = x - xp - c;
            double g = gauss1(t, sigma);
            G[(long)x * N + xp] = g;
            if (Gd) Gd[(long)x * N + xp] = g * t / (sigma * sigma);
        }
}

/* out(y,x) = sum_{y',x'} Gy[y,y'] Gx[x,x'] in(y',x') over the whole N x N grid:
 * the convolution of `in` with the separable kernel r = g(dx) g(dy) (Eq. 3). */
static void sep_apply(const double *in, int N, const double *Gy, const double *Gx, double *out,
                      double *tmp)
{
    for (int yp = 0; yp < N; ++yp)
        for (int x = 0; x < N; ++x) {
            double acc = 0.0;
            for (int xp = 0; xp < N; ++xp) acc += Gx[(long)x * N + xp] * in[(long)yp * N + xp];
            tmp[(long)yp * N + x] = acc;
        }
    for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x) {
            double acc = 0.0;
            for (int yp = 0; yp < N; ++yp) acc += Gy[(long)y * N + yp] * tmp[(long)yp * N + x];
            out[(long)y * N + x] = acc;
        }
}

/* transpose of sep_apply: out(y',x') = sum_{y,x} Gy[y,y'] Gx[x,x'] in(y,x) */
static void sep_apply_T(const double *in, int N, const double *Gy, const double *Gx, double *out,
                        double *tmp)
{
    for (int yp = 0; yp < N; ++yp)
        for (int x = 0; x < N; ++x) {
            double acc = 0.0;
            for (int y = 0; y < N; ++y) acc += Gy[(long)y * N + yp] * in[(long)y * N + x];
            tmp[(long)yp * N + x] = acc;
        }
    for (int yp = 0; yp < N; ++yp)
        for (int xp = 0; xp < N; ++xp) {
            double acc = 0.0;
            for (int x = 0; x < N; ++x) acc += Gx[(long)x * N + xp] * tmp[(long)yp * N + x];
            out[(long)yp * N + xp] = acc;
        }
}

/* Narrow PSF s = m(eta_M) + b (Eq. 2). */
void ora_psf_render(int N, const double *params, double *s_out)
{
    long NN = (long)N * N;
    ora_moffat(N, params, s_out, NULL);
    for (long p = 0; p < NN; ++p) s_out[p] += params[5 + p];
}

/* Star models m_k = D(s * a_k r_k), packed S x n^2 with n = N/s_sub (Eq. 3). */
void ora_psf_model(int S, int n, int ssub, int N, double fwhm, const double *params,
                   double *model)
{
    long NN = (long)N * N;
    double sigma = ora_sigma_from_fwhm(fwhm);
    double *s = (double *)malloc(sizeof(double) * NN);
    ora_psf_render(N, params, s);
    const double *a = params + 5 + NN;
    const double *c = a + S;
    int k;
#pragma omp parallel for schedule(dynamic)
    for (k = 0; k < S; ++k) {
        double *u = (double *)malloc(sizeof(double) * NN);
        double *tmp = (double *)malloc(sizeof(double) * NN);
        double *Gx = (double *)malloc(sizeof(double) * NN);
        double *Gy = (double *)malloc(sizeof(double) * NN);
        gauss_tables(N, c[2 * k], sigma, Gx, NULL);
        gauss_tables(N, c[2 * k + 1], sigma, Gy, NULL);
        sep_apply(s, N, Gy, Gx, u, tmp);
        for (long p = 0; p < NN; ++p) u[p] *= a[k];
        block_sum(u, n, ssub, model + (long)k * n * n);
        free(u);
        free(tmp);
        free(Gx);
        free(Gy);
    }
    free(s);
}

void ora_psf_loss_grad(int S, int n, int ssub, int N, int J, int w_stride, double lambda,
                       double fwhm, const double *data, const double *invvar, const double *W,
                       const double *params, double *grad, double *loss,
                       const signed char *sgn_override)
{
    long NN = (long)N * N;
    long nd = (long)S * n * n;
    double sigma = ora_sigma_from_fwhm(fwhm);
    double *model = (double *)malloc(sizeof(double) * (nd > 0 ? nd : 1));
    double *rho = (double *)malloc(sizeof(double) * (nd > 0 ? nd : 1));
    ora_psf_model(S, n, ssub, N, fwhm, params, model);
    double chi = 0.0;
    for (long p = 0; p < nd; ++p) {
        double r = model[p] - data[p];
        rho[p] = invvar[p] * r;
        chi += 0.5 * invvar[p] * r * r;
    }
    const double *b = params + 5;
    double *alpha = (double *)malloc(sizeof(double) * J * NN);
    double *z = (double *)malloc(sizeof(double) * J * NN);
    ora_starlet_fwd(N, J, b, alpha);
    double l1 = l1_prior(N, J, alpha, W, w_stride, lambda, sgn_override, z);
    loss[0] = chi;
    loss[1] = l1;
    loss[2] = chi + l1;

    if (grad) {
        const double *a = params + 5 + NN;
        const double *c = a + S;
        double *s = (double *)malloc(sizeof(double) * NN);
        double *mof = (double *)malloc(sizeof(double) * NN);
        double *dm = (double *)malloc(sizeof(double) * 5 * NN);
        ora_psf_render(N, params, s);
        ora_moffat(N, params, mof, dm);
        double *gs_star = (double *)calloc((size_t)S * NN, sizeof(double));
        double *ga = grad + 5 + NN;
        double *gc = ga + S;
        int k;
#pragma omp parallel for schedule(dynamic)
        for (k = 0; k < S; ++k) {
            double *gh = (double *)malloc(sizeof(double) * NN);
            double *tmp = (double *)malloc(sizeof(double) * NN);
            double *Gx = (double *)malloc(sizeof(double) * NN);
            double *Gy = (double *)malloc(sizeof(double) * NN);
            double *Gdx = (double *)malloc(sizeof(double) * NN);
            double *Gdy = (double *)malloc(sizeof(double) * NN);
            double *v = (double *)malloc(sizeof(double) * NN);
            block_sum_adj(rho + (long)k * n * n, n, ssub, gh);
            gauss_tables(N, c[2 * k], sigma, Gx, Gdx);
            gauss_tables(N, c[2 * k + 1], sigma, Gy, Gdy);
            /* dchi/ds = a_k R_k^T D^T rho_k */
            sep_apply_T(gh, N, Gy, Gx, gs_star + (long)k * NN, tmp);
            for (long p = 0; p < NN; ++p) gs_star[(long)k * NN + p] *= a[k];
            /* dchi/da_k = < D^T rho_k, s * r_k > */
            sep_apply(s, N, Gy, Gx, v, tmp);
            double sa = 0.0;
            for (long p = 0; p < NN; ++p) sa += gh[p] * v[p];
            /* dchi/dc_k: the Gaussian factor of the shifted axis is replaced by its
             * derivative with respect to the centre */
            sep_apply(s, N, Gy, Gdx, v, tmp);
            double scx = 0.0;
            for (long p = 0; p < NN; ++p) scx += gh[p] * v[p];
            sep_apply(s, N, Gdy, Gx, v, tmp);
            double scy = 0.0;
            for (long p = 0; p < NN; ++p) scy += gh[p] * v[p];
            ga[k] = sa;
            gc[2 * k] = a[k] * scx;
            gc[2 * k + 1] = a[k] * scy;
            free(gh);
            free(tmp);
            free(Gx);
            free(Gy);
            free(Gdx);
            free(Gdy);
            free(v);
        }
        /* g_s = sum_k (per-star contributions), summed in star order */
        double *gs = (double *)calloc(NN, sizeof(double));
        for (int kk = 0; kk < S; ++kk)
            for (long p = 0; p < NN; ++p) gs[p] += gs_star[(long)kk * NN + p];
        /* dchi/deta_M = sum_x g_s(x) dm/deta_M(x) */
        for (int e = 0; e < 5; ++e) {
            double acc = 0.0;
            for (long p = 0; p < NN; ++p) acc += gs[p] * dm[(long)e * NN + p];
            grad[e] = acc;
        }
        double *pz = (double *)malloc(sizeof(double) * NN);
        ora_starlet_adj(N, J, z, pz);
        for (long p = 0; p < NN; ++p) grad[5 + p] = gs[p] + pz[p];
        free(pz);
        free(gs);
        free(gs_star);
        free(s);
        free(mof);
        free(dm);
    }
    free(alpha);
    free(z);
    free(model);
    free(rho);
}

/* ------------------------------------------------------------------------- */
/* Noise propagated to the starlet coefficients (Sec. 2.3, App. B)           */
/* ------------------------------------------------------------------------- */

/* Exact variance maps of W's Monte Carlo estimate. White noise delta_d on the
 * fine window of frame 1 with diagonal covariance C_up (the data-pixel variance
 * sigma2_data replicated over each s x s block) is propagated as
 * Phi^T S_1^T C_up^-1 delta_d. Its coefficient (j, X) has variance
 *   Var_j(X) = sum_y [Phi^T S_1^T]_{(j,X), y}^2 / sigma_up^2(y),
 * accumulated here column by column: for every fine pixel y, the image
 * S_1^T e_y (the correlation of a unit impulse with the kernel) is placed in the
 * window of h and transformed. var_out: J x N x N. */
void ora_noise_variance(int n1, int K1, int s, int N, int J, const double *kernel1,
                        const double *sigma2_data, double *var_out)
{
    int F = s * n1, o = (N - F) / 2;
    long NN = (long)N * N;
    double *e = (double *)calloc((size_t)F * F, sizeof(double));
    double *g = (double *)malloc(sizeof(double) * F * F);
    double *img = (double *)calloc(NN, sizeof(double));
    double *co = (double *)malloc(sizeof(double) * J * NN);
    for (long q = 0; q < J * NN; ++q) var_out[q] = 0.0;
    for (int y = 0; y < F; ++y)
        for (int x = 0; x < F; ++x) {
            e[(long)y * F + x] = 1.0;
            corr_same(e, F, kernel1, K1, g);
            e[(long)y * F + x] = 0.0;
            for (int yy = 0; yy < F; ++yy)
                for (int xx = 0; xx < F; ++xx) img[(long)(yy + o) * N + xx + o] = g[(long)yy * F + xx];
            ora_starlet_fwd(N, J, img, co);
            double s2 = sigma2_data[(long)(y / s) * n1 + (x / s)];
            for (long q = 0; q < J * NN; ++q) var_out[q] += co[q] * co[q] / s2;
        }
    free(e);
    free(g);
    free(img);
    free(co);
}

/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of the
 * multiply-hi/lo bijection on a 4-word counter with a 2-word key, the key
 * bumped by the Weyl constants between rounds. */
void ora_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Standard normal draw number `idx` of realization `real` (the draw convention
 * shared with the device generator): Philox4x32-10 of counter (idx/4, real, 0, 0)
 * and key (seed low, seed high) gives four words; each is mapped to
 * u = (word >> 8) + 1/2) / 2^24 in (0, 1), and Box-Muller turns the pairs
 * (u0, u1), (u2, u3) into (r cos, r sin) with r = sqrt(-2 ln u_first) and angle
 * 2 pi u_second. */
double ora_normal(uint64_t seed, uint32_t real, uint32_t idx)
{
    const uint32_t ctr[4] = {idx / 4u, real, 0u, 0u};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    ora_philox4x32_10(ctr, key, w);
    const int pair = (int)(idx % 4u) / 2, second = (int)(idx % 2u);
    const double u1 = ((double)(w[2 * pair] >> 8) + 0.5) / 16777216.0;
    const double u2 = ((double)(w[2 * pair + 1] >> 8) + 0.5) / 16777216.0;
    const double r = sqrt(-2.0 * log(u1));
    const double ang = 6.283185307179586476925286766559 * u2;  /* 2 pi */
    return second ? r * sin(ang) : r * cos(ang);
}

/* Monte Carlo estimate of W (Sec. 2.3): for each realization r < R the white
 * noise delta_d on frame f's fine window (variance sigma2_data of the data pixel
 * replicated over its s x s block) is weighted by C_up^-1, correlated with the
 * frame's kernel (S^T), placed in the window of h and transformed; W is the
 * standard deviation (mean removed, divided by R) of each coefficient over the
 * realizations (per_pixel: J x N x N) or of all coefficients of each scale over
 * the realizations (J values). normals: R x F^2 standard normal draws, or NULL
 * for the Philox draws of ora_normal(seed, r, pixel). */
void ora_noise_weights_mc(int n1, int K1, int s, int N, int J, const double *kernel1, const double *sigma2_data,
                          int R, const double *normals, uint64_t seed, int per_pixel, double *W_out)
{
    int F = s * n1, o = (N - F) / 2;
    long NN = (long)N * N;
    double *s1 = (double *)calloc((size_t)J * NN, sizeof(double));
    double *s2 = (double *)calloc((size_t)J * NN, sizeof(double));
    double *dl = (double *)malloc(sizeof(double) * F * F);
    double *g = (double *)malloc(sizeof(double) * F * F);
    double *img = (double *)calloc(NN, sizeof(double));
    double *co = (double *)malloc(sizeof(double) * J * NN);
    for (int r = 0; r < R; ++r) {
        for (int y = 0; y < F; ++y)
            for (int x = 0; x < F; ++x) {
                const long i = (long)y * F + x;
                const double z = normals ? normals[(long)r * F * F + i] : ora_normal(seed, (uint32_t)r, (uint32_t)i);
                const double s2u = sigma2_data[(long)(y / s) * n1 + (x / s)];
                dl[i] = sqrt(s2u) * z / s2u; /* C_up^-1 delta_d, delta_d = sigma_up z */
            }
        corr_same(dl, F, kernel1, K1, g);
        for (int yy = 0; yy < F; ++yy)
            for (int xx = 0; xx < F; ++xx) img[(long)(yy + o) * N + xx + o] = g[(long)yy * F + xx];
        ora_starlet_fwd(N, J, img, co);
        for (long q = 0; q < J * NN; ++q) {
            s1[q] += co[q];
            s2[q] += co[q] * co[q];
        }
    }
    for (int j = 0; j < J; ++j) {
        if (per_pixel) {
            for (long q = 0; q < NN; ++q) {
                const double m = s1[j * NN + q] / R, v = s2[j * NN + q] / R - m * m;
                W_out[j * NN + q] = sqrt(v > 0.0 ? v : 0.0);
            }
        } else {
            double a = 0.0, b = 0.0;
            for (long q = 0; q < NN; ++q) {
                a += s1[j * NN + q];
                b += s2[j * NN + q];
            }
            const double cnt = (double)R * (double)NN, m = a / cnt, v = b / cnt - m * m;
            W_out[j] = sqrt(v > 0.0 ? v : 0.0);
        }
    }
    free(s1);
    free(s2);
    free(dl);
    free(g);
    free(img);
    free(co);
}

/* ------------------------------------------------------------------------- */
/* Adam update (Kingma & Ba 2015), the optimiser step of the gradient-based   */
/* fit (Sec. 2.4). lr is per element.                                         */
/* ------------------------------------------------------------------------- */

void ora_adam_step(long P, double *params, const double *grad, double *m, double *v, int t,
                   const double *lr, double beta1, double beta2, double eps)
{
    double bc1 = 1.0 - pow(beta1, t);
    double bc2 = 1.0 - pow(beta2, t);
    for (long p = 0; p < P; ++p) {
        m[p] = beta1 * m[p] + (1.0 - beta1) * grad[p];
        v[p] = beta2 * v[p] + (1.0 - beta2) * grad[p] * grad[p];
        double mh = m[p] / bc1;
        double vh = v[p] / bc2;
        params[p] -= lr[p] * mh / (sqrt(vh) + eps);
    }
}

/* AdaBelief (Zhuang et al., NeurIPS 2020): the second moment tracks the squared
 * deviation of the gradient from the updated first moment, plus eps_root; the
 * bias corrections and the step are Adam's. lr per parameter. */
void ora_adabelief_step(long P, double *params, const double *grad, double *m, double *v, int t,
                        const double *lr, double beta1, double beta2, double eps, double eps_root)
{
    double bc1 = 1.0 - pow(beta1, t);
    double bc2 = 1.0 - pow(beta2, t);
    for (long p = 0; p < P; ++p) {
        m[p] = beta1 * m[p] + (1.0 - beta1) * grad[p];
        const double d = grad[p] - m[p];
        v[p] = beta2 * v[p] + (1.0 - beta2) * d * d + eps_root;
        params[p] -= lr[p] * (m[p] / bc1) / (sqrt(v[p] / bc2) + eps);
    }
}

/* L-BFGS two-loop recursion (Nocedal & Wright, Numerical Optimization, Alg. 7.4):
 * d = -H g for the inverse-Hessian approximation built from the `count` newest
 * pairs (s_i, y_i) of the ring buffers S, Y ([m][n], newest at slot `newest`,
 * older ones before it modulo m) and H_0 = gamma I, gamma = s^T y / y^T y of the
 * newest pair. count = 0 gives d = -g. */
void ora_lbfgs_direction(long n, const double *g, const double *S, const double *Y, int m, int count, int newest,
                         double *d)
{
    double *q = (double *)malloc(sizeof(double) * n);
    double *alpha = (double *)malloc(sizeof(double) * (m > 0 ? m : 1));
    for (long p = 0; p < n; ++p) q[p] = g[p];
    for (int c = 0; c < count; ++c) {
        const int i = ((newest - c) % m + m) % m;
        const double *s = S + (long)i * n, *y = Y + (long)i * n;
        double sy = 0.0, sq = 0.0;
        for (long p = 0; p < n; ++p) {
            sy += s[p] * y[p];
            sq += s[p] * q[p];
        }
        alpha[c] = sq / sy;
        for (long p = 0; p < n; ++p) q[p] -= alpha[c] * y[p];
    }
    double gamma = 1.0;
    if (count > 0) {
        const double *s = S + (long)newest * n, *y = Y + (long)newest * n;
        double sy = 0.0, yy = 0.0;
        for (long p = 0; p < n; ++p) {
            sy += s[p] * y[p];
            yy += y[p] * y[p];
        }
        gamma = sy / yy;
    }
    for (long p = 0; p < n; ++p) q[p] *= gamma;
    for (int c = count - 1; c >= 0; --c) {
        const int i = ((newest - c) % m + m) % m;
        const double *s = S + (long)i * n, *y = Y + (long)i * n;
        double sy = 0.0, yr = 0.0;
        for (long p = 0; p < n; ++p) {
            sy += s[p] * y[p];
            yr += y[p] * q[p];
        }
        const double beta = yr / sy;
        for (long p = 0; p < n; ++p) q[p] += s[p] * (alpha[c] - beta);
    }
    for (long p = 0; p < n; ++p) d[p] = -q[p];
    free(q);
    free(alpha);
}

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the frame loops (n <= 0: every processor). */
void ora_set_num_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------- */
/* Per-frame shifts and rotations (Conclusion: all epochs processed together  */
/* while modelling shifts and rotations between frames; Sec. 4.1: per-epoch   */
/* dithering offsets recovered by the fit).                                   */
/* Frame i with transform t_i = (dx_i, dy_i, theta_i) observes the scene at   */
/*   u_i(X) = R(theta_i) (X - C) + C + (dx_i, dy_i),  C = ((N-1)/2, (N-1)/2), */
/* X a fine pixel of its window in grid coordinates, R the counter-clockwise  */
/* rotation [[cos, -sin], [sin, cos]]. The extended channel is read there by  */
/* bilinear interpolation of h (zero outside the grid); point source k adds   */
/* a_ik r(u_i(X) - c_k).  t_i = 0 gives Eq. (9) exactly.                      */
/* ------------------------------------------------------------------------- */

static double h_at(const double *h, int N, long X, long Y)
{
    if (X < 0 || X >= N || Y < 0 || Y >= N) return 0.0;
    return h[Y * N + X];
}

/* bilinear interpolation of h at (ux, uy) and its two partial derivatives */
static double bilerp(const double *h, int N, double ux, double uy, double *dx_out, double *dy_out)
{
    const double fx = floor(ux), fy = floor(uy);
    const long X0 = (long)fx, Y0 = (long)fy;
    const double tx = ux - fx, ty = uy - fy;
    const double h00 = h_at(h, N, X0, Y0), h10 = h_at(h, N, X0 + 1, Y0);
    const double h01 = h_at(h, N, X0, Y0 + 1), h11 = h_at(h, N, X0 + 1, Y0 + 1);
    if (dx_out) *dx_out = (1.0 - ty) * (h10 - h00) + ty * (h11 - h01);
    if (dy_out) *dy_out = (1.0 - tx) * (h01 - h00) + tx * (h11 - h10);
    return (1.0 - tx) * (1.0 - ty) * h00 + tx * (1.0 - ty) * h10 + (1.0 - tx) * ty * h01 + tx * ty * h11;
}

static void frame_map(int N, const double *t, double X, double Y, double *ux, double *uy)
{
    const double C = 0.5 * (N - 1), cs = cos(t[2]), sn = sin(t[2]);
    const double vx = X - C, vy = Y - C;
    *ux = cs * vx - sn * vy + C + t[0];
    *uy = sn * vx + cs * vy + C + t[1];
}

/* scene of every frame under its transform (xf: E x 3 = dx, dy, theta) */
void ora_render_scene_xf(int E, const int *n, int s, int N, int M, double fwhm, const double *params,
                         const double *xf, double *scene)
{
    const double *h = params;
    const double *Gam = params + (long)N * N;
    const double *a = Gam + E;
    const double *c = a + (long)E * M;
    const double sigma = ora_sigma_from_fwhm(fwhm);
    int *o = (int *)malloc(sizeof(int) * (E > 0 ? E : 1));
    ora_frame_offsets(E, n, s, N, o);
    for (int i = 0; i < E; ++i) {
        const int F = s * n[i];
        double *f = scene + fine_offset(E, n, s, i);
        for (int y = 0; y < F; ++y)
            for (int x = 0; x < F; ++x) {
                double ux, uy;
                frame_map(N, xf + 3 * i, x + o[i], y + o[i], &ux, &uy);
                double v = Gam[i] + bilerp(h, N, ux, uy, NULL, NULL);
                for (int k = 0; k < M; ++k)
                    v += a[(long)i * M + k] * gauss2(ux - c[2 * k], uy - c[2 * k + 1], sigma);
                f[(long)y * F + x] = v;
            }
    }
    free(o);
}

/* Loss and gradient with per-frame transforms (Eqs. 9-11 with the scene above).
 * grad: [h | Gamma | a | c] as ora_loss_grad; gxf (E x 3, may be NULL): dL/d(dx_i,
 * dy_i, theta_i). The h block's data term is the literal transpose of the
 * interpolation: every frame pixel scatters its g onto the four pixels it read. */
void ora_loss_grad_xf(int E, const int *n, const int *K, int s, int N, int M, int J, int w_stride, double lambda,
                      double fwhm, const double *data, const double *invvar, const double *kernels, const double *W,
                      const double *params, const double *xf, double *grad, double *gxf, double *loss,
                      const signed char *sgn_override)
{
    const long NN = (long)N * N;
    const long nfine = fine_offset(E, n, s, E);
    const long ndata = data_offset(n, E);
    const double sigma = ora_sigma_from_fwhm(fwhm), s2 = sigma * sigma;
    int *o = (int *)malloc(sizeof(int) * (E > 0 ? E : 1));
    ora_frame_offsets(E, n, s, N, o);
    double *scene = (double *)malloc(sizeof(double) * (nfine > 0 ? nfine : 1));
    double *model = (double *)malloc(sizeof(double) * (ndata > 0 ? ndata : 1));
    double *rho = (double *)malloc(sizeof(double) * (ndata > 0 ? ndata : 1));
    ora_render_scene_xf(E, n, s, N, M, fwhm, params, xf, scene);
    ora_conv_sub(E, n, K, s, kernels, scene, model);
    double chi = 0.0;
    for (long p = 0; p < ndata; ++p) {
        const double r = model[p] - data[p];
        rho[p] = invvar[p] * r;
        chi += 0.5 * invvar[p] * r * r;
    }
    double *alpha = (double *)malloc(sizeof(double) * J * NN);
    double *z = (double *)malloc(sizeof(double) * J * NN);
    ora_starlet_fwd(N, J, params, alpha);
    const double l1 = l1_prior(N, J, alpha, W, w_stride, lambda, sgn_override, z);
    loss[0] = chi;
    loss[1] = l1;
    loss[2] = chi + l1;
    if (grad) {
        const double *h = params;
        const double *a = params + NN + E;
        const double *c = a + (long)E * M;
        double *gh = grad, *gG = grad + NN, *ga = gG + E, *gc = ga + (long)E * M;
        double *gscene = (double *)malloc(sizeof(double) * (nfine > 0 ? nfine : 1));
        ora_conv_sub_adj(E, n, K, s, kernels, rho, gscene);
        for (long p = 0; p < NN; ++p) gh[p] = 0.0;
        for (long q = 0; q < 2L * M; ++q) gc[q] = 0.0;
        for (int i = 0; i < E; ++i) {
            const int F = s * n[i];
            const double *g = gscene + fine_offset(E, n, s, i);
            const double *t = xf + 3 * i;
            const double cs = cos(t[2]), sn = sin(t[2]), C = 0.5 * (N - 1);
            double sG = 0.0, gdx = 0.0, gdy = 0.0, gth = 0.0;
            for (int k = 0; k < M; ++k) ga[(long)i * M + k] = 0.0;
            for (int y = 0; y < F; ++y)
                for (int x = 0; x < F; ++x) {
                    const double gv = g[(long)y * F + x];
                    const double X = x + o[i], Y = y + o[i];
                    double ux, uy, hx, hy;
                    frame_map(N, t, X, Y, &ux, &uy);
                    bilerp(h, N, ux, uy, &hx, &hy);
                    sG += gv;
                    /* transpose of the interpolation */
                    const double fx = floor(ux), fy = floor(uy);
                    const long X0 = (long)fx, Y0 = (long)fy;
                    const double tx = ux - fx, ty = uy - fy;
                    const double wts[4] = {(1 - tx) * (1 - ty), tx * (1 - ty), (1 - tx) * ty, tx * ty};
                    const long xs[4] = {X0, X0 + 1, X0, X0 + 1}, ys[4] = {Y0, Y0, Y0 + 1, Y0 + 1};
                    for (int q = 0; q < 4; ++q)
                        if (xs[q] >= 0 && xs[q] < N && ys[q] >= 0 && ys[q] < N) gh[ys[q] * N + xs[q]] += gv * wts[q];
                    /* d scene / d u at this pixel */
                    double dux = hx, duy = hy;
                    for (int k = 0; k < M; ++k) {
                        const double ex = ux - c[2 * k], ey = uy - c[2 * k + 1];
                        const double r = gauss2(ex, ey, sigma);
                        const double aik = a[(long)i * M + k];
                        ga[(long)i * M + k] += gv * r;
                        gc[2 * k] += gv * aik * r * ex / s2;       /* d r(u - c)/d c = r (u - c)/sigma^2 */
                        gc[2 * k + 1] += gv * aik * r * ey / s2;
                        dux -= aik * r * ex / s2;
                        duy -= aik * r * ey / s2;
                    }
                    /* u = R (X - C) + C + d:  du/dd = I,  du/dtheta = R'(theta) (X - C) */
                    const double vx = X - C, vy = Y - C;
                    gdx += gv * dux;
                    gdy += gv * duy;
                    gth += gv * (dux * (-sn * vx - cs * vy) + duy * (cs * vx - sn * vy));
                }
            gG[i] = sG;
            if (gxf) {
                gxf[3 * i] = gdx;
                gxf[3 * i + 1] = gdy;
                gxf[3 * i + 2] = gth;
            }
        }
        double *pz = (double *)malloc(sizeof(double) * NN);
        ora_starlet_adj(N, J, z, pz);
        for (long p = 0; p < NN; ++p) gh[p] += pz[p];
        free(pz);
        free(gscene);
    }
    free(alpha);
    free(z);
    free(scene);
    free(model);
    free(rho);
    free(o);
}
