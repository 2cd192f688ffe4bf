// Internal declarations shared by the host side of the library and the kernels.
// Not part of the public C ABI (include/starred.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace starred {

// Per-frame description kept in device memory (deconvolution mode).
//
// Direct algorithm: the fused S_i + D forward is the stride-s correlation
//   m(p,q) = sum_{a,b < Kp} kf(a,b) f(s p + A0 + a, s q + A0 + b),  A0 = cp - (Kp - 1),
// with kf the flipped kernel box-folded over s x s (side Kp = K + s - 1) and
// cp = floor(K/2) + s - 1. kf is stored [a][psi][t], b = s t + psi, t < Tpad.
// The adjoint is split into s^2 phases: for phase (py, px)
//   g(s P + py, s Q + px) = sum_{al < Ar, be < Bpad} kp(al,be) rho(P + dmin + al, Q + dmin + be),
// kp stored [py][px][al][be].
struct FrameDev {
    int n;      // data side
    int F;      // fine side s*n
    int K;      // kernel side
    int Kp;     // folded kernel side K + s - 1
    int o;      // window offset inside h
    int cp;     // floor(K/2) + s - 1
    int Tpad;   // forward taps per residue, padded to a multiple of 4
    int Ar;     // adjoint phase-kernel rows
    int Bpad;   // adjoint phase-kernel columns, padded to a multiple of 4
    int dmin;   // adjoint row/column offset of phase kernels
    int pad0, pad1;
    long long data_off;  // into packed n_i^2 arrays
    long long fine_off;  // into packed (s n_i)^2 arrays
    long long kern_off;  // into packed K_i^2 kernels
    long long kf_off;    // into the forward folded kernels
    long long ka_off;    // into the adjoint phase kernels
};

// One work item of a tiled launch: frame and tile origin (data pixels),
// plus the slot of its partial results (frame-major enumeration).
struct Item {
    int frame;
    int p0;
    int q0;
    int slot;
};

// Tile shapes of the direct kernels (data pixels; every thread owns 4
// consecutive outputs of one row).
constexpr int kFwdTP = 16, kFwdTQ = 32, kFwdCA = 16;
constexpr int kAdjTP = 16, kAdjTQ = 32;
constexpr int kFwdThreads = kFwdTP * kFwdTQ / 4;
constexpr int kAdjThreads = kAdjTP * kAdjTQ / 4;

constexpr int kGaussRadius = 8;  // r is evaluated within +-8 fine px of c_k
constexpr size_t kMaxLds = 160 * 1024;

size_t fwd_lds_bytes(int s, int Tmax);
size_t adj_lds_bytes(int Ar_max, int Bpad_max);

// ---- kernel launchers (starred_kernels.hip) ----
hipError_t launch_prep_kernels(hipStream_t st, const FrameDev *fr_dev, const FrameDev *fr_host,
                               int E, int s, const float *psf, float *kf, float *ka);
// flist (device, nlist frame indices) restricts a launch to those frames; null: every frame
// xf (device, E x 3 = dx, dy, theta, or null): per-frame transforms of the scene
hipError_t launch_render(hipStream_t st, const FrameDev *fr, int E, int Fmax, int N, int M,
                         float sigma, const float *params, float *scene, const int *flist = nullptr,
                         int nlist = 0, const float *xf = nullptr);
// Persistent launches: at most `groups` work groups walk the item list (0: one per item).
hipError_t launch_fwd_direct(hipStream_t st, int s, const FrameDev *fr, const Item *items,
                             int n_items, int Tmax, const float *scene, const float *kf,
                             const float *data, const float *invvar, float *out, double *part_chi,
                             int groups = 0);
hipError_t launch_adj_direct(hipStream_t st, int s, const FrameDev *fr, const Item *items,
                             int n_items, int Ar_max, int Bpad_max, const float *rho,
                             const float *ka, float *g, int groups = 0);
// with xf: sums in scene coordinates, and (gxf non-null) dL/d(dx, dy, theta) per frame
// gxf (with xf): the transforms' gradient, through gxfp (xf_grad_parts(E) FP64 partials)
hipError_t launch_frame_sums(hipStream_t st, const FrameDev *fr, int E, int N, int M, float sigma,
                             const float *params, const float *g, double *fsum, bool with_gamma,
                             const int *flist = nullptr, int nlist = 0, const float *xf = nullptr,
                             float *gxf = nullptr, double *gxfp = nullptr);
int xf_grad_parts(int E);
hipError_t launch_finalize_h(hipStream_t st, const FrameDev *fr, int E, int N, const float *g,
                             const float *prior, float *grad_h, float *part, const int *flist = nullptr,
                             int nlist = 0, const float *xf = nullptr);
// work groups of the direct kernels that fit on the device at once (persistent grid)
int direct_fwd_groups(int s, int Tmax);
int direct_adj_groups(int s, int Ar_max, int Bpad_max);
int finalize_h_chunks(int E, bool xf = false);
// Update of one parameter (bias-corrected moments, per-block learning rate):
// Adam (v tracks g^2) or, with belief, AdaBelief (v tracks (g - m)^2 + eps_root
// with the updated m).
__device__ __forceinline__ void adam_update(float &param, float &m, float &v, float g, float lr, float beta1,
                                            float beta2, float bc1, float bc2, float eps, bool belief = false,
                                            float eps_root = 0.f)
{
    m = beta1 * m + (1.f - beta1) * g;
    if (belief) {
        const float dg = g - m;
        v = beta2 * v + (1.f - beta2) * dg * dg + eps_root;
    } else {
        v = beta2 * v + (1.f - beta2) * g * g;
    }
    param -= lr * (m / bc1) / (sqrtf(v / bc2) + eps);
}

// Optimiser state for an update fused into the final reduction launch (params null: none).
struct AdamDev {
    float *params = nullptr, *m = nullptr, *v = nullptr;
    const int *d_t = nullptr;
    float lr[4] = {0.f, 0.f, 0.f, 0.f};
    float beta1 = 0.f, beta2 = 0.f, eps = 0.f;
    int rule = 0;
    float eps_root = 0.f;
};

struct ClassFft;
struct DenseStar;
// With classes (FFT path), the launch also writes dL/dh = prior + the classes'
// window contributions hcls. pts (3M, or null): the point-source prior's
// additions to dL/da_ik (every i) and dL/dc_k.
hipError_t launch_finalize_small(hipStream_t st, int E, int M, int n_chi, const double *part_chi,
                                 int n_l1, const double *part_l1, double lambda,
                                 const double *fsum, const float *params, int N,
                                 float *grad, double *loss, const int *gcsr_off = nullptr,
                                 const int *gcsr_item = nullptr, const double *gpart = nullptr,
                                 int *tick = nullptr, const ClassFft *classes = nullptr, int ncls = 0,
                                 const float *hcls = nullptr, const float *prior = nullptr,
                                 const AdamDev &adam = AdamDev(), const double *pts = nullptr,
                                 const DenseStar *psum = nullptr);
hipError_t launch_copy_probe(hipStream_t st, const float *src, float *dst, long long n);
hipError_t launch_idle(hipStream_t st, int iters);

// partial L1 slots the forward transform writes for an N x N image and J planes
int starlet_l1_slots(int N, int J);
hipError_t launch_starlet_fwd(hipStream_t st, int N, int J, const float *img, float *coeffs,
                              float *z, const float *W, int w_stride, float lam, float *c_a,
                              float *c_b, float *tmp, double *part_l1, int *n_l1);
hipError_t launch_starlet_prior(hipStream_t st, int N, int J, int B, const float *img, float *z, const float *W,
                                int w_stride, float lam0, float lam1, float *c_a, float *c_b, double *part_l1,
                                int *n_l1);
// Starlet prior through the per-scale composite filters (starred_starlet.hip)
struct DenseStar;
constexpr int kDenseMaxN = 256;
constexpr size_t kDenseMaxLds = 128 * 1024;
bool dense_fits(int N, int J);  // images and scale counts the composite filters handle
int dense_rows_per_job(int N);
int dense_rows_for(int N, int threads);  // rows per x-pass job for work groups of `threads`
int dense_num_taps(int J);
void dense_taps(int J, double *out);  // host: the composite filters of levels 1 .. J-1
size_t dense_lds_x(int N, int J);
size_t dense_lds_xr(int N, int J, int rx);  // rx rows per job
size_t dense_lds_y(int J);
size_t dense_lds_d(int J);
// L1 partials (part_l1, if set) and, with out set, the subgradient's image
hipError_t launch_dense_prior(hipStream_t st, const DenseStar &d);
// coefficients alpha [B][J][N][N] of d.img
hipError_t launch_dense_coeffs(hipStream_t st, const DenseStar &d, float *coeffs);
// out = Phi zin
hipError_t launch_dense_adjoint(hipStream_t st, const DenseStar &d);
hipError_t launch_starlet_adj_batch(hipStream_t st, int N, int J, int B, const float *z, float *out, float *v_a,
                                    float *v_b);
hipError_t launch_pts_render(hipStream_t st, int N, int E, int M, float sigma, const float *params, float *h_out,
                             float *P_out);
hipError_t launch_pts_dots(hipStream_t st, int N, int E, int M, float sigma, const float *params, const float *q,
                           double *pts);
hipError_t launch_pts_images(hipStream_t st, int N, int E, int M, float sigma, const float *params, float *out);
hipError_t launch_pts_sums(hipStream_t st, int B, int n, const double *part, int N, int E, int M, const float *params,
                           double *out);
hipError_t launch_starlet_fwd_batch(hipStream_t st, int N, int J, int B, const float *img, float *coeffs,
                                    float *c_a, float *c_b, const float *wzero);
hipError_t launch_starlet_adj(hipStream_t st, int N, int J, const float *z, float *out,
                              float *v_a, float *v_b, float *tmp);


hipError_t launch_adam(hipStream_t st, long long P, const long long *seg_end, const float *lr,
                       float *params, const float *grad, float *m, float *v, int *d_t, float beta1,
                       float beta2, float eps, int rule = 0, float eps_root = 0.f);
hipError_t launch_set_step(hipStream_t st, int *d_t, int value);

hipError_t launch_fill(hipStream_t st, float *p, long long n, float v);

// plain (unfused, per-epoch) baseline: one launch per operator per frame
hipError_t launch_render_frame(hipStream_t st, const FrameDev *fr, int E, int i, int F, int N, int M,
                               float sigma, const float *params, float *scene);
// op 0: m = D u; op 1: rho = w (m - d) with chi partials; op 2: gh = D^T rho
hipError_t launch_plain_frame_ops(hipStream_t st, int op, const FrameDev *fr, int i, int n, int F, int s,
                                  const float *a, const float *data, const float *invvar, float *out,
                                  double *part);
hipError_t launch_frame_sums_one(hipStream_t st, const FrameDev *fr, int E, int i, int N, int M, float sigma,
                                 const float *params, const float *g, double *fsum);

// noise propagation (starred_noise.hip)
// delta[b][y][x] = z / sigma_up(y, x), z = normals[r0 + b] or the device Philox draws
hipError_t launch_noise_draw(hipStream_t st, int B, int nb, int r0, int n, int s, const float *sigma2_data,
                             const float *normals, unsigned long long seed, float *delta);
// img[b] = zero N x N with g[b] (F x F) at offset o
hipError_t launch_noise_embed(hipStream_t st, int B, int F, int N, int o, const float *g, float *img);
// s1 += sum_b c, s2 += sum_b c^2 over the first nb of B coefficient sets (each count floats)
hipError_t launch_noise_moments(hipStream_t st, int nb, long long count, const float *coeffs, double *s1,
                                double *s2);
// W from the moments of R realizations: per pixel (count = J N^2) or per scale (J values)
hipError_t launch_noise_finish(hipStream_t st, int J, long long NN, int R, int per_pixel, const double *s1,
                               const double *s2, float *W);
hipError_t launch_fill_d(hipStream_t st, double *p, long long n);

// L-BFGS vector kernels (starred_opt.hip)
hipError_t launch_lbfgs_direction(hipStream_t st, long long n, const float *g, const float *S, const float *Y, int m,
                                  int count, int newest, float *d, double *alpha_scratch);
hipError_t launch_trial_point(hipStream_t st, long long n, const float *x, const float *d, float step, const float *lo,
                              const float *hi, float *xt);
hipError_t launch_dots(hipStream_t st, long long n, const float *a, const float *b, const float *c, double *out);
hipError_t launch_history(hipStream_t st, long long n, const float *xn, float *xo, const float *gn, float *go,
                          float *s, float *y, int store);

// PSF mode (starred_psf.hip)
hipError_t launch_psf_render(hipStream_t st, int N, const float *params, float *s_out);
// dm (or null): the Moffat derivatives per pixel, [5][N^2]; tick (or null): the step
// counter, advanced by this launch
hipError_t launch_psf_render64(hipStream_t st, int N, const float *params, double *s64, float *dm,
                               int *tick = nullptr);
// model (or null): the star models alone into model (S x n^2; data, invvar, rho and part unused)
hipError_t launch_psf_fwd(hipStream_t st, int S, int n, int ss, int N, float sigma, const float *params,
                          const double *s64, const float *data, const float *invvar, float *rho, double *part,
                          float *model = nullptr);
hipError_t launch_psf_adjsum(hipStream_t st, int S, int n, int ss, int N, float sigma, const float *params,
                             const float *rho, const float *dm, float *grad, double *part_eta);
// the loss, the gradient's small blocks, grad_b += prior, and (adam.params non-null) the update
hipError_t launch_psf_finalize(hipStream_t st, int S, int N, int tiles, const double *part, int n_l1,
                               const double *part_l1, int n_eta, const double *part_eta, const float *params,
                               const float *prior, float *grad, double *loss, const AdamDev &adam = AdamDev());
int psf_fwd_tiles(int n);   // forward tiles per star (four FP64 partials each)
int psf_adj_tiles(int N);   // adjoint tiles (five FP64 partials each)
size_t psf_fwd_lds(int s);
size_t psf_adj_lds(int s, int S);

}  // namespace starred
