/*
 * starred.h -- C ABI of the MI355X (gfx950) library that evaluates the loss and
 * gradient of STARRED's joint multi-epoch two-channel deconvolution and of its
 * PSF-reconstruction mode (Millon et al., "Image deconvolution and PSF
 * reconstruction with STARRED", Sec. 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All float* / double* arguments are DEVICE pointers owned by the caller. The
 *    library never frees them. Pointers passed to starred_set_frames are kept by
 *    the plan (not copied) and must stay valid until the next starred_set_frames
 *    or starred_plan_destroy.
 *  - The plan owns its scratch memory, its device tables and its captured graph.
 *  - Every call enqueues work on the plan's stream and returns without
 *    synchronising (starred_plan_create / starred_set_frames synchronise once).
 *  - Status codes: 0 = STARRED_OK; negative = error. Argument errors are found
 *    on the host before anything is launched. The message of the last error of
 *    the calling thread is returned by starred_last_error().
 *  - A plan must not be used from two host threads at once.
 *  - Images are square, row-major, FP32. Fine pixel (y, x) has its centre at
 *    coordinate (x, y) in fine-pixel units. Data pixel (p, q) covers the fine
 *    pixels [s p, s p + s) x [s q, s q + s) (the subsampling operator D of
 *    Eq. 3 and Eq. 8 is the block sum).
 *  - Frame i of data side n_i sees the central window of the fine grid h with
 *    offset o_i = (N - s n_i)/2, which must be a non-negative integer.
 *  - Per-frame arrays are packed frame after frame: data and inverse variance
 *    n_i^2 each, scenes (s n_i)^2 each, kernels K_i^2 each.
 */
#ifndef STARRED_H
#define STARRED_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STARRED_ABI_VERSION 1

enum {
    STARRED_OK = 0,
    STARRED_EINVAL = -1,      /* bad argument, detected before any launch */
    STARRED_ENOMEM = -2,      /* device allocation failed */
    STARRED_EHIP = -3,        /* HIP runtime error (see starred_last_error) */
    STARRED_EUNSUPPORTED = -4,/* valid request this build does not support */
    STARRED_ESTATE = -5       /* call out of order (e.g. loss_grad before set_frames) */
};

enum { STARRED_DECONV = 0, STARRED_PSF = 1 };

/* Convolution algorithm for the S_i / D pair of the deconvolution mode. */
enum { STARRED_CONV_AUTO = 0, STARRED_CONV_DIRECT = 1, STARRED_CONV_FFT = 2 };

typedef struct starred_plan starred_plan;

/* Problem description (Sec. 2.1 Eqs. 2-7 for STARRED_PSF, Sec. 2.2 Eqs. 8-11
 * for STARRED_DECONV).
 *   mode        STARRED_DECONV or STARRED_PSF.
 *   n_frames    E epochs (deconvolution) or S star stamps (PSF mode), >= 1.
 *   side_host   host array [n_frames]: data side n_i of each frame (PSF mode: all
 *               equal to grid_side / subsample).
 *   ksize_host  host array [n_frames]: side K_i of each narrow-PSF kernel s_i
 *               (deconvolution only; NULL in PSF mode). Centre at floor(K_i/2).
 *   subsample   s >= 1 (1, 2 or 3 in this build).
 *   grid_side   N: side of h (deconvolution) or of the PSF grid (PSF mode).
 *   n_sources   M point sources (deconvolution), >= 0.
 *   n_scales    J starlet planes including the coarse one, >= 1, with
 *               2^(J-1) <= N-1 so that one mirror fold covers every tap.
 *   w_pixel_stride  0: W holds J per-scale values; 1: W holds J*N*N maps.
 *   lambda      regularisation strength of the starlet L1 term (Eq. 6, Eq. 11).
 *   gauss_fwhm  FWHM of the target Gaussian r in fine pixels (2 in the paper,
 *               Sec. 2.1); at most about 3.04 (sigma <= 8/6.2), since r is evaluated
 *               within +-8 fine pixels of its centre (EINVAL above).
 *   conv_algo   STARRED_CONV_AUTO / DIRECT / FFT (deconvolution only). */
typedef struct {
    int32_t mode;
    int32_t n_frames;
    const int32_t *side_host;
    const int32_t *ksize_host;
    int32_t subsample;
    int32_t grid_side;
    int32_t n_sources;
    int32_t n_scales;
    int32_t w_pixel_stride;
    int32_t conv_algo;
    double lambda;
    double gauss_fwhm;
} starred_desc;

/* Optimiser hyper-parameters; lr is given per parameter block:
 *   deconvolution: lr[0] h, lr[1] Gamma, lr[2] a, lr[3] c
 *   PSF mode:      lr[0] eta_M, lr[1] b, lr[2] a, lr[3] c
 * rule: STARRED_ADAM (Kingma & Ba: v tracks g^2) or STARRED_ADABELIEF (Zhuang et
 * al.: v tracks (g - m)^2 + eps_root, m the updated first moment); both use the
 * bias corrections 1 - beta^t and the step lr m_hat / (sqrt(v_hat) + eps).
 * A zero-initialised struct's rule is Adam (eps_root is then unused). */
enum { STARRED_ADAM = 0, STARRED_ADABELIEF = 1 };
typedef struct {
    float lr[4];
    float beta1, beta2, eps;
    int32_t rule;
    float eps_root;
} starred_adam;

/* Create a plan: validates the description, builds the frame tables and the
 * work lists, allocates scratch. stream is a hipStream_t (NULL = default stream).
 * Returns EINVAL for bad descriptions, ENOMEM / EHIP on device failures. */
int starred_plan_create(const starred_desc *desc, void *stream, starred_plan **plan_out);
int starred_plan_destroy(starred_plan *plan);

/* Number of float parameters of the flat parameter vector:
 *   deconvolution: [h N^2 | Gamma E | a E*M (epoch-major, a[i*M+k]) | c M*2 (x,y)]
 *   PSF mode:      [eta_M 5 = (A, alpha_x, alpha_y, phi, beta) | b N^2 | a S | c S*2]
 * and of the packed data arrays (sum of n_i^2) and scenes (sum of (s n_i)^2). */
int64_t starred_num_params(const starred_plan *plan);
int64_t starred_num_data(const starred_plan *plan);
int64_t starred_num_scene(const starred_plan *plan);

/* Bind the observations (Eq. 4 and Eq. 10): data d_i (or star stamps t_k),
 * inverse variance w_i = diagonal of C^-1 (0 masks a pixel), the per-epoch
 * narrow-PSF kernels s_i (packed K_i^2; NULL in PSF mode) and the starlet weights
 * W (J values or J*N*N maps, see w_pixel_stride). The kernels are preprocessed
 * on the device (box-folded and phase-split copies owned by the plan); data,
 * inv_var and W are referenced, not copied. Synchronises the plan's stream. */
int starred_set_frames(starred_plan *plan, const float *data, const float *inv_var,
                       const float *psf, const float *W);

/* Eq. 9: scene f_i = Gamma_i + h[window_i] + sum_k a_ki r_k for every frame,
 * written packed (s n_i)^2. r_k is the Gaussian of FWHM gauss_fwhm centred at
 * c_k (unit integral, point-sampled). PSF mode: writes the narrow PSF
 * s = m(eta_M) + b (Eq. 2) on the N x N grid instead. */
int starred_render_scene(starred_plan *plan, const float *params, float *scene);

/* Eq. 8 without noise: model m_i = D S_i f_i for every frame (deconvolution).
 * scene packed (s n_i)^2, model packed n_i^2. S_i is the linear 'same'
 * convolution with zero padding. */
int starred_convolve_subsample(starred_plan *plan, const float *scene, float *model);

/* Adjoint of starred_convolve_subsample: grad_scene_i = S_i^T D^T resid_i.
 * Both are deconvolution-mode operators (EUNSUPPORTED in PSF mode). */
int starred_convolve_subsample_adj(starred_plan *plan, const float *resid, float *grad_scene);

/* PSF mode, Eq. 3 without noise: star models m_k = D(s * a_k r_k), s = m(eta_M) + b,
 * r_k the Gaussian of FWHM gauss_fwhm shifted by c_k from the grid centre
 * floor(N/2). params in the PSF-mode layout; model packed S x n^2. */
int starred_psf_model(starred_plan *plan, const float *params, float *model);

/* Starlet transform Phi^T (Eq. 6): coeffs = J planes of N^2; plane j < J-1 is
 * c_j - c_{j+1}, plane J-1 the coarse c_{J-1}; c_0 = img, c_{j+1} = H_j c_j with
 * the B3 filter [1,4,6,4,1]/16 at dilation 2^j and a whole-sample mirror
 * boundary. starred_starlet_adj applies the exact transpose Phi. */
int starred_starlet_fwd(starred_plan *plan, const float *img, float *coeffs);
int starred_starlet_adj(starred_plan *plan, const float *coeffs, float *img);

/* Loss and gradient (Eq. 11 with lambda_pts = 0, or Eq. 7 in PSF mode).
 * loss_out: device double[3] = {1/2 chi^2, lambda ||W o Phi^T h||_1, total}.
 * grad (same layout as params) may be NULL: forward only (line searches).
 * Deterministic: no floating-point atomics; repeated calls give identical bits. */
int starred_loss_grad(starred_plan *plan, const float *params, float *grad, double *loss_out);

/* Baseline for measurement: the same loss and gradient computed the plain way,
 * epoch after epoch with one launch per operator (render, full-resolution
 * convolution S_i, block sum D, residual, D^T, full-resolution correlation
 * S_i^T, per-frame sums) and no fusion or graph. Results equal
 * starred_loss_grad's up to rounding. The psf kernels passed to
 * starred_set_frames must stay valid (they are re-read on the first call). */
int starred_loss_grad_plain(starred_plan *plan, const float *params, float *grad, double *loss_out);

/* One optimiser step: loss_grad at params, then the update (hp->rule: Adam or
 * AdaBelief) of params, m and v in place, t = step number starting at 1. The plan keeps
 * the gradient in its own scratch. loss_out as above (may be NULL). */
int starred_step(starred_plan *plan, float *params, float *m, float *v, int32_t t,
                 const starred_adam *hp, double *loss_out);

/* n_steps >= 1 consecutive optimiser steps, the same as starred_step with t, t+1,
 * ..., t+n_steps-1 (bitwise: the same launches in the same order); in graph mode
 * several steps share one graph launch. loss_out holds the last step's loss. The
 * paper's fits run hundreds of such steps (Sec. 2.4). */
int starred_steps(starred_plan *plan, float *params, float *m, float *v, int32_t t,
                  const starred_adam *hp, int32_t n_steps, double *loss_out);

/* The two-loop recursion alone (Nocedal & Wright Alg. 7.4): d_out = -H grad for the
 * `count` newest pairs of the caller's ring buffers S, Y ([m][num_params] floats,
 * device, newest pair at slot `newest`, older ones before it modulo m) and
 * H_0 = gamma I, gamma = s^T y / y^T y of the newest pair; count = 0: -grad.
 * count <= min(m, 1024). One launch on the plan's stream. */
int starred_lbfgs_direction(starred_plan *plan, const float *grad, const float *S, const float *Y, int32_t m,
                            int32_t count, int32_t newest, float *d_out);

/* L-BFGS-B (Byrd, Lu, Nocedal & Zhu; the projected subspace step of Morales &
 * Nocedal), the bound-constrained quasi-Newton method of the paper's PSF fits, as a
 * host-side iteration in FP64 driven by reverse communication: each iteration
 * takes the generalized Cauchy point of the quadratic model along the projected
 * steepest-descent path, minimises the model over the variables free there (the
 * result projected onto the box, or cut back to it when the projection is not a
 * descent direction), then searches the line with Moré-Thuente steps (sufficient
 * decrease 1e-3, curvature 0.9, first trial 1, or 1/|d| on the first iteration when
 * not every variable is bounded, never past the box) and stores the correction
 * pair when s^T y is safely positive (history m). Stops when the projected
 * gradient's largest entry is <= pgtol or the relative decrease of f is below
 * factr times the machine epsilon (scipy's defaults: m 10, factr 1e7, pgtol 1e-5,
 * maxls 20).
 * create: n variables, host bounds lo/hi (NULL or +-inf entries: unbounded).
 * iterate: x (host, n doubles) is projected into the box and returned on the first
 * call (task FG); afterwards pass f and g (host) at the current x each time. Tasks:
 * FG (evaluate at the updated x and call again), NEW_X (an iteration ended at x:
 * call again with the same f, g to continue), CONVERGED, ABNORMAL (no descent or
 * the line search failed without history). counts: iterations done and
 * evaluations requested. */
enum { STARRED_LBFGSB_FG = 1, STARRED_LBFGSB_NEW_X = 2, STARRED_LBFGSB_CONVERGED = 3, STARRED_LBFGSB_ABNORMAL = 4 };
typedef struct starred_lbfgsb starred_lbfgsb;
int starred_lbfgsb_create(int64_t n, int32_t m, const double *lo, const double *hi, double factr, double pgtol,
                          int32_t maxls, starred_lbfgsb **out);
int starred_lbfgsb_destroy(starred_lbfgsb *state);
int starred_lbfgsb_iterate(starred_lbfgsb *state, double *x, double f, const double *g, int32_t *task);
int starred_lbfgsb_counts(const starred_lbfgsb *state, int32_t *iterations, int32_t *evaluations);

/* L-BFGS-B on the plan's loss: the iteration of starred_lbfgsb_* (history m, scipy's
 * defaults otherwise) on the host, with the loss and gradient evaluated on the device
 * at every point it asks for (each evaluation synchronises the plan's stream and
 * copies the loss and the gradient to the host). lo, hi (device, num_params floats,
 * or NULL; +-inf entries are unbounded): box bounds, copied at creation. */
typedef struct starred_lbfgs starred_lbfgs;
int starred_lbfgs_create(starred_plan *plan, int32_t m, const float *lo, const float *hi, starred_lbfgs **state_out);
int starred_lbfgs_destroy(starred_lbfgs *state);
/* Forget the history and the stored gradient (call after changing x elsewhere). */
int starred_lbfgs_reset(starred_lbfgs *state);
/* Up to n_iter iterations from x (device, num_params floats, updated in place; it
 * must not change between calls except here, else reset first; the first call
 * projects it into the box). Stops early at convergence (projected gradient <= 1e-5
 * or relative decrease <= 1e7 eps) or when no descent is possible. *loss_out (host):
 * the loss at the final x; *n_evals_out (host, may be NULL): evaluations used. */
int starred_lbfgs_run(starred_lbfgs *state, float *x, int32_t n_iter, double *loss_out, int32_t *n_evals_out);

/* Graph mode. When enabled, starred_loss_grad and starred_step capture their
 * launch sequence into a HIP graph on the first call and replay it while the
 * argument pointers (and, for step, the Adam hyper-parameters) stay the same;
 * a change re-captures. The step number t lives in device memory and is
 * advanced by the step itself, so consecutive steps replay one graph. Needs a
 * non-default stream. 0 disables and frees the graphs. In graph mode stage
 * timing reports one STARRED_STAGE_GRAPH interval per call. */
int starred_set_graph_mode(starred_plan *plan, int32_t enable);

/* Eq. 11, third term: lambda_pts ||W (.) Phi^T sum_k <a_k> r_k||_1 with <a_k> the
 * mean over the epochs of a_ik and r_k rendered on the N x N grid of h. 0 (the
 * default) leaves the term out. Deconvolution mode; lambda_pts >= 0. Its gradient
 * reaches every a_ik (through <a_k>) and c_k. Drops captured graphs. */
int starred_set_lambda_pts(starred_plan *plan, double lambda_pts);

/* The image that term regularises: P_out (device, N x N) = sum_k <a_k> r_k at
 * params (r_k within 8 fine pixels of c_k, as in the scene). */
int starred_pts_image(starred_plan *plan, const float *params, float *P_out);

/* App. C: the estimate of lambda_pts at params (device, num_params floats),
 *   lambda (||W (.) Phi^T f||_1 - ||W (.) Phi^T h||_1) / sum_k <a_k> ||W (.) Phi^T r_k||_1,
 * f = <Gamma> + h + sum_k <a_k> r_k the epoch average of the scene on the N x N grid,
 * W the bound weights. Writes the value to *lambda_pts_out (host) and synchronises
 * the plan's stream. Deconvolution mode with n_sources >= 1; set_frames first. */
int starred_estimate_lambda_pts(starred_plan *plan, const float *params, double *lambda_pts_out);

/* FFT algorithm, loss and gradient: frames whose Q x Q model and residual
 * spectra fit in LDS (Q = P/s, see the FFT notes of starred_plan_create) run the
 * forward of Eqs. 8 and 10 in one launch with a work group per frame; with
 * enable = 0 every frame takes the batched line passes instead (same results up
 * to rounding order). Default 1. Drops captured graphs. */
int starred_set_fft_fused(starred_plan *plan, int32_t enable);

/* Which convolution algorithm the plan runs (STARRED_CONV_DIRECT or _FFT). */
int starred_conv_algo(const starred_plan *plan);

/* Shape classes of a deconvolution plan: the frames that share a (data side,
 * kernel side) pair. For each, the convolution algorithm it runs and, on the FFT
 * algorithm, the transform lengths P (fine grid) and Q = P/s (data grid) and
 * whether its forward is the one-launch form (fused = 1 with two LDS planes, 2 with
 * one plane transformed in place, for frames whose two planes do not fit) or the
 * batched line passes (0). starred_num_classes returns the count (>= 0) or a negative status;
 * starred_get_class_info fills *out for class c in [0, count). */
typedef struct {
    int32_t n, K, n_frames;
    int32_t algo;
    int32_t P, Q;
    int32_t fused;
    int32_t pad;
    double tune_ms[3];  /* autotuner: ms per loss+gradient evaluation of the whole plan with
                           this class on the direct algorithm, the FFT one-launch forward,
                           the FFT line passes (-1: not tried) */
} starred_class_info;
int starred_num_classes(const starred_plan *plan);
int starred_get_class_info(const starred_plan *plan, int32_t c, starred_class_info *out);

/* The autotuner (STARRED_CONV_AUTO, run by starred_set_frames): each shape class
 * gets the direct algorithm, the FFT algorithm with the one-launch forward or the
 * FFT algorithm with the line passes, by coordinate descent over the classes (most
 * costly first), each candidate timed as whole loss+gradient evaluations on the
 * plan's stream; then the launch shapes of the FFT path (work groups aimed at by
 * the spectral adjoint and by the line passes). Decisions are cached per process
 * by the plan's shapes (subsampling, grid, sources, scales and the multiset of
 * (n_i, K_i)) and device, so a second plan of the same shapes reuses them.
 * starred_autotune_info reports the host milliseconds of the tuning that made the
 * plan's decision (0 when none ran; with a cached decision, the time of the tuning
 * that filled the cache), whether the decision came from the cache, and the launch
 * shapes in use: work groups aimed at by the frequency-domain adjoint and by the
 * line passes, frames per adjoint chunk, whether the one-launch forward runs on a
 * stream of its own, and whether the prior forks after the forward (any pointer may be
 * NULL). */
int starred_autotune_info(const starred_plan *plan, double *wall_ms_out, int32_t *cached_out,
                          int32_t *adj_blocks_out, int32_t *line_groups_out, int32_t *adj_frames_out,
                          int32_t *split_forward_out, int32_t *prior_late_out);

/* Per-frame shifts and rotations (the joint processing of epochs that differ by a
 * shift and a rotation, as in the paper's conclusions; the per-epoch dithering
 * offsets of its supernova application). xf: device array [n_frames][3] =
 * (dx_i, dy_i, theta_i), referenced, not copied. Frame i then observes the scene
 * at u = R(theta_i)(X - C) + C + (dx_i, dy_i) for its fine pixel at grid position X,
 * C = ((N-1)/2, (N-1)/2), R the counter-clockwise rotation: h is read there by
 * bilinear interpolation (zero outside the grid) and point source k contributes
 * a_ik r(u - c_k); t_i = 0 is Eq. 9. The data term's gradient in h is the exact
 * transpose of that interpolation. grad_xf (device [n_frames][3], or NULL):
 * loss_grad also writes dL/d(dx_i, dy_i, theta_i) there, so that offsets can be
 * fitted. Each frame's scene is rendered under its transform; setting transforms
 * moves every class off the shared class spectra (EUNSUPPORTED when the kernels
 * exceed the direct tiles), and algo chooses how the rendered frames are convolved:
 * STARRED_CONV_DIRECT (the direct kernels), STARRED_CONV_FFT (each frame through its
 * own spectrum: a P-size forward transform of its rendered window, the spectral
 * product and alias fold, and a P-size inverse in the adjoint), or STARRED_CONV_AUTO
 * (both timed on the bound data when frames are bound, else the spectra). xf = NULL
 * clears them and restores the previous choices. Drops captured graphs. The plain
 * baseline does not support them. */
int starred_set_frame_transforms(starred_plan *plan, const float *xf, float *grad_xf, int32_t algo);
/* The convolution chosen for frames with transforms (*algo_out: STARRED_CONV_DIRECT or
 * STARRED_CONV_FFT, 0 when none are set) and, when STARRED_CONV_AUTO timed it, the
 * milliseconds per loss+gradient evaluation with each (ms_out[2]: direct, spectra;
 * -1 when not timed). Either pointer may be NULL. */
int starred_frame_transforms_info(const starred_plan *plan, int32_t *algo_out, double *ms_out);

/* Launch shapes of the deconvolution FFT path (what the autotuner chooses; 0 keeps
 * the current value): adj_frames, frames per chunk of the frequency-domain adjoint
 * (2 or 4; 8 with at most one point source; 1 with more than eight; one summed
 * spectrum per chunk goes through memory; a chunk of one frame takes 16 sources per
 * pass over its spectra, two frames 8 when there are more than four, otherwise 4);
 * adj_blocks, work groups its launch aims at; line_groups, work groups a line pass
 * aims at; split_forward (-1 keeps it): 1
 * runs the one-launch forward of the smaller classes on a second stream of the plan,
 * beside the line passes of the larger ones (forked from and joined back into the
 * plan's stream, also inside captured graphs), 0 runs everything in order. Results
 * agree up to rounding for every choice (bitwise for split_forward). prior_late (-1
 * keeps it): 1 forks the starlet prior onto its stream after the forward's launches, so
 * that it runs beside the adjoint, 0 at the start of the evaluation, beside the forward
 * (bitwise the same results); 2 carries its passes in the evaluation's own launches as
 * extra work groups where they can ride (every frame on the FFT algorithm with the
 * one-launch forward, composite filters, no point-source prior; otherwise as 1); 3 forks
 * it after the adjoint's spectral products, beside the chunk sums and the dL/dh inverse
 * (with a gradient; otherwise as 1). Drops captured graphs. EINVAL for other values. */
int starred_set_fft_shapes(starred_plan *plan, int32_t adj_frames, int32_t adj_blocks, int32_t line_groups,
                           int32_t split_forward, int32_t prior_late);

/* Force the algorithm of shape class c: STARRED_CONV_DIRECT, or STARRED_CONV_FFT with
 * the one-launch forward (fused = 1, where it fits) or the line passes (fused = 0).
 * Frames of different classes may run different algorithms in one evaluation; the
 * results agree up to rounding. Drops captured graphs. EUNSUPPORTED when the class's
 * kernels do not fit the direct path's tiles. */
int starred_set_class_algo(starred_plan *plan, int32_t c, int32_t algo, int32_t fused);

/* Stage timing, for measurement. While enabled, loss_grad and step record a
 * pair of HIP events on the plan's stream around each stage below, and each
 * call first runs a short idle kernel (about 1 ms) on that stream, so that the
 * call's launches are queued before they run and an interval holds device
 * time only, not host launch gaps.
 * starred_profile_read synchronises the stream, returns per stage the summed
 * milliseconds (ms_out[STARRED_NUM_STAGES]) and the number of timed launches
 * (count_out[STARRED_NUM_STAGES]; either pointer may be NULL), then resets. */
enum {
    STARRED_STAGE_RENDER = 0,   /* scene rendering (Eq. 9) */
    STARRED_STAGE_CONV_FWD,     /* S_i and D with the residual and chi-square (Eqs. 8, 10) */
    STARRED_STAGE_CONV_ADJ,     /* S_i^T D^T of the weighted residuals */
    STARRED_STAGE_GRAD_SUMS,    /* per-frame sums for Gamma, a and c */
    STARRED_STAGE_STARLET,      /* starlet transform, L1 term, subgradient and adjoint (Eq. 6) */
    STARRED_STAGE_FINALIZE,     /* cross-frame gradient of h and the final reductions */
    STARRED_STAGE_ADAM,         /* optimiser update */
    STARRED_STAGE_SPECTRA,      /* FFT path: spectra shared by all frames */
    STARRED_STAGE_GRAPH,        /* graph mode: one whole captured loss_grad or step */
    STARRED_STAGE_FFT_SPEC,     /* FFT path, inside CONV_FWD: spectral product and alias fold */
    STARRED_STAGE_FFT_MCOLS,    /* ... inverse along the first axis of the model spectra */
    STARRED_STAGE_FFT_MROWS,    /* ... inverse rows, residual, chi-square, forward rows of rho */
    STARRED_STAGE_FFT_RCOLS,    /* FFT path, inside CONV_ADJ: forward columns of rho */
    STARRED_STAGE_FFT_ACOLS,    /* ... kernel-spectrum products, their sum over frames and the
                                   per-frame dot products for Gamma, a and c */
    STARRED_STAGE_FFT_AROWS,    /* ... inverse transform of the summed spectra (dL/dh) */
    STARRED_STAGE_FFT_FSUM,     /* ... sums of the frame-chunk spectra and of the per-block
                                   dot products per frame */
    STARRED_STAGE_FFT_FUSED,    /* FFT path, inside CONV_FWD: one-launch forward of the frames
                                   whose spectra fit in LDS (product, both 2-D transforms,
                                   residual, chi-square) */
    STARRED_STAGE_DIRECT_FWD,   /* the direct algorithm's fused S_i + D forward with the residual
                                   and chi-square, over the frames of the classes that run it */
    STARRED_STAGE_DIRECT_ADJ,   /* the direct algorithm's S_i^T D^T over those frames */
    STARRED_NUM_STAGES
};
int starred_set_profiling(starred_plan *plan, int32_t enable);
int starred_profile_read(starred_plan *plan, double *ms_out, int64_t *count_out);

/* Sec. 2.3 and App. B: the starlet weights W by noise propagation (Monte Carlo).
 * Deconvolution mode, after starred_set_frames. For n_real realizations, white
 * noise is drawn on the fine grid of frame `frame` (side s n_f) with the variance
 * of its data pixel replicated over each s x s block (C_up: sigma2_data, device,
 * n_f^2 values, > 0; the caller chooses the map, e.g. the frame's own or that of
 * the co-added data), weighted by C_up^-1, correlated with the frame's bound
 * kernel (S^T), placed in the frame's window of the N x N grid and transformed
 * (Phi^T). W_out (device) receives the standard deviation over the realizations
 * (mean removed, divided by n_real) of every coefficient, J x N x N
 * (per_pixel = 1), or of all coefficients of each scale, J values (per_pixel = 0);
 * these are the W inputs of set_frames with w_pixel_stride 1 or 0.
 * normals: device array [n_real][(s n_f)^2] of standard normal draws, or NULL to
 * draw them on the device: draw k of realization r is the Box-Muller value of
 * Philox4x32-10 with counter (k/4, r, 0, 0) and key (seed low, seed high), words
 * mapped to ((w >> 8) + 1/2) / 2^24, pairs (0,1) and (2,3), cosine then sine.
 * n_real >= 2. The plan allocates its working memory on the first call (kept
 * until destroy); the call synchronises the plan's stream. */
int starred_noise_weights(starred_plan *plan, int32_t frame, const float *sigma2_data, int32_t n_real,
                          uint64_t seed, const float *normals, int32_t per_pixel, float *W_out);

/* Measurement aid: the device time of one stage's launches alone. Runs one
 * loss+gradient evaluation at params (device, num_params floats) so that every
 * buffer the stage reads holds real data, then launches the stage reps times back
 * to back between two HIP events on the plan's stream (after a short idle lead-in,
 * so that the launches are queued ahead of the device) and writes the average
 * milliseconds per repetition to *ms_out (host). Blocks until done. Stages:
 * deconvolution mode, FFT algorithm: SPECTRA, FFT_FUSED, FFT_SPEC, FFT_MCOLS,
 * FFT_MROWS, FFT_RCOLS, FFT_ACOLS, FFT_FSUM, FFT_AROWS; direct algorithm: RENDER, CONV_FWD,
 * CONV_ADJ, GRAD_SUMS; both: STARLET. Other stages, PSF mode: STARRED_EUNSUPPORTED.
 * The plan's internal work buffers are left in an unspecified state (the next
 * evaluation recomputes them); caller-owned memory is not touched. */
int starred_time_stage(starred_plan *plan, const float *params, int32_t stage, int32_t reps, double *ms_out);

/* Measurement aid: a plain device copy of n floats (n a multiple of 4) from src to
 * dst on the plan's stream; its memory-counter readings calibrate the ones of the
 * library's kernels. */
int starred_copy_probe(starred_plan *plan, const float *src, float *dst, int64_t n);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, hosts that forbid allocation): the starlet transform of
 * starred_starlet_fwd without a plan. img (N x N) and coeffs (J planes of N^2) are
 * the caller's device arrays; the two working planes of the cascade live in one
 * fixed device array of the library (2 x 512 x 512 floats plus 16, about 2 MiB,
 * held on each device it runs on until the process ends), so the call allocates
 * nothing. Limits: 2 <= N <= 512, 1 <= J <= 16, 2^(J-1) <= N-1; larger requests
 * return STARRED_EINVAL. Enqueues on stream (a hipStream_t, NULL = default) without
 * synchronising. Every call on a device shares that device's working array, so
 * calls that may overlap on one device (different streams or host threads without
 * ordering) race; calls on one stream are ordered and safe. Coefficients equal
 * starred_starlet_fwd's up to rounding (that call may evaluate the scales by
 * composite filters in FP64). */
int starred_starlet_fwd_noalloc(int32_t N, int32_t J, const float *img, float *coeffs, void *stream);

const char *starred_last_error(void);
int starred_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STARRED_H */
