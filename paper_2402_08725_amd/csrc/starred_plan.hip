// Host side of the C ABI (include/starred.h): plan validation, frame tables,
// work lists, scratch ownership and the launch sequences of loss_grad / step.
#include "starred.h"
#include "starred_dense.h"
#include "starred_fft.h"
#include "starred_finalize.h"
#include "starred_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <mutex>
#include <cmath>
#include <complex>
#include <map>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace starred;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *msg)
{
    g_last_error = msg;
    return code;
}

int fail_hip(hipError_t e, const char *where)
{
    char buf[512];
    snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    g_last_error = buf;
    return e == hipErrorOutOfMemory ? STARRED_ENOMEM : STARRED_EHIP;
}

// s_sleep periods of the idle lead-in that stage timing puts before each call
constexpr int kProfIdleIters = 300;
// noise propagation: realizations per batch
constexpr int kNoiseBatch = 32;

#define HIP_TRY(expr)                                     \
    do {                                                  \
        hipError_t _e = (expr);                           \
        if (_e != hipSuccess) return fail_hip(_e, #expr); \
    } while (0)

int round_up(int a, int b) { return (a + b - 1) / b * b; }
int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

template <typename T>
int dev_alloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) return fail_hip(e, "hipMalloc");
    return STARRED_OK;
}

}  // namespace

// the calling thread's last error, for the entry points of other files
int starred_set_error(int code, const char *msg) { return fail(code, msg); }

struct starred_plan {
    int mode = 0, E = 0, s = 1, N = 0, M = 0, J = 1, w_stride = 0, algo = STARRED_CONV_DIRECT;
    double lam = 0.0, fwhm = 2.0;
    float sigma = 0.f;
    hipStream_t st = nullptr;

    std::vector<int> n, K;
    std::vector<FrameDev> fr;
    FrameDev *d_fr = nullptr;
    std::vector<Item> fwd_items, adj_items;
    Item *d_fwd_items = nullptr, *d_adj_items = nullptr;
    int Tmax = 0, Ar_max = 0, Bpad_max = 0, Fmax = 0;
    long long ndata = 0, nfine = 0, nparams = 0, nkern = 0, nkf = 0, nka = 0;

    const float *data = nullptr, *invvar = nullptr, *W = nullptr;
    bool frames_set = false;

    float *d_kf = nullptr, *d_ka = nullptr;
    float *d_scene = nullptr, *d_rho = nullptr, *d_g = nullptr;
    double *d_part_chi = nullptr, *d_part_l1 = nullptr, *d_fsum = nullptr;
    float *d_z = nullptr, *d_ca = nullptr, *d_cb = nullptr, *d_tmp = nullptr, *d_prior = nullptr;
    // Eq. 11, third term: weight, [h | P] images, shares of dL/da and dL/dc (3M)
    double lam_pts = 0.0;
    float *d_pair = nullptr;
    double *d_pts = nullptr;
    double *d_lbfgs_alpha = nullptr;  // two-loop coefficients of starred_lbfgs_direction
    // its App. C estimate: images [f | h | r_k], L1 partials, norms and <a_k>
    float *est_img = nullptr;
    double *est_part = nullptr, *est_out = nullptr;
    float *d_grad = nullptr;
    float *d_wzero = nullptr;
    // the prior through the per-scale composite filters (when they fit): taps and
    // the row-filtered, smoothed and adjoint planes, for up to dense_b images
    bool dense = false;
    int dense_b = 0;
    double *d_dense_taps = nullptr, *d_dense_T = nullptr, *d_dense_C = nullptr, *d_dense_U = nullptr;
    float *d_hpart = nullptr;
    int hpart_chunks = 0;  // partial planes d_hpart holds
    double *d_gxfp = nullptr;  // partials of the transforms' gradient
    std::vector<void *> owned;
    // noise propagation: an s = 1 plan applying S_f^T to a batch of noise fields
    starred_plan *noise_aux = nullptr;
    int noise_frame = -1, noise_B = 0;
    float *nz_kern = nullptr, *nz_zero = nullptr, *nz_one = nullptr, *nz_w = nullptr;
    float *nz_delta = nullptr, *nz_g = nullptr, *nz_img = nullptr, *nz_ca = nullptr, *nz_cb = nullptr;
    float *nz_coef = nullptr;
    double *nz_s1 = nullptr, *nz_s2 = nullptr;

    // FFT path
    bool fft_ready = false;
    bool fft_fused = true;
    FftPlanDev fd;
    std::vector<ClassFft> cls;
    std::vector<FrameFft> ffr;
    std::vector<int> fcls;        // class of each frame
    std::vector<int> cls_frames;  // frames in class order
    std::vector<int> cls_fits;    // per class: the one-launch forward fits in LDS (1: two planes, 2: one in place)
    double *d_part_chi_fft = nullptr;  // chi-square partials: FFT groups, then direct tiles
    int n_fft_chi = 0;
    // launch shapes of the FFT path: work groups aimed at by the spectral adjoint
    // and by the line passes (the autotuner may change them)
    int adj_blocks = kAdjBlocks, line_groups = 1024, adj_fc = kAdjFrames;
    // frames of the classes that run the direct algorithm, and their LDS extents
    std::vector<int> fdir;
    int *d_fdir = nullptr;
    int Tdir = 0, Ardir = 0, Bpdir = 0, Fdir = 0;
    int fwd_groups = 0, adj_groups = 0;  // persistent grids of the direct kernels
    float *d_hdir = nullptr;  // prior gradient plus the direct frames' windows of dL/dh
    // per-frame transforms (device E x 3: dx, dy, theta; caller-owned) and the
    // caller's buffer for their gradient (or null); the class choices before they
    // were set (restored when they are cleared)
    const float *xf = nullptr;
    float *gxf = nullptr;
    std::vector<int> xf_prev_choice;
    // autotuner: per class the ms of an evaluation with each choice tried
    // (direct, FFT one-launch forward, FFT line passes; < 0 = not tried), the
    // host time it took and whether its decision came from the cache
    std::vector<std::array<double, 3>> cls_tune;
    double tune_wall_ms = 0.0;
    int tune_cached = 0;
    // work lists (rebuilt with the per-class choices): freed on rebuild
    std::vector<void *> list_owned;
    // plain per-epoch baseline (s = 1 tables at fine resolution)
    bool plain_ready = false;
    std::vector<FrameDev> frp;
    FrameDev *d_frp = nullptr;
    Item *d_pfwd = nullptr, *d_padj = nullptr;
    std::vector<int> pfwd_start, padj_start, pchi_start;
    int pTmax = 0, pAr_max = 0, pBpad_max = 0, n_pchi = 0;
    float *d_pkf = nullptr, *d_pka = nullptr, *d_u = nullptr, *d_gh = nullptr, *d_m = nullptr;
    double *d_pchi = nullptr;
    const float *psf_bound = nullptr;

    // PSF mode
    int psf_n = 0;
    float *d_dm = nullptr;
    double *d_s64 = nullptr;
    double *d_part_eta = nullptr;
    int algo_req = STARRED_CONV_AUTO;
    bool direct_ok = true;

    // starlet branch: a second stream forked from and joined back into st
    hipStream_t st2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // FFT path: the one-launch forward on a third stream, beside the line passes of
    // the larger classes (their frames are independent until the adjoint)
    hipStream_t st3 = nullptr;
    hipEvent_t ev_fork3 = nullptr, ev_join3 = nullptr;
    int fwd_split = 1;
    // FFT path, prior on the forked stream: forked after the forward's launches (beside
    // the adjoint) instead of at the start of the evaluation (beside the forward)
    int prior_late = 0;
    // frames with per-frame transforms: convolved through their own spectra (1) or by the
    // direct kernels (0)
    int xf_fft = 0;
    double xf_ms[2] = {-1.0, -1.0};  // timings of that choice: direct, spectra (-1: not timed)
    int *d_t = nullptr;
    int next_t = -1;  // step number the device counter will produce next (-1: unknown)

    // captured graphs (slot 0: loss_grad, slot 1: step, slot 2: kStepsPerGraph steps)
    bool graph_mode = false;
    struct GraphSlot {
        bool valid = false;
        hipGraph_t g = nullptr;
        hipGraphExec_t x = nullptr;
        std::vector<uintptr_t> key;
    } gs[3];

    // stage timing
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_next = 0;
    struct Rec { int stage; hipEvent_t a, b; };
    std::vector<Rec> recs;
    double prof_ms[STARRED_NUM_STAGES] = {};
    long long prof_cnt[STARRED_NUM_STAGES] = {};

    hipEvent_t prof_start(hipStream_t s = nullptr)
    {
        if (!prof_on) return nullptr;
        if (ev_next == ev_pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            ev_pool.push_back(e);
        }
        hipEvent_t e = ev_pool[ev_next++];
        (void)hipEventRecord(e, s ? s : st);
        return e;
    }
    void prof_stop(int stage, hipEvent_t a, hipStream_t s = nullptr)
    {
        if (!prof_on || !a) return;
        hipEvent_t b = prof_start(s);
        if (b) recs.push_back({stage, a, b});
    }
    void drop_graphs()
    {
        for (auto &g : gs) {
            if (g.x) (void)hipGraphExecDestroy(g.x);
            if (g.g) (void)hipGraphDestroy(g.g);
            g = GraphSlot();
        }
    }
    int prof_collect()
    {
        if (recs.empty()) return STARRED_OK;
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
        for (const Rec &r : recs) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, r.a, r.b);
            if (e != hipSuccess) return fail_hip(e, "hipEventElapsedTime");
            prof_ms[r.stage] += ms;
            prof_cnt[r.stage] += 1;
        }
        recs.clear();
        ev_next = 0;
        return STARRED_OK;
    }

    ~starred_plan();
    void destroy_members()
    {
        drop_graphs();
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (st2) (void)hipStreamDestroy(st2);
        if (ev_fork3) (void)hipEventDestroy(ev_fork3);
        if (ev_join3) (void)hipEventDestroy(ev_join3);
        if (st3) (void)hipStreamDestroy(st3);
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        for (void *p : owned) (void)hipFree(p);
        free_lists();
    }
    template <typename T>
    int alloc(T **p, size_t count)
    {
        int rc = dev_alloc(p, count);
        if (rc == STARRED_OK) owned.push_back((void *)*p);
        return rc;
    }
    template <typename T>
    int alloc_list(T **p, size_t count)
    {
        int rc = dev_alloc(p, count);
        if (rc == STARRED_OK) list_owned.push_back((void *)*p);
        return rc;
    }
    void free_lists()
    {
        for (void *q : list_owned) (void)hipFree(q);
        list_owned.clear();
    }
};

extern "C" {

const char *starred_last_error(void) { return g_last_error.c_str(); }
int starred_abi_version(void) { return STARRED_ABI_VERSION; }

static int validate(const starred_desc *d)
{
    if (!d) return fail(STARRED_EINVAL, "desc is NULL");
    if (d->mode != STARRED_DECONV && d->mode != STARRED_PSF) return fail(STARRED_EINVAL, "unknown mode");
    if (d->n_frames < 1) return fail(STARRED_EINVAL, "n_frames must be >= 1");
    if (!d->side_host) return fail(STARRED_EINVAL, "side_host is NULL");
    if (d->subsample < 1 || d->subsample > 3) return fail(STARRED_EINVAL, "subsample must be 1, 2 or 3");
    if (d->grid_side < 2 || d->grid_side > 4096) return fail(STARRED_EINVAL, "grid_side out of range");
    if (d->n_scales < 1) return fail(STARRED_EINVAL, "n_scales must be >= 1");
    if (d->n_scales > 1 && (1 << (d->n_scales - 1)) > d->grid_side - 1)
        return fail(STARRED_EINVAL, "2^(J-1) must not exceed grid_side-1");
    if (d->w_pixel_stride != 0 && d->w_pixel_stride != 1) return fail(STARRED_EINVAL, "w_pixel_stride must be 0 or 1");
    if (!(d->gauss_fwhm > 0.0)) return fail(STARRED_EINVAL, "gauss_fwhm must be > 0");
    // r is evaluated within +-kGaussRadius fine pixels of its centre: the mass beyond
    // the box must stay negligible (below 1e-9 of the total: sigma <= R / 6.2)
    if (d->gauss_fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0))) > kGaussRadius / 6.2)
        return fail(STARRED_EINVAL, "gauss_fwhm above 3.0 fine pixels: r would be cut by its +-8 px evaluation box");
    if (!(d->lambda >= 0.0)) return fail(STARRED_EINVAL, "lambda must be >= 0");
    if (d->n_sources < 0) return fail(STARRED_EINVAL, "n_sources must be >= 0");
    for (int i = 0; i < d->n_frames; ++i) {
        const int n = d->side_host[i];
        if (n < 1) return fail(STARRED_EINVAL, "frame side must be >= 1");
        const int F = d->subsample * n;
        if (F > d->grid_side || ((d->grid_side - F) & 1))
            return fail(STARRED_EINVAL, "s*n_i must fit the grid with an integer central offset");
        if (d->mode == STARRED_DECONV) {
            if (!d->ksize_host) return fail(STARRED_EINVAL, "ksize_host is NULL");
            const int K = d->ksize_host[i];
            if (K < 1 || K > 512) return fail(STARRED_EINVAL, "kernel side must be in [1, 512]");
        }
    }
    if (d->mode == STARRED_DECONV) {
        if (d->conv_algo < STARRED_CONV_AUTO || d->conv_algo > STARRED_CONV_FFT)
            return fail(STARRED_EINVAL, "unknown conv_algo");
    } else {
        for (int i = 0; i < d->n_frames; ++i)
            if (d->side_host[i] * d->subsample != d->grid_side)
                return fail(STARRED_EINVAL, "PSF mode: every star stamp must have side grid_side/subsample");
    }
    return STARRED_OK;
}

// The composite-filter prior: taps and planes for up to B images, when the
// grid and the scale count fit it (else the prior runs the cascade).
static int dense_setup(starred_plan *p, int B)
{
    p->dense = dense_fits(p->N, p->J);
    if (!p->dense) return STARRED_OK;
    p->dense_b = B;
    const size_t planes = (size_t)B * p->J * p->N * p->N;
    int rc;
    if ((rc = p->alloc(&p->d_dense_taps, (size_t)dense_num_taps(p->J)))) return rc;
    if ((rc = p->alloc(&p->d_dense_T, planes))) return rc;
    if ((rc = p->alloc(&p->d_dense_C, planes))) return rc;
    if ((rc = p->alloc(&p->d_dense_U, planes))) return rc;
    std::vector<double> taps(dense_num_taps(p->J));
    dense_taps(p->J, taps.data());
    HIP_TRY(hipMemcpy(p->d_dense_taps, taps.data(), sizeof(double) * taps.size(), hipMemcpyHostToDevice));
    return STARRED_OK;
}

static DenseStar dense_desc(const starred_plan *p, int B, const float *img)
{
    DenseStar d;
    d.N = p->N;
    d.J = p->J;
    d.B = B;
    d.rx = dense_rows_per_job(p->N);
    d.taps = p->d_dense_taps;
    d.img = img;
    d.T = p->d_dense_T;
    d.C = p->d_dense_C;
    d.U = p->d_dense_U;
    d.W = p->W;
    d.w_stride = p->w_stride;
    d.lam0 = d.lam1 = (float)p->lam;
    return d;
}

static size_t dense_l1_slots(const starred_plan *p)
{
    return p->dense ? (size_t)dense_desc(p, p->dense_b, nullptr).l1_slots() : 0;
}

static int build_deconv(starred_plan *p)
{
    const int s = p->s, E = p->E;
    p->fr.resize(E);
    long long doff = 0, foff = 0, koff = 0, kfoff = 0, kaoff = 0;
    for (int i = 0; i < E; ++i) {
        FrameDev &f = p->fr[i];
        memset(&f, 0, sizeof f);
        f.n = p->n[i];
        f.F = s * f.n;
        f.K = p->K[i];
        f.Kp = f.K + s - 1;
        f.o = (p->N - f.F) / 2;
        f.cp = f.K / 2 + s - 1;
        f.Tpad = round_up((f.Kp + s - 1) / s, 4);
        f.dmin = -(f.cp / s);  // ceil(-cp/s) = -floor(cp/s): the smallest row shift of any phase
        const int dmax = floor_div(f.Kp - 1 + s - 1 - f.cp, s);
        f.Ar = dmax - f.dmin + 1;
        f.Bpad = round_up(f.Ar, 4);
        f.data_off = doff;
        f.fine_off = foff;
        f.kern_off = koff;
        f.kf_off = kfoff;
        f.ka_off = kaoff;
        doff += (long long)f.n * f.n;
        foff += (long long)f.F * f.F;
        koff += (long long)f.K * f.K;
        kfoff += (long long)f.Kp * s * f.Tpad;
        kaoff += (long long)s * s * f.Ar * f.Bpad;
        p->Tmax = std::max(p->Tmax, f.Tpad);
        p->Ar_max = std::max(p->Ar_max, f.Ar);
        p->Bpad_max = std::max(p->Bpad_max, f.Bpad);
        p->Fmax = std::max(p->Fmax, f.F);
    }
    p->ndata = doff;
    p->nfine = foff;
    p->nkern = koff;
    p->nkf = kfoff;
    p->nka = kaoff;
    p->nparams = (long long)p->N * p->N + E + (long long)E * p->M + 2LL * p->M;

    int rc;
    if ((rc = p->alloc(&p->d_fr, E))) return rc;
    HIP_TRY(hipMemcpy(p->d_fr, p->fr.data(), sizeof(FrameDev) * E, hipMemcpyHostToDevice));

    const long long NN = (long long)p->N * p->N;
    if ((rc = p->alloc(&p->d_kf, p->nkf))) return rc;
    if ((rc = p->alloc(&p->d_ka, p->nka))) return rc;
    if ((rc = p->alloc(&p->d_scene, p->nfine))) return rc;
    if ((rc = p->alloc(&p->d_rho, p->ndata))) return rc;
    if ((rc = p->alloc(&p->d_g, p->nfine))) return rc;
    if ((rc = dense_setup(p, 2))) return rc;
    if ((rc = p->alloc(&p->d_part_l1, std::max((size_t)2 * starlet_l1_slots(p->N, p->J), dense_l1_slots(p)))))
        return rc;
    if ((rc = p->alloc(&p->d_fsum, (size_t)E * (1 + 3 * p->M)))) return rc;
    // two images (h and the point-source image P of Eq. 11) for the prior buffers
    if ((rc = p->alloc(&p->d_z, (size_t)2 * p->J * NN))) return rc;
    if ((rc = p->alloc(&p->d_ca, 2 * NN))) return rc;
    if ((rc = p->alloc(&p->d_cb, 2 * NN))) return rc;
    if ((rc = p->alloc(&p->d_pair, 2 * NN))) return rc;
    if ((rc = p->alloc(&p->d_pts, (size_t)3 * std::max(1, p->M)))) return rc;
    if ((rc = p->alloc(&p->d_tmp, NN))) return rc;
    if ((rc = p->alloc(&p->d_prior, 2 * NN))) return rc;
    p->hpart_chunks = finalize_h_chunks(E);
    if ((rc = p->alloc(&p->d_hpart, (size_t)p->hpart_chunks * NN))) return rc;
    if ((rc = p->alloc(&p->d_gxfp, (size_t)xf_grad_parts(E)))) return rc;
    if ((rc = p->alloc(&p->d_hdir, NN))) return rc;
    if ((rc = p->alloc(&p->d_grad, p->nparams))) return rc;
    if ((rc = p->alloc(&p->d_wzero, (size_t)p->J * NN))) return rc;
    HIP_TRY(hipMemset(p->d_wzero, 0, sizeof(float) * p->J * NN));
    return STARRED_OK;
}

// The direct path's work lists over the frames of the classes that run it
// (every frame when the plan has no classes yet): tiles of those frames; the
// partial-result slots are enumerated frame by frame, the launch order is
// longest first (cost ~ folded kernel area) so that ragged batches balance
// across the compute units, and the launches are persistent (a fixed grid that
// walks the list).
static int build_direct_lists(starred_plan *p)
{
    const int s = p->s, E = p->E;
    p->fwd_items.clear();
    p->adj_items.clear();
    p->fdir.clear();
    p->Tdir = p->Ardir = p->Bpdir = p->Fdir = 0;
    for (int i = 0; i < E; ++i)
        if (p->cls.empty() || p->cls[p->fcls[i]].direct) {
            const FrameDev &f = p->fr[i];
            p->fdir.push_back(i);
            p->Tdir = std::max(p->Tdir, f.Tpad);
            p->Ardir = std::max(p->Ardir, f.Ar);
            p->Bpdir = std::max(p->Bpdir, f.Bpad);
            p->Fdir = std::max(p->Fdir, f.F);
        }
    struct Cost { long long c; Item it; };
    std::vector<Cost> fw, ad;
    int slot = 0;
    for (int i : p->fdir) {
        const FrameDev &f = p->fr[i];
        for (int p0 = 0; p0 < f.n; p0 += kFwdTP)
            for (int q0 = 0; q0 < f.n; q0 += kFwdTQ) {
                Item it{i, p0, q0, slot++};
                fw.push_back({(long long)f.Kp * s * f.Tpad, it});
            }
    }
    slot = 0;
    for (int i : p->fdir) {
        const FrameDev &f = p->fr[i];
        for (int p0 = 0; p0 < f.n; p0 += kAdjTP)
            for (int q0 = 0; q0 < f.n; q0 += kAdjTQ) {
                Item it{i, p0, q0, slot++};
                ad.push_back({(long long)s * s * f.Ar * f.Bpad, it});
            }
    }
    auto by_cost = [](const Cost &a, const Cost &b) { return a.c > b.c; };
    std::stable_sort(fw.begin(), fw.end(), by_cost);
    std::stable_sort(ad.begin(), ad.end(), by_cost);
    for (auto &c : fw) p->fwd_items.push_back(c.it);
    for (auto &c : ad) p->adj_items.push_back(c.it);
    if (!p->fdir.empty()) {
        p->fwd_groups = direct_fwd_groups(s, p->Tdir);
        p->adj_groups = direct_adj_groups(s, p->Ardir, p->Bpdir);
    }
    int rc;
    if ((rc = p->alloc_list(&p->d_fwd_items, std::max<size_t>(1, p->fwd_items.size())))) return rc;
    if ((rc = p->alloc_list(&p->d_adj_items, std::max<size_t>(1, p->adj_items.size())))) return rc;
    if ((rc = p->alloc_list(&p->d_fdir, std::max<size_t>(1, p->fdir.size())))) return rc;
    if (!p->fwd_items.empty())
        HIP_TRY(hipMemcpy(p->d_fwd_items, p->fwd_items.data(), sizeof(Item) * p->fwd_items.size(),
                          hipMemcpyHostToDevice));
    if (!p->adj_items.empty())
        HIP_TRY(hipMemcpy(p->d_adj_items, p->adj_items.data(), sizeof(Item) * p->adj_items.size(),
                          hipMemcpyHostToDevice));
    if (!p->fdir.empty())
        HIP_TRY(hipMemcpy(p->d_fdir, p->fdir.data(), sizeof(int) * p->fdir.size(), hipMemcpyHostToDevice));
    return STARRED_OK;
}

// ---- FFT path: shape classes, transform lengths, line passes ----

static bool smooth235(int v)
{
    for (int f : {2, 3, 5})
        while (v % f == 0) v /= f;
    return v == 1;
}

// smallest P >= need with P a multiple of 2s and P = 2^a 3^b 5^c
static int good_size(int need, int s)
{
    for (int P = need;; ++P)
        if (P % (2 * s) == 0 && smooth235(P)) return P;
}

static FftLen make_len(int L, std::map<int, long long> &tw_offsets, long long &tw_total)
{
    FftLen f;
    memset(&f, 0, sizeof f);
    f.L = L;
    int v = L;
    while (v % 4 == 0) { f.rad[f.nst++] = 4; v /= 4; }
    while (v % 2 == 0) { f.rad[f.nst++] = 2; v /= 2; }
    while (v % 3 == 0) { f.rad[f.nst++] = 3; v /= 3; }
    while (v % 5 == 0) { f.rad[f.nst++] = 5; v /= 5; }
    auto it = tw_offsets.find(L);
    if (it == tw_offsets.end()) {
        tw_offsets[L] = tw_total;
        f.tw_off = tw_total;
        tw_total += L;
    } else {
        f.tw_off = it->second;
    }
    return f;
}

static int build_fft_lists(starred_plan *p);

// Shape classes, transform lengths, factor tables and the per-frame spectra (fixed
// for the plan); the work lists, which depend on each class's algorithm and
// forward form, follow in build_fft_lists.
static int build_fft(starred_plan *p)
{
    const int s = p->s, E = p->E;
    std::map<std::pair<int, int>, int> cls_of;  // (n, K) -> class
    std::map<int, long long> tw_off;
    long long tw_total = 0;
    std::vector<int> &fcls = p->fcls;
    fcls.assign(E, 0);
    for (int i = 0; i < E; ++i) {
        auto key = std::make_pair(p->n[i], p->K[i]);
        auto it = cls_of.find(key);
        if (it == cls_of.end()) {
            ClassFft c;
            memset(&c, 0, sizeof c);
            c.n = p->n[i];
            c.F = s * c.n;
            c.K = p->K[i];
            c.o = (p->N - c.F) / 2;
            c.P = good_size(c.F + c.K / 2, s);
            c.Q = c.P / s;
            if (c.P > 4096) return fail(STARRED_EUNSUPPORTED, "FFT size above 4096");
            c.fP = make_len(c.P, tw_off, tw_total);
            c.fQ = make_len(c.Q, tw_off, tw_total);
            c.sscale = (float)(1.0 / ((double)s * s * (double)c.Q * c.Q));
            cls_of[key] = (int)p->cls.size();
            p->cls.push_back(c);
            fcls[i] = (int)p->cls.size() - 1;
        } else {
            fcls[i] = it->second;
        }
    }
    const int M = p->M;
    long long th = 0, hh = 0, tb = 0;
    for (auto &c : p->cls) {
        const long long HP = c.P / 2 + 1;
        c.th_off = th;
        th += (long long)c.F * HP;
        c.hh_off = hh;
        hh += (long long)c.P * HP;
        c.tab_off = tb;
        tb += (long long)(1 + 4 * M) * c.P;
    }
    // classes whose Q-grid planes fit in LDS may take the one-launch forward
    p->cls_fits.clear();
    for (auto &c : p->cls) {
        // the one-launch forward: two LDS planes (1), one plane in place (2), or none (0)
        int fit = 0;
        if (fused_lds_bytes(c.Q, c.n, c.P, p->M, 2) <= kFusedLdsMax) fit = 1;
        else if (c.Q > 64 && fft_ip_length(c.Q) && !(p->M > 4 && p->M <= 8) &&
                 fused_lds_bytes(c.Q, c.n, c.P, p->M, 1) <= kFusedLdsMax)
            fit = 2;  // (5-8 sources: the source factors take the registers the in-place form needs)
        p->cls_fits.push_back(fit);
        c.fused = fit ? 1 : 0;
        c.direct = 0;
    }
    // class-ordered frame list
    std::vector<int> &cls_frames = p->cls_frames;
    cls_frames.clear();
    for (int c = 0; c < (int)p->cls.size(); ++c) {
        p->cls[c].cf_off = (int)cls_frames.size();
        for (int i = 0; i < E; ++i)
            if (fcls[i] == c) cls_frames.push_back(i);
        p->cls[c].ncf = (int)cls_frames.size() - p->cls[c].cf_off;
    }
    p->ffr.resize(E);
    long long so = 0, to = 0, ro = 0, t3o = 0;
    for (int i = 0; i < E; ++i) {
        const ClassFft &c = p->cls[fcls[i]];
        FrameFft &f = p->ffr[i];
        memset(&f, 0, sizeof f);
        f.cls = fcls[i];
        f.kern_off = p->fr[i].kern_off;
        f.data_off = p->fr[i].data_off;
        f.fine_off = p->fr[i].fine_off;
        const long long HP = c.P / 2 + 1, HQ = c.Q / 2 + 1;
        f.s_off = so;
        so += (long long)c.P * HP;
        f.t_off = to;
        to += (long long)c.n * HQ;
        f.r_off = ro;
        ro += (long long)c.Q * HQ;
        f.t3_off = t3o;
        t3o += (long long)c.P * HP;
    }
    // frequency-domain adjoint: summed spectra per chunk of frames, room for the
    // smallest chunks allowed (the chunk size is chosen with the work lists): one frame
    // with more than kAdjSBWide point sources, else two
    const int min_fc = p->M > kAdjSBWide ? 1 : 2;
    long long gp = 0, hc = 0;
    for (ClassFft &cl : p->cls) {
        cl.gfch = kAdjFrames;
        cl.ngch = (cl.ncf + kAdjFrames - 1) / kAdjFrames;
        cl.ngch_cap = (cl.ncf + min_fc - 1) / min_fc;
        cl.gp_off = gp;
        gp += (long long)cl.ngch_cap * cl.P * (cl.P / 2 + 1);
        cl.hc_off = hc;
        hc += (long long)cl.F * cl.F;
    }
    int rc;
    FftPlanDev &d = p->fd;
    d.n_classes = (int)p->cls.size();
    d.n_frames = E;
    if ((rc = p->alloc(&d.classes, p->cls.size()))) return rc;
    if ((rc = p->alloc(&d.frames, E))) return rc;
    if ((rc = p->alloc(&d.tw, tw_total))) return rc;
    if ((rc = p->alloc(&d.S, so))) return rc;
    if ((rc = p->alloc(&d.T, to))) return rc;
    if ((rc = p->alloc(&d.T2, to))) return rc;
    if ((rc = p->alloc(&d.Rh, ro))) return rc;
    if ((rc = p->alloc(&d.T3, t3o))) return rc;
    if ((rc = p->alloc(&d.Th, th))) return rc;
    if ((rc = p->alloc(&d.Hh, hh))) return rc;
    if ((rc = p->alloc(&d.tab, tb))) return rc;
    if ((rc = p->alloc(&d.Gp, gp))) return rc;
    if ((rc = p->alloc(&d.hcls, hc))) return rc;
    if ((rc = p->alloc(&d.cls_frames, cls_frames.size()))) return rc;
    HIP_TRY(hipMemcpy(d.cls_frames, cls_frames.data(), sizeof(int) * cls_frames.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d.frames, p->ffr.data(), sizeof(FrameFft) * E, hipMemcpyHostToDevice));

    // twiddles e^{-2 pi i m / L} rounded from double
    std::vector<float2> tw(tw_total);
    for (auto &kv : tw_off)
        for (int m = 0; m < kv.first; ++m) {
            const double a = -2.0 * M_PI * m / kv.first;
            tw[kv.second + m] = make_float2((float)std::cos(a), (float)std::sin(a));
        }
    // static window factor of every class: w(K) = sum_{x < F} e^{-2 pi i K x / P}
    std::vector<float2> tabh(tb, make_float2(0.f, 0.f));
    for (auto &c : p->cls)
        for (int K = 0; K < c.P; ++K) {
            std::complex<double> acc = 0.0;
            for (int x = 0; x < c.F; ++x) {
                const long long m = ((long long)K * x) % c.P;
                acc += std::polar(1.0, -2.0 * M_PI * (double)m / c.P);
            }
            tabh[c.tab_off + K] = make_float2((float)acc.real(), (float)acc.imag());
        }
    HIP_TRY(hipMemcpy(d.tw, tw.data(), sizeof(float2) * tw_total, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d.tab, tabh.data(), sizeof(float2) * tb, hipMemcpyHostToDevice));
    // the kernel-spectrum passes cover every frame (set_frames prepares both forms)
    p->fft_ready = true;
    return build_fft_lists(p);
}

// The FFT path's work lists for the classes that run it (cls[c].direct == 0), and
// the direct path's for the frames of the others: rebuilt when the autotuner
// changes a class's algorithm, its forward form or the launch shapes.
static int build_fft_lists(starred_plan *p)
{
    const int E = p->E, M = p->M;
    const std::vector<int> &fcls = p->fcls;
    const std::vector<int> &cls_frames = p->cls_frames;
    FftPlanDev &d = p->fd;
    p->free_lists();
    int rc;
    auto is_direct = [&](int c) { return p->cls[c].direct != 0; };
    // forward spectral product items: 256 bins x a chunk of frames, longest first
    // (every FFT class, and for the loss the classes without the one-launch forward)
    for (int lg = 0; lg < 2; ++lg) {
        std::vector<SpecItem> sp;
        for (int c = 0; c < (int)p->cls.size(); ++c) {
            const ClassFft &cl = p->cls[c];
            if (is_direct(c) || (lg && cl.fused)) continue;
            const int nbins = cl.Q * (cl.Q / 2 + 1);
            const int nbb = (nbins + kFftThreads - 1) / kFftThreads;
            // enough frame chunks to give every compute unit several groups; with more than
            // 16 point sources a chunk holds at least a whole frame group of the product
            // (the sources' table values are loaded once per group)
            int fch = std::max(1, std::min(8, (int)((long long)nbb * cl.ncf / 1024)));
            if (p->M > 16) fch = std::max(fch, std::min(cl.ncf, kFwdFrames));
            for (int f0 = 0; f0 < cl.ncf; f0 += fch)
                for (int bb = 0; bb < nbb; ++bb)
                    sp.push_back(SpecItem{c, f0, std::min(fch, cl.ncf - f0), bb * kFftThreads});
        }
        std::stable_sort(sp.begin(), sp.end(), [&](const SpecItem &a, const SpecItem &b) {
            return p->cls[a.cls].P > p->cls[b.cls].P;
        });
        int &ns = lg ? d.n_spec_lg : d.n_spec;
        SpecItem *&dst = lg ? d.spec_lg : d.spec;
        ns = (int)sp.size();
        if ((rc = p->alloc_list(&dst, sp.size()))) return rc;
        if (!sp.empty()) HIP_TRY(hipMemcpy(dst, sp.data(), sizeof(SpecItem) * sp.size(), hipMemcpyHostToDevice));
    }
    // frames of the one-launch forward, largest transforms first
    {
        std::vector<int> fi;
        size_t lds = 0;
        for (int i = 0; i < E; ++i)
            if (!is_direct(fcls[i]) && p->cls[fcls[i]].fused) {
                fi.push_back(i);
                const ClassFft &cl = p->cls[fcls[i]];
                lds = std::max(lds, fused_lds_bytes(cl.Q, cl.n, cl.P, M, p->cls_fits[fcls[i]] == 2 ? 1 : 2));
            }
        std::stable_sort(fi.begin(), fi.end(), [&](int a, int b) { return p->cls[fcls[a]].Q > p->cls[fcls[b]].Q; });
        std::vector<FusedItem> fu;
        for (int i : fi) {
            const ClassFft &cl = p->cls[fcls[i]];
            const FrameFft &f = p->ffr[i];
            FusedItem it{};
            it.frame = i;
            it.cls = fcls[i];
            it.P = cl.P;
            it.Q = cl.Q;
            it.n = cl.n;
            it.inplace = p->cls_fits[fcls[i]] == 2 ? 1 : 0;
            it.tw_off = cl.fQ.tw_off;
            it.s_off = f.s_off;
            it.data_off = f.data_off;
            it.r_off = f.r_off;
            it.tab_off = cl.tab_off;
            it.hh_off = cl.hh_off;
            fu.push_back(it);
        }
        d.n_fused = (int)fu.size();
        d.fused_lds = lds;
        if ((rc = p->alloc_list(&d.fused, std::max<size_t>(1, fu.size())))) return rc;
        if (!fu.empty()) HIP_TRY(hipMemcpy(d.fused, fu.data(), sizeof(FusedItem) * fu.size(), hipMemcpyHostToDevice));
    }
    // frequency-domain adjoint: items over chunks of p->adj_fc frames x ranges of
    // rows of the P half spectrum, about p->adj_blocks of them per launch (chunks of
    // up to 8 frames with one source per pass, up to 4 with four, 2 with eight, 1 with 16)
    {
        const int fc = p->adj_fc;
        d.adj_fc = fc;
        std::vector<AdjItem> sp;
        int maxpb = 1, nchunks = 0;
        for (ClassFft &cl : p->cls) {
            cl.gfch = fc;
            cl.ngch = (cl.ncf + fc - 1) / fc;
            if (cl.ngch > cl.ngch_cap)  // the chunk spectra would overrun the class's region
                return fail(STARRED_EINVAL, "adjoint chunk size below the smallest the plan was built for");
        }
        for (int c = 0; c < (int)p->cls.size(); ++c)
            if (!is_direct(c)) nchunks += p->cls[c].ngch;
        for (int c = 0; c < (int)p->cls.size(); ++c) {
            ClassFft &cl = p->cls[c];
            cl.arr = cl.nrr = 0;
            if (is_direct(c)) continue;
            const int HP = cl.P / 2 + 1, nbins = cl.P * HP;
            const int CX = adj_lanes(HP), RG = kFftThreads / CX;
            const int want = std::max(1, (p->adj_blocks + nchunks - 1) / std::max(1, nchunks));
            // a block takes the 2s rows of each of its representatives y <= Q/2 (the rows
            // congruent to y or -y modulo Q): at least kAdjMinRows rows per thread, at
            // most kAdjMaxRows rows
            const int S2 = 2 * (cl.P / cl.Q), nrep = cl.Q / 2 + 1;
            const int rows = std::max(kAdjMinRows * RG, (cl.P + want - 1) / want);
            int arr = std::max(1, (rows + S2 - 1) / S2);
            arr = std::min(arr, kAdjMaxRows / S2);
            cl.arr = arr;
            cl.nrr = (nrep + arr - 1) / arr;
            maxpb = std::max(maxpb, cl.nrr);
            for (int f0 = 0; f0 < cl.ncf; f0 += fc)
                for (int r = 0; r < cl.nrr; ++r) {
                    AdjItem it{};
                    it.cls = c;
                    it.nf = std::min(fc, cl.ncf - f0);
                    it.y0 = r * arr;
                    it.y1 = std::min(nrep, it.y0 + arr);
                    it.P = cl.P;
                    it.Q = cl.Q;
                    it.pb = r;
                    for (int f = 0; f < kAdjMaxFrames; ++f) {
                        const int fi = f < it.nf ? cls_frames[cl.cf_off + f0 + f] : -1;
                        it.fid[f] = fi;
                        // a slot past the chunk's frames reads the chunk's first frame again
                        // (computed spectra: finite values, which the kernel then discards)
                        it.soff[f] = fi >= 0 ? p->ffr[fi].s_off : it.soff[0];
                        it.roff[f] = fi >= 0 ? p->ffr[fi].r_off : it.roff[0];
                    }
                    it.tab_off = cl.tab_off;
                    it.gout = cl.gp_off + (long long)(f0 / cl.gfch) * nbins;
                    sp.push_back(it);
                }
        }
        std::stable_sort(sp.begin(), sp.end(), [&](const AdjItem &a, const AdjItem &b) {
            return p->cls[a.cls].P > p->cls[b.cls].P;
        });
        d.n_aspec = (int)sp.size();
        d.maxpb = maxpb;
        d.total_bins = 0;
        for (int c = 0; c < (int)p->cls.size(); ++c)
            if (!is_direct(c)) d.total_bins += (long long)p->cls[c].P * (p->cls[c].P / 2 + 1);
        if ((rc = p->alloc_list(&d.aspec, std::max<size_t>(1, sp.size())))) return rc;
        if ((rc = p->alloc_list(&d.apart, (size_t)E * maxpb * (1 + 3 * M) + 1))) return rc;
        if (!sp.empty()) HIP_TRY(hipMemcpy(d.aspec, sp.data(), sizeof(AdjItem) * sp.size(), hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMemcpy(d.classes, p->cls.data(), sizeof(ClassFft) * p->cls.size(), hipMemcpyHostToDevice));

    // line passes: groups of lines of one frame (or class), longest transforms first
    std::vector<LineItem> last_items;
    // all: every frame, whatever its class runs (the kernel-spectrum passes of set_frames)
    auto make_pass = [&](LinePass &lp, bool per_class, auto lines_of, auto len_of, bool skip_fused = false,
                         bool all = false) -> int {
        struct G { int L; LineItem it; };
        std::vector<G> g;
        const int nunits = per_class ? (int)p->cls.size() : E;
        auto skip = [&](int u) {
            const int c = per_class ? u : fcls[u];
            if (all) return false;
            return is_direct(c) || (skip_fused && !per_class && p->cls[c].fused);
        };
        long long total_lines = 0;
        for (int u = 0; u < nunits; ++u)
            if (!skip(u)) total_lines += lines_of(p->cls[per_class ? u : fcls[u]]);
        // lines per work group: about kFftTargetElems elements, fewer when the
        // pass is small so that every compute unit gets work
        const long long want_groups = p->line_groups;
        const int cap = (int)std::max(1LL, total_lines / want_groups);
        int maxL = 1;
        for (int u = 0; u < nunits; ++u) {
            if (skip(u)) continue;
            const int c = per_class ? u : fcls[u];
            const ClassFft &cl = p->cls[c];
            const int L = len_of(cl);
            const int lines = lines_of(cl);
            const int lpw = std::max(1, std::min(kFftTargetElems / L, cap));
            maxL = std::max(maxL, (L + 1) * lpw);
            for (int l0 = 0; l0 < lines; l0 += lpw)
                g.push_back({L, LineItem{c, per_class ? -1 : u, l0, std::min(lpw, lines - l0)}});
        }
        std::stable_sort(g.begin(), g.end(), [](const G &a, const G &b) { return a.L > b.L; });
        std::vector<LineItem> items;
        for (auto &x : g) items.push_back(x.it);
        last_items = items;
        lp.n_items = (int)items.size();
        lp.lds_bytes = (size_t)2 * maxL * sizeof(float2);
        int rc2 = p->alloc_list(&lp.items, std::max<size_t>(1, items.size()));
        if (rc2) return rc2;
        if (!items.empty()) {
            hipError_t e = hipMemcpy(lp.items, items.data(), sizeof(LineItem) * items.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) return fail_hip(e, "hipMemcpy(line items)");
        }
        return STARRED_OK;
    };
    auto LP = [](const ClassFft &c) { return c.P; };
    auto LQ = [](const ClassFft &c) { return c.Q; };
    if ((rc = make_pass(d.hrows, true, [](const ClassFft &c) { return c.F; }, LP))) return rc;
    if ((rc = make_pass(d.hcols, true, [](const ClassFft &c) { return c.P / 2 + 1; }, LP))) return rc;
    if ((rc = make_pass(d.krows, false, [](const ClassFft &c) { return c.P; }, LP, false, true))) return rc;
    if ((rc = make_pass(d.kcols, false, [](const ClassFft &c) { return c.P / 2 + 1; }, LP, false, true))) return rc;
    if ((rc = make_pass(d.fcols, false, [](const ClassFft &c) { return c.Q / 2 + 1; }, LQ))) return rc;
    if ((rc = make_pass(d.frows, false, [](const ClassFft &c) { return c.n; }, LQ))) return rc;
    if ((rc = make_pass(d.rrows, false, [](const ClassFft &c) { return c.n; }, LQ))) return rc;
    if ((rc = make_pass(d.rcols, false, [](const ClassFft &c) { return c.Q / 2 + 1; }, LQ))) return rc;
    if ((rc = make_pass(d.fcols_lg, false, [](const ClassFft &c) { return c.Q / 2 + 1; }, LQ, true))) return rc;
    if ((rc = make_pass(d.frows_lg, false, [](const ClassFft &c) { return c.n; }, LQ, true))) return rc;
    if ((rc = make_pass(d.rcols_lg, false, [](const ClassFft &c) { return c.Q / 2 + 1; }, LQ, true))) return rc;
    if ((rc = make_pass(d.acols, false, [](const ClassFft &c) { return c.P / 2 + 1; }, LP))) return rc;
    if ((rc = make_pass(d.arows, false, [](const ClassFft &c) { return c.F; }, LP))) return rc;
    {
        std::vector<int> off(E + 1, 0), item;
        for (const LineItem &li : last_items) off[li.frame + 1]++;
        for (int i = 0; i < E; ++i) off[i + 1] += off[i];
        item.resize(last_items.size());
        std::vector<int> fill(off.begin(), off.end() - 1);
        for (int q = 0; q < (int)last_items.size(); ++q) item[fill[last_items[q].frame]++] = q;
        if ((rc = p->alloc_list(&d.gpart, std::max<size_t>(1, last_items.size())))) return rc;
        if ((rc = p->alloc_list(&d.gcsr_off, E + 1))) return rc;
        if ((rc = p->alloc_list(&d.gcsr_item, std::max<size_t>(1, item.size())))) return rc;
        HIP_TRY(hipMemcpy(d.gcsr_off, off.data(), sizeof(int) * (E + 1), hipMemcpyHostToDevice));
        if (!item.empty()) HIP_TRY(hipMemcpy(d.gcsr_item, item.data(), sizeof(int) * item.size(), hipMemcpyHostToDevice));
    }
    if ((rc = make_pass(d.srows, false, [](const ClassFft &c) { return c.F; }, LP))) return rc;
    if ((rc = make_pass(d.scols, false, [](const ClassFft &c) { return c.P / 2 + 1; }, LP))) return rc;
    if ((rc = make_pass(d.gcols, true, [](const ClassFft &c) { return c.P / 2 + 1; }, LP))) return rc;
    if ((rc = make_pass(d.grows, true, [](const ClassFft &c) { return c.F; }, LP))) return rc;
    // every frame: the per-frame convolution of the rendered scenes (frame transforms)
    if ((rc = make_pass(d.srows_x, false, [](const ClassFft &c) { return c.F; }, LP, false, true))) return rc;
    if ((rc = make_pass(d.scols_x, false, [](const ClassFft &c) { return c.P / 2 + 1; }, LP, false, true))) return rc;
    if ((rc = make_pass(d.fcols_x, false, [](const ClassFft &c) { return c.Q / 2 + 1; }, LQ, false, true))) return rc;
    if ((rc = make_pass(d.frows_x, false, [](const ClassFft &c) { return c.n; }, LQ, false, true))) return rc;
    if ((rc = make_pass(d.rcols_x, false, [](const ClassFft &c) { return c.Q / 2 + 1; }, LQ, false, true))) return rc;
    if ((rc = make_pass(d.acols_x, false, [](const ClassFft &c) { return c.P / 2 + 1; }, LP, false, true))) return rc;
    if ((rc = make_pass(d.arows_x, false, [](const ClassFft &c) { return c.F; }, LP, false, true))) return rc;
    if ((rc = p->alloc_list(&d.gpart_x, std::max<size_t>(1, (size_t)d.arows_x.n_items)))) return rc;
    // the direct path's lists for the frames of the direct classes
    if ((rc = build_direct_lists(p))) return rc;
    // chi-square partials: the FFT line-pass row groups (or, with the one-launch
    // forward, its row groups and then one per fused frame), then the direct tiles
    p->n_fft_chi = std::max(std::max(d.frows.n_items, d.frows_lg.n_items + d.n_fused), d.frows_x.n_items);
    if ((rc = p->alloc_list(&p->d_part_chi_fft, (size_t)p->n_fft_chi + p->fwd_items.size() + 1))) return rc;
    return STARRED_OK;
}

static int build_psf(starred_plan *p)
{
    const int S = p->E, n = p->n[0], N = p->N;
    p->psf_n = n;
    p->nparams = 5 + (long long)N * N + 3LL * S;
    p->ndata = (long long)S * n * n;
    p->nfine = (long long)N * N;
    const long long NN = (long long)N * N;
    if (psf_fwd_lds(p->s) > kMaxLds || psf_adj_lds(p->s, S) > kMaxLds)
        return fail(STARRED_EUNSUPPORTED, "PSF tiles too large for one work group");
    int rc;
    if ((rc = p->alloc(&p->d_s64, NN))) return rc;
    if ((rc = p->alloc(&p->d_dm, 5 * NN))) return rc;
    if ((rc = p->alloc(&p->d_rho, p->ndata))) return rc;
    if ((rc = p->alloc(&p->d_part_chi, (size_t)S * psf_fwd_tiles(n) * 4))) return rc;
    if ((rc = p->alloc(&p->d_part_eta, (size_t)psf_adj_tiles(N) * 5))) return rc;
    if ((rc = dense_setup(p, 1))) return rc;
    if ((rc = p->alloc(&p->d_part_l1, std::max((size_t)starlet_l1_slots(p->N, p->J), dense_l1_slots(p))))) return rc;
    if ((rc = p->alloc(&p->d_z, (size_t)p->J * NN))) return rc;
    if ((rc = p->alloc(&p->d_ca, NN))) return rc;
    if ((rc = p->alloc(&p->d_cb, NN))) return rc;
    if ((rc = p->alloc(&p->d_tmp, NN))) return rc;
    if ((rc = p->alloc(&p->d_prior, NN))) return rc;
    if ((rc = p->alloc(&p->d_grad, p->nparams))) return rc;
    if ((rc = p->alloc(&p->d_wzero, (size_t)p->J * NN))) return rc;
    HIP_TRY(hipMemset(p->d_wzero, 0, sizeof(float) * p->J * NN));
    return STARRED_OK;
}

static int loss_grad_impl(starred_plan *p, const float *params, float *grad, double *loss_out, int *tick = nullptr,
                          const AdamDev *adam = nullptr);
static int autotune(starred_plan *p);

// Per-class algorithm choices: the direct algorithm, the FFT algorithm with the
// one-launch forward (where it fits), the FFT algorithm with the line passes.
enum { kChDirect = 0, kChFused = 1, kChLines = 2 };

// Whether the direct kernels' LDS tiles hold the frames of class c.
static bool class_direct_ok(const starred_plan *p, int c)
{
    const FrameDev &f = p->fr[p->cls_frames[p->cls[c].cf_off]];
    return fwd_lds_bytes(p->s, f.Tpad) <= kMaxLds && adj_lds_bytes(f.Ar, f.Bpad) <= kMaxLds;
}

static int class_choice(const starred_plan *p, int c)
{
    const ClassFft &cl = p->cls[c];
    return cl.direct ? kChDirect : (cl.fused ? kChFused : kChLines);
}

// Set every class's algorithm and forward form, then rebuild the work lists.
static int apply_choices(starred_plan *p, const std::vector<int> &ch)
{
    bool any_fft = false;
    for (int c = 0; c < (int)p->cls.size(); ++c) {
        ClassFft &cl = p->cls[c];
        cl.direct = ch[c] == kChDirect ? 1 : 0;
        cl.fused = (ch[c] == kChFused && p->cls_fits[c]) ? 1 : 0;
        any_fft = any_fft || !cl.direct;
    }
    p->algo = any_fft ? STARRED_CONV_FFT : STARRED_CONV_DIRECT;
    p->drop_graphs();
    return build_fft_lists(p);
}

int starred_plan_create(const starred_desc *desc, void *stream, starred_plan **plan_out)
{
    if (!plan_out) return fail(STARRED_EINVAL, "plan_out is NULL");
    *plan_out = nullptr;
    int rc = validate(desc);
    if (rc) return rc;
    starred_plan *p = new starred_plan();
    p->mode = desc->mode;
    p->E = desc->n_frames;
    p->s = desc->subsample;
    p->N = desc->grid_side;
    p->M = desc->n_sources;
    p->J = desc->n_scales;
    p->w_stride = desc->w_pixel_stride;
    p->lam = desc->lambda;
    p->fwhm = desc->gauss_fwhm;
    p->sigma = (float)(desc->gauss_fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0))));
    p->st = (hipStream_t)stream;
    {
        hipError_t e = hipStreamCreate(&p->st2);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming);
        if (e == hipSuccess) e = hipStreamCreate(&p->st3);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork3, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join3, hipEventDisableTiming);
        if (e != hipSuccess) {
            delete p;
            return fail_hip(e, "stream/event creation");
        }
        rc = p->alloc(&p->d_t, 1);
        if (rc) {
            delete p;
            return rc;
        }
    }
    p->n.assign(desc->side_host, desc->side_host + p->E);
    if (desc->ksize_host) p->K.assign(desc->ksize_host, desc->ksize_host + p->E);
    if (p->mode == STARRED_PSF) {
        p->algo_req = p->algo = STARRED_CONV_DIRECT;
        rc = build_psf(p);
        if (rc) {
            delete p;
            return rc;
        }
        *plan_out = p;
        return STARRED_OK;
    }
    p->algo_req = desc->conv_algo;
    p->algo = STARRED_CONV_FFT;  // every class on the FFT algorithm until told or tuned otherwise
    rc = build_deconv(p);
    if (!rc) rc = build_fft(p);
    if (rc) {
        delete p;
        return rc;
    }
    p->direct_ok = true;
    for (int c = 0; c < (int)p->cls.size(); ++c) p->direct_ok = p->direct_ok && class_direct_ok(p, c);
    if (p->algo_req == STARRED_CONV_DIRECT) {
        if (!p->direct_ok) {
            delete p;
            return fail(STARRED_EUNSUPPORTED, "kernels too large for the direct path's LDS tiles");
        }
        rc = apply_choices(p, std::vector<int>(p->cls.size(), kChDirect));
        if (rc) {
            delete p;
            return rc;
        }
    }
    *plan_out = p;
    return STARRED_OK;
}

starred_plan::~starred_plan()
{
    if (noise_aux) (void)starred_plan_destroy(noise_aux);
    destroy_members();
}

int starred_plan_destroy(starred_plan *p)
{
    if (!p) return fail(STARRED_EINVAL, "plan is NULL");
    if (p->st) (void)hipStreamSynchronize(p->st);
    else (void)hipDeviceSynchronize();
    delete p;
    return STARRED_OK;
}

int64_t starred_num_params(const starred_plan *p) { return p ? p->nparams : -1; }
int64_t starred_num_data(const starred_plan *p) { return p ? p->ndata : -1; }
int64_t starred_num_scene(const starred_plan *p) { return p ? p->nfine : -1; }
int starred_conv_algo(const starred_plan *p) { return p ? p->algo : STARRED_EINVAL; }

int starred_num_classes(const starred_plan *p)
{
    if (!p) return fail(STARRED_EINVAL, "plan is NULL");
    return p->mode == STARRED_DECONV ? (int)p->cls.size() : 0;
}

int starred_get_class_info(const starred_plan *p, int32_t c, starred_class_info *out)
{
    if (!p || !out) return fail(STARRED_EINVAL, "NULL argument");
    if (p->mode != STARRED_DECONV || c < 0 || c >= (int)p->cls.size()) return fail(STARRED_EINVAL, "no such class");
    const ClassFft &cl = p->cls[c];
    memset(out, 0, sizeof *out);
    out->n = cl.n;
    out->K = cl.K;
    out->n_frames = cl.ncf;
    out->algo = cl.direct ? STARRED_CONV_DIRECT : STARRED_CONV_FFT;
    out->P = cl.P;
    out->Q = cl.Q;
    out->fused = (!cl.direct && p->fft_fused && cl.fused) ? p->cls_fits[c] : 0;
    for (int k = 0; k < 3; ++k) out->tune_ms[k] = c < (int)p->cls_tune.size() ? p->cls_tune[c][k] : -1.0;
    return STARRED_OK;
}

int starred_autotune_info(const starred_plan *p, double *wall_ms_out, int32_t *cached_out, int32_t *adj_blocks_out,
                          int32_t *line_groups_out, int32_t *adj_frames_out, int32_t *split_forward_out,
                          int32_t *prior_late_out)
{
    if (prior_late_out && p) *prior_late_out = p->prior_late;
    if (split_forward_out && p) *split_forward_out = p->fwd_split;
    if (!p) return fail(STARRED_EINVAL, "plan is NULL");
    if (wall_ms_out) *wall_ms_out = p->tune_wall_ms;
    if (cached_out) *cached_out = p->tune_cached;
    if (adj_blocks_out) *adj_blocks_out = p->adj_blocks;
    if (line_groups_out) *line_groups_out = p->line_groups;
    if (adj_frames_out) *adj_frames_out = p->fd.adj_fc;
    return STARRED_OK;
}

int starred_set_class_algo(starred_plan *p, int32_t c, int32_t algo, int32_t fused)
{
    if (!p) return fail(STARRED_EINVAL, "plan is NULL");
    if (p->mode != STARRED_DECONV || c < 0 || c >= (int)p->cls.size()) return fail(STARRED_EINVAL, "no such class");
    if (algo != STARRED_CONV_DIRECT && algo != STARRED_CONV_FFT) return fail(STARRED_EINVAL, "algo must be DIRECT or FFT");
    if (algo == STARRED_CONV_DIRECT && !class_direct_ok(p, c))
        return fail(STARRED_EUNSUPPORTED, "kernels of this class too large for the direct path's LDS tiles");
    if (algo == STARRED_CONV_FFT && p->xf)
        return fail(STARRED_EUNSUPPORTED, "frames with per-frame transforms run the direct algorithm");
    std::vector<int> ch(p->cls.size());
    for (int k = 0; k < (int)p->cls.size(); ++k) ch[k] = class_choice(p, k);
    ch[c] = algo == STARRED_CONV_DIRECT ? kChDirect : (fused && p->cls_fits[c] ? kChFused : kChLines);
    return apply_choices(p, ch);
}

// chunk sizes of the frequency-domain adjoint (8 only with at most one point source:
// four sources per pass need the registers)
static bool adj_shape_ok(int fc, int M)
{
    return fc == 2 || fc == 4 || (fc == 8 && M <= 1) || (fc == 1 && M > kAdjSBWide);
}

int starred_set_fft_shapes(starred_plan *p, int32_t adj_frames, int32_t adj_blocks, int32_t line_groups,
                           int32_t split_forward, int32_t prior_late)
{
    if (!p) return fail(STARRED_EINVAL, "plan is NULL");
    if (p->mode != STARRED_DECONV) return fail(STARRED_EUNSUPPORTED, "launch shapes of the deconvolution FFT path");
    if (adj_frames && !adj_shape_ok(adj_frames, p->M))
        return fail(STARRED_EINVAL,
                    "adj_frames must be 2 or 4 (or 8 with at most one point source, 1 with more than eight)");
    if (adj_blocks < 0 || adj_blocks > (1 << 20) || line_groups < 0 || line_groups > (1 << 20))
        return fail(STARRED_EINVAL, "work-group targets must lie in [1, 2^20] (0 keeps the current one)");
    if (split_forward < -1 || split_forward > 1) return fail(STARRED_EINVAL, "split_forward must be -1, 0 or 1");
    if (prior_late < -1 || prior_late > 3) return fail(STARRED_EINVAL, "prior_late must be -1, 0, 1, 2 or 3");
    if (prior_late >= 0) p->prior_late = prior_late;
    if (split_forward >= 0) p->fwd_split = split_forward;
    if (adj_frames) p->adj_fc = adj_frames;
    if (adj_blocks) p->adj_blocks = adj_blocks;
    if (line_groups) p->line_groups = line_groups;
    p->drop_graphs();
    // taken up by the next list build (binding frames, or a class moving onto the FFT path)
    if (p->algo != STARRED_CONV_FFT || !p->data || p->cls.empty()) return STARRED_OK;
    return build_fft_lists(p);
}

static int time_plan(starred_plan *p, const float *params, double *loss, hipEvent_t a, hipEvent_t b, double *ms);

// The convolution of frames with per-frame transforms: the direct kernels or each
// frame's own spectra; STARRED_CONV_AUTO times both on the bound data (h = 0) when
// frames are bound, else takes the spectra.
static int choose_xf_algo(starred_plan *p, int algo)
{
    p->xf_ms[0] = p->xf_ms[1] = -1.0;
    const bool fft_ok = !p->cls.empty() && p->fd.frows_x.n_items > 0 && p->fd.srows_x.n_items > 0;
    if (algo == STARRED_CONV_FFT && !fft_ok) return fail(STARRED_EUNSUPPORTED, "this plan has no FFT structures");
    if (algo == STARRED_CONV_DIRECT || !fft_ok) {
        p->xf_fft = 0;
        return STARRED_OK;
    }
    if (algo == STARRED_CONV_FFT || !p->frames_set) {
        p->xf_fft = 1;
        return STARRED_OK;
    }
    float *params = nullptr;
    double *loss = nullptr;
    int rc = dev_alloc(&params, p->nparams);
    if (!rc) rc = dev_alloc(&loss, 3);
    hipEvent_t a = nullptr, b = nullptr;
    if (!rc && hipEventCreate(&a) != hipSuccess) rc = fail(STARRED_EHIP, "hipEventCreate");
    if (!rc && hipEventCreate(&b) != hipSuccess) rc = fail(STARRED_EHIP, "hipEventCreate");
    if (!rc && launch_fill(p->st, params, p->nparams, 0.f) != hipSuccess) rc = fail(STARRED_EHIP, "fill");
    const bool prof = p->prof_on;
    p->prof_on = false;
    for (int v = 0; v < 2 && !rc; ++v) {
        p->xf_fft = v;
        rc = time_plan(p, params, loss, a, b, &p->xf_ms[v]);
    }
    p->prof_on = prof;
    if (!rc) p->xf_fft = p->xf_ms[1] < p->xf_ms[0] ? 1 : 0;
    (void)hipStreamSynchronize(p->st);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (params) (void)hipFree(params);
    if (loss) (void)hipFree(loss);
    return rc;
}

int starred_frame_transforms_info(const starred_plan *p, int32_t *algo_out, double *ms_out)
{
    if (!p) return fail(STARRED_EINVAL, "plan is NULL");
    if (algo_out) *algo_out = !p->xf ? 0 : (p->xf_fft ? STARRED_CONV_FFT : STARRED_CONV_DIRECT);
    if (ms_out) {
        ms_out[0] = p->xf_ms[0];
        ms_out[1] = p->xf_ms[1];
    }
    return STARRED_OK;
}

int starred_set_frame_transforms(starred_plan *p, const float *xf, float *grad_xf, int32_t algo)
{
    if (!p) return fail(STARRED_EINVAL, "plan is NULL");
    if (p->mode != STARRED_DECONV) return fail(STARRED_EUNSUPPORTED, "per-frame transforms need deconvolution mode");
    if (!xf && grad_xf) return fail(STARRED_EINVAL, "grad_xf without transforms");
    if (algo != STARRED_CONV_AUTO && algo != STARRED_CONV_DIRECT && algo != STARRED_CONV_FFT)
        return fail(STARRED_EINVAL, "algo must be STARRED_CONV_AUTO, DIRECT or FFT");
    if (xf && !p->direct_ok)
        return fail(STARRED_EUNSUPPORTED, "per-frame transforms run the direct algorithm, whose tiles these kernels exceed");
    p->drop_graphs();
    if (xf && !p->xf) {
        // every class onto the direct algorithm (the FFT path assumes untransformed windows)
        p->xf_prev_choice.resize(p->cls.size());
        for (int c = 0; c < (int)p->cls.size(); ++c) p->xf_prev_choice[c] = class_choice(p, c);
        int rc = apply_choices(p, std::vector<int>(p->cls.size(), kChDirect));
        if (rc) return rc;
    } else if (!xf && p->xf && !p->xf_prev_choice.empty()) {
        p->xf = nullptr;
        p->gxf = nullptr;
        return apply_choices(p, p->xf_prev_choice);
    }
    p->xf = xf;
    p->gxf = xf ? grad_xf : nullptr;
    if (!xf) return STARRED_OK;
    if (p->hpart_chunks < finalize_h_chunks(p->E, true)) {
        // transformed frames are summed into dL/dh in smaller chunks: more partial planes
        p->hpart_chunks = finalize_h_chunks(p->E, true);
        int rc = p->alloc(&p->d_hpart, (size_t)p->hpart_chunks * p->N * p->N);
        if (rc) return rc;
    }
    int rc = choose_xf_algo(p, algo);
    p->drop_graphs();
    return rc;
}

int starred_set_frames(starred_plan *p, const float *data, const float *inv_var, const float *psf,
                       const float *W)
{
    if (!p) return fail(STARRED_EINVAL, "plan is NULL");
    if (!data || !inv_var || !W) return fail(STARRED_EINVAL, "data, inv_var and W must be non-NULL");
    if (p->mode == STARRED_DECONV && !psf) return fail(STARRED_EINVAL, "psf kernels are required in deconvolution mode");
    // captured graphs hold the bound pointers as kernel arguments: re-capture
    // after any re-bind
    p->drop_graphs();
    p->data = data;
    p->invvar = inv_var;
    p->W = W;
    p->psf_bound = psf;
    if (p->plain_ready) {
        HIP_TRY(launch_prep_kernels(p->st, p->d_frp, p->frp.data(), p->E, 1, psf, p->d_pkf, p->d_pka));
    }
    if (p->mode == STARRED_PSF) {
        p->frames_set = true;
        return STARRED_OK;
    }
    HIP_TRY(launch_prep_kernels(p->st, p->d_fr, p->fr.data(), p->E, p->s, psf, p->d_kf, p->d_ka));
    if (p->fft_ready) HIP_TRY(fft_prep_kernels(p->st, p->fd, psf, p->s));
    HIP_TRY(hipStreamSynchronize(p->st));
    p->frames_set = true;
    if (p->algo_req == STARRED_CONV_AUTO && !p->xf) return autotune(p);
    return STARRED_OK;
}

int starred_render_scene(starred_plan *p, const float *params, float *scene)
{
    if (!p || !params || !scene) return fail(STARRED_EINVAL, "NULL argument");
    if (p->mode == STARRED_PSF) {
        HIP_TRY(launch_psf_render(p->st, p->N, params, scene));
        return STARRED_OK;
    }
    HIP_TRY(launch_render(p->st, p->d_fr, p->E, p->Fmax, p->N, p->M, p->sigma, params, scene, nullptr, 0, p->xf));
    return STARRED_OK;
}

int starred_convolve_subsample(starred_plan *p, const float *scene, float *model)
{
    if (!p || !scene || !model) return fail(STARRED_EINVAL, "NULL argument");
    if (p->mode == STARRED_PSF) return fail(STARRED_EUNSUPPORTED, "deconvolution-mode operator called on a PSF-mode plan");
    if (!p->frames_set) return fail(STARRED_ESTATE, "set_frames has not been called");
    // frames of FFT classes by the transforms, frames of direct classes by the direct kernel
    if (p->algo == STARRED_CONV_FFT) HIP_TRY(fft_scene_model(p->st, p->fd, scene, p->s, model));
    HIP_TRY(launch_fwd_direct(p->st, p->s, p->d_fr, p->d_fwd_items, (int)p->fwd_items.size(), p->Tdir,
                              scene, p->d_kf, nullptr, nullptr, model, nullptr, p->fwd_groups));
    return STARRED_OK;
}

int starred_convolve_subsample_adj(starred_plan *p, const float *resid, float *grad_scene)
{
    if (!p || !resid || !grad_scene) return fail(STARRED_EINVAL, "NULL argument");
    if (p->mode == STARRED_PSF) return fail(STARRED_EUNSUPPORTED, "deconvolution-mode operator called on a PSF-mode plan");
    if (!p->frames_set) return fail(STARRED_ESTATE, "set_frames has not been called");
    if (p->algo == STARRED_CONV_FFT) {
        HIP_TRY(fft_resid_rows(p->st, p->fd, resid));
        HIP_TRY(fft_adjoint(p->st, p->fd, grad_scene));
    }
    HIP_TRY(launch_adj_direct(p->st, p->s, p->d_fr, p->d_adj_items, (int)p->adj_items.size(), p->Ardir,
                              p->Bpdir, resid, p->d_ka, grad_scene, p->adj_groups));
    return STARRED_OK;
}

int starred_starlet_fwd(starred_plan *p, const float *img, float *coeffs)
{
    if (!p || !img || !coeffs) return fail(STARRED_EINVAL, "NULL argument");
    if (p->dense) {
        HIP_TRY(launch_dense_coeffs(p->st, dense_desc(p, 1, img), coeffs));
        return STARRED_OK;
    }
    // the transform alone: zero weights, no L1 partials, no subgradient
    HIP_TRY(launch_starlet_fwd(p->st, p->N, p->J, img, coeffs, nullptr, p->d_wzero, 0, 0.f,
                               p->d_ca, p->d_cb, p->d_tmp, nullptr, nullptr));
    return STARRED_OK;
}

int starred_starlet_adj(starred_plan *p, const float *coeffs, float *img)
{
    if (!p || !coeffs || !img) return fail(STARRED_EINVAL, "NULL argument");
    if (p->dense) {
        DenseStar d = dense_desc(p, 1, nullptr);
        d.zin = coeffs;
        d.out = img;
        HIP_TRY(launch_dense_adjoint(p->st, d));
        return STARRED_OK;
    }
    HIP_TRY(launch_starlet_adj(p->st, p->N, p->J, coeffs, img, p->d_ca, p->d_cb, p->d_tmp));
    return STARRED_OK;
}

// Starlet transform, L1 term, subgradient and adjoint of the image part of
// params (h, or b in PSF mode) on the second stream: fork from st, join with
// ev_join (the caller waits on it before the final reductions).
// The prior terms on stream st: lambda ||W (.) Phi^T img||_1 with its gradient
// Phi z in d_prior and, when lambda_pts != 0 (deconvolution), the point-source
// term of Eq. 11 transformed together with h (a batch of two images): its
// gradient's shares of dL/da and dL/dc land in d_pts.
static int prior_launches(starred_plan *p, hipStream_t st, const float *img, bool want_grad, int *n_l1)
{
    if (p->dense) {
        // every scale from the image(s) directly: four passes over all scales
        const bool pts = p->mode == STARRED_DECONV && p->lam_pts != 0.0;
        const long long NN = (long long)p->N * p->N;
        if (pts) HIP_TRY(launch_pts_render(st, p->N, p->E, p->M, p->sigma, img, nullptr, p->d_pair + NN));
        DenseStar d = dense_desc(p, pts ? 2 : 1, img);
        if (pts) {
            d.img1 = p->d_pair + NN;  // the point-source image
            d.lam1 = (float)p->lam_pts;
        }
        d.part_l1 = p->d_part_l1;
        d.out = want_grad ? p->d_prior : nullptr;
        HIP_TRY(launch_dense_prior(st, d));
        *n_l1 = d.l1_slots();
        if (pts && want_grad) HIP_TRY(launch_pts_dots(st, p->N, p->E, p->M, p->sigma, img, p->d_prior + NN, p->d_pts));
        return STARRED_OK;
    }
    if (p->mode == STARRED_DECONV && p->lam_pts != 0.0) {
        const long long NN = (long long)p->N * p->N;
        HIP_TRY(launch_pts_render(st, p->N, p->E, p->M, p->sigma, img, p->d_pair, p->d_pair + NN));
        HIP_TRY(launch_starlet_prior(st, p->N, p->J, 2, p->d_pair, want_grad ? p->d_z : nullptr, p->W, p->w_stride,
                                     (float)p->lam, (float)p->lam_pts, p->d_ca, p->d_cb, p->d_part_l1, n_l1));
        if (want_grad) {
            HIP_TRY(launch_starlet_adj_batch(st, p->N, p->J, 2, p->d_z, p->d_prior, p->d_ca, p->d_cb));
            HIP_TRY(launch_pts_dots(st, p->N, p->E, p->M, p->sigma, img, p->d_prior + NN, p->d_pts));
        }
        return STARRED_OK;
    }
    HIP_TRY(launch_starlet_fwd(st, p->N, p->J, img, nullptr, want_grad ? p->d_z : nullptr, p->W, p->w_stride,
                               (float)p->lam, p->d_ca, p->d_cb, p->d_tmp, p->d_part_l1, n_l1));
    if (want_grad) HIP_TRY(launch_starlet_adj(st, p->N, p->J, p->d_z, p->d_prior, p->d_ca, p->d_cb, p->d_tmp));
    return STARRED_OK;
}

// The prior on the second stream: fork from st, join with ev_join (the caller
// waits on it before the final reductions). The fork point is the work st holds
// when starlet_fork records it; starlet_launch may follow later launches on st.
// (A captured graph's executor keeps a node's hardware queue for the child that
// was captured first and moves the others to further queues; launching the main
// stream's next kernel before the branch keeps a step's longer chain on one queue,
// so that the prior is the one crossing queues, each crossing costing several
// microseconds.)
static int starlet_fork(starred_plan *p)
{
    HIP_TRY(hipEventRecord(p->ev_fork, p->st));
    return STARRED_OK;
}

static int starlet_launch(starred_plan *p, const float *img, bool want_grad, int *n_l1)
{
    HIP_TRY(hipStreamWaitEvent(p->st2, p->ev_fork, 0));
    hipEvent_t e0 = p->prof_start(p->st2);
    int rc = prior_launches(p, p->st2, img, want_grad, n_l1);
    if (rc) return rc;
    p->prof_stop(STARRED_STAGE_STARLET, e0, p->st2);
    HIP_TRY(hipEventRecord(p->ev_join, p->st2));
    return STARRED_OK;
}

// tick: the device step counter a step advances; adam (FFT path only): the
// update fused into the final launch, which the counter then feeds.
static int loss_grad_impl(starred_plan *p, const float *params, float *grad, double *loss_out, int *tick,
                          const AdamDev *adam)
{
    // fft: some class runs the FFT algorithm; dir: some frames run the direct one
    // (both in one evaluation when the classes differ)
    const bool fft = (p->algo == STARRED_CONV_FFT);
    const bool dir = !p->fdir.empty();
    // per-frame transforms through the frames' own spectra (every class is on the direct
    // algorithm while transforms are set; only its convolution changes)
    const bool xf_fft = p->xf && p->xf_fft && !fft;
    hipEvent_t e0;
    int n_chi = 0;
    const double *part_chi = p->d_part_chi_fft;
    int n_l1 = 0;
    const bool fused = fft && p->fft_fused && p->fd.n_fused > 0;
    // the one-launch forward beside the line passes when both have frames
    const bool split = fused && p->fwd_split && p->fd.frows_lg.n_items > 0;
    // one class covering the whole grid: the row inverse of dL/dh carries the final
    // reductions and the update (one launch fewer)
    const bool fin_rows = fft && !dir && grad && p->fd.n_classes == 1 && p->cls[0].F == p->N;
    // The starlet prior depends on h only. With the composite filters, the
    // one-launch forward and (for the gradient) the row inverse above, its passes
    // ride in the step's own launches as extra work groups (A: the h-row launch,
    // B: the h-column launch, C with z and the L1 share: the forward, D1 with each
    // level's adjoint term: the dL/dh column launch; the row inverse sums the
    // terms per pixel); otherwise, and with the point-source term, the prior runs
    // on the forked stream.
    const bool pts = p->lam_pts != 0.0;
    // several FFT classes, no direct frames: the passes ride too when asked (prior_late 2),
    // the final launch summing the per-level terms per pixel
    const bool ride_multi = p->prior_late == 2 && fft && !dir;
    const bool ride = fused && p->dense && !pts && (!grad || fin_rows || ride_multi);
    DensePiece pa, pb, pc, pd;
    DenseStar dd;
    if (ride) {
        dd = dense_desc(p, 1, params);
        dd.part_l1 = p->d_part_l1;
        dd.out = grad ? p->d_prior : nullptr;  // (pass C builds U_j only when set)
        pa.d = pb.d = pd.d = dd;
        pc.d = dd;
        pc.d.rx = dense_rows_for(p->N, kFusedThreads);  // the forward's work groups are wider
        pa.pass = 0;
        pa.jobs = pa.d.jobs_a();
        pb.pass = 1;
        pb.jobs = pb.d.jobs_b();
        pc.pass = 2;
        pc.jobs = pc.d.jobs_c();
        if (grad) {
            pd.pass = 4;  // each level's term into its own plane; the h-row inverse sums them
            pd.jobs = pd.d.jobs_d1();
        }
        n_l1 = pc.d.l1_slots();
    }
    // the fork of the prior: at the start, after the forward's launches (1, and 2 where it
    // cannot ride), or after the adjoint's spectral products (3, with a gradient)
    const bool late_adj = !ride && fft && grad && p->prior_late == 3;
    const bool late = !ride && fft && p->prior_late && !late_adj;
    // the prior's branch is launched after the main stream's next launch (see starlet_fork)
    bool prior_pending = false;
    auto prior_flush = [&]() -> int {
        if (!prior_pending) return STARRED_OK;
        prior_pending = false;
        return starlet_launch(p, params, grad != nullptr, &n_l1);
    };
    if (!ride && !late && !late_adj) {
        int rc = starlet_fork(p);
        if (rc) return rc;
        prior_pending = true;
    }
    if (fft) {
        e0 = p->prof_start();
        // with the fused update the counter advances in the first launch of the step
        HIP_TRY(fft_spectra(p->st, p->fd, params, p->N, p->E, p->M, p->sigma, adam ? tick : nullptr,
                            ride ? &pa : nullptr, ride ? &pb : nullptr));
        p->prof_stop(STARRED_STAGE_SPECTRA, e0);
        if (int rc = prior_flush()) return rc;
        e0 = p->prof_start();
        hipEvent_t e1;
        // chi-square partials: the line-pass frames' row groups, then one per fused frame
        const int n_rows = fused ? p->fd.frows_lg.n_items : p->fd.frows.n_items;
        if (fused) {
            hipStream_t sf = p->st;
            if (split) {
                HIP_TRY(hipEventRecord(p->ev_fork3, p->st));
                HIP_TRY(hipStreamWaitEvent(p->st3, p->ev_fork3, 0));
                sf = p->st3;
            }
            e1 = p->prof_start(sf);
            HIP_TRY(fft_fused_fwd(sf, p->fd, params, p->N, p->E, p->M, p->s, p->data, p->invvar,
                                  p->d_part_chi_fft + n_rows, ride ? &pc : nullptr));
            p->prof_stop(STARRED_STAGE_FFT_FUSED, e1, sf);
            if (split) HIP_TRY(hipEventRecord(p->ev_join3, p->st3));
        }
        e1 = p->prof_start();
        HIP_TRY(fft_spec_fwd(p->st, p->fd, params, p->N, p->E, p->M, p->s, fused));
        p->prof_stop(STARRED_STAGE_FFT_SPEC, e1);
        e1 = p->prof_start();
        HIP_TRY(fused ? fft_model_cols_lg(p->st, p->fd) : fft_model_cols(p->st, p->fd));
        p->prof_stop(STARRED_STAGE_FFT_MCOLS, e1);
        e1 = p->prof_start();
        HIP_TRY(fused ? fft_model_rows_lg(p->st, p->fd, p->data, p->invvar, p->d_part_chi_fft)
                      : fft_model_rows(p->st, p->fd, p->data, p->invvar, p->d_part_chi_fft, nullptr));
        p->prof_stop(STARRED_STAGE_FFT_MROWS, e1);
        p->prof_stop(STARRED_STAGE_CONV_FWD, e0);
        n_chi = n_rows + (fused ? p->fd.n_fused : 0);
        if (late) {
            int rc = starlet_fork(p);
            if (rc) return rc;
            prior_pending = true;
        }
    }
    if (dir) {
        // the direct classes' frames: their chi-square partials follow the FFT ones
        const bool all = !fft;
        e0 = p->prof_start();
        HIP_TRY(launch_render(p->st, p->d_fr, p->E, p->Fdir, p->N, p->M, p->sigma, params, p->d_scene,
                              all ? nullptr : p->d_fdir, (int)p->fdir.size(), p->xf));
        p->prof_stop(STARRED_STAGE_RENDER, e0);
        if (int rc = prior_flush()) return rc;
        e0 = p->prof_start();
        hipEvent_t e1 = p->prof_start();
        if (xf_fft) {
            // transformed frames through their own spectra (every frame: all classes run
            // this path while transforms are set)
            HIP_TRY(fft_xf_forward(p->st, p->fd, p->d_scene, p->s, p->data, p->invvar, p->d_part_chi_fft + n_chi));
            n_chi += p->fd.frows_x.n_items;
        } else {
            HIP_TRY(launch_fwd_direct(p->st, p->s, p->d_fr, p->d_fwd_items, (int)p->fwd_items.size(), p->Tdir,
                                      p->d_scene, p->d_kf, p->data, p->invvar, p->d_rho, p->d_part_chi_fft + n_chi,
                                      p->fwd_groups));
            n_chi += (int)p->fwd_items.size();
        }
        p->prof_stop(STARRED_STAGE_DIRECT_FWD, e1);
        if (!fft) p->prof_stop(STARRED_STAGE_CONV_FWD, e0);
    }
    if (grad) {
        e0 = p->prof_start();
        if (fft) {
            // frequency domain: the frames' adjoint spectra are summed per shape class
            // before one inverse transform, and the per-frame dot products for Gamma, a
            // and c are taken there (Parseval)
            hipEvent_t e1 = p->prof_start();
            HIP_TRY(fused ? fft_rho_cols_lg(p->st, p->fd) : fft_rho_cols(p->st, p->fd));
            p->prof_stop(STARRED_STAGE_FFT_RCOLS, e1);
            if (split) HIP_TRY(hipStreamWaitEvent(p->st, p->ev_join3, 0));
            e1 = p->prof_start();
            HIP_TRY(fft_spec_adj(p->st, p->fd, p->M));
            p->prof_stop(STARRED_STAGE_FFT_ACOLS, e1);
            if (int rc = prior_flush()) return rc;
            if (late_adj) {
                int rc = starlet_fork(p);
                if (rc) return rc;
                prior_pending = true;
            }
            e1 = p->prof_start();
            HIP_TRY(fft_adj_sums(p->st, p->fd, p->M, p->d_fsum));
            p->prof_stop(STARRED_STAGE_FFT_FSUM, e1);
            if (int rc = prior_flush()) return rc;
            e1 = p->prof_start();
            HIP_TRY(fin_rows ? fft_grad_h_cols(p->st, p->fd, ride ? &pd : nullptr)
                             : fft_grad_h_inverse(p->st, p->fd, ride ? &pd : nullptr));
            p->prof_stop(STARRED_STAGE_FFT_AROWS, e1);
        }
        if (dir) {
            hipEvent_t e1 = p->prof_start();
            if (xf_fft)
                HIP_TRY(fft_xf_adjoint(p->st, p->fd, p->d_g));
            else
                HIP_TRY(launch_adj_direct(p->st, p->s, p->d_fr, p->d_adj_items, (int)p->adj_items.size(), p->Ardir,
                                          p->Bpdir, p->d_rho, p->d_ka, p->d_g, p->adj_groups));
            p->prof_stop(STARRED_STAGE_DIRECT_ADJ, e1);
        }
        p->prof_stop(STARRED_STAGE_CONV_ADJ, e0);
        if (dir) {
            e0 = p->prof_start();
            HIP_TRY(launch_frame_sums(p->st, p->d_fr, p->E, p->N, p->M, p->sigma, params, p->d_g, p->d_fsum, true,
                                      fft ? p->d_fdir : nullptr, (int)p->fdir.size(), p->xf, p->gxf, p->d_gxfp));
            p->prof_stop(STARRED_STAGE_GRAD_SUMS, e0);
        }
    }
    if (int rc = prior_flush()) return rc;
    if (split && !grad) HIP_TRY(hipStreamWaitEvent(p->st, p->ev_join3, 0));
    if (!ride) HIP_TRY(hipStreamWaitEvent(p->st, p->ev_join, 0));
    e0 = p->prof_start();
    if (fin_rows) {
        FinalArgs fa;
        fa.E = p->E;
        fa.M = p->M;
        fa.N = p->N;
        fa.n_chi = n_chi;
        fa.n_l1 = n_l1;
        fa.part_chi = part_chi;
        fa.part_l1 = p->d_part_l1;
        fa.fsum = p->d_fsum;
        fa.params = params;
        fa.grad = grad;
        fa.loss = loss_out;
        fa.tick = adam ? nullptr : tick;
        if (adam) fa.adam = *adam;
        fa.pts = p->lam_pts != 0.0 ? p->d_pts : nullptr;
        HIP_TRY(fft_grad_h_rows_final(p->st, p->fd, p->d_prior, fa, ride ? &dd : nullptr));
        p->prof_stop(STARRED_STAGE_FINALIZE, e0);
        return STARRED_OK;
    }
    // dL/dh: the prior gradient plus the direct frames' windows (directly into grad
    // when every frame is direct; else into d_hdir, which the final launch adds to
    // the FFT classes' windows, pixel by pixel in the same launch as the update)
    if (grad && dir)
        HIP_TRY(launch_finalize_h(p->st, p->d_fr, p->E, p->N, p->d_g, p->d_prior, fft ? p->d_hdir : grad,
                                  p->d_hpart, fft ? p->d_fdir : nullptr, (int)p->fdir.size(), p->xf));
    HIP_TRY(launch_finalize_small(p->st, p->E, p->M, n_chi, part_chi, n_l1, p->d_part_l1, p->lam, p->d_fsum,
                                  params, p->N, grad, loss_out, nullptr, nullptr, nullptr,
                                  (fft && adam) ? nullptr : tick, fft ? p->fd.classes : nullptr, p->fd.n_classes,
                                  p->fd.hcls, ride ? nullptr : ((fft && dir) ? p->d_hdir : p->d_prior),
                                  (fft && adam) ? *adam : AdamDev(),
                                  (p->lam_pts != 0.0 && grad) ? p->d_pts : nullptr, (ride && grad) ? &dd : nullptr));
    p->prof_stop(STARRED_STAGE_FINALIZE, e0);
    return STARRED_OK;
}

// ---- autotuner ----
// Per-class algorithm and forward form, then the FFT path's launch shapes, chosen
// by timing whole loss+gradient evaluations (one warm-up, kTuneReps timed) on the
// plan's stream at h = 0 with the bound data. Coordinate descent over the classes,
// most costly first; a change is kept when it saves more than 2 %.
constexpr int kTuneReps = 8;
constexpr double kTuneGain = 0.98;

struct TuneEntry {
    std::vector<int> choice;
    int adj_blocks = kAdjBlocks, line_groups = 1024, adj_fc = kAdjFrames, fwd_split = 1, prior_late = 0;
    std::vector<std::array<double, 3>> tried;  // the timings the decision came from
    double wall_ms = 0.0;                      // how long that tuning took
};

static std::mutex g_tune_mu;
static std::map<std::string, TuneEntry> g_tune_cache;

// The plan's shapes and the device: what the timings depend on.
static std::string tune_key(const starred_plan *p)
{
    std::map<std::pair<int, int>, int> cnt;
    for (int i = 0; i < p->E; ++i) cnt[{p->n[i], p->K[i]}]++;
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    std::string k = "s" + std::to_string(p->s) + " N" + std::to_string(p->N) + " M" + std::to_string(p->M) + " J" +
                    std::to_string(p->J) + " w" + std::to_string(p->w_stride) + " cu" + std::to_string(cus) + ":";
    for (auto &kv : cnt)
        k += " " + std::to_string(kv.first.first) + "/" + std::to_string(kv.first.second) + "x" +
             std::to_string(kv.second);
    return k;
}

static int time_plan(starred_plan *p, const float *params, double *loss, hipEvent_t a, hipEvent_t b, double *ms)
{
    int rc = loss_grad_impl(p, params, p->d_grad, loss);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(a, p->st));
    for (int r = 0; r < kTuneReps && !rc; ++r) rc = loss_grad_impl(p, params, p->d_grad, loss);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(b, p->st));
    HIP_TRY(hipEventSynchronize(b));
    float f = 0.f;
    HIP_TRY(hipEventElapsedTime(&f, a, b));
    *ms = (double)f / kTuneReps;
    return STARRED_OK;
}

static int autotune(starred_plan *p)
{
    const auto t_start = std::chrono::steady_clock::now();
    const int C = (int)p->cls.size();
    p->cls_tune.assign(C, {-1.0, -1.0, -1.0});
    const std::string key = tune_key(p);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            p->adj_blocks = it->second.adj_blocks;
            p->line_groups = it->second.line_groups;
            p->adj_fc = it->second.adj_fc;
            p->fwd_split = it->second.fwd_split;
            p->prior_late = it->second.prior_late;
            p->tune_cached = 1;
            p->cls_tune = it->second.tried;
            p->tune_wall_ms = it->second.wall_ms;
            const std::vector<int> ch = it->second.choice;
            return apply_choices(p, ch);
        }
    }
    p->tune_cached = 0;
    float *params = nullptr;
    double *loss = nullptr;
    int rc = dev_alloc(&params, p->nparams);
    if (rc) return rc;
    rc = dev_alloc(&loss, 3);
    if (rc) {
        (void)hipFree(params);
        return rc;
    }
    const bool prof = p->prof_on;
    p->prof_on = false;
    hipEvent_t a = nullptr, b = nullptr;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    // h = 0 (a fill kernel: the tuning's launches may be the first on this stream)
    if (launch_fill(p->st, params, p->nparams, 0.f) != hipSuccess) rc = fail(STARRED_EHIP, "autotune fill");
    // start: every class on the FFT algorithm, the one-launch forward where it fits
    std::vector<int> ch(C);
    for (int c = 0; c < C; ++c) ch[c] = p->cls_fits[c] ? kChFused : kChLines;
    double best = 0.0;
    if (!rc) rc = apply_choices(p, ch);
    if (!rc) rc = time_plan(p, params, loss, a, b, &best);
    for (int c = 0; c < C && !rc; ++c) p->cls_tune[c][ch[c]] = best;
    // classes in order of FFT cost: frames x P^2
    std::vector<int> order(C);
    for (int c = 0; c < C; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return (double)p->cls[x].ncf * p->cls[x].P * p->cls[x].P > (double)p->cls[y].ncf * p->cls[y].P * p->cls[y].P;
    });
    for (int c : order) {
        if (rc) break;
        for (int alt : {kChDirect, kChFused, kChLines}) {
            if (alt == ch[c]) continue;
            if (alt == kChDirect && !class_direct_ok(p, c)) continue;
            if (alt == kChFused && !p->cls_fits[c]) continue;
            std::vector<int> t = ch;
            t[c] = alt;
            double ms = 0.0;
            rc = apply_choices(p, t);
            if (!rc) rc = time_plan(p, params, loss, a, b, &ms);
            if (rc) break;
            p->cls_tune[c][alt] = ms;
            if (ms < kTuneGain * best) {
                best = ms;
                ch = t;
            }
        }
        if (!rc) p->cls_tune[c][ch[c]] = best;
    }
    if (!rc) rc = apply_choices(p, ch);
    // launch shapes of the FFT path: frames per adjoint chunk and adjoint work groups
    // together (they interact: the chunk count sets the rows per group), then the
    // line-pass work groups, then the one-launch forward on its own stream or not
    if (!rc && p->algo == STARRED_CONV_FFT) {
        const std::vector<int> abs_ = {256, 512, 1024, 2048};
        const int keep_fc = p->adj_fc, keep_ab = p->adj_blocks;
        int best_fc = keep_fc, best_ab = keep_ab;
        for (int fc : {1, 2, 4, 8})
            for (int ab : abs_) {
                if (rc || !adj_shape_ok(fc, p->M) || (fc == keep_fc && ab == keep_ab)) continue;
                p->adj_fc = fc;
                p->adj_blocks = ab;
                double ms = 0.0;
                rc = build_fft_lists(p);
                if (!rc) rc = time_plan(p, params, loss, a, b, &ms);
                if (!rc && ms < kTuneGain * best) {
                    best = ms;
                    best_fc = fc;
                    best_ab = ab;
                }
            }
        p->adj_fc = best_fc;
        p->adj_blocks = best_ab;
        for (int which = 0; which < 3 && !rc; ++which) {
            int &knob = which == 0 ? p->line_groups : (which == 1 ? p->fwd_split : p->prior_late);
            const int keep = knob;
            int best_v = keep;
            // prior placement: forked at the start (0), after the forward (1) or after the
            // adjoint's spectral products (3), or its passes carried by the step's own
            // launches (2, where they can ride)
            const std::vector<int> cands = which == 0   ? std::vector<int>{512, 1024, 2048}
                                           : which == 1 ? std::vector<int>{0, 1}
                                                        : std::vector<int>{0, 1, 2, 3};
            for (int v : cands) {
                if (v == keep) continue;
                knob = v;
                double ms = 0.0;
                rc = build_fft_lists(p);
                if (!rc) rc = time_plan(p, params, loss, a, b, &ms);
                if (rc) break;
                if (ms < kTuneGain * best) {
                    best = ms;
                    best_v = v;
                }
            }
            knob = best_v;
        }
        if (!rc) rc = build_fft_lists(p);
    }
    p->drop_graphs();
    p->prof_on = prof;
    (void)hipStreamSynchronize(p->st);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(params);
    (void)hipFree(loss);
    p->tune_wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (!rc) {
        TuneEntry e;
        e.choice = ch;
        e.adj_blocks = p->adj_blocks;
        e.line_groups = p->line_groups;
        e.adj_fc = p->adj_fc;
        e.fwd_split = p->fwd_split;
        e.prior_late = p->prior_late;
        e.tried = p->cls_tune;
        e.wall_ms = p->tune_wall_ms;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = e;
    }
    return rc;
}

// tick: the device step counter the step advances (its first launch); adam: the update
// fused into the final launch (which also adds the prior's gradient to grad_b)
static int psf_loss_grad_impl(starred_plan *p, const float *params, float *grad, double *loss_out, int *tick = nullptr,
                              const AdamDev *adam = nullptr)
{
    const int S = p->E, n = p->psf_n, N = p->N;
    int n_l1 = 0;
    // the prior's branch first: its chain is about as long as the stars' (render, forward,
    // adjoint), and launching it ahead of them measured faster than after the render
    int rc = starlet_fork(p);
    if (!rc) rc = starlet_launch(p, params + 5, grad != nullptr, &n_l1);
    if (rc) return rc;
    hipEvent_t e0 = p->prof_start();
    HIP_TRY(launch_psf_render64(p->st, N, params, p->d_s64, grad ? p->d_dm : nullptr, tick));
    p->prof_stop(STARRED_STAGE_RENDER, e0);
    e0 = p->prof_start();
    HIP_TRY(launch_psf_fwd(p->st, S, n, p->s, N, p->sigma, params, p->d_s64, p->data, p->invvar, p->d_rho,
                           p->d_part_chi));
    p->prof_stop(STARRED_STAGE_CONV_FWD, e0);
    if (grad) {
        e0 = p->prof_start();
        HIP_TRY(launch_psf_adjsum(p->st, S, n, p->s, N, p->sigma, params, p->d_rho, p->d_dm, grad, p->d_part_eta));
        p->prof_stop(STARRED_STAGE_CONV_ADJ, e0);
    }
    // the L1 partials and the prior's gradient come from the starlet branch
    HIP_TRY(hipStreamWaitEvent(p->st, p->ev_join, 0));
    e0 = p->prof_start();
    HIP_TRY(launch_psf_finalize(p->st, S, N, psf_fwd_tiles(n), p->d_part_chi, n_l1, p->d_part_l1, psf_adj_tiles(N),
                                p->d_part_eta, params, grad ? p->d_prior : nullptr, grad, loss_out,
                                adam ? *adam : AdamDev()));
    p->prof_stop(STARRED_STAGE_FINALIZE, e0);
    return STARRED_OK;
}

int starred_psf_model(starred_plan *p, const float *params, float *model)
{
    if (!p || !params || !model) return fail(STARRED_EINVAL, "NULL argument");
    if (p->mode != STARRED_PSF) return fail(STARRED_EUNSUPPORTED, "starred_psf_model needs a PSF-mode plan");
    // the forward's tiles in model mode over the FP64 PSF
    HIP_TRY(launch_psf_render64(p->st, p->N, params, p->d_s64, nullptr));
    HIP_TRY(launch_psf_fwd(p->st, p->E, p->psf_n, p->s, p->N, p->sigma, params, p->d_s64, nullptr, nullptr, nullptr,
                           nullptr, model));
    return STARRED_OK;
}

// ---- plain baseline: per-epoch, full-resolution convolution, one launch per operator ----
static int build_plain(starred_plan *p)
{
    const int E = p->E;
    p->frp.resize(E);
    long long kfoff = 0, kaoff = 0;
    std::vector<Item> fw, ad;
    int nchi = 0;
    for (int i = 0; i < E; ++i) {
        const FrameDev &r = p->fr[i];
        FrameDev &f = p->frp[i];
        memset(&f, 0, sizeof f);
        f.n = r.F;  // the plain convolution runs at fine resolution
        f.F = r.F;
        f.K = r.K;
        f.Kp = r.K;
        f.o = r.o;
        f.cp = r.K / 2;
        f.Tpad = round_up(f.Kp, 4);
        f.dmin = -f.cp;
        const int dmax = f.Kp - 1 - f.cp;
        f.Ar = dmax - f.dmin + 1;
        f.Bpad = round_up(f.Ar, 4);
        f.data_off = r.fine_off;
        f.fine_off = r.fine_off;
        f.kern_off = r.kern_off;
        f.kf_off = kfoff;
        f.ka_off = kaoff;
        kfoff += (long long)f.Kp * f.Tpad;
        kaoff += (long long)f.Ar * f.Bpad;
        p->pTmax = std::max(p->pTmax, f.Tpad);
        p->pAr_max = std::max(p->pAr_max, f.Ar);
        p->pBpad_max = std::max(p->pBpad_max, f.Bpad);
        p->pfwd_start.push_back((int)fw.size());
        for (int p0 = 0; p0 < f.n; p0 += kFwdTP)
            for (int q0 = 0; q0 < f.n; q0 += kFwdTQ) fw.push_back(Item{i, p0, q0, 0});
        p->padj_start.push_back((int)ad.size());
        for (int p0 = 0; p0 < f.n; p0 += kAdjTP)
            for (int q0 = 0; q0 < f.n; q0 += kAdjTQ) ad.push_back(Item{i, p0, q0, 0});
        p->pchi_start.push_back(nchi);
        nchi += (r.n * r.n + 255) / 256;
    }
    p->pfwd_start.push_back((int)fw.size());
    p->padj_start.push_back((int)ad.size());
    p->n_pchi = nchi;
    if (fwd_lds_bytes(1, p->pTmax) > kMaxLds || adj_lds_bytes(p->pAr_max, p->pBpad_max) > kMaxLds)
        return fail(STARRED_EUNSUPPORTED, "kernels too large for the plain baseline");
    int rc;
    if ((rc = p->alloc(&p->d_frp, E))) return rc;
    if ((rc = p->alloc(&p->d_pfwd, fw.size()))) return rc;
    if ((rc = p->alloc(&p->d_padj, ad.size()))) return rc;
    if ((rc = p->alloc(&p->d_pkf, kfoff))) return rc;
    if ((rc = p->alloc(&p->d_pka, kaoff))) return rc;
    if ((rc = p->alloc(&p->d_u, p->nfine))) return rc;
    if ((rc = p->alloc(&p->d_gh, p->nfine))) return rc;
    if ((rc = p->alloc(&p->d_m, p->ndata))) return rc;
    if ((rc = p->alloc(&p->d_pchi, std::max(1, nchi)))) return rc;
    HIP_TRY(hipMemcpy(p->d_frp, p->frp.data(), sizeof(FrameDev) * E, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->d_pfwd, fw.data(), sizeof(Item) * fw.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->d_padj, ad.data(), sizeof(Item) * ad.size(), hipMemcpyHostToDevice));
    HIP_TRY(launch_prep_kernels(p->st, p->d_frp, p->frp.data(), E, 1, p->psf_bound, p->d_pkf, p->d_pka));
    HIP_TRY(hipStreamSynchronize(p->st));
    p->plain_ready = true;
    return STARRED_OK;
}

int starred_loss_grad_plain(starred_plan *p, const float *params, float *grad, double *loss_out)
{
    if (p && p->xf) return fail(STARRED_EUNSUPPORTED, "the plain baseline has no per-frame transforms");
    if (!p || !params || !loss_out) return fail(STARRED_EINVAL, "NULL argument");
    if (p->mode != STARRED_DECONV) return fail(STARRED_EUNSUPPORTED, "the plain baseline is a deconvolution-mode path");
    if (!p->frames_set) return fail(STARRED_ESTATE, "set_frames has not been called");
    if (!p->plain_ready) {
        int rc = build_plain(p);
        if (rc) return rc;
    }
    for (int i = 0; i < p->E; ++i) {
        const FrameDev &f = p->fr[i];
        HIP_TRY(launch_render_frame(p->st, p->d_fr, p->E, i, f.F, p->N, p->M, p->sigma, params, p->d_scene));
        HIP_TRY(launch_fwd_direct(p->st, 1, p->d_frp, p->d_pfwd + p->pfwd_start[i],
                                  p->pfwd_start[i + 1] - p->pfwd_start[i], p->pTmax, p->d_scene, p->d_pkf,
                                  nullptr, nullptr, p->d_u, nullptr));
        HIP_TRY(launch_plain_frame_ops(p->st, 0, p->d_fr, i, f.n, f.F, p->s, p->d_u, nullptr, nullptr, p->d_m,
                                       nullptr));
        HIP_TRY(launch_plain_frame_ops(p->st, 1, p->d_fr, i, f.n, f.F, p->s, p->d_m, p->data, p->invvar, p->d_rho,
                                       p->d_pchi + p->pchi_start[i]));
        if (grad) {
            HIP_TRY(launch_plain_frame_ops(p->st, 2, p->d_fr, i, f.n, f.F, p->s, p->d_rho, nullptr, nullptr,
                                           p->d_gh, nullptr));
            HIP_TRY(launch_adj_direct(p->st, 1, p->d_frp, p->d_padj + p->padj_start[i],
                                      p->padj_start[i + 1] - p->padj_start[i], p->pAr_max, p->pBpad_max, p->d_gh,
                                      p->d_pka, p->d_g));
            HIP_TRY(launch_frame_sums_one(p->st, p->d_fr, p->E, i, p->N, p->M, p->sigma, params, p->d_g, p->d_fsum));
        }
    }
    int n_l1 = 0;
    int rc = prior_launches(p, p->st, params, grad != nullptr, &n_l1);
    if (rc) return rc;
    if (grad) HIP_TRY(launch_finalize_h(p->st, p->d_fr, p->E, p->N, p->d_g, p->d_prior, grad, p->d_hpart));
    HIP_TRY(launch_finalize_small(p->st, p->E, p->M, p->n_pchi, p->d_pchi, n_l1, p->d_part_l1, p->lam, p->d_fsum,
                                  params, p->N, grad, loss_out, nullptr, nullptr, nullptr, nullptr, nullptr, 0,
                                  nullptr, nullptr, AdamDev(), (p->lam_pts != 0.0 && grad) ? p->d_pts : nullptr));
    return STARRED_OK;
}

// Run `body` through a captured HIP graph: replay the graph of `slot` when the
// key (argument pointers and by-value parameters) matches, otherwise capture
// the launch sequence on st (the forked starlet stream joins the capture
// through its events) and instantiate it.
extern "C++" {
template <class Body>
static int run_graph(starred_plan *p, int slot, const std::vector<uintptr_t> &key, Body body)
{
    auto &g = p->gs[slot];
    if (!g.valid || g.key != key) {
        if (g.x) (void)hipGraphExecDestroy(g.x);
        if (g.g) (void)hipGraphDestroy(g.g);
        g = starred_plan::GraphSlot();
        const bool prof = p->prof_on;
        p->prof_on = false;
        HIP_TRY(hipStreamBeginCapture(p->st, hipStreamCaptureModeThreadLocal));
        int rc = body();
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(p->st, &graph);
        p->prof_on = prof;
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail_hip(e, "hipGraphInstantiate");
        }
        e = hipGraphUpload(exec, p->st);  // device-side set-up once, not at every launch
        if (e != hipSuccess) {
            (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
            return fail_hip(e, "hipGraphUpload");
        }
        g.g = graph;
        g.x = exec;
        g.key = key;
        g.valid = true;
    }
    hipEvent_t e0 = p->prof_start();
    HIP_TRY(hipGraphLaunch(g.x, p->st));
    p->prof_stop(STARRED_STAGE_GRAPH, e0);
    return STARRED_OK;
}
}  // extern "C++"

int starred_loss_grad(starred_plan *p, const float *params, float *grad, double *loss_out)
{
    if (!p || !params || !loss_out) return fail(STARRED_EINVAL, "NULL argument");
    if (!p->frames_set) return fail(STARRED_ESTATE, "set_frames has not been called");
    if (p->prof_on) HIP_TRY(launch_idle(p->st, kProfIdleIters));
    auto body = [&]() -> int {
        return (p->mode == STARRED_PSF) ? psf_loss_grad_impl(p, params, grad, loss_out)
                                         : loss_grad_impl(p, params, grad, loss_out);
    };
    if (!p->graph_mode) return body();
    std::vector<uintptr_t> key = {(uintptr_t)params, (uintptr_t)grad, (uintptr_t)loss_out, (uintptr_t)p->algo};
    return run_graph(p, 0, key, body);
}

// Steps a graph replay of starred_steps covers (the device-side gap between two
// graph launches is paid once per kStepsPerGraph steps).
constexpr int kStepsPerGraph = 8;

// n consecutive optimiser steps from step number t
static int run_steps(starred_plan *p, float *params, float *m, float *v, int32_t t, const starred_adam *hp,
                     int32_t n, double *loss_out)
{
    if (!p || !params || !m || !v || !hp) return fail(STARRED_EINVAL, "NULL argument");
    if (t < 1) return fail(STARRED_EINVAL, "t must be >= 1");
    if (n < 1) return fail(STARRED_EINVAL, "the number of steps must be >= 1");
    if (hp->rule != STARRED_ADAM && hp->rule != STARRED_ADABELIEF) return fail(STARRED_EINVAL, "unknown update rule");
    if (!p->frames_set) return fail(STARRED_ESTATE, "set_frames has not been called");
    // the device step counter is advanced inside the step; resynchronise it when
    // the caller's step number is not the next one
    if (t != p->next_t) HIP_TRY(launch_set_step(p->st, p->d_t, t - 1));
    if (p->prof_on) HIP_TRY(launch_idle(p->st, kProfIdleIters));
    // FFT path and PSF mode: the update runs inside the final reduction launch
    const bool fused_adam = p->mode == STARRED_PSF || p->algo == STARRED_CONV_FFT;
    AdamDev ad;
    ad.params = params;
    ad.m = m;
    ad.v = v;
    ad.d_t = p->d_t;
    for (int k = 0; k < 4; ++k) ad.lr[k] = hp->lr[k];
    ad.beta1 = hp->beta1;
    ad.beta2 = hp->beta2;
    ad.eps = hp->eps;
    ad.rule = hp->rule;
    ad.eps_root = hp->eps_root;
    auto one = [&]() -> int {
        int rc = (p->mode == STARRED_PSF) ? psf_loss_grad_impl(p, params, p->d_grad, loss_out, p->d_t, &ad)
                                          : loss_grad_impl(p, params, p->d_grad, loss_out, p->d_t,
                                                           fused_adam ? &ad : nullptr);
        if (rc) return rc;
        if (fused_adam) return STARRED_OK;
        const long long NN = (long long)p->N * p->N;
        const long long seg[3] = {NN, NN + p->E, NN + p->E + (long long)p->E * p->M};
        hipEvent_t e0 = p->prof_start();
        HIP_TRY(launch_adam(p->st, p->nparams, seg, hp->lr, params, p->d_grad, m, v, p->d_t, hp->beta1, hp->beta2,
                            hp->eps, hp->rule, hp->eps_root));
        p->prof_stop(STARRED_STAGE_ADAM, e0);
        return STARRED_OK;
    };
    if (!p->graph_mode) {
        for (int i = 0; i < n; ++i) {
            int rc = one();
            if (rc) return rc;
        }
    } else {
        uint32_t hb[9];
        memcpy(hb, hp->lr, sizeof(float) * 4);
        memcpy(hb + 4, &hp->beta1, sizeof(float));
        memcpy(hb + 5, &hp->beta2, sizeof(float));
        memcpy(hb + 6, &hp->eps, sizeof(float));
        memcpy(hb + 7, &hp->rule, sizeof(int32_t));
        memcpy(hb + 8, &hp->eps_root, sizeof(float));
        std::vector<uintptr_t> key = {(uintptr_t)params, (uintptr_t)m, (uintptr_t)v, (uintptr_t)loss_out,
                                      (uintptr_t)p->algo};
        for (uint32_t x : hb) key.push_back(x);
        // whole groups of steps as one graph, the rest one step per graph
        int left = n;
        while (left >= kStepsPerGraph) {
            int rc = run_graph(p, 2, key, [&]() -> int {
                for (int i = 0; i < kStepsPerGraph; ++i) {
                    int rc2 = one();
                    if (rc2) return rc2;
                }
                return STARRED_OK;
            });
            if (rc) return rc;
            left -= kStepsPerGraph;
        }
        for (; left > 0; --left) {
            int rc = run_graph(p, 1, key, one);
            if (rc) return rc;
        }
    }
    p->next_t = t + n;
    return STARRED_OK;
}

int starred_step(starred_plan *p, float *params, float *m, float *v, int32_t t,
                 const starred_adam *hp, double *loss_out)
{
    return run_steps(p, params, m, v, t, hp, 1, loss_out);
}

int starred_steps(starred_plan *p, float *params, float *m, float *v, int32_t t, const starred_adam *hp,
                  int32_t n_steps, double *loss_out)
{
    return run_steps(p, params, m, v, t, hp, n_steps, loss_out);
}

int starred_set_fft_fused(starred_plan *p, int32_t enable)
{
    if (!p) return fail(STARRED_EINVAL, "plan is NULL");
    p->drop_graphs();
    p->fft_fused = enable != 0;
    return STARRED_OK;
}

int starred_set_lambda_pts(starred_plan *p, double lambda_pts)
{
    if (!p) return fail(STARRED_EINVAL, "plan is NULL");
    if (p->mode != STARRED_DECONV) return fail(STARRED_EUNSUPPORTED, "the point-source prior is a deconvolution term");
    if (!(lambda_pts >= 0.0)) return fail(STARRED_EINVAL, "lambda_pts must be >= 0");
    p->drop_graphs();
    p->lam_pts = lambda_pts;
    return STARRED_OK;
}

int starred_pts_image(starred_plan *p, const float *params, float *P_out)
{
    if (!p || !params || !P_out) return fail(STARRED_EINVAL, "NULL argument");
    if (p->mode != STARRED_DECONV) return fail(STARRED_EUNSUPPORTED, "the point-source prior is a deconvolution term");
    HIP_TRY(launch_pts_render(p->st, p->N, p->E, p->M, p->sigma, params, nullptr, P_out));
    return STARRED_OK;
}

int starred_estimate_lambda_pts(starred_plan *p, const float *params, double *lambda_pts_out)
{
    if (!p || !params || !lambda_pts_out) return fail(STARRED_EINVAL, "NULL argument");
    if (p->mode != STARRED_DECONV) return fail(STARRED_EUNSUPPORTED, "the point-source prior is a deconvolution term");
    if (!p->frames_set) return fail(STARRED_ESTATE, "set_frames has not been called");
    if (p->M < 1) return fail(STARRED_EUNSUPPORTED, "no point sources");
    const long long NN = (long long)p->N * p->N;
    const int B = p->M + 2, slots = starlet_l1_slots(p->N, p->J);
    if (!p->est_img) {
        int rc = p->alloc(&p->est_img, (size_t)B * NN);
        if (!rc) rc = p->alloc(&p->est_part, (size_t)B * slots);
        if (!rc) rc = p->alloc(&p->est_out, (size_t)B + p->M);
        if (rc) return rc;
    }
    HIP_TRY(launch_fill_d(p->st, p->est_part, (long long)B * slots));
    HIP_TRY(launch_pts_images(p->st, p->N, p->E, p->M, p->sigma, params, p->est_img));
    for (int b = 0; b < B; ++b)
        HIP_TRY(launch_starlet_fwd(p->st, p->N, p->J, p->est_img + b * NN, nullptr, nullptr, p->W, p->w_stride, 1.f,
                                   p->d_ca, p->d_cb, p->d_tmp, p->est_part + (long long)b * slots, nullptr));
    HIP_TRY(launch_pts_sums(p->st, B, slots, p->est_part, p->N, p->E, p->M, params, p->est_out));
    std::vector<double> h(B + p->M);
    HIP_TRY(hipMemcpyAsync(h.data(), p->est_out, sizeof(double) * h.size(), hipMemcpyDeviceToHost, p->st));
    HIP_TRY(hipStreamSynchronize(p->st));
    double den = 0.0;
    for (int k = 0; k < p->M; ++k) den += h[B + k] * h[2 + k];
    if (!(den != 0.0)) return fail(STARRED_EINVAL, "the point sources' norms sum to zero");
    *lambda_pts_out = p->lam * (h[0] - h[1]) / den;
    return STARRED_OK;
}

int starred_set_graph_mode(starred_plan *p, int32_t enable)
{
    if (!p) return fail(STARRED_EINVAL, "plan is NULL");
    if (enable && !p->st) return fail(STARRED_EUNSUPPORTED, "graph capture needs a non-default stream");
    if (!enable) p->drop_graphs();
    p->graph_mode = enable != 0;
    return STARRED_OK;
}

int starred_noise_weights(starred_plan *p, int32_t frame, const float *sigma2_data, int32_t n_real, uint64_t seed,
                          const float *normals, int32_t per_pixel, float *W_out)
{
    if (!p || !sigma2_data || !W_out) return fail(STARRED_EINVAL, "NULL argument");
    if (p->mode != STARRED_DECONV) return fail(STARRED_EUNSUPPORTED, "noise propagation needs deconvolution mode");
    if (!p->frames_set) return fail(STARRED_ESTATE, "set_frames has not been called");
    if (frame < 0 || frame >= p->E) return fail(STARRED_EINVAL, "frame out of range");
    if (n_real < 2) return fail(STARRED_EINVAL, "n_real must be >= 2");
    const int n = p->n[frame], K = p->K[frame], s = p->s, F = s * n, N = p->N, J = p->J;
    const int o = (N - F) / 2;
    const long long FF = (long long)F * F, NN = (long long)N * N;
    const int B = std::min(n_real, kNoiseBatch);
    if (!p->noise_aux || p->noise_frame != frame || p->noise_B < B) {
        if (p->noise_aux) {
            (void)starred_plan_destroy(p->noise_aux);
            p->noise_aux = nullptr;
        }
        // S_f^T on the fine grid = the adjoint of an s = 1 plan with B copies of the frame
        std::vector<int32_t> sides(B, F), ks(B, K);
        starred_desc d{};
        d.mode = STARRED_DECONV;
        d.n_frames = B;
        d.side_host = sides.data();
        d.ksize_host = ks.data();
        d.subsample = 1;
        d.grid_side = N;
        d.n_sources = 0;
        d.n_scales = J;
        d.w_pixel_stride = 0;
        d.conv_algo = STARRED_CONV_FFT;
        d.lambda = 0.0;
        d.gauss_fwhm = p->fwhm;
        int rc = starred_plan_create(&d, p->st, &p->noise_aux);
        if (rc) return rc;
        p->noise_frame = frame;
        p->noise_B = B;
        const long long kk = (long long)K * K;
        if ((rc = p->alloc(&p->nz_kern, (size_t)B * kk))) return rc;
        if ((rc = p->alloc(&p->nz_zero, (size_t)B * FF))) return rc;
        if ((rc = p->alloc(&p->nz_one, (size_t)B * FF))) return rc;
        if ((rc = p->alloc(&p->nz_w, (size_t)J))) return rc;
        if ((rc = p->alloc(&p->nz_delta, (size_t)B * FF))) return rc;
        if ((rc = p->alloc(&p->nz_g, (size_t)B * FF))) return rc;
        if ((rc = p->alloc(&p->nz_img, (size_t)B * NN))) return rc;
        if ((rc = p->alloc(&p->nz_ca, (size_t)B * NN))) return rc;
        if ((rc = p->alloc(&p->nz_cb, (size_t)B * NN))) return rc;
        if ((rc = p->alloc(&p->nz_coef, (size_t)B * J * NN))) return rc;
        if ((rc = p->alloc(&p->nz_s1, (size_t)J * NN))) return rc;
        if ((rc = p->alloc(&p->nz_s2, (size_t)J * NN))) return rc;
        const float *kf = p->psf_bound + p->fr[frame].kern_off;
        for (int b = 0; b < B; ++b)
            HIP_TRY(hipMemcpyAsync(p->nz_kern + b * kk, kf, sizeof(float) * kk, hipMemcpyDeviceToDevice, p->st));
        HIP_TRY(launch_fill(p->st, p->nz_zero, (long long)B * FF, 0.f));
        HIP_TRY(launch_fill(p->st, p->nz_one, (long long)B * FF, 1.f));
        HIP_TRY(launch_fill(p->st, p->nz_w, J, 0.f));
        rc = starred_set_frames(p->noise_aux, p->nz_zero, p->nz_one, p->nz_kern, p->nz_w);
        if (rc) return rc;
    }
    HIP_TRY(launch_fill_d(p->st, p->nz_s1, (long long)J * NN));
    HIP_TRY(launch_fill_d(p->st, p->nz_s2, (long long)J * NN));
    for (int r0 = 0; r0 < n_real; r0 += B) {
        const int nb = std::min(B, n_real - r0);
        HIP_TRY(launch_noise_draw(p->st, B, nb, r0, n, s, sigma2_data, normals, (unsigned long long)seed,
                                  p->nz_delta));
        int rc = starred_convolve_subsample_adj(p->noise_aux, p->nz_delta, p->nz_g);
        if (rc) return rc;
        HIP_TRY(launch_noise_embed(p->st, B, F, N, o, p->nz_g, p->nz_img));
        if (J == 1) {
            HIP_TRY(hipMemcpyAsync(p->nz_coef, p->nz_img, sizeof(float) * B * NN, hipMemcpyDeviceToDevice, p->st));
        } else {
            HIP_TRY(launch_starlet_fwd_batch(p->st, N, J, nb, p->nz_img, p->nz_coef, p->nz_ca, p->nz_cb,
                                             p->d_wzero));
        }
        HIP_TRY(launch_noise_moments(p->st, nb, (long long)J * NN, p->nz_coef, p->nz_s1, p->nz_s2));
    }
    HIP_TRY(launch_noise_finish(p->st, J, NN, n_real, per_pixel, p->nz_s1, p->nz_s2, W_out));
    HIP_TRY(hipStreamSynchronize(p->st));
    return STARRED_OK;
}

// ---------------------------------------------------------------------------
// L-BFGS-B on the plan's loss: the iteration control (starred_lbfgsb_*, FP64 on
// the host) asks for the loss and gradient at a point, the device evaluates them
// there, and the two are copied back (one synchronisation per evaluation).
// starred_lbfgs_direction: the two-loop recursion on the device (L-BFGS direction).
// ---------------------------------------------------------------------------
extern "C++" {
struct starred_lbfgs {
    starred_plan *p = nullptr;
    int m = 0;
    long long n = 0;
    std::vector<double> lo, hi;
    bool has_lo = false, has_hi = false;
    starred_lbfgsb *core = nullptr;
    std::vector<double> xh, gh;
    std::vector<float> buf;
    float *gdev = nullptr;
    double *loss = nullptr;
    double f = 0.0;
    int task = 0;
    bool started = false, done = false;
    std::vector<void *> owned;
    ~starred_lbfgs()
    {
        if (core) (void)starred_lbfgsb_destroy(core);
        for (void *q : owned) (void)hipFree(q);
    }
    template <typename T>
    int alloc(T **q, size_t cnt)
    {
        int rc = dev_alloc(q, cnt);
        if (rc == STARRED_OK) owned.push_back((void *)*q);
        return rc;
    }
};
}  // extern "C++"

int starred_lbfgs_direction(starred_plan *p, const float *grad, const float *S, const float *Y, int32_t m,
                            int32_t count, int32_t newest, float *d_out)
{
    if (!p || !grad || !d_out || (count > 0 && (!S || !Y))) return fail(STARRED_EINVAL, "NULL argument");
    if (m < 1 || count < 0 || count > m || (count > 0 && (newest < 0 || newest >= m)))
        return fail(STARRED_EINVAL, "history indices out of range");
    if (!p->d_lbfgs_alpha) {
        int rc = p->alloc(&p->d_lbfgs_alpha, 1024);
        if (rc) return rc;
    }
    if (count > 1024) return fail(STARRED_EINVAL, "history longer than 1024");
    HIP_TRY(launch_lbfgs_direction(p->st, p->nparams, grad, S, Y, m, count, count > 0 ? newest : 0, d_out,
                                   p->d_lbfgs_alpha));
    return STARRED_OK;
}

int starred_lbfgs_create(starred_plan *p, int32_t m, const float *lo, const float *hi, starred_lbfgs **out)
{
    if (!p || !out) return fail(STARRED_EINVAL, "NULL argument");
    *out = nullptr;
    if (m < 1) return fail(STARRED_EINVAL, "history length must be >= 1");
    starred_lbfgs *L = new starred_lbfgs();
    L->p = p;
    L->m = m;
    L->n = p->nparams;
    int rc = L->alloc(&L->gdev, (size_t)L->n);
    if (!rc) rc = L->alloc(&L->loss, 3);
    L->buf.resize(L->n);
    // bounds copied to the host once (FP32 values; +-inf or a NULL array: unbounded)
    auto copy_bound = [&](const float *src, std::vector<double> &dst, double inf) -> int {
        dst.assign(L->n, inf);
        if (!src) return STARRED_OK;
        HIP_TRY(hipMemcpy(L->buf.data(), src, sizeof(float) * L->n, hipMemcpyDeviceToHost));
        for (long long i = 0; i < L->n; ++i) dst[i] = (double)L->buf[i];
        return STARRED_OK;
    };
    if (!rc) rc = copy_bound(lo, L->lo, -HUGE_VAL);
    if (!rc) rc = copy_bound(hi, L->hi, HUGE_VAL);
    if (rc) {
        delete L;
        return rc;
    }
    *out = L;
    return STARRED_OK;
}

int starred_lbfgs_destroy(starred_lbfgs *L)
{
    if (!L) return fail(STARRED_EINVAL, "state is NULL");
    if (L->p && L->p->st) (void)hipStreamSynchronize(L->p->st);
    delete L;
    return STARRED_OK;
}

int starred_lbfgs_reset(starred_lbfgs *L)
{
    if (!L) return fail(STARRED_EINVAL, "state is NULL");
    if (L->core) (void)starred_lbfgsb_destroy(L->core);
    L->core = nullptr;
    L->started = L->done = false;
    return STARRED_OK;
}

int starred_lbfgs_run(starred_lbfgs *L, float *x, int32_t n_iter, double *loss_out, int32_t *n_evals_out)
{
    if (!L || !x) return fail(STARRED_EINVAL, "NULL argument");
    starred_plan *p = L->p;
    if (!p->frames_set) return fail(STARRED_ESTATE, "set_frames has not been called");
    const long long n = L->n;
    int evals = 0, rc;
    // the loss and gradient at the device vector x, into L->f and L->gh
    auto evaluate = [&]() -> int {
        int r = (p->mode == STARRED_PSF) ? psf_loss_grad_impl(p, x, L->gdev, L->loss)
                                         : loss_grad_impl(p, x, L->gdev, L->loss);
        if (r) return r;
        double h[3];
        HIP_TRY(hipMemcpyAsync(h, L->loss, sizeof(double) * 3, hipMemcpyDeviceToHost, p->st));
        HIP_TRY(hipMemcpyAsync(L->buf.data(), L->gdev, sizeof(float) * n, hipMemcpyDeviceToHost, p->st));
        HIP_TRY(hipStreamSynchronize(p->st));
        L->f = h[2];
        for (long long i = 0; i < n; ++i) L->gh[i] = (double)L->buf[i];
        ++evals;
        return STARRED_OK;
    };
    auto put_x = [&]() -> int {
        for (long long i = 0; i < n; ++i) L->buf[i] = (float)L->xh[i];
        HIP_TRY(hipMemcpyAsync(x, L->buf.data(), sizeof(float) * n, hipMemcpyHostToDevice, p->st));
        HIP_TRY(hipStreamSynchronize(p->st));
        return STARRED_OK;
    };
    if (!L->started) {
        L->xh.resize(n);
        L->gh.assign(n, 0.0);
        HIP_TRY(hipMemcpyAsync(L->buf.data(), x, sizeof(float) * n, hipMemcpyDeviceToHost, p->st));
        HIP_TRY(hipStreamSynchronize(p->st));
        for (long long i = 0; i < n; ++i) L->xh[i] = (double)L->buf[i];
        if ((rc = starred_lbfgsb_create(n, L->m, L->lo.data(), L->hi.data(), 1e7, 1e-5, 20, &L->core))) return rc;
        int32_t task = 0;
        if ((rc = starred_lbfgsb_iterate(L->core, L->xh.data(), 0.0, nullptr, &task))) return rc;
        L->task = task;  // FG at the projected start
        L->started = true;
        L->done = false;
    }
    int iters = 0;
    while (!L->done && iters < n_iter) {
        int32_t task = L->task;
        if (task == STARRED_LBFGSB_FG) {
            if ((rc = put_x())) return rc;
            if ((rc = evaluate())) return rc;
        }
        if ((rc = starred_lbfgsb_iterate(L->core, L->xh.data(), L->f, L->gh.data(), &task))) return rc;
        L->task = task;
        if (task == STARRED_LBFGSB_NEW_X) ++iters;
        if (task == STARRED_LBFGSB_CONVERGED || task == STARRED_LBFGSB_ABNORMAL) L->done = true;
    }
    // x holds the last iterate; after a failed search the iterate is the previous
    // point, whose loss is evaluated again
    if ((rc = put_x())) return rc;
    if (L->task == STARRED_LBFGSB_ABNORMAL && (rc = evaluate())) return rc;
    if (loss_out) *loss_out = L->f;
    if (n_evals_out) *n_evals_out = evals;
    return STARRED_OK;
}

int starred_time_stage(starred_plan *p, const float *params, int32_t stage, int32_t reps, double *ms_out)
{
    if (!p || !params || !ms_out) return fail(STARRED_EINVAL, "NULL argument");
    if (reps < 1) return fail(STARRED_EINVAL, "reps must be >= 1");
    if (p->mode != STARRED_DECONV) return fail(STARRED_EUNSUPPORTED, "stage timing needs deconvolution mode");
    if (!p->frames_set) return fail(STARRED_ESTATE, "set_frames has not been called");
    const bool fft = (p->algo == STARRED_CONV_FFT);
    const bool fused = fft && p->fft_fused && p->fd.n_fused > 0;
    int n_l1 = 0;
    auto launch = [&]() -> int {
        switch (stage) {
        case STARRED_STAGE_STARLET:
            return prior_launches(p, p->st, params, true, &n_l1);
        case STARRED_STAGE_SPECTRA:
            if (!fft) break;
            HIP_TRY(fft_spectra(p->st, p->fd, params, p->N, p->E, p->M, p->sigma));
            return STARRED_OK;
        case STARRED_STAGE_FFT_FUSED:
            if (!fft) break;
            HIP_TRY(fft_fused_fwd(p->st, p->fd, params, p->N, p->E, p->M, p->s, p->data, p->invvar,
                                  p->d_part_chi_fft + p->fd.frows_lg.n_items));
            return STARRED_OK;
        case STARRED_STAGE_FFT_SPEC:
            if (!fft) break;
            HIP_TRY(fft_spec_fwd(p->st, p->fd, params, p->N, p->E, p->M, p->s, fused));
            return STARRED_OK;
        case STARRED_STAGE_FFT_MCOLS:
            if (!fft) break;
            HIP_TRY(fused ? fft_model_cols_lg(p->st, p->fd) : fft_model_cols(p->st, p->fd));
            return STARRED_OK;
        case STARRED_STAGE_FFT_MROWS:
            if (!fft) break;
            HIP_TRY(fused ? fft_model_rows_lg(p->st, p->fd, p->data, p->invvar, p->d_part_chi_fft)
                          : fft_model_rows(p->st, p->fd, p->data, p->invvar, p->d_part_chi_fft, nullptr));
            return STARRED_OK;
        case STARRED_STAGE_FFT_RCOLS:
            if (!fft) break;
            HIP_TRY(fused ? fft_rho_cols_lg(p->st, p->fd) : fft_rho_cols(p->st, p->fd));
            return STARRED_OK;
        case STARRED_STAGE_FFT_ACOLS:
            if (!fft) break;
            HIP_TRY(fft_spec_adj(p->st, p->fd, p->M));
            return STARRED_OK;
        case STARRED_STAGE_FFT_FSUM:
            if (!fft) break;
            HIP_TRY(fft_adj_sums(p->st, p->fd, p->M, p->d_fsum));
            return STARRED_OK;
        case STARRED_STAGE_FFT_AROWS:
            if (!fft) break;
            HIP_TRY(fft_grad_h_inverse(p->st, p->fd));
            return STARRED_OK;
        // the direct stages over the frames of the direct classes
        case STARRED_STAGE_RENDER:
            if (p->fdir.empty()) break;
            HIP_TRY(launch_render(p->st, p->d_fr, p->E, p->Fdir, p->N, p->M, p->sigma, params, p->d_scene,
                                  p->d_fdir, (int)p->fdir.size(), p->xf));
            return STARRED_OK;
        case STARRED_STAGE_CONV_FWD:
        case STARRED_STAGE_DIRECT_FWD:
            if (p->fdir.empty()) break;
            if (p->xf && p->xf_fft) {
                HIP_TRY(fft_xf_forward(p->st, p->fd, p->d_scene, p->s, p->data, p->invvar, p->d_part_chi_fft));
                return STARRED_OK;
            }
            HIP_TRY(launch_fwd_direct(p->st, p->s, p->d_fr, p->d_fwd_items, (int)p->fwd_items.size(), p->Tdir,
                                      p->d_scene, p->d_kf, p->data, p->invvar, p->d_rho, p->d_part_chi_fft,
                                      p->fwd_groups));
            return STARRED_OK;
        case STARRED_STAGE_CONV_ADJ:
        case STARRED_STAGE_DIRECT_ADJ:
            if (p->fdir.empty()) break;
            if (p->xf && p->xf_fft) {
                HIP_TRY(fft_xf_adjoint(p->st, p->fd, p->d_g));
                return STARRED_OK;
            }
            HIP_TRY(launch_adj_direct(p->st, p->s, p->d_fr, p->d_adj_items, (int)p->adj_items.size(), p->Ardir,
                                      p->Bpdir, p->d_rho, p->d_ka, p->d_g, p->adj_groups));
            return STARRED_OK;
        case STARRED_STAGE_GRAD_SUMS:
            if (p->fdir.empty()) break;
            HIP_TRY(launch_frame_sums(p->st, p->d_fr, p->E, p->N, p->M, p->sigma, params, p->d_g, p->d_fsum, true,
                                      p->d_fdir, (int)p->fdir.size(), p->xf, p->gxf, p->d_gxfp));
            return STARRED_OK;
        default:
            break;
        }
        return fail(STARRED_EUNSUPPORTED, "stage cannot be timed alone with this plan's algorithm");
    };
    if (stage < 0 || stage >= STARRED_NUM_STAGES) return fail(STARRED_EINVAL, "unknown stage");
    const bool prof = p->prof_on;
    p->prof_on = false;
    int rc = STARRED_OK;
    double *loss = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    rc = dev_alloc(&loss, 3);
    if (!rc && hipEventCreate(&a) != hipSuccess) rc = fail(STARRED_EHIP, "hipEventCreate");
    if (!rc && hipEventCreate(&b) != hipSuccess) rc = fail(STARRED_EHIP, "hipEventCreate");
    if (!rc) rc = loss_grad_impl(p, params, p->d_grad, loss);
    if (!rc) rc = launch(); // rejects unsupported stages before any timing
    if (!rc) {
        hipError_t e = launch_idle(p->st, kProfIdleIters);
        if (e == hipSuccess) e = hipEventRecord(a, p->st);
        for (int r = 0; r < reps && e == hipSuccess && !rc; ++r) rc = launch();
        if (e == hipSuccess && !rc) e = hipEventRecord(b, p->st);
        if (e == hipSuccess && !rc) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess && !rc) e = hipEventElapsedTime(&ms, a, b);
        if (e != hipSuccess && !rc) rc = fail_hip(e, "stage timing");
        if (!rc) *ms_out = (double)ms / reps;
    }
    if (hipStreamSynchronize(p->st) != hipSuccess && !rc) rc = fail(STARRED_EHIP, "stage timing synchronisation");
    p->prof_on = prof;
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (loss) (void)hipFree(loss);
    return rc;
}

int starred_copy_probe(starred_plan *p, const float *src, float *dst, int64_t n)
{
    if (!p || !src || !dst || n < 0 || (n % 4)) return fail(STARRED_EINVAL, "bad copy probe arguments");
    HIP_TRY(launch_copy_probe(p->st, src, dst, n));
    return STARRED_OK;
}

int starred_set_profiling(starred_plan *p, int32_t enable)
{
    if (!p) return fail(STARRED_EINVAL, "plan is NULL");
    if (!enable) {
        int rc = p->prof_collect();
        p->prof_on = false;
        return rc;
    }
    p->prof_on = true;
    return STARRED_OK;
}

int starred_profile_read(starred_plan *p, double *ms_out, int64_t *count_out)
{
    if (!p) return fail(STARRED_EINVAL, "plan is NULL");
    int rc = p->prof_collect();
    if (rc) return rc;
    for (int i = 0; i < STARRED_NUM_STAGES; ++i) {
        if (ms_out) ms_out[i] = p->prof_ms[i];
        if (count_out) count_out[i] = p->prof_cnt[i];
        p->prof_ms[i] = 0.0;
        p->prof_cnt[i] = 0;
    }
    return STARRED_OK;
}

}  // extern "C"
