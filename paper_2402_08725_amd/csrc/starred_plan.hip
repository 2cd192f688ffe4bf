// Host side of the C ABI (include/starred.h): plan validation, frame tables,
// work lists, scratch ownership and the launch sequences of loss_grad / step.
#include "starred.h"
#include "starred_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
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
    float *d_grad = nullptr;
    float *d_wzero = nullptr;
    std::vector<void *> owned;

    // stage timing
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_next = 0;
    struct Rec { int stage; hipEvent_t a, b; };
    std::vector<Rec> recs;
    double prof_ms[STARRED_NUM_STAGES] = {};
    long long prof_cnt[STARRED_NUM_STAGES] = {};

    hipEvent_t prof_start()
    {
        if (!prof_on) return nullptr;
        if (ev_next == ev_pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            ev_pool.push_back(e);
        }
        hipEvent_t e = ev_pool[ev_next++];
        (void)hipEventRecord(e, st);
        return e;
    }
    void prof_stop(int stage, hipEvent_t a)
    {
        if (!prof_on || !a) return;
        hipEvent_t b = prof_start();
        if (b) recs.push_back({stage, a, b});
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

    ~starred_plan()
    {
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        for (void *p : owned) (void)hipFree(p);
    }
    template <typename T>
    int alloc(T **p, size_t count)
    {
        int rc = dev_alloc(p, count);
        if (rc == STARRED_OK) owned.push_back((void *)*p);
        return rc;
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
    }
    return STARRED_OK;
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

    // Work lists: frame-major enumeration fixes the partial-result slots; the
    // launch order is longest-first (cost ~ folded kernel area) so that ragged
    // batches balance across the compute units.
    struct Cost { long long c; Item it; };
    std::vector<Cost> fw, ad;
    int slot = 0;
    for (int i = 0; i < E; ++i) {
        const FrameDev &f = p->fr[i];
        for (int p0 = 0; p0 < f.n; p0 += kFwdTP)
            for (int q0 = 0; q0 < f.n; q0 += kFwdTQ) {
                Item it{i, p0, q0, slot++};
                fw.push_back({(long long)f.Kp * s * f.Tpad, it});
            }
    }
    slot = 0;
    for (int i = 0; i < E; ++i) {
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

    int rc;
    if ((rc = p->alloc(&p->d_fr, E))) return rc;
    if ((rc = p->alloc(&p->d_fwd_items, p->fwd_items.size()))) return rc;
    if ((rc = p->alloc(&p->d_adj_items, p->adj_items.size()))) return rc;
    HIP_TRY(hipMemcpy(p->d_fr, p->fr.data(), sizeof(FrameDev) * E, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->d_fwd_items, p->fwd_items.data(), sizeof(Item) * p->fwd_items.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->d_adj_items, p->adj_items.data(), sizeof(Item) * p->adj_items.size(), hipMemcpyHostToDevice));

    const long long NN = (long long)p->N * p->N;
    const int nb_star = (int)((NN + 255) / 256);
    if ((rc = p->alloc(&p->d_kf, p->nkf))) return rc;
    if ((rc = p->alloc(&p->d_ka, p->nka))) return rc;
    if ((rc = p->alloc(&p->d_scene, p->nfine))) return rc;
    if ((rc = p->alloc(&p->d_rho, p->ndata))) return rc;
    if ((rc = p->alloc(&p->d_g, p->nfine))) return rc;
    if ((rc = p->alloc(&p->d_part_chi, p->fwd_items.size()))) return rc;
    if ((rc = p->alloc(&p->d_part_l1, (size_t)std::max(1, p->J - 1) * nb_star))) return rc;
    if ((rc = p->alloc(&p->d_fsum, (size_t)E * (1 + 3 * p->M)))) return rc;
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

int starred_plan_create(const starred_desc *desc, void *stream, starred_plan **plan_out)
{
    if (!plan_out) return fail(STARRED_EINVAL, "plan_out is NULL");
    *plan_out = nullptr;
    int rc = validate(desc);
    if (rc) return rc;
    if (desc->mode == STARRED_PSF) return fail(STARRED_EUNSUPPORTED, "PSF mode is not available in this build");
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
    p->n.assign(desc->side_host, desc->side_host + p->E);
    if (desc->ksize_host) p->K.assign(desc->ksize_host, desc->ksize_host + p->E);
    p->algo = (desc->conv_algo == STARRED_CONV_FFT) ? STARRED_CONV_FFT : STARRED_CONV_DIRECT;
    if (p->algo == STARRED_CONV_FFT) {
        delete p;
        return fail(STARRED_EUNSUPPORTED, "FFT convolution is not available in this build");
    }
    rc = build_deconv(p);
    if (rc) {
        delete p;
        return rc;
    }
    *plan_out = p;
    return STARRED_OK;
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

int starred_set_frames(starred_plan *p, const float *data, const float *inv_var, const float *psf,
                       const float *W)
{
    if (!p) return fail(STARRED_EINVAL, "plan is NULL");
    if (!data || !inv_var || !W) return fail(STARRED_EINVAL, "data, inv_var and W must be non-NULL");
    if (p->mode == STARRED_DECONV && !psf) return fail(STARRED_EINVAL, "psf kernels are required in deconvolution mode");
    p->data = data;
    p->invvar = inv_var;
    p->W = W;
    HIP_TRY(launch_prep_kernels(p->st, p->d_fr, p->fr.data(), p->E, p->s, psf, p->d_kf, p->d_ka));
    HIP_TRY(hipStreamSynchronize(p->st));
    p->frames_set = true;
    return STARRED_OK;
}

int starred_render_scene(starred_plan *p, const float *params, float *scene)
{
    if (!p || !params || !scene) return fail(STARRED_EINVAL, "NULL argument");
    HIP_TRY(launch_render(p->st, p->d_fr, p->E, p->Fmax, p->N, p->M, p->sigma, params, scene));
    return STARRED_OK;
}

int starred_convolve_subsample(starred_plan *p, const float *scene, float *model)
{
    if (!p || !scene || !model) return fail(STARRED_EINVAL, "NULL argument");
    if (!p->frames_set) return fail(STARRED_ESTATE, "set_frames has not been called");
    HIP_TRY(launch_fwd_direct(p->st, p->s, p->d_fr, p->d_fwd_items, (int)p->fwd_items.size(), p->Tmax,
                              scene, p->d_kf, nullptr, nullptr, model, nullptr));
    return STARRED_OK;
}

int starred_convolve_subsample_adj(starred_plan *p, const float *resid, float *grad_scene)
{
    if (!p || !resid || !grad_scene) return fail(STARRED_EINVAL, "NULL argument");
    if (!p->frames_set) return fail(STARRED_ESTATE, "set_frames has not been called");
    HIP_TRY(launch_adj_direct(p->st, p->s, p->d_fr, p->d_adj_items, (int)p->adj_items.size(), p->Ar_max,
                              p->Bpad_max, resid, p->d_ka, grad_scene));
    return STARRED_OK;
}

int starred_starlet_fwd(starred_plan *p, const float *img, float *coeffs)
{
    if (!p || !img || !coeffs) return fail(STARRED_EINVAL, "NULL argument");
    // the transform alone: zero weights, no L1 partials, no subgradient
    HIP_TRY(launch_starlet_fwd(p->st, p->N, p->J, img, coeffs, nullptr, p->d_wzero, 0, 0.f,
                               p->d_ca, p->d_cb, p->d_tmp, nullptr, nullptr));
    return STARRED_OK;
}

int starred_starlet_adj(starred_plan *p, const float *coeffs, float *img)
{
    if (!p || !coeffs || !img) return fail(STARRED_EINVAL, "NULL argument");
    HIP_TRY(launch_starlet_adj(p->st, p->N, p->J, coeffs, img, p->d_ca, p->d_cb, p->d_tmp));
    return STARRED_OK;
}

static int loss_grad_impl(starred_plan *p, const float *params, float *grad, double *loss_out)
{
    hipEvent_t e0 = p->prof_start();
    HIP_TRY(launch_render(p->st, p->d_fr, p->E, p->Fmax, p->N, p->M, p->sigma, params, p->d_scene));
    p->prof_stop(STARRED_STAGE_RENDER, e0);
    e0 = p->prof_start();
    HIP_TRY(launch_fwd_direct(p->st, p->s, p->d_fr, p->d_fwd_items, (int)p->fwd_items.size(), p->Tmax,
                              p->d_scene, p->d_kf, p->data, p->invvar, p->d_rho, p->d_part_chi));
    p->prof_stop(STARRED_STAGE_CONV_FWD, e0);
    int n_l1 = 0;
    e0 = p->prof_start();
    HIP_TRY(launch_starlet_fwd(p->st, p->N, p->J, params, nullptr, grad ? p->d_z : nullptr, p->W, p->w_stride,
                               (float)p->lam, p->d_ca, p->d_cb, p->d_tmp, p->d_part_l1, &n_l1));
    if (grad) HIP_TRY(launch_starlet_adj(p->st, p->N, p->J, p->d_z, p->d_prior, p->d_ca, p->d_cb, p->d_tmp));
    p->prof_stop(STARRED_STAGE_STARLET, e0);
    if (grad) {
        e0 = p->prof_start();
        HIP_TRY(launch_adj_direct(p->st, p->s, p->d_fr, p->d_adj_items, (int)p->adj_items.size(), p->Ar_max,
                                  p->Bpad_max, p->d_rho, p->d_ka, p->d_g));
        p->prof_stop(STARRED_STAGE_CONV_ADJ, e0);
        e0 = p->prof_start();
        HIP_TRY(launch_frame_sums(p->st, p->d_fr, p->E, p->N, p->M, p->sigma, params, p->d_g, p->d_fsum));
        p->prof_stop(STARRED_STAGE_GRAD_SUMS, e0);
    }
    e0 = p->prof_start();
    if (grad) HIP_TRY(launch_finalize_h(p->st, p->d_fr, p->E, p->N, p->d_g, p->d_prior, grad));
    HIP_TRY(launch_finalize_small(p->st, p->E, p->M, (int)p->fwd_items.size(), p->d_part_chi, n_l1,
                                  p->d_part_l1, p->lam, p->d_fsum, params, p->N, grad, loss_out));
    p->prof_stop(STARRED_STAGE_FINALIZE, e0);
    return STARRED_OK;
}

int starred_loss_grad(starred_plan *p, const float *params, float *grad, double *loss_out)
{
    if (!p || !params || !loss_out) return fail(STARRED_EINVAL, "NULL argument");
    if (!p->frames_set) return fail(STARRED_ESTATE, "set_frames has not been called");
    return loss_grad_impl(p, params, grad, loss_out);
}

int starred_step(starred_plan *p, float *params, float *m, float *v, int32_t t,
                 const starred_adam *hp, double *loss_out)
{
    if (!p || !params || !m || !v || !hp) return fail(STARRED_EINVAL, "NULL argument");
    if (t < 1) return fail(STARRED_EINVAL, "t must be >= 1");
    if (!p->frames_set) return fail(STARRED_ESTATE, "set_frames has not been called");
    int rc = loss_grad_impl(p, params, p->d_grad, loss_out);
    if (rc) return rc;
    const long long NN = (long long)p->N * p->N;
    long long seg[3] = {NN, NN + p->E, NN + p->E + (long long)p->E * p->M};
    hipEvent_t e0 = p->prof_start();
    HIP_TRY(launch_adam(p->st, p->nparams, seg, hp->lr, params, p->d_grad, m, v, t, hp->beta1, hp->beta2,
                        hp->eps));
    p->prof_stop(STARRED_STAGE_ADAM, e0);
    return STARRED_OK;
}

int starred_set_graph_mode(starred_plan *p, int32_t enable)
{
    if (!p) return fail(STARRED_EINVAL, "plan is NULL");
    if (enable) return fail(STARRED_EUNSUPPORTED, "graph mode is not available in this build");
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
