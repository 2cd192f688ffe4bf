// PSF-reconstruction mode (Sec. 2.1, Eqs. 2-7): narrow PSF s = m(eta_M) + b on
// an N x N grid; star k's model is m_k = D(s * a_k r_k), r_k the Gaussian of
// FWHM 2 fine px centred at c_k, D the s x s block sum.
//
// r = g(dx) g(dy) is separable, and D folds into the 1-D factors: with
// xb(q) = s q - floor(cx) - R - 1,
//   Gx[t] = sum_{b < s} g(b + floor(cx) + R + 1 - t - cx),   t < T = 2R + s + 2,
//   m_k(p, q) = a_k sum_t Gy[t] sum_u Gx[u] s(yb(p) + t, xb(q) + u),
// so each star is two banded passes over the grid (no dependence of the taps on
// p or q). Derivative taps dGx (the derivative of Gx with respect to cx) give
// the centre gradient. One work group per star; everything deterministic.
#include "starred_internal.h"
#include "starred_fft.h"

#include <hip/hip_runtime.h>

namespace starred {

constexpr int kPsfThreads = 256;
constexpr int kPsfMaxT = 2 * kGaussRadius + 3 + 2;  // s <= 3

// Moffat profile and its parameter derivatives at pixel (y, x). The profile's
// wings enter the chi-square multiplied by star amplitudes up to 1e6, so the
// transcendental part is evaluated in FP64 (N^2 evaluations per call) and rounded.
__device__ __forceinline__ void moffat_eval(const float *eta, int N, int y, int x, float &m, float d[5])
{
    const double A = eta[0], ax = eta[1], ay = eta[2], phi = eta[3], beta = eta[4];
    double sn, cs;
    sincos(phi, &sn, &cs);
    const double dx = (double)(x - N / 2), dy = (double)(y - N / 2);
    const double u = cs * dx + sn * dy;
    const double v = -sn * dx + cs * dy;
    const double qx = u / ax, qy = v / ay;
    const double Q = qx * qx + qy * qy;
    const double l1q = log1p(Q);
    const double base = exp(-beta * l1q);
    const double md = A * base;
    m = (float)md;
    if (d) {
        const double dQ = -beta * md / (1.0 + Q);
        d[0] = (float)base;
        d[1] = (float)(dQ * (-2.0 * u * u / (ax * ax * ax)));
        d[2] = (float)(dQ * (-2.0 * v * v / (ay * ay * ay)));
        d[3] = (float)(dQ * (2.0 * u * v * (1.0 / (ax * ax) - 1.0 / (ay * ay))));
        d[4] = (float)(-md * l1q);
    }
}

// s = m(eta_M) + b   (Eq. 2)
__global__ void k_psf_render(int N, const float *__restrict__ params, float *__restrict__ s_img)
{
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= N * N) return;
    float m;
    moffat_eval(params, N, pix / N, pix % N, m, nullptr);
    s_img[pix] = m + params[5 + pix];
}

hipError_t launch_psf_render(hipStream_t st, int N, const float *params, float *s_out)
{
    hipLaunchKernelGGL(k_psf_render, dim3((N * N + 255) / 256), dim3(256), 0, st, N, params, s_out);
    return hipGetLastError();
}

// Tap tables of one star: G[t] and its centre derivative dG[t].
__device__ __forceinline__ void psf_taps(float c, int s, float sigma, int T, float *G, float *dG)
{
    const float fc = floorf(c);
    const float inv2s2 = 1.0f / (2.0f * sigma * sigma), invs2 = 1.0f / (sigma * sigma);
    const float norm = 1.0f / (2.50662827463100050f * sigma);
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
        float g = 0.f, dg = 0.f;
        for (int b = 0; b < s; ++b) {
            const float arg = ((float)b + fc + (float)(kGaussRadius + 1 - t)) - c;
            const float e = norm * expf(-arg * arg * inv2s2);
            g += e;
            dg += e * arg * invs2;
        }
        G[t] = g;
        dG[t] = dg;
    }
}

// FP64 copy of the narrow PSF for the forward model: with star amplitudes up to
// 1e6 the chi-square near the truth is set by model errors far below an FP32
// ulp of the brightest pixels, so the (small) PSF-mode forward runs in FP64.
__global__ void k_psf_render64(int N, const float *__restrict__ params, double *__restrict__ s64)
{
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= N * N) return;
    const int y = pix / N, x = pix % N;
    const double A = params[0], ax = params[1], ay = params[2], phi = params[3], beta = params[4];
    double sn, cs;
    sincos(phi, &sn, &cs);
    const double dx = (double)(x - N / 2), dy = (double)(y - N / 2);
    const double u = cs * dx + sn * dy, v = -sn * dx + cs * dy;
    const double Q = (u / ax) * (u / ax) + (v / ay) * (v / ay);
    s64[pix] = A * exp(-beta * log1p(Q)) + (double)params[5 + pix];
}

hipError_t launch_psf_render64(hipStream_t st, int N, const float *params, double *s64)
{
    hipLaunchKernelGGL(k_psf_render64, dim3((N * N + 255) / 256), dim3(256), 0, st, N, params, s64);
    return hipGetLastError();
}

__device__ __forceinline__ void psf_taps64(double c, int s, double sigma, int T, double *G, double *dG)
{
    const double fc = floor(c);
    const double inv2s2 = 1.0 / (2.0 * sigma * sigma), invs2 = 1.0 / (sigma * sigma);
    const double norm = 1.0 / (2.5066282746310002 * sigma);
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
        double g = 0.0, dg = 0.0;
        for (int b = 0; b < s; ++b) {
            const double arg = ((double)b + fc + (double)(kGaussRadius + 1 - t)) - c;
            const double e = norm * exp(-arg * arg * inv2s2);
            g += e;
            dg += e * arg * invs2;
        }
        G[t] = g;
        dG[t] = dg;
    }
}

constexpr int kPsfRowChunk = 8;  // data rows per pass of the forward

// One work group per star: unit model u and centre derivatives ux, uy (FP64),
// residual rho = w (m - d) (stored FP32 for the adjoint), chi-square, and
// dchi/da, dchi/dc of the star. params = [eta 5 | b N^2 | a S | c 2S]
__global__ __launch_bounds__(kPsfThreads) void k_psf_fwd(
    int S, int n, int s, int N, float sigma, const float *__restrict__ params,
    const double *__restrict__ s64, const float *__restrict__ data, const float *__restrict__ invvar,
    float *__restrict__ rho, double *__restrict__ part_chi, float *__restrict__ grad)
{
    extern __shared__ double smd[];
    __shared__ double G[2][kPsfMaxT], dG[2][kPsfMaxT];
    __shared__ double red[kPsfThreads / 64];
    const int k = blockIdx.x;
    const long long NN = (long long)N * N;
    const double a = params[5 + NN + k];
    const double cx = params[5 + NN + S + 2 * k], cy = params[5 + NN + S + 2 * k + 1];
    const int T = 2 * kGaussRadius + s + 2;
    psf_taps64(cx, s, (double)sigma, T, G[0], dG[0]);
    psf_taps64(cy, s, (double)sigma, T, G[1], dG[1]);
    __syncthreads();
    const int fx = (int)floor(cx), fy = (int)floor(cy);
    const int rows = kPsfRowChunk * s + T;  // grid rows one chunk of data rows needs
    double *T1 = smd;
    double *T1x = smd + (long long)rows * n;
    double chi = 0.0, sa = 0.0, sx = 0.0, sy = 0.0;
    const long long doff = (long long)k * n * n;
    for (int p0 = 0; p0 < n; p0 += kPsfRowChunk) {
        const int y0 = s * p0 - fy - kGaussRadius - 1;  // grid row of T1 row 0
        __syncthreads();
        // T1(y', q) = sum_u Gx[u] s(y', xb(q) + u), T1x with dGx
        for (int e = threadIdx.x; e < rows * n; e += blockDim.x) {
            const int r = e / n, q = e - r * n;
            const int yp = y0 + r;
            double acc = 0.0, accx = 0.0;
            if (yp >= 0 && yp < N) {
                const int xb = s * q - fx - kGaussRadius - 1;
                const double *row = s64 + (long long)yp * N;
                for (int u = 0; u < T; ++u) {
                    const int xx = xb + u;
                    if (xx >= 0 && xx < N) {
                        const double v = row[xx];
                        acc = fma(G[0][u], v, acc);
                        accx = fma(dG[0][u], v, accx);
                    }
                }
            }
            T1[e] = acc;
            T1x[e] = accx;
        }
        __syncthreads();
        const int np = min(kPsfRowChunk, n - p0);
        for (int e = threadIdx.x; e < np * n; e += blockDim.x) {
            const int pl = e / n, q = e - pl * n;
            const int p = p0 + pl;
            const int rb = s * pl;  // T1 row of tap 0 for this data row
            double u = 0.0, ux = 0.0, uy = 0.0;
            for (int t = 0; t < T; ++t) {
                const double v = T1[(rb + t) * n + q];
                u = fma(G[1][t], v, u);
                uy = fma(dG[1][t], v, uy);
                ux = fma(G[1][t], T1x[(rb + t) * n + q], ux);
            }
            const long long idx = doff + (long long)p * n + q;
            const double r = a * u - (double)data[idx];
            const double w = invvar[idx];
            const double rh = w * r;
            rho[idx] = (float)rh;
            chi += 0.5 * w * r * r;
            sa += rh * u;
            sx += rh * ux;
            sy += rh * uy;
        }
    }
    chi = block_sum_d_fft(chi, red);
    sa = block_sum_d_fft(sa, red);
    sx = block_sum_d_fft(sx, red);
    sy = block_sum_d_fft(sy, red);
    if (threadIdx.x == 0) {
        if (part_chi) part_chi[k] = chi;
        if (grad) {
            grad[5 + NN + k] = (float)sa;
            grad[5 + NN + S + 2 * k] = (float)(a * sx);
            grad[5 + NN + S + 2 * k + 1] = (float)(a * sy);
        }
    }
}

// star models only (no data): m_k packed S x n^2
__global__ __launch_bounds__(kPsfThreads) void k_psf_model(int S, int n, int s, int N, float sigma,
                                                           const float *__restrict__ params,
                                                           const float *__restrict__ s_img,
                                                           float *__restrict__ model)
{
    extern __shared__ float sm[];
    __shared__ float G[2][kPsfMaxT], dG[2][kPsfMaxT];
    const int k = blockIdx.x;
    const long long NN = (long long)N * N;
    const float a = params[5 + NN + k];
    const float cx = params[5 + NN + S + 2 * k], cy = params[5 + NN + S + 2 * k + 1];
    const int T = 2 * kGaussRadius + s + 2;
    psf_taps(cx, s, sigma, T, G[0], dG[0]);
    psf_taps(cy, s, sigma, T, G[1], dG[1]);
    __syncthreads();
    const int fx = (int)floorf(cx), fy = (int)floorf(cy);
    float *T1 = sm;
    for (int e = threadIdx.x; e < N * n; e += blockDim.x) {
        const int yp = e / n, q = e - yp * n;
        const int xb = s * q - fx - kGaussRadius - 1;
        const float *row = s_img + (long long)yp * N;
        float acc = 0.f;
        for (int u = 0; u < T; ++u) {
            const int xx = xb + u;
            if (xx >= 0 && xx < N) acc = fmaf(G[0][u], row[xx], acc);
        }
        T1[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int p = e / n, q = e - p * n;
        const int yb = s * p - fy - kGaussRadius - 1;
        float u = 0.f;
        for (int t = 0; t < T; ++t) {
            const int yy = yb + t;
            if (yy >= 0 && yy < N) u = fmaf(G[1][t], T1[yy * n + q], u);
        }
        model[(long long)k * n * n + e] = a * u;
    }
}

// Adjoint of star k: gstar_k(y', x') = a_k sum_p Gy[t(p,y')] sum_q Gx[u(q,x')] rho_k(p, q),
// written per star (summed over stars, in star order, by k_psf_sum).
__global__ __launch_bounds__(kPsfThreads) void k_psf_adj(int S, int n, int s, int N, float sigma,
                                                         const float *__restrict__ params,
                                                         const float *__restrict__ rho,
                                                         float *__restrict__ gstar)
{
    extern __shared__ float sm[];
    __shared__ float G[2][kPsfMaxT], dG[2][kPsfMaxT];
    const int k = blockIdx.x;
    const long long NN = (long long)N * N;
    const float a = params[5 + NN + k];
    const float cx = params[5 + NN + S + 2 * k], cy = params[5 + NN + S + 2 * k + 1];
    const int T = 2 * kGaussRadius + s + 2;
    psf_taps(cx, s, sigma, T, G[0], dG[0]);
    psf_taps(cy, s, sigma, T, G[1], dG[1]);
    __syncthreads();
    const int fx = (int)floorf(cx), fy = (int)floorf(cy);
    const float *rk = rho + (long long)k * n * n;
    // U(p, x') = sum_q rho(p, q) Gx[x' - xb(q)]   (n rows x N columns)
    float *U = sm;
    for (int e = threadIdx.x; e < n * N; e += blockDim.x) {
        const int p = e / N, xp = e - p * N;
        float acc = 0.f;
        // q with 0 <= xp - (s q - fx - R - 1) < T
        const int base = xp + fx + kGaussRadius + 1;  // = s q + u
        int qhi = base / s;
        int qlo = (base - T + 1 + s - 1) / s;
        if (base - T + 1 < 0) qlo = 0;
        if (qhi > n - 1) qhi = n - 1;
        for (int q = max(qlo, 0); q <= qhi; ++q) {
            const int u = base - s * q;
            if (u >= 0 && u < T) acc = fmaf(G[0][u], rk[p * n + q], acc);
        }
        U[e] = acc;
    }
    __syncthreads();
    float *gk = gstar + (long long)k * NN;
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int yp = e / N, xp = e - yp * N;
        const int base = yp + fy + kGaussRadius + 1;
        int phi = base / s;
        int plo = (base - T + 1 + s - 1) / s;
        if (base - T + 1 < 0) plo = 0;
        if (phi > n - 1) phi = n - 1;
        float acc = 0.f;
        for (int p = max(plo, 0); p <= phi; ++p) {
            const int t = base - s * p;
            if (t >= 0 && t < T) acc = fmaf(G[1][t], U[p * N + xp], acc);
        }
        gk[e] = a * acc;
    }
}

// dchi/ds = sum over stars (in order); dchi/deta = sum_x dchi/ds(x) dm/deta(x);
// grad_b = dchi/ds + prior (the L1 gradient, Phi z).
constexpr int kPsfSumThreads = 256;
__global__ __launch_bounds__(kPsfSumThreads) void k_psf_sum(int S, int N, const float *__restrict__ params,
                                                            const float *__restrict__ gstar,
                                                            const float *__restrict__ prior,
                                                            float *__restrict__ grad,
                                                            double *__restrict__ part_eta)
{
    __shared__ double red[kPsfSumThreads / 64];
    const long long NN = (long long)N * N;
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    float de[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if (pix < NN) {
        float gs = 0.f;
        for (int k = 0; k < S; ++k) gs += gstar[(long long)k * NN + pix];
        float m;
        float d[5];
        moffat_eval(params, N, pix / N, pix % N, m, d);
        for (int e = 0; e < 5; ++e) de[e] = gs * d[e];
        grad[5 + pix] = gs + (prior ? prior[pix] : 0.f);
    }
    for (int e = 0; e < 5; ++e) {
        const double t = block_sum_d_fft((double)de[e], red);
        if (threadIdx.x == 0) part_eta[(long long)blockIdx.x * 5 + e] = t;
    }
}

__global__ __launch_bounds__(256) void k_psf_finalize_small(int S, int n_chi, const double *__restrict__ part_chi,
                                                            int n_l1, const double *__restrict__ part_l1,
                                                            int n_eta, const double *__restrict__ part_eta,
                                                            float *__restrict__ grad, double *__restrict__ loss,
                                                            int *__restrict__ tick)
{
    if (tick && threadIdx.x == 0) *tick += 1;  // the Adam step that follows reads it
    __shared__ double red[4];
    double a = 0.0;
    for (int i = threadIdx.x; i < n_chi; i += 256) a += part_chi[i];
    const double chi = block_sum_d_fft(a, red);
    double b = 0.0;
    for (int i = threadIdx.x; i < n_l1; i += 256) b += part_l1[i];
    const double l1 = block_sum_d_fft(b, red);
    if (threadIdx.x == 0 && loss) {
        loss[0] = chi;
        loss[1] = l1;
        loss[2] = chi + l1;
    }
    if (grad && threadIdx.x < 5) {
        double acc = 0.0;
        for (int i = 0; i < n_eta; ++i) acc += part_eta[(long long)i * 5 + threadIdx.x];
        grad[threadIdx.x] = (float)acc;
    }
}

size_t psf_fwd_lds(int n, int s) { return (size_t)2 * (kPsfRowChunk * s + 2 * kGaussRadius + s + 2) * n * sizeof(double); }
size_t psf_adj_lds(int n, int N) { return (size_t)n * N * sizeof(float); }

hipError_t launch_psf_fwd(hipStream_t st, int S, int n, int ss, int N, float sigma, const float *params,
                          const double *s64, const float *data, const float *invvar, float *rho,
                          double *part_chi, float *grad)
{
    hipLaunchKernelGGL(k_psf_fwd, dim3(S), dim3(kPsfThreads), psf_fwd_lds(n, ss), st, S, n, ss, N, sigma, params,
                       s64, data, invvar, rho, part_chi, grad);
    return hipGetLastError();
}

hipError_t launch_psf_model(hipStream_t st, int S, int n, int ss, int N, float sigma, const float *params,
                            const float *s_img, float *model)
{
    hipLaunchKernelGGL(k_psf_model, dim3(S), dim3(kPsfThreads), psf_adj_lds(n, N), st, S, n, ss, N, sigma,
                       params, s_img, model);
    return hipGetLastError();
}

hipError_t launch_psf_adj(hipStream_t st, int S, int n, int ss, int N, float sigma, const float *params,
                          const float *rho, float *gstar)
{
    hipLaunchKernelGGL(k_psf_adj, dim3(S), dim3(kPsfThreads), psf_adj_lds(n, N), st, S, n, ss, N, sigma, params,
                       rho, gstar);
    return hipGetLastError();
}

int psf_sum_blocks(int N) { return (N * N + kPsfSumThreads - 1) / kPsfSumThreads; }

hipError_t launch_psf_sum(hipStream_t st, int S, int N, const float *params, const float *gstar,
                          const float *prior, float *grad, double *part_eta)
{
    hipLaunchKernelGGL(k_psf_sum, dim3(psf_sum_blocks(N)), dim3(kPsfSumThreads), 0, st, S, N, params, gstar, prior,
                       grad, part_eta);
    return hipGetLastError();
}

hipError_t launch_psf_finalize_small(hipStream_t st, int S, int n_chi, const double *part_chi, int n_l1,
                                     const double *part_l1, int n_eta, const double *part_eta, float *grad,
                                     double *loss, int *tick)
{
    hipLaunchKernelGGL(k_psf_finalize_small, dim3(1), dim3(256), 0, st, S, n_chi, part_chi, n_l1, part_l1, n_eta,
                       part_eta, grad, loss, tick);
    return hipGetLastError();
}

}  // namespace starred
