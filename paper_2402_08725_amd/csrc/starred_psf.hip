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

__device__ __forceinline__ void moffat_eval(const float *eta, int N, int y, int x, float &m, float d[5])
{
    const float A = eta[0], ax = eta[1], ay = eta[2], phi = eta[3], beta = eta[4];
    float sn, cs;
    sincosf(phi, &sn, &cs);
    const float dx = (float)(x - N / 2), dy = (float)(y - N / 2);
    const float u = cs * dx + sn * dy;
    const float v = -sn * dx + cs * dy;
    const float qx = u / ax, qy = v / ay;
    const float Q = qx * qx + qy * qy;
    const float l1q = log1pf(Q);
    const float base = expf(-beta * l1q);
    m = A * base;
    if (d) {
        const float dQ = -beta * m / (1.0f + Q);
        d[0] = base;
        d[1] = dQ * (-2.0f * u * u / (ax * ax * ax));
        d[2] = dQ * (-2.0f * v * v / (ay * ay * ay));
        d[3] = dQ * (2.0f * u * v * (1.0f / (ax * ax) - 1.0f / (ay * ay)));
        d[4] = -m * l1q;
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

// One work group per star: unit model u, centre derivatives ux, uy; model,
// residual rho = w (m - d), chi-square, and dchi/da, dchi/dc of the star.
// params = [eta 5 | b N^2 | a S | c 2S]
__global__ __launch_bounds__(kPsfThreads) void k_psf_fwd(
    int S, int n, int s, int N, float sigma, const float *__restrict__ params,
    const float *__restrict__ s_img, const float *__restrict__ data, const float *__restrict__ invvar,
    float *__restrict__ rho, double *__restrict__ part_chi, float *__restrict__ grad)
{
    extern __shared__ float sm[];
    __shared__ float G[2][kPsfMaxT], dG[2][kPsfMaxT];
    __shared__ double red[kPsfThreads / 64];
    const int k = blockIdx.x;
    const long long NN = (long long)N * N;
    const float a = params[5 + NN + k];
    const float cx = params[5 + NN + S + 2 * k], cy = params[5 + NN + S + 2 * k + 1];
    const int T = 2 * kGaussRadius + s + 2;
    psf_taps(cx, s, sigma, T, G[0], dG[0]);
    psf_taps(cy, s, sigma, T, G[1], dG[1]);
    __syncthreads();
    const int fx = (int)floorf(cx), fy = (int)floorf(cy);
    // T1(y', q) = sum_u Gx[u] s(y', xb(q) + u), T1x with dGx  (N rows x n columns each)
    float *T1 = sm;
    float *T1x = sm + (long long)N * n;
    for (int e = threadIdx.x; e < N * n; e += blockDim.x) {
        const int yp = e / n, q = e - yp * n;
        const int xb = s * q - fx - kGaussRadius - 1;
        const float *row = s_img + (long long)yp * N;
        float acc = 0.f, accx = 0.f;
        for (int u = 0; u < T; ++u) {
            const int xx = xb + u;
            if (xx >= 0 && xx < N) {
                const float v = row[xx];
                acc = fmaf(G[0][u], v, acc);
                accx = fmaf(dG[0][u], v, accx);
            }
        }
        T1[e] = acc;
        T1x[e] = accx;
    }
    __syncthreads();
    double chi = 0.0, sa = 0.0, sx = 0.0, sy = 0.0;
    const long long doff = (long long)k * n * n;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int p = e / n, q = e - p * n;
        const int yb = s * p - fy - kGaussRadius - 1;
        float u = 0.f, ux = 0.f, uy = 0.f;
        for (int t = 0; t < T; ++t) {
            const int yy = yb + t;
            if (yy >= 0 && yy < N) {
                const float v = T1[yy * n + q];
                u = fmaf(G[1][t], v, u);
                uy = fmaf(dG[1][t], v, uy);
                ux = fmaf(G[1][t], T1x[yy * n + q], ux);
            }
        }
        const float m = a * u;
        const float r = m - data[doff + e];
        const float w = invvar[doff + e];
        const float rh = w * r;
        rho[doff + e] = rh;
        chi += 0.5 * (double)w * (double)r * (double)r;
        sa += (double)(rh * u);
        sx += (double)(rh * ux);
        sy += (double)(rh * uy);
    }
    chi = block_sum_d_fft(chi, red);
    sa = block_sum_d_fft(sa, red);
    sx = block_sum_d_fft(sx, red);
    sy = block_sum_d_fft(sy, red);
    if (threadIdx.x == 0) {
        if (part_chi) part_chi[k] = chi;
        if (grad) {
            grad[5 + NN + k] = (float)sa;
            grad[5 + NN + S + 2 * k] = (float)((double)a * sx);
            grad[5 + NN + S + 2 * k + 1] = (float)((double)a * sy);
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
                                                            float *__restrict__ grad, double *__restrict__ loss)
{
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

size_t psf_fwd_lds(int n, int N) { return (size_t)2 * N * n * sizeof(float); }
size_t psf_adj_lds(int n, int N) { return (size_t)n * N * sizeof(float); }

hipError_t launch_psf_fwd(hipStream_t st, int S, int n, int ss, int N, float sigma, const float *params,
                          const float *s_img, const float *data, const float *invvar, float *rho,
                          double *part_chi, float *grad)
{
    hipLaunchKernelGGL(k_psf_fwd, dim3(S), dim3(kPsfThreads), psf_fwd_lds(n, N), st, S, n, ss, N, sigma, params,
                       s_img, data, invvar, rho, part_chi, grad);
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
                                     double *loss)
{
    hipLaunchKernelGGL(k_psf_finalize_small, dim3(1), dim3(256), 0, st, S, n_chi, part_chi, n_l1, part_l1, n_eta,
                       part_eta, grad, loss);
    return hipGetLastError();
}

}  // namespace starred
