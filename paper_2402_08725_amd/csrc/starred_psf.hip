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
// the centre gradient. The forward runs one work group per (data tile, star),
// the adjoint one per grid tile with every star summed inside it, so a few tens
// of stars still fill the chip; every reduction runs in a fixed order.
#include "starred_internal.h"
#include "starred_fft.h"

#include <hip/hip_runtime.h>

namespace starred {

constexpr int kPsfThreads = 256;
constexpr int kPsfMaxT = 2 * kGaussRadius + 3 + 2;  // s <= 3

// Deterministic block sums of NV doubles per thread (NT threads) with one barrier:
// each wave's butterfly, then thread 0 adds the waves in order (v holds the sums there).
template <int NT, int NV>
__device__ __forceinline__ void block_sum_vec(double (&v)[NV], double (*sh)[NV])
{
#pragma unroll
    for (int j = 0; j < NV; ++j) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[j] += __shfl_xor(v[j], off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) sh[threadIdx.x >> 6][j] = v[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double r = 0.0;
#pragma unroll
            for (int i = 0; i < NT / 64; ++i) r += sh[i][j];
            v[j] = r;
        }
    }
}

// Moffat profile and its parameter derivatives at pixel (y, x). The profile's
// wings enter the chi-square multiplied by star amplitudes up to 1e6, so the
// transcendental part is evaluated in FP64 (N^2 evaluations per call) and rounded.
__device__ __forceinline__ void moffat_eval(const float *eta, int N, int y, int x, double &m, float d[5])
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
    m = md;
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
    double m;
    moffat_eval(params, N, pix / N, pix % N, m, nullptr);
    s_img[pix] = (float)m + params[5 + pix];
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
// dm (or null): the Moffat derivatives dm/deta per pixel, [5][N^2], for the adjoint.
// tick (or null): the step counter, advanced here (the step's first launch) for the
// update at its end.
__global__ void k_psf_render64(int N, const float *__restrict__ params, double *__restrict__ s64,
                               float *__restrict__ dm, int *__restrict__ tick)
{
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    const long long NN = (long long)N * N;
    if (pix >= NN) return;
    if (tick && pix == 0) *tick += 1;
    double m;
    float d[5];
    moffat_eval(params, N, pix / N, pix % N, m, d);
    s64[pix] = m + (double)params[5 + pix];
    if (dm) {
#pragma unroll
        for (int e = 0; e < 5; ++e) dm[e * NN + pix] = d[e];
    }
}

hipError_t launch_psf_render64(hipStream_t st, int N, const float *params, double *s64, float *dm, int *tick)
{
    hipLaunchKernelGGL(k_psf_render64, dim3((N * N + 255) / 256), dim3(256), 0, st, N, params, s64, dm, tick);
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

constexpr int kPsfRowChunk = 8;   // data rows of one forward tile
constexpr int kPsfColTile = 32;   // data columns of one forward tile
static_assert(kPsfRowChunk * kPsfColTile == kPsfThreads, "one thread per data pixel of a forward tile");

int psf_fwd_tiles(int n) { return ((n + kPsfRowChunk - 1) / kPsfRowChunk) * ((n + kPsfColTile - 1) / kPsfColTile); }

// Grid window one forward tile reads: rows x columns
template <int SS> struct PsfFwdWin {
    static constexpr int T = 2 * kGaussRadius + SS + 2;
    static constexpr int RM = SS * (kPsfRowChunk - 1) + T;
    static constexpr int CM = SS * (kPsfColTile - 1) + T;
    static_assert(CM <= 128, "the window's columns map onto 128 lanes");
    static constexpr size_t lds = ((size_t)RM * CM + 2 * (size_t)RM * kPsfColTile) * sizeof(double);
};

// LDS of one forward tile: the grid window it reads (FP64) and its two x-pass planes
size_t psf_fwd_lds(int s)
{
    return s == 1 ? PsfFwdWin<1>::lds : s == 2 ? PsfFwdWin<2>::lds : PsfFwdWin<3>::lds;
}

// One work group per (8-row x 32-column data tile, star): unit model u and centre
// derivatives ux, uy (FP64), residual rho = w (m - d) (stored FP32 for the
// adjoint), and the tile's chi-square, dchi/da and the two sums dchi/dc needs
// (divided by a_k), as four FP64 partials in part[(k * tiles + tile) * 4 ..].
// params = [eta 5 | b N^2 | a S | c 2S]
template <int SS>
__global__ __launch_bounds__(kPsfThreads) void k_psf_fwd(
    int S, int n, int N, float sigma, const float *__restrict__ params,
    const double *__restrict__ s64, const float *__restrict__ data, const float *__restrict__ invvar,
    float *__restrict__ rho, double *__restrict__ part, float *__restrict__ model)
{
    using Win = PsfFwdWin<SS>;
    constexpr int T = Win::T, RM = Win::RM, CM = Win::CM, QT = kPsfColTile;
    extern __shared__ double smd[];
    __shared__ double G[2][kPsfMaxT], dG[2][kPsfMaxT];
    __shared__ double red[kPsfThreads / 64][4];
    const int k = blockIdx.z;
    const long long NN = (long long)N * N;
    const int p0 = blockIdx.x * kPsfRowChunk, q0 = blockIdx.y * QT;
    // this thread's data pixel, loaded first: it does not depend on the star's centre
    const int pl = threadIdx.x / QT, ql = threadIdx.x % QT;
    const bool own = p0 + pl < n && q0 + ql < n;
    const long long idx = (long long)k * n * n + (long long)(p0 + pl) * n + q0 + ql;
    // (model != null: the star models alone, m_k = a_k u, no data)
    const bool fit = own && !model;
    const double dat = fit ? (double)data[idx] : 0.0, wgt = fit ? (double)invvar[idx] : 0.0;
    const double a = params[5 + NN + k];
    const double cx = params[5 + NN + S + 2 * k], cy = params[5 + NN + S + 2 * k + 1];
    const int fx = (int)floor(cx), fy = (int)floor(cy);
    const int y0 = SS * p0 - fy - kGaussRadius - 1;  // grid row of window row 0
    const int x0 = SS * q0 - fx - kGaussRadius - 1;  // grid column of window column 0
    double *W = smd;              // RM x CM window of s, zero off the grid
    double *T1 = W + RM * CM;     // T1(y', q) = sum_u Gx[u] s(y', xb(q) + u): RM x 32
    double *T1x = T1 + RM * QT;   // the same with dGx
    // the window, two rows per pass of the work group, every load of a thread in
    // flight at once (and in flight while the taps are computed)
    const int wc = threadIdx.x & 127, wr = threadIdx.x >> 7;
    constexpr int NR = (RM + 1) / 2;
    double win[NR];
    {
        const int xx = x0 + wc;
        const bool cin = wc < CM && xx >= 0 && xx < N;
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const int yy = y0 + wr + 2 * i;
            win[i] = (cin && wr + 2 * i < RM && yy >= 0 && yy < N) ? s64[(long long)yy * N + xx] : 0.0;
        }
    }
    psf_taps64(cx, SS, (double)sigma, T, G[0], dG[0]);
    psf_taps64(cy, SS, (double)sigma, T, G[1], dG[1]);
#pragma unroll
    for (int i = 0; i < NR; ++i)
        if (wc < CM && wr + 2 * i < RM) W[(wr + 2 * i) * CM + wc] = win[i];
    __syncthreads();
    {
        // four consecutive outputs of a window row per thread: together they read
        // 3s + T window values, each loaded once for every output its taps reach
        // (rather than 4T loads); each output still adds its taps in order
        constexpr int QB = 4, NW = SS * (QB - 1) + T, NG = QT / QB;
        for (int task = threadIdx.x; task < RM * NG; task += kPsfThreads) {
            const int r = task / NG, q0 = (task % NG) * QB;
            const double *w = W + r * CM + SS * q0;
            double acc[QB], accx[QB];
#pragma unroll
            for (int i = 0; i < QB; ++i) acc[i] = accx[i] = 0.0;
#pragma unroll
            for (int j = 0; j < NW; ++j) {
                const double v = w[j];
#pragma unroll
                for (int i = 0; i < QB; ++i) {
                    const int u = j - SS * i;
                    if (u >= 0 && u < T) {
                        acc[i] = fma(G[0][u], v, acc[i]);
                        accx[i] = fma(dG[0][u], v, accx[i]);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < QB; ++i) {
                T1[r * QT + q0 + i] = acc[i];
                T1x[r * QT + q0 + i] = accx[i];
            }
        }
    }
    __syncthreads();
    double sums[4] = {0.0, 0.0, 0.0, 0.0};  // chi-square, then rho u, rho ux, rho uy
    if (own) {
        const int rb = SS * pl;  // window row of tap 0 for this data row
        double u = 0.0, ux = 0.0, uy = 0.0;
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const double v = T1[(rb + t) * QT + ql];
            u = fma(G[1][t], v, u);
            uy = fma(dG[1][t], v, uy);
            ux = fma(G[1][t], T1x[(rb + t) * QT + ql], ux);
        }
        if (model) {
            model[idx] = (float)(a * u);
        } else {
            const double r = a * u - dat;
            const double rh = wgt * r;
            rho[idx] = (float)rh;
            sums[0] = 0.5 * wgt * r * r;
            sums[1] = rh * u;
            sums[2] = rh * ux;
            sums[3] = rh * uy;
        }
    }
    block_sum_vec<kPsfThreads, 4>(sums, red);
    if (threadIdx.x == 0 && part) {
        double *o = part + ((long long)k * gridDim.x * gridDim.y + (long long)blockIdx.y * gridDim.x + blockIdx.x) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) o[j] = sums[j];
    }
}

// Adjoint, summed over stars: dchi/ds(y', x') = sum_k a_k sum_p Gy_k[t(p,y')]
// sum_q Gx_k[u(q,x')] rho_k(p, q), with t = y' + floor(cy_k) + R + 1 - s p and
// u likewise. One work group per 8 x 16 tile of the grid; stars are taken in
// batches: the batch's residual windows and taps go to LDS, then
// U_k(p, x') = sum_q Gx_k[u] rho_k(p, q) for the window's rows, then each of four
// thread groups adds a contiguous quarter of the batch's stars per pixel, in star
// order, and the four sums are added in group order. The pixel then writes grad_b = dchi/ds
// (the prior's L1 gradient Phi z is added after the starlet branch joins) and its share of dchi/deta = sum_x dchi/ds(x)
// dm/deta(x), one block partial per tile (five values).
constexpr int kPsfAdjTy = 8, kPsfAdjTx = 16, kPsfAdjPix = kPsfAdjTy * kPsfAdjTx;
constexpr int kPsfAdjGroups = 4;  // thread groups of a tile, each adding a quarter of the batch's stars
constexpr int kPsfAdjThreads = kPsfAdjGroups * kPsfAdjPix;
constexpr size_t kPsfAdjLds = 48 * 1024;

template <int SS> struct PsfAdjWin {
    static constexpr int T = 2 * kGaussRadius + SS + 2;
    static constexpr int PR = (kPsfAdjTy + T - 2) / SS + 1;  // residual rows one tile reads
    static constexpr int QC = (kPsfAdjTx + T - 2) / SS + 1;  // residual columns
    static constexpr int KT = (T - 1) / SS + 1;               // taps per output, at most
    // per star: window, U rows, taps (x then y), four ints, a_k and c_k
    static constexpr size_t per_star = ((size_t)PR * QC + (size_t)PR * kPsfAdjTx + 2 * T + 7) * sizeof(float);
};

static size_t psf_adj_per_star(int s)
{
    return s == 1 ? PsfAdjWin<1>::per_star : s == 2 ? PsfAdjWin<2>::per_star : PsfAdjWin<3>::per_star;
}

static int psf_adj_batch(int s, int S)
{
    return (int)std::max<size_t>(1, std::min<size_t>((size_t)S, kPsfAdjLds / psf_adj_per_star(s)));
}

int psf_adj_tiles(int N) { return ((N + kPsfAdjTx - 1) / kPsfAdjTx) * ((N + kPsfAdjTy - 1) / kPsfAdjTy); }

// floor(a / b) for b > 0
__device__ __forceinline__ int psf_fdiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

template <int SS>
__global__ __launch_bounds__(kPsfAdjThreads) void k_psf_adjsum(int S, int n, int N, float sigma, int kb,
                                                               const float *__restrict__ params,
                                                               const float *__restrict__ rho,
                                                               const float *__restrict__ dm,
                                                               float *__restrict__ grad,
                                                               double *__restrict__ part_eta)
{
    using Win = PsfAdjWin<SS>;
    constexpr int T = Win::T, PR = Win::PR, QC = Win::QC, KT = Win::KT, TX = kPsfAdjTx;
    extern __shared__ float sm[];
    __shared__ double red[kPsfAdjThreads / 64][5];
    int *sp = (int *)sm;                    // per star: first residual row, first column, floor(cx), floor(cy)
    float *sa = sm + 4 * kb;                // a_k
    float *sc = sa + kb;                    // c_k: [kb][2]
    float *Gt = sc + 2 * kb;                // taps: [kb][2][T] (x, then y)
    float *Rt = Gt + 2 * kb * T;            // residual windows [kb][PR][QC]
    float *U = Rt + (size_t)kb * PR * QC;   // [kb][PR][TX]
    const long long NN = (long long)N * N;
    const int X0 = blockIdx.x * TX, Y0 = blockIdx.y * kPsfAdjTy;
    const int pix_l = threadIdx.x % kPsfAdjPix, grp = threadIdx.x / kPsfAdjPix;
    const int xl = pix_l % TX, yl = pix_l / TX;
    const int xp = X0 + xl, yp = Y0 + yl;
    const bool own = grp == 0 && xp < N && yp < N;
    // this pixel's Moffat derivatives dm/deta, loaded first (used at the end)
    float dmp[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if (own) {
#pragma unroll
        for (int e = 0; e < 5; ++e) dmp[e] = dm[e * NN + (long long)yp * N + xp];
    }
    const float fc_norm = 1.0f / (2.50662827463100050f * sigma);
    const float inv2s2 = 1.0f / (2.0f * sigma * sigma);
    constexpr int R1 = kGaussRadius + 1;
    float gs = 0.f;
    for (int k0 = 0; k0 < S; k0 += kb) {
        const int nk = min(kb, S - k0);
        __syncthreads();  // the previous batch is done with the LDS
        // per (star, direction): c, floor(c) and the first residual row (column), by the
        // last threads (the first group's are loading their pixel's derivatives)
        for (int j = kPsfAdjThreads - 1 - threadIdx.x; j < 2 * nk; j += kPsfAdjThreads) {
            const int kk = j >> 1, dir = j & 1, k = k0 + kk;
            const float c = params[5 + NN + S + 2 * k + dir];
            const int f = (int)floorf(c);
            // rows p (columns q) with 0 <= y' + f + R + 1 - s p < T for some y' (x') of the tile
            sp[4 * kk + 1 - dir] = -psf_fdiv(-((dir ? Y0 : X0) + f + R1 - T + 1), SS);
            sp[4 * kk + 2 + dir] = f;
            sc[j] = c;
            if (dir == 0) sa[kk] = params[5 + NN + k];
        }
        __syncthreads();
        // taps G[t] = sum_{b < s} g(b + floor(c) + R + 1 - t - c) and the residual
        // windows, sixteen loads of a thread in flight at once
        for (int e = threadIdx.x; e < nk * 2 * T; e += kPsfAdjThreads) {
            const int j = e / T, t = e - j * T;
            const float c = sc[j];
            const float fc = floorf(c);
            float g = 0.f;
#pragma unroll
            for (int b = 0; b < SS; ++b) {
                const float arg = ((float)b + fc + (float)(R1 - t)) - c;
                g += fc_norm * expf(-arg * arg * inv2s2);
            }
            Gt[e] = g;
        }
        {
            const int tot = nk * PR * QC;
            for (int e0 = threadIdx.x; e0 < tot; e0 += 16 * kPsfAdjThreads) {
                float v[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int e = e0 + j * kPsfAdjThreads;
                    const int kk = e / (PR * QC), r = e - kk * (PR * QC), i = r / QC, c = r - i * QC;
                    const int pp = e < tot ? sp[4 * kk] + i : -1, qq = e < tot ? sp[4 * kk + 1] + c : -1;
                    v[j] = (pp >= 0 && pp < n && qq >= 0 && qq < n)
                               ? rho[(long long)(k0 + kk) * n * n + (long long)pp * n + qq]
                               : 0.f;
                }
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    if (e0 + j * kPsfAdjThreads < tot) Rt[e0 + j * kPsfAdjThreads] = v[j];
            }
        }
        __syncthreads();
        // U_k(p, x') over the tile's columns, one thread per (star, column) for all the
        // window's rows: q ascending from the first that reaches x'. Taps past the
        // last q are zero and read a clamped (finite) residual.
        for (int e = threadIdx.x; e < nk * TX; e += kPsfAdjThreads) {
            const int kk = e / TX, xc = e - kk * TX;
            const int base = X0 + xc + sp[4 * kk + 2] + R1;  // = s q + u
            const int qa = -psf_fdiv(-(base - T + 1), SS);
            const int u0 = base - SS * qa;                   // tap of q = qa, < T
            const int j0 = qa - sp[4 * kk + 1];               // window column of q = qa, >= 0
            const float *g = Gt + kk * 2 * T;
            float gj[KT];
            int jc[KT];
#pragma unroll
            for (int jj = 0; jj < KT; ++jj) {
                const int u = u0 - SS * jj;
                gj[jj] = u >= 0 ? g[max(u, 0)] : 0.f;
                jc[jj] = min(j0 + jj, QC - 1);
            }
            const float *rr = Rt + (size_t)kk * PR * QC;
            float *uo = U + (size_t)kk * PR * TX + xc;
#pragma unroll
            for (int i = 0; i < PR; ++i) {
                float acc = 0.f;
#pragma unroll
                for (int jj = 0; jj < KT; ++jj) acc = fmaf(gj[jj], rr[i * QC + jc[jj]], acc);
                uo[i * TX] = acc;
            }
        }
        __syncthreads();
        const int base_y = yp + R1;
        const int qk = (nk + kPsfAdjGroups - 1) / kPsfAdjGroups;
        const int kk_end = min(nk, (grp + 1) * qk);
#pragma unroll 2
        for (int kk = grp * qk; kk < kk_end; ++kk) {
            const int by = base_y + sp[4 * kk + 3];
            const int pa = -psf_fdiv(-(by - T + 1), SS);
            const int t0 = by - SS * pa;       // tap of p = pa, < T
            const int i0 = pa - sp[4 * kk];    // window row of p = pa, >= 0
            const float *g = Gt + kk * 2 * T + T;
            const float *uu = U + (size_t)kk * PR * TX + xl;
            float acc = 0.f;
#pragma unroll
            for (int ii = 0; ii < KT; ++ii) {
                const int t = t0 - SS * ii;
                acc = fmaf(t >= 0 ? g[max(t, 0)] : 0.f, uu[min(i0 + ii, PR - 1) * TX], acc);
            }
            gs += sa[kk] * acc;
        }
    }
    __shared__ float gsum[kPsfAdjGroups][kPsfAdjPix];
    gsum[grp][pix_l] = gs;
    __syncthreads();
    double de[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (own) {
        gs = gsum[0][pix_l];
#pragma unroll
        for (int g = 1; g < kPsfAdjGroups; ++g) gs += gsum[g][pix_l];
#pragma unroll
        for (int e = 0; e < 5; ++e) de[e] = (double)(gs * dmp[e]);
        grad[5 + (long long)yp * N + xp] = gs;
    }
    block_sum_vec<kPsfAdjThreads, 5>(de, red);
    if (threadIdx.x == 0) {
        const long long tile = (long long)blockIdx.y * gridDim.x + blockIdx.x;
#pragma unroll
        for (int e = 0; e < 5; ++e) part_eta[tile * 5 + e] = de[e];
    }
}

size_t psf_adj_lds(int s, int S) { return psf_adj_per_star(s) * psf_adj_batch(s, S); }

// Completion of the loss and gradient once the starlet branch has joined, and (ad.params
// non-null) the optimiser update of every parameter. Work group 0: the chi-square over
// every forward tile and the L1 partials, dchi/da_k and dchi/dc_k = a_k sum rho du/dc
// from the star's tiles, dchi/deta from the adjoint tiles (every sum a fixed-order
// strided pass and a fixed-order reduction), then the update of eta, a and c. Work
// groups 1..: grad_b = dchi/ds + the prior's gradient, per pixel, and its update.
__global__ __launch_bounds__(256) void k_psf_finalize(int S, int N, int tiles, const double *__restrict__ part,
                                                      int n_l1, const double *__restrict__ part_l1,
                                                      int n_eta, const double *__restrict__ part_eta,
                                                      const float *params,  // updated through ad.params
                                                      const float *__restrict__ prior,
                                                      float *__restrict__ grad, double *__restrict__ loss,
                                                      AdamDev ad)
{
    if (blockIdx.x > 0) {
        const long long NN = (long long)N * N;
        const long long i = (long long)(blockIdx.x - 1) * blockDim.x + threadIdx.x;
        if (!grad || i >= NN) return;
        const float g = grad[5 + i] + (prior ? prior[i] : 0.f);
        grad[5 + i] = g;
        if (ad.params) {
            const float t = (float)(*ad.d_t);
            const float bc1 = 1.f - powf(ad.beta1, t), bc2 = 1.f - powf(ad.beta2, t);
            float pi = ad.params[5 + i], mi = ad.m[5 + i], vi = ad.v[5 + i];
            adam_update(pi, mi, vi, g, ad.lr[1], ad.beta1, ad.beta2, bc1, bc2, ad.eps, ad.rule == 1, ad.eps_root);
            ad.m[5 + i] = mi;
            ad.v[5 + i] = vi;
            ad.params[5 + i] = pi;
        }
        return;
    }
    const long long NN = (long long)N * N;
    if (grad) {
        // eight lanes per star: lane l adds tiles l, l + 8, ... in order, then a
        // butterfly over the eight lanes (lane 0's order fixed)
        for (int k0 = 0; k0 < S; k0 += 32) {
            const int k = k0 + (threadIdx.x >> 3), l = threadIdx.x & 7;
            double sa = 0.0, sx = 0.0, sy = 0.0;
            if (k < S) {
                const double *o = part + (long long)k * tiles * 4;
#pragma unroll 4
                for (int t = l; t < tiles; t += 8) {
                    sa += o[4 * t + 1];
                    sx += o[4 * t + 2];
                    sy += o[4 * t + 3];
                }
            }
#pragma unroll
            for (int off = 4; off > 0; off >>= 1) {
                sa += __shfl_xor(sa, off, 64);
                sx += __shfl_xor(sx, off, 64);
                sy += __shfl_xor(sy, off, 64);
            }
            if (k < S && l == 0) {
                const double ak = params[5 + NN + k];
                grad[5 + NN + k] = (float)sa;
                grad[5 + NN + S + 2 * k] = (float)(ak * sx);
                grad[5 + NN + S + 2 * k + 1] = (float)(ak * sy);
            }
        }
    }
    // chi-square, L1 and the five dchi/deta sums: strided per-thread sums, then one
    // fixed-order reduction of all seven
    double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const long long n_chi = (long long)S * tiles;
#pragma unroll 4
    for (long long i = threadIdx.x; i < n_chi; i += 256) v[0] += part[i * 4];
#pragma unroll 4
    for (int i = threadIdx.x; i < n_l1; i += 256) v[1] += part_l1[i];
    if (grad) {
#pragma unroll 2
        for (int i = threadIdx.x; i < n_eta; i += 256)
#pragma unroll
            for (int e = 0; e < 5; ++e) v[2 + e] += part_eta[(long long)i * 5 + e];
    }
    __shared__ double red[4][7];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[j] += __shfl_xor(v[j], off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int j = 0; j < 7; ++j) red[threadIdx.x >> 6][j] = v[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r[7];
#pragma unroll
        for (int j = 0; j < 7; ++j) r[j] = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
        if (loss) {
            loss[0] = r[0];
            loss[1] = r[1];
            loss[2] = r[0] + r[1];
        }
        if (grad) {
#pragma unroll
            for (int e = 0; e < 5; ++e) grad[e] = (float)r[2 + e];
        }
    }
    if (!grad || !ad.params) return;
    // eta, a and c: their gradients are final (written above by this group); the a
    // values read for dchi/dc were taken before the reduction's barrier
    __syncthreads();
    const float t = (float)(*ad.d_t);
    const float bc1 = 1.f - powf(ad.beta1, t), bc2 = 1.f - powf(ad.beta2, t);
    for (long long e = threadIdx.x; e < 5 + 3LL * S; e += blockDim.x) {
        const long long i = e < 5 ? e : NN + e;  // past the b block
        const float lr = i < 5 ? ad.lr[0] : (i < 5 + NN + S ? ad.lr[2] : ad.lr[3]);
        float pi = ad.params[i], mi = ad.m[i], vi = ad.v[i];
        adam_update(pi, mi, vi, grad[i], lr, ad.beta1, ad.beta2, bc1, bc2, ad.eps, ad.rule == 1, ad.eps_root);
        ad.m[i] = mi;
        ad.v[i] = vi;
        ad.params[i] = pi;
    }
}

hipError_t launch_psf_fwd(hipStream_t st, int S, int n, int ss, int N, float sigma, const float *params,
                          const double *s64, const float *data, const float *invvar, float *rho, double *part,
                          float *model)
{
    const dim3 grid((n + kPsfRowChunk - 1) / kPsfRowChunk, (n + kPsfColTile - 1) / kPsfColTile, S);
    auto kern = ss == 1 ? k_psf_fwd<1> : ss == 2 ? k_psf_fwd<2> : k_psf_fwd<3>;
    hipLaunchKernelGGL(kern, grid, dim3(kPsfThreads), psf_fwd_lds(ss), st, S, n, N, sigma, params, s64, data, invvar,
                       rho, part, model);
    return hipGetLastError();
}

hipError_t launch_psf_adjsum(hipStream_t st, int S, int n, int ss, int N, float sigma, const float *params,
                             const float *rho, const float *dm, float *grad, double *part_eta)
{
    const int kb = psf_adj_batch(ss, S);
    const dim3 grid((N + kPsfAdjTx - 1) / kPsfAdjTx, (N + kPsfAdjTy - 1) / kPsfAdjTy);
    auto kern = ss == 1 ? k_psf_adjsum<1> : ss == 2 ? k_psf_adjsum<2> : k_psf_adjsum<3>;
    hipLaunchKernelGGL(kern, grid, dim3(kPsfAdjThreads), psf_adj_per_star(ss) * kb, st, S, n, N, sigma, kb, params,
                       rho, dm, grad, part_eta);
    return hipGetLastError();
}

hipError_t launch_psf_finalize(hipStream_t st, int S, int N, int tiles, const double *part, int n_l1,
                               const double *part_l1, int n_eta, const double *part_eta, const float *params,
                               const float *prior, float *grad, double *loss, const AdamDev &adam)
{
    const long long NN = (long long)N * N;
    const unsigned groups = grad ? 1 + (unsigned)((NN + 255) / 256) : 1;
    hipLaunchKernelGGL(k_psf_finalize, dim3(groups), dim3(256), 0, st, S, N, tiles, part, n_l1, part_l1, n_eta,
                       part_eta, params, prior, grad, loss, adam);
    return hipGetLastError();
}

}  // namespace starred
