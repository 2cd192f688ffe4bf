// Vector kernels of the L-BFGS iteration: the two-loop recursion, the projected
// trial point, dot products and the history update. Every reduction is a fixed
// tree in FP64, so the iteration is deterministic.
#include "starred_internal.h"

#include <hip/hip_runtime.h>

namespace starred {

constexpr int kOptThreads = 1024;

// Work-group sum of one double per thread (fixed order); every thread gets it.
__device__ double wg_sum(double v, double *sh)
{
    #pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();  // sh free from any previous use
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    #pragma unroll
    for (int i = 0; i < kOptThreads / 64; ++i) r += sh[i];
    return r;
}

// Two-loop recursion (one work group): d = -H g over the `count` newest pairs of
// the ring buffers S, Y ([m][n], newest at `newest`), H_0 = gamma I with gamma =
// s^T y / y^T y of the newest pair.
__global__ __launch_bounds__(kOptThreads) void k_lbfgs_direction(long long n, const float *__restrict__ g,
                                                                 const float *__restrict__ S,
                                                                 const float *__restrict__ Y, int m, int count,
                                                                 int newest, float *__restrict__ d,
                                                                 double *__restrict__ alpha)
{
    __shared__ double sh[kOptThreads / 64];
    for (long long p = threadIdx.x; p < n; p += kOptThreads) d[p] = g[p];  // d holds q
    __syncthreads();
    for (int c = 0; c < count; ++c) {
        const int i = ((newest - c) % m + m) % m;
        const float *s = S + (long long)i * n, *y = Y + (long long)i * n;
        double sy = 0.0, sq = 0.0;
        for (long long p = threadIdx.x; p < n; p += kOptThreads) {
            sy += (double)s[p] * y[p];
            sq += (double)s[p] * d[p];
        }
        sy = wg_sum(sy, sh);
        sq = wg_sum(sq, sh);
        const double a = sq / sy;
        if (threadIdx.x == 0) alpha[c] = a;
        for (long long p = threadIdx.x; p < n; p += kOptThreads) d[p] = (float)(d[p] - a * y[p]);
        __syncthreads();
    }
    double gamma = 1.0;
    if (count > 0) {
        const float *s = S + (long long)newest * n, *y = Y + (long long)newest * n;
        double sy = 0.0, yy = 0.0;
        for (long long p = threadIdx.x; p < n; p += kOptThreads) {
            sy += (double)s[p] * y[p];
            yy += (double)y[p] * y[p];
        }
        sy = wg_sum(sy, sh);
        yy = wg_sum(yy, sh);
        gamma = sy / yy;
    }
    for (long long p = threadIdx.x; p < n; p += kOptThreads) d[p] = (float)(gamma * d[p]);
    __syncthreads();
    for (int c = count - 1; c >= 0; --c) {
        const int i = ((newest - c) % m + m) % m;
        const float *s = S + (long long)i * n, *y = Y + (long long)i * n;
        double sy = 0.0, yr = 0.0;
        for (long long p = threadIdx.x; p < n; p += kOptThreads) {
            sy += (double)s[p] * y[p];
            yr += (double)y[p] * d[p];
        }
        sy = wg_sum(sy, sh);
        yr = wg_sum(yr, sh);
        const double b = yr / sy, a = alpha[c];
        for (long long p = threadIdx.x; p < n; p += kOptThreads) d[p] = (float)(d[p] + s[p] * (a - b));
        __syncthreads();
    }
    for (long long p = threadIdx.x; p < n; p += kOptThreads) d[p] = -d[p];
}

hipError_t launch_lbfgs_direction(hipStream_t st, long long n, const float *g, const float *S, const float *Y, int m,
                                  int count, int newest, float *d, double *alpha_scratch)
{
    hipLaunchKernelGGL(k_lbfgs_direction, dim3(1), dim3(kOptThreads), 0, st, n, g, S, Y, m, count, newest, d,
                       alpha_scratch);
    return hipGetLastError();
}

// xt = clamp(x + step d, lo, hi) (bounds optional)
__global__ void k_trial_point(long long n, const float *__restrict__ x, const float *__restrict__ d, float step,
                              const float *__restrict__ lo, const float *__restrict__ hi, float *__restrict__ xt)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float v = x[p] + step * d[p];
    if (lo) v = fmaxf(v, lo[p]);
    if (hi) v = fminf(v, hi[p]);
    xt[p] = v;
}

hipError_t launch_trial_point(hipStream_t st, long long n, const float *x, const float *d, float step, const float *lo,
                              const float *hi, float *xt)
{
    hipLaunchKernelGGL(k_trial_point, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, x, d, step, lo, hi, xt);
    return hipGetLastError();
}

// out[0] = a^T (b - c) (c optional: a^T b), out[1] = a^T a (one work group)
__global__ __launch_bounds__(kOptThreads) void k_dots(long long n, const float *__restrict__ a,
                                                      const float *__restrict__ b, const float *__restrict__ c,
                                                      double *__restrict__ out)
{
    __shared__ double sh[kOptThreads / 64];
    double ab = 0.0, aa = 0.0;
    for (long long p = threadIdx.x; p < n; p += kOptThreads) {
        const double bv = c ? (double)b[p] - c[p] : (double)b[p];
        ab += (double)a[p] * bv;
        aa += (double)a[p] * a[p];
    }
    ab = wg_sum(ab, sh);
    aa = wg_sum(aa, sh);
    if (threadIdx.x == 0) {
        out[0] = ab;
        out[1] = aa;
    }
}

hipError_t launch_dots(hipStream_t st, long long n, const float *a, const float *b, const float *c, double *out)
{
    hipLaunchKernelGGL(k_dots, dim3(1), dim3(kOptThreads), 0, st, n, a, b, c, out);
    return hipGetLastError();
}

// s = x_new - x_old, y = g_new - g_old into history slot `slot`; then x_old = x_new,
// g_old = g_new
__global__ void k_history(long long n, const float *__restrict__ xn, float *__restrict__ xo,
                          const float *__restrict__ gn, float *__restrict__ go, float *__restrict__ s,
                          float *__restrict__ y, int store)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    if (store) {
        s[p] = xn[p] - xo[p];
        y[p] = gn[p] - go[p];
    }
    xo[p] = xn[p];
    go[p] = gn[p];
}

hipError_t launch_history(hipStream_t st, long long n, const float *xn, float *xo, const float *gn, float *go,
                          float *s, float *y, int store)
{
    hipLaunchKernelGGL(k_history, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, xn, xo, gn, go, s, y,
                       store);
    return hipGetLastError();
}

}  // namespace starred
