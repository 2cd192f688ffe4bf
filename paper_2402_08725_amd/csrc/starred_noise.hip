// Monte Carlo noise propagation to the starlet coefficients (Sec. 2.3, App. B):
// noise draws on the fine grid, their embedding in the h grid, and the moment
// accumulation that yields the weights W. S^T and the starlet transform are the
// library's own operators (an auxiliary s = 1 plan and the batched level kernels).
#include "starred_internal.h"

#include <hip/hip_runtime.h>

namespace starred {

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of the
// multiply-hi/lo bijection, the key bumped by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k)
{
    #pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k.x += 0x9E3779B9u;
            k.y += 0xBB67AE85u;
        }
        const unsigned hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
        const unsigned hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    }
    return c;
}

// Draw idx of realization real: Philox of counter (idx/4, real, 0, 0), key (seed
// low, seed high); words mapped to ((w >> 8) + 1/2) / 2^24 and paired (0,1), (2,3)
// by Box-Muller (r cos, r sin), r = sqrt(-2 ln u_first), angle 2 pi u_second.
__device__ __forceinline__ float normal_draw(unsigned long long seed, unsigned real, unsigned idx)
{
    const uint4 w = philox4x32_10(make_uint4(idx >> 2, real, 0u, 0u),
                                  make_uint2((unsigned)seed, (unsigned)(seed >> 32)));
    const int pair = (idx >> 1) & 1;
    const unsigned a = pair ? w.z : w.x, b = pair ? w.w : w.y;
    const float u1 = ((float)(a >> 8) + 0.5f) * (1.0f / 16777216.0f);
    const float u2 = ((float)(b >> 8) + 0.5f) * (1.0f / 16777216.0f);
    const float r = sqrtf(-2.0f * logf(u1));
    float sn, cs;
    sincosf(6.28318530717958647692f * u2, &sn, &cs);
    return (idx & 1) ? r * sn : r * cs;
}

__global__ void k_noise_draw(int nb, int r0, int n, int s, const float *__restrict__ sigma2_data,
                             const float *__restrict__ normals, unsigned long long seed, float *__restrict__ delta)
{
    const int F = s * n;
    const long long FF = (long long)F * F;
    const int b = blockIdx.y;
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= FF) return;
    float v = 0.f;
    if (b < nb) {
        const int y = (int)(pix / F), x = (int)(pix % F);
        const float z = normals ? normals[(long long)(r0 + b) * FF + pix]
                                : normal_draw(seed, (unsigned)(r0 + b), (unsigned)pix);
        // C_up^-1 delta_d with delta_d = sigma_up z
        v = z / sqrtf(sigma2_data[(long long)(y / s) * n + (x / s)]);
    }
    delta[(long long)b * FF + pix] = v;
}

hipError_t launch_noise_draw(hipStream_t st, int B, int nb, int r0, int n, int s, const float *sigma2_data,
                             const float *normals, unsigned long long seed, float *delta)
{
    const long long FF = (long long)s * n * s * n;
    hipLaunchKernelGGL(k_noise_draw, dim3((unsigned)((FF + 255) / 256), B), dim3(256), 0, st, nb, r0, n, s,
                       sigma2_data, normals, seed, delta);
    return hipGetLastError();
}

__global__ void k_noise_embed(int F, int N, int o, const float *__restrict__ g, float *__restrict__ img)
{
    const int b = blockIdx.y;
    const long long NN = (long long)N * N;
    const long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= NN) return;
    const int y = (int)(pix / N) - o, x = (int)(pix % N) - o;
    img[b * NN + pix] = (y >= 0 && y < F && x >= 0 && x < F) ? g[(long long)b * F * F + (long long)y * F + x] : 0.f;
}

hipError_t launch_noise_embed(hipStream_t st, int B, int F, int N, int o, const float *g, float *img)
{
    const long long NN = (long long)N * N;
    hipLaunchKernelGGL(k_noise_embed, dim3((unsigned)((NN + 255) / 256), B), dim3(256), 0, st, F, N, o, g, img);
    return hipGetLastError();
}

// realizations summed in order for every coefficient (FP64)
__global__ void k_noise_moments(int nb, long long count, const float *__restrict__ coeffs, double *__restrict__ s1,
                                double *__restrict__ s2)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    double a = s1[q], b2 = s2[q];
    for (int b = 0; b < nb; ++b) {
        const double c = coeffs[(long long)b * count + q];
        a += c;
        b2 += c * c;
    }
    s1[q] = a;
    s2[q] = b2;
}

hipError_t launch_noise_moments(hipStream_t st, int nb, long long count, const float *coeffs, double *s1,
                                double *s2)
{
    hipLaunchKernelGGL(k_noise_moments, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, nb, count, coeffs,
                       s1, s2);
    return hipGetLastError();
}

__global__ void k_noise_pixel(long long count, int R, const double *__restrict__ s1, const double *__restrict__ s2,
                              float *__restrict__ W)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const double m = s1[q] / R, v = s2[q] / R - m * m;
    W[q] = (float)sqrt(v > 0.0 ? v : 0.0);
}

// one work group per scale: pooled moments over the plane in a fixed order
__global__ __launch_bounds__(256) void k_noise_scale(long long NN, int R, const double *__restrict__ s1,
                                                     const double *__restrict__ s2, float *__restrict__ W)
{
    __shared__ double ra[256], rb[256];
    const int j = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (long long q = threadIdx.x; q < NN; q += 256) {
        a += s1[j * NN + q];
        b += s2[j * NN + q];
    }
    ra[threadIdx.x] = a;
    rb[threadIdx.x] = b;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            ra[threadIdx.x] += ra[threadIdx.x + h];
            rb[threadIdx.x] += rb[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double cnt = (double)R * (double)NN, m = ra[0] / cnt, v = rb[0] / cnt - m * m;
        W[j] = (float)sqrt(v > 0.0 ? v : 0.0);
    }
}

hipError_t launch_noise_finish(hipStream_t st, int J, long long NN, int R, int per_pixel, const double *s1,
                               const double *s2, float *W)
{
    if (per_pixel) {
        const long long count = (long long)J * NN;
        hipLaunchKernelGGL(k_noise_pixel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, R, s1, s2,
                           W);
    } else {
        hipLaunchKernelGGL(k_noise_scale, dim3(J), dim3(256), 0, st, NN, R, s1, s2, W);
    }
    return hipGetLastError();
}

__global__ void k_fill_d(double *p, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

hipError_t launch_fill_d(hipStream_t st, double *p, long long n)
{
    hipLaunchKernelGGL(k_fill_d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace starred
