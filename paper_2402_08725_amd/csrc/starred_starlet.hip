// Starlet prior through the per-scale composite filters (starred_dense.h):
// standalone launches of the four passes, the coefficient and adjoint forms,
// and the host-side construction of the composite taps.
#include "starred_dense.h"
#include "starred_internal.h"

#include <hip/hip_runtime.h>

#include <vector>

namespace starred {

__global__ __launch_bounds__(kDenseThreads) void k_dense_a(DenseStar d)
{
    extern __shared__ double lds[];
    dense_job_a(d, blockIdx.x, lds);
}

__global__ __launch_bounds__(kDenseThreads) void k_dense_b(DenseStar d)
{
    extern __shared__ double lds[];
    dense_job_b(d, blockIdx.x, lds);
}

__global__ __launch_bounds__(kDenseThreads) void k_dense_c(DenseStar d)
{
    extern __shared__ double lds[];
    __shared__ double red[kDenseThreads / 64];
    dense_job_c(d, blockIdx.x, lds, red);
}

__global__ __launch_bounds__(kDenseThreads) void k_dense_d(DenseStar d)
{
    extern __shared__ double lds[];
    dense_job_d(d, blockIdx.x, lds);
}

// alpha_j (FP32) of every scale: [B][J][N][N]
__global__ void k_dense_coeffs(DenseStar d, float *coeffs)
{
    const long long NN = (long long)d.N * d.N, n = (long long)d.B * d.J * NN;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int b = (int)(e / (d.J * NN)), j = (int)((e / NN) % d.J);
    const long long pix = e % NN;
    coeffs[e] = (float)dense_alpha(d, b, j, (int)(pix / d.N), (int)(pix % d.N));
}

size_t dense_lds_xr(int N, int J, int rx)
{
    return sizeof(double) * ((size_t)rx * (N + 2 * DenseStar::bw(J - 1)) + kDenseXTail);
}

size_t dense_lds_x(int N, int J) { return dense_lds_xr(N, J, dense_rows_per_job(N)); }

size_t dense_lds_y(int J)
{
    return sizeof(double) * (kDenseTile * (size_t)(kDenseTile + 2 * DenseStar::bw(J - 1)) + kDenseYTail);
}

size_t dense_lds_d(int J)
{
    size_t n = kDenseYTail;
    for (int j = 1; j < J; ++j) n += (size_t)(kDenseTile + 2 * DenseStar::bw(j)) * kDenseTile;
    return sizeof(double) * n;
}

int dense_rows_for(int N, int threads) { return N >= threads ? 1 : threads / N; }

int dense_rows_per_job(int N) { return dense_rows_for(N, kDenseThreads); }

bool dense_fits(int N, int J)
{
    return J >= 2 && J <= kDenseMaxJ - 1 && N <= kDenseMaxN && DenseStar::bw(J - 1) <= N - 1 &&
           dense_lds_d(J) <= kDenseMaxLds && dense_lds_x(N, J) <= kDenseMaxLds;
}

int dense_num_taps(int J) { return J >= 2 ? DenseStar::toff(J) : 0; }

void dense_taps(int J, double *out)
{
    // a_j = h_0 * ... * h_{j-1}, h_l = B3 (1 4 6 4 1)/16 with holes 2^l
    std::vector<double> a{1.0};
    for (int j = 1; j < J; ++j) {
        const int d = 1 << (j - 1);
        std::vector<double> n(a.size() + 4 * d, 0.0);
        const double h[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
        for (size_t i = 0; i < a.size(); ++i)
            for (int t = 0; t < 5; ++t) n[i + t * d] += a[i] * h[t];
        a.swap(n);
        for (int i = 0; i < DenseStar::plen(j); ++i) out[DenseStar::toff(j) + i] = i < (int)a.size() ? a[i] : 0.0;
    }
}

static hipError_t dense_launch(void (*k)(DenseStar), int jobs, size_t lds, hipStream_t st, const DenseStar &d)
{
    if (jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k, dim3(jobs), dim3(kDenseThreads), lds, st, d);
    return hipGetLastError();
}

hipError_t launch_dense_prior(hipStream_t st, const DenseStar &d)
{
    hipError_t e;
    if ((e = dense_launch(k_dense_a, d.jobs_a(), dense_lds_x(d.N, d.J), st, d)) != hipSuccess) return e;
    if ((e = dense_launch(k_dense_b, d.jobs_b(), dense_lds_y(d.J), st, d)) != hipSuccess) return e;
    if ((e = dense_launch(k_dense_c, d.jobs_c(), dense_lds_x(d.N, d.J), st, d)) != hipSuccess) return e;
    if (!d.out) return hipSuccess;
    return dense_launch(k_dense_d, d.jobs_d(), dense_lds_d(d.J), st, d);
}

hipError_t launch_dense_coeffs(hipStream_t st, const DenseStar &d, float *coeffs)
{
    hipError_t e;
    if ((e = dense_launch(k_dense_a, d.jobs_a(), dense_lds_x(d.N, d.J), st, d)) != hipSuccess) return e;
    if ((e = dense_launch(k_dense_b, d.jobs_b(), dense_lds_y(d.J), st, d)) != hipSuccess) return e;
    const long long n = (long long)d.B * d.J * d.N * d.N;
    hipLaunchKernelGGL(k_dense_coeffs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d, coeffs);
    return hipGetLastError();
}

hipError_t launch_dense_adjoint(hipStream_t st, const DenseStar &d)
{
    if (!d.zin || !d.out) return hipErrorInvalidValue;
    hipError_t e;
    if ((e = dense_launch(k_dense_c, d.jobs_c(), dense_lds_x(d.N, d.J), st, d)) != hipSuccess) return e;
    return dense_launch(k_dense_d, d.jobs_d(), dense_lds_d(d.J), st, d);
}

}  // namespace starred
