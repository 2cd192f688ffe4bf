// An entry point that allocates nothing: the starlet transform Phi^T (Eq. 6)
// without a plan, for callers that cannot allocate device memory (code under
// graph capture, tight loops, hosts that forbid allocation). Its working planes
// live in one fixed device array of this file, `scratch`, whose device address
// is looked up once per device; inputs and outputs are the caller's.
#include "starred.h"
#include "starred_internal.h"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>
#include <string>

using namespace starred;

namespace {

// Two smoothed planes c_a, c_b of the cascade (N^2 floats each, N <= kStaticMaxSide)
// followed by the J per-scale weights the transform-only launch reads (zero).
constexpr int kStaticMaxSide = 512;
constexpr int kStaticMaxScales = 16;
constexpr size_t kScratchFloats = 2 * (size_t)kStaticMaxSide * kStaticMaxSide + kStaticMaxScales;

static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
float *g_ptr[kMaxDevices] = {};

__global__ void k_zero(float *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

}  // namespace

// defined with the plan (sets the calling thread's message)
int starred_set_error(int code, const char *msg);

extern "C" int starred_starlet_fwd_noalloc(int32_t N, int32_t J, const float *img, float *coeffs, void *stream)
{
    if (!img || !coeffs) return starred_set_error(STARRED_EINVAL, "NULL argument");
    if (N < 2 || J < 1) return starred_set_error(STARRED_EINVAL, "N must be >= 2 and J >= 1");
    if (J > 1 && (1 << (J - 1)) > N - 1) return starred_set_error(STARRED_EINVAL, "2^(J-1) must not exceed N-1");
    if (N > kStaticMaxSide || J > kStaticMaxScales)
        return starred_set_error(STARRED_EINVAL, "starred_starlet_fwd_noalloc: N above 512 or J above 16 "
                                                 "(the fixed working array holds two 512 x 512 planes)");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return starred_set_error(STARRED_EHIP, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return starred_set_error(STARRED_EUNSUPPORTED, "device index above 63");
    float *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_ptr[dev]) {
            // the array's device address on this device (the host-side name is not one)
            void *ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr) {
                char buf[256];
                snprintf(buf, sizeof buf, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
                return starred_set_error(STARRED_EHIP, buf);
            }
            g_ptr[dev] = (float *)ptr;
        }
        base = g_ptr[dev];
    }
    hipStream_t st = (hipStream_t)stream;
    const size_t NN = (size_t)N * N;
    float *c_a = base, *c_b = base + NN, *wz = base + 2 * NN;
    // the weights the transform-only launch reads must be zero: a fill kernel
    // (every call, since calls share the array)
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, wz, J);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_starlet_fwd(st, N, J, img, coeffs, nullptr, wz, 0, 0.f, c_a, c_b, nullptr,
                                                nullptr, nullptr);
    if (e != hipSuccess) return starred_set_error(STARRED_EHIP, hipGetErrorString(e));
    return STARRED_OK;
}
