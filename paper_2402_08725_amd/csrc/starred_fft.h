// FFT-path data structures shared by the plan (host) and the FFT kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "starred_internal.h"

namespace starred {

constexpr int kFftThreads = 256;
constexpr int kFftTargetElems = 2048;  // complex elements per work group and buffer
constexpr int kAdjBins = 4;            // spectral adjoint: bins per thread
constexpr int kAdjFrames = 4;          // spectral adjoint: frames held in registers at once
constexpr int kAdjQB = 8;              // spectral adjoint: dot products reduced per LDS pass

// A 1-D transform length L = product of radices (4, 2, 3, 5) and the offset of
// its twiddle table e^{-2 pi i m / L}, m < L.
struct FftLen {
    int L;
    int nst;
    int rad[8];
    long long tw_off;
};

// One shape class: frames with the same fine side F, kernel side K and window.
// P is the circular size (P >= F + floor(K/2), a multiple of 2s), Q = P/s.
struct ClassFft {
    int P, Q, F, n, o, K;
    FftLen fP, fQ;
    long long th_off;   // [F][P/2+1]   rows of the h window
    long long hh_off;   // [P][P/2+1]   spectrum of the h window
    long long tab_off;  // [(1 + 2M) P] window and point-source factor tables
    float sscale;       // 1 / (s^2 Q^2)
    int cf_off;         // first entry of this class in the class-ordered frame list
    int ncf;            // number of frames of the class
    int ngch;           // frame chunks of the frequency-domain adjoint
    int gfch;           // frames per chunk
    long long gp_off;   // [ngch][P][P/2+1] summed adjoint spectra of each chunk
    long long hc_off;   // [F][F] the class's contribution to dL/dh (its window)
};

struct FrameFft {
    int cls;
    int pad;
    long long kern_off;  // packed K^2 kernels
    long long s_off;     // [P][P/2+1] kernel spectrum S''
    long long t_off;     // [n][Q/2+1] row spectra (model / rho)
    long long r_off;     // [Q][Q/2+1] rho_hat
    long long t3_off;    // [P][P/2+1] scratch of the adjoint (and of the kernel transform)
    long long data_off;  // packed n^2
    long long fine_off;  // packed F^2
};

// A group of consecutive lines of one frame (or one class) handled by one work group.
struct LineItem {
    int cls;
    int frame;
    int line0;
    int nl;
};

// A block of output bins of one class and a chunk of that class's frames.
struct SpecItem {
    int cls;
    int f0;
    int nf;
    int bin0;
};

struct LinePass {
    LineItem *items = nullptr;  // device
    int n_items = 0;
    size_t lds_bytes = 0;
};

struct FftPlanDev {
    ClassFft *classes = nullptr;
    FrameFft *frames = nullptr;
    int n_classes = 0;
    float2 *tw = nullptr;
    float2 *S = nullptr, *T = nullptr, *T2 = nullptr, *Rh = nullptr, *T3 = nullptr;
    float2 *Th = nullptr, *Hh = nullptr, *tab = nullptr;
    LinePass hrows, hcols, krows, kcols, fcols, frows, rrows, rcols, acols, arows, srows, scols;
    SpecItem *spec = nullptr;
    int n_spec = 0;
    int *cls_frames = nullptr;
    // per-frame sums of g from the adjoint row pass: partial per line group and,
    // for each frame, the list of its groups (CSR)
    double *gpart = nullptr;
    int *gcsr_off = nullptr, *gcsr_item = nullptr;
    // frequency-domain adjoint
    int n_frames = 0;
    SpecItem *aspec = nullptr;
    int n_aspec = 0;
    int maxpb = 0;           // per-wave partial slots per frame
    double *apart = nullptr; // [E][maxpb][1 + 3M]
    float2 *Gp = nullptr;
    float *hcls = nullptr;
    LinePass gcols, grows;
};

// Deterministic block sum of one double per thread (kFftThreads); thread 0 holds it.
__device__ __forceinline__ double block_sum_d_fft(double v, double *sh)
{
    #pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        #pragma unroll
        for (int i = 0; i < kFftThreads / 64; ++i) r += sh[i];
    }
    __syncthreads();
    return r;
}

hipError_t fft_prep_kernels(hipStream_t st, const FftPlanDev &d, const float *psf, int s);
hipError_t fft_spectra(hipStream_t st, const FftPlanDev &d, const float *params, int N, int E, int M,
                       float sigma);
hipError_t fft_spec_fwd(hipStream_t st, const FftPlanDev &d, const float *params, int N, int E, int M, int s);
hipError_t fft_model_cols(hipStream_t st, const FftPlanDev &d);
hipError_t fft_model_rows(hipStream_t st, const FftPlanDev &d, const float *data, const float *invvar,
                          double *part_chi, float *model);
hipError_t fft_rho_cols(hipStream_t st, const FftPlanDev &d);
hipError_t fft_adj_cols(hipStream_t st, const FftPlanDev &d);
hipError_t fft_adj_rows(hipStream_t st, const FftPlanDev &d, float *g);
hipError_t fft_resid_rows(hipStream_t st, const FftPlanDev &d, const float *resid);
hipError_t fft_adjoint(hipStream_t st, const FftPlanDev &d, float *g);
hipError_t fft_spec_adj(hipStream_t st, const FftPlanDev &d, int M, double *fsum);
hipError_t fft_grad_h_inverse(hipStream_t st, const FftPlanDev &d);
hipError_t fft_finalize_h(hipStream_t st, const FftPlanDev &d, int N, const float *prior, float *grad_h);
hipError_t fft_scene_model(hipStream_t st, const FftPlanDev &d, const float *scene, int s, float *model);

}  // namespace starred
