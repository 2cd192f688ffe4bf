// FFT-path data structures shared by the plan (host) and the FFT kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "starred_dense.h"
#include "starred_internal.h"

namespace starred {

constexpr int kFftThreads = 256;
constexpr int kFftTargetElems = 2048;  // complex elements per work group and buffer
constexpr int kFusedThreads = 1024;     // one-launch forward: threads per frame
constexpr size_t kFusedLdsMax = 150 * 1024;  // one-launch forward: LDS of its two Q x (Q+1) planes
constexpr int kFwdFrames = 4;          // spectral product: frames whose loads are issued together
constexpr int kProdPairQ = 128;        // one-launch forward: columns of at least this length load two rows at once
constexpr int kAdjFrames = 2;          // spectral adjoint: frames of a work group (a chunk), default
constexpr int kAdjMaxFrames = 8;       // spectral adjoint: most frames of a chunk
constexpr int kAdjSB = 4;              // spectral adjoint: sources per pass over the rows (M > 1)
constexpr int kAdjSBWide = 8;          // the same with 2-frame chunks and more than kAdjSB sources
constexpr int kAdjSBOne = 16;          // the same with 1-frame chunks (more than kAdjSBWide sources)
constexpr int kAdjBlocks = 512;        // spectral adjoint: work groups aimed at per launch
constexpr int kAdjMinRows = 4;         // spectral adjoint: fewest rows per thread
constexpr int kAdjMaxRows = 64;        // spectral adjoint: most rows per work group
constexpr int kAdjRB = 3;              // spectral adjoint: rows of a thread whose loads are issued together
constexpr int kSumBins = 64;           // chunk-spectrum sums: bins of a work group
constexpr int kSumParts = 4;           // chunk-spectrum sums: runs of chunks per bin (threads)
constexpr int kSumBatch = 16;          // chunk-spectrum sums: loads of a run in flight together
// spectral adjoint: column lanes of a work group (64, 128 or 256, a divisor of its
// threads), the smallest that covers the P/2+1 columns
__host__ __device__ inline int adj_lanes(int HP) { return HP <= 64 ? 64 : (HP <= 128 ? 128 : 256); }

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
    int ngch_cap;       // chunks the class's gp region holds (its smallest allowed chunks)
    long long gp_off;   // [ngch][P][P/2+1] summed adjoint spectra of each chunk (total in chunk 0)
    long long hc_off;   // [F][F] the class's contribution to dL/dh (its window)
    int fused;          // frames of this class take the one-launch forward (spectra fit in LDS)
    int arr;            // spectral adjoint: row representatives per work group (2s rows each)
    int nrr;            // spectral adjoint: row ranges (per-frame partial slots)
    int direct;         // the class runs the direct algorithm (the FFT launches skip it)
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

// A work group of the one-launch forward: its frame with the offsets it reads,
// resolved on the host (the class record itself is only needed for the
// transforms' factor tables, later).
struct FusedItem {
    int frame, cls;
    int P, Q, n;          // sizes
    int inplace;          // one LDS plane transformed in place (else two planes)
    long long tw_off;     // the Q-point twiddles
    long long s_off;      // kernel spectrum S''
    long long data_off;   // data and inverse variances
    long long r_off;      // rho_hat (output)
    long long tab_off;    // the class's factor tables
    long long hh_off;     // the class's spectrum of h
};

// A work group of the frequency-domain adjoint: a chunk of frames and a range of
// rows of one class, with everything the group needs resolved on the host (so
// its loads depend on this item alone).
struct AdjItem {
    int cls;
    int nf;                      // frames in the chunk
    int y0, y1;                  // representatives [y0, y1) of the rows (y <= Q/2: rows = +-y mod Q)
    int P, Q;
    int pb;                      // row range index (the per-frame partial slot)
    int pad;
    int fid[kAdjMaxFrames];         // frame indices (-1 past nf)
    long long soff[kAdjMaxFrames];  // kernel spectra S'' (the chunk's first frame again past nf)
    long long roff[kAdjMaxFrames];  // rho_hat (the chunk's first frame again past nf)
    long long tab_off;           // the class's factor tables
    long long gout;              // the chunk's slot in the chunk spectra
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
    AdjItem *aspec = nullptr;
    int n_aspec = 0;
    int adj_fc = kAdjFrames;   // frames per chunk of the current items
    int maxpb = 0;           // per-frame partial slots (largest nrr)
    long long total_bins = 0;  // sum over classes of P (P/2 + 1)
    double *apart = nullptr; // [E][maxpb][1 + 3M]
    float2 *Gp = nullptr;
    float *hcls = nullptr;
    LinePass gcols, grows;
    // loss+gradient forward: frames of fused classes in one launch (a work group
    // per frame); the line passes below cover the remaining frames
    SpecItem *spec_lg = nullptr;
    int n_spec_lg = 0;
    FusedItem *fused = nullptr;
    int n_fused = 0;
    size_t fused_lds = 0;
    LinePass fcols_lg, frows_lg, rcols_lg;
    // every frame, whatever its class runs: the per-frame convolution of rendered
    // scenes (frames with per-frame transforms), and its per-group sums of g
    LinePass srows_x, scols_x, fcols_x, frows_x, rcols_x, acols_x, arows_x;
    double *gpart_x = nullptr;
};

// Deterministic block sum of one double per thread (NT threads); thread 0 holds it.
template <int NT = kFftThreads>
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
        for (int i = 0; i < NT / 64; ++i) r += sh[i];
    }
    __syncthreads();
    return r;
}

hipError_t fft_prep_kernels(hipStream_t st, const FftPlanDev &d, const float *psf, int s);
// tick: a step counter the launch advances (the first launch of a fused step), or null
// pa, pb: passes of the starlet prior carried by the row and column launches (or null)
hipError_t fft_spectra(hipStream_t st, const FftPlanDev &d, const float *params, int N, int E, int M,
                       float sigma, int *tick = nullptr, DensePiece *pa = nullptr, DensePiece *pb = nullptr);
hipError_t fft_spec_fwd(hipStream_t st, const FftPlanDev &d, const float *params, int N, int E, int M, int s,
                        bool lg = false);
hipError_t fft_model_cols(hipStream_t st, const FftPlanDev &d);
hipError_t fft_model_rows(hipStream_t st, const FftPlanDev &d, const float *data, const float *invvar,
                          double *part_chi, float *model);
hipError_t fft_rho_cols(hipStream_t st, const FftPlanDev &d);
hipError_t fft_adj_cols(hipStream_t st, const FftPlanDev &d);
hipError_t fft_adj_rows(hipStream_t st, const FftPlanDev &d, float *g);
hipError_t fft_resid_rows(hipStream_t st, const FftPlanDev &d, const float *resid);
hipError_t fft_adjoint(hipStream_t st, const FftPlanDev &d, float *g);
hipError_t fft_spec_adj(hipStream_t st, const FftPlanDev &d, int M);
hipError_t fft_adj_sums(hipStream_t st, const FftPlanDev &d, int M, double *fsum);
struct FinalArgs;
// dL/dh of the classes: the column inverse alone, and (one class whose window
// is the whole grid) the row inverse that also writes dL/dh, updates h and does
// the evaluation's small reductions in an extra work group
hipError_t fft_grad_h_cols(hipStream_t st, const FftPlanDev &d, DensePiece *pd = nullptr);
// psum (or null): the composite-filter prior's planes after pass D1, summed per pixel instead of reading prior
hipError_t fft_grad_h_rows_final(hipStream_t st, const FftPlanDev &d, const float *prior, const FinalArgs &fin,
                                 const DenseStar *psum = nullptr);
// lines of each LDS plane of the one-launch forward: the Q/2+1 columns of the half
// spectrum, or the (n+1)/2 pairs of real rows (two rows share a complex transform)
__host__ __device__ inline int fused_plane_lines(int Q, int n)
{
    const int pairs = (n + 1) / 2;
    return (Q / 2 + 1) > pairs ? (Q / 2 + 1) : pairs;
}
// bytes of LDS the one-launch forward needs for a class: `planes` (two, or one
// transformed in place) of fused_plane_lines lines of Q+1 values, the Q twiddles
// and the (1+4M) P table values
inline size_t fused_lds_bytes(int Q, int n, int P, int M, int planes = 2)
{
    const int rows = fused_plane_lines(Q, n);
    return ((size_t)planes * rows * (Q + 1) + Q + (size_t)(1 + 4 * M) * P) * 8;
}
// transform lengths with a single-plane (in-place) form in the one-launch forward
__host__ __device__ inline bool fft_ip_length(int L) { return L == 128 || L == 144 || L == 160 || L == 192; }
hipError_t fft_fused_fwd(hipStream_t st, const FftPlanDev &d, const float *params, int N, int E, int M, int s,
                         const float *data, const float *invvar, double *part_chi, DensePiece *pc = nullptr);
hipError_t fft_model_cols_lg(hipStream_t st, const FftPlanDev &d);
hipError_t fft_model_rows_lg(hipStream_t st, const FftPlanDev &d, const float *data, const float *invvar,
                             double *part_chi);
hipError_t fft_rho_cols_lg(hipStream_t st, const FftPlanDev &d);
hipError_t fft_grad_h_inverse(hipStream_t st, const FftPlanDev &d, DensePiece *pd = nullptr);
hipError_t fft_scene_model(hipStream_t st, const FftPlanDev &d, const float *scene, int s, float *model);
// Frames with per-frame transforms: S_i and D of each frame's rendered scene (fine
// grid, per-frame layout) through its own spectrum, the weighted residual and its
// chi-square partials (one per row group of frows_x), rho_hat kept for the adjoint.
hipError_t fft_xf_forward(hipStream_t st, const FftPlanDev &d, const float *scene, int s, const float *data,
                          const float *invvar, double *part_chi);
// ... and D^T S_i^T of those residuals into g (fine grid, per-frame layout).
hipError_t fft_xf_adjoint(hipStream_t st, const FftPlanDev &d, float *g);

}  // namespace starred
