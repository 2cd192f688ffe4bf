// The starlet prior (Eq. 11's L1 term and its subgradient) with every scale
// computed directly from the image instead of through the a-trous cascade.
//
// With mirror boundaries, one smoothing level along an axis is the filter
// h_j = B3 with holes 2^j applied to the whole-sample symmetric extension of
// the line (period 2N - 2), and such extensions are kept by symmetric filters,
// so the cascade up to level j is ONE filter on the extension: the composite
// a_j = h_0 * h_1 * ... * h_{j-1} (half width 2^{j+1} - 2, dyadic taps). In
// matrix form c_j = M_j x M_j^T with M_j the N x N operator of a_j, and the
// coefficients alpha_j = c_j - c_{j+1} (alpha_{J-1} = c_{J-1}) are independent
// of one another. The subgradient's image is sum_j M_j^T (z_j - z_{j-1}) M_j
// (z_{-1} = 0), and M_j D is symmetric for D = diag(2, 1, ..., 1, 2), so
// M_j^T Y M_j = D^-1 M_j (D Y D) M_j^T D^-1: the adjoint is the same mirror
// filtering with the end samples scaled by exact powers of two.
//
// Four passes, each over all scales at once (FP64 accumulation):
//   A  T_j = x M_j^T           (rows, j >= 1)
//   B  c_j = M_j T_j           (columns, j >= 1)
//   C  alpha_j, z_j, the L1 share, and U_j = (D Y_j D) M_j^T, Y_j = z_j - z_{j-1}
//      (rows; U_0 = z_0)
//   D  out = U_0 + sum_{j >= 1} D^-1 (M_j U_j) D^-1   (columns)
// The job bodies take the work-group index as an argument so that other
// launches can carry them as extra work groups.
#pragma once

#include <hip/hip_runtime.h>

namespace starred {

constexpr int kDenseMaxJ = 8;  // at most 7 scales (eight need more LDS than the cap: the cascade)
constexpr int kDenseTile = 16;  // y-pass output tiles
constexpr int kDenseThreads = 256;

struct DenseStar {
    int N = 0, J = 0, B = 0;
    int rx = 1;                  // rows per x-pass job
    const double *taps = nullptr;  // levels 1 .. J-1 one after the other (plen(j) entries each)
    const float *img = nullptr;  // image 0 (N x N)
    const float *img1 = nullptr; // image 1 (N x N), when B = 2
    double *T = nullptr;         // [B][J][N][N]: plane j >= 1 = x M_j^T, then (pass D1) D^-1 (M_j U_j) D^-1
    double *C = nullptr;         // [B][J][N][N]: plane j >= 1 = c_j
    double *U = nullptr;         // [B][J][N][N]: plane 0 = z_0, plane j >= 1 = (D Y_j D) M_j^T
    const float *W = nullptr;    // weights: per pixel [J][N][N] (w_stride != 0) or per scale [J]
    int w_stride = 0;
    float lam0 = 0.f, lam1 = 0.f;  // image 0's and image 1's weight
    const float *zin = nullptr;  // given coefficients' subgradient (adjoint alone): z [B][J][N][N]
    float *out = nullptr;        // [B][N][N]
    double *part_l1 = nullptr;   // [B][J][rows jobs]

    // half width of level j's composite filter, 2^{j+1} - 2; its 2 bw + 1 taps
    // zero-padded to plen(j), a multiple of 16 (the filter loops read whole blocks
    // of 16), at offset toff(j)
    __host__ __device__ static constexpr int bw(int j) { return (2 << j) - 2; }
    __host__ __device__ static constexpr int plen(int j) { return (2 * bw(j) + 1 + 15) & ~15; }
    // sum of plen(l) for l < j: 16 for level 1, 2^{l+2} for l >= 2
    __host__ __device__ static constexpr int toff(int j) { return j >= 2 ? (4 << j) : 0; }
    __host__ __device__ int xjobs() const { return (N + rx - 1) / rx; }
    __host__ __device__ int tiles() const { return (N + kDenseTile - 1) / kDenseTile; }
    __host__ __device__ int jobs_a() const { return B * (J - 1) * xjobs(); }
    __host__ __device__ int jobs_b() const { return B * (J - 1) * tiles() * tiles(); }
    __host__ __device__ int jobs_c() const { return B * J * xjobs(); }
    __host__ __device__ int jobs_d() const { return B * tiles() * tiles(); }
    __host__ __device__ int jobs_d1() const { return B * (J - 1) * tiles() * tiles(); }
    __host__ __device__ int l1_slots() const { return B * J * xjobs(); }
    __host__ __device__ const float *image(int b) const { return b ? img1 : img; }
    __host__ __device__ long long plane(int b, int j) const { return ((long long)b * J + j) * N * N; }
};

__device__ __forceinline__ int dmirror(int i, int N)
{
    i = i < 0 ? -i : i;
    return i > N - 1 ? 2 * (N - 1) - i : i;
}

__device__ __forceinline__ double dend(int i, int N) { return (i == 0 || i == N - 1) ? 2.0 : 1.0; }

__device__ __forceinline__ float dsgn(double v) { return (float)((v > 0.0) - (v < 0.0)); }

// Deterministic sum of one double per thread over a work group of any size
// (at most 1024 threads); the result is valid in thread 0.
__device__ __forceinline__ double dense_block_sum(double v, double *sh)
{
    #pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < nw; ++i) r += sh[i];
    __syncthreads();
    return r;
}

// sum_t a[t] s[t stride] (taps uniform across the work group, s in LDS), in
// whole blocks of 16 taps whose loads are in flight together: the taps past nt
// are the level's zero padding, against staged samples (or the staging's zero
// tail), so they add exact zeros
__device__ __forceinline__ double dense_dot(const double *a, const double *s, int stride, int nt)
{
    double acc = 0.0;
    for (int t = 0; t < nt; t += 16) {
        double av[16], sv[16];
        #pragma unroll
        for (int u = 0; u < 16; ++u) {
            av[u] = a[t + u];
            sv[u] = s[(t + u) * stride];
        }
        #pragma unroll
        for (int u = 0; u < 16; ++u) acc = fma(av[u], sv[u], acc);
    }
    return acc;
}

// The composite taps of the levels up to kDenseConstLevels, built at compile time
// (a_j = a_{j-1} * h_{j-1}, h_l the B3 kernel (1 4 6 4 1)/16 with holes 2^l). Each tap
// is a dyadic rational with at most 20 significant bits, so it is an exact FP64
// instruction literal: the filter loops of these levels load no taps at all (a tap
// read from memory costs a dependent round trip per block of 16 taps).
constexpr int kDenseConstLevels = 5;
struct DenseConstTaps {
    double v[DenseStar::toff(kDenseConstLevels + 1)];
};
constexpr DenseConstTaps dense_const_taps()
{
    constexpr int kLen = 2 * DenseStar::bw(kDenseConstLevels) + 1;
    DenseConstTaps t{};
    double a[kLen] = {}, n[kLen] = {};
    const double h[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
    int len = 1;
    a[0] = 1.0;
    for (int j = 1; j <= kDenseConstLevels; ++j) {
        const int d = 1 << (j - 1), nl = len + 4 * d;
        for (int i = 0; i < nl; ++i) n[i] = 0.0;
        for (int i = 0; i < len; ++i)
            for (int k = 0; k < 5; ++k) n[i + k * d] += a[i] * h[k];
        for (int i = 0; i < nl; ++i) {
            a[i] = n[i];
            t.v[DenseStar::toff(j) + i] = n[i];
        }
        len = nl;
    }
    return t;
}
constexpr DenseConstTaps kDenseConstTaps = dense_const_taps();

// Level LV's filter, sum_t a[t] s[t stride], with literal taps (four interleaved sums)
template <int LV>
__device__ __forceinline__ double dense_dot_lv(const double *s, int stride)
{
    constexpr int nt = 2 * DenseStar::bw(LV) + 1, off = DenseStar::toff(LV);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    #pragma unroll
    for (int t = 0; t < nt; ++t) acc[t & 3] = fma(kDenseConstTaps.v[off + t], s[t * stride], acc[t & 3]);
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// Level j's filter: literal taps up to kDenseConstLevels, the padded table beyond
__device__ __forceinline__ double dense_dot_level(const DenseStar &d, int j, const double *s, int stride)
{
    switch (j) {
    case 1: return dense_dot_lv<1>(s, stride);
    case 2: return dense_dot_lv<2>(s, stride);
    case 3: return dense_dot_lv<3>(s, stride);
    case 4: return dense_dot_lv<4>(s, stride);
    case 5: return dense_dot_lv<5>(s, stride);
    default: return dense_dot(d.taps + d.toff(j), s, stride, 2 * d.bw(j) + 1);
    }
}

// Stages n values through LDS with kDenseBatch independent loads in flight per
// thread, then nz zeros after them; load(e) is only called with e < n.
constexpr int kDenseBatch = 8;
constexpr int kDenseXTail = 16;       // zeros after an x-pass job's rows
constexpr int kDenseYTail = 15 * 16;  // zero rows after a y-pass strip (16 wide)
template <class Load>
__device__ __forceinline__ void dense_stage(double *lds, int n, int nz, Load load)
{
    for (int base = threadIdx.x; base < n; base += kDenseBatch * blockDim.x) {
        double v[kDenseBatch];
        #pragma unroll
        for (int u = 0; u < kDenseBatch; ++u) v[u] = load(min(base + u * (int)blockDim.x, n - 1));
        #pragma unroll
        for (int u = 0; u < kDenseBatch; ++u) {
            const int e = base + u * blockDim.x;
            if (e < n) lds[e] = v[u];
        }
    }
    for (int e = threadIdx.x; e < nz; e += blockDim.x) lds[n + e] = 0.0;
}

// Rows y0 .. y0+ny-1, filtered along x by level j's composite filter through
// the mirror: lds holds the extended rows (ny (N + 2 bw) doubles).
template <class Src, class Dst>
__device__ __forceinline__ void dense_xpass(const DenseStar &d, int j, int y0, int ny, double *lds, Src src, Dst dst)
{
    const int N = d.N, bw = d.bw(j), L = N + 2 * bw;
    dense_stage(lds, ny * L, kDenseXTail, [&](int e) {
        const int r = e / L, i = e - r * L - bw;
        return src(y0 + r, dmirror(i, N));
    });
    __syncthreads();
    for (int o = threadIdx.x; o < ny * N; o += blockDim.x) {
        const int r = o / N, x = o - r * N;
        dst(y0 + r, x, dense_dot_level(d, j, lds + r * L + x, 1));
    }
}

// Stages the column strip of output tile (y0, x0) for level j's filter along y
// through the mirror: (kDenseTile + 2 bw) x kDenseTile doubles (rows past the
// last one a tap reaches, and columns past N, are zero).
// value of the extended strip of level j at (r, c) for output tile (y0, x0)
template <class Src>
__device__ __forceinline__ double dense_strip_at(const DenseStar &d, int j, int y0, int x0, int e, Src src)
{
    const int N = d.N, bw = d.bw(j);
    const int r = e / kDenseTile, c = e - r * kDenseTile, x = x0 + c, y = y0 - bw + r;
    const bool in = x < N && y <= N - 1 + bw;
    const double v = src(dmirror(in ? y : 0, N), in ? x : 0);
    return in ? v : 0.0;
}

template <class Src>
__device__ __forceinline__ void dense_ystage(const DenseStar &d, int j, int y0, int x0, double *lds, Src src)
{
    const int R = kDenseTile + 2 * d.bw(j);
    dense_stage(lds, R * kDenseTile, kDenseYTail, [&](int e) { return dense_strip_at(d, j, y0, x0, e, src); });
}

// Level j's filter along y at output (y0 + ty, x0 + tx) from a staged strip.

__device__ __forceinline__ double dense_ysum(const DenseStar &d, int j, const double *lds, int ty, int tx)
{
    return dense_dot_level(d, j, lds + ty * kDenseTile + tx, kDenseTile);
}

// ---- pass A: T_j = x M_j^T ----
__device__ __forceinline__ void dense_job_a(const DenseStar &d, int job, double *lds)
{
    const int xj = d.xjobs(), per_b = (d.J - 1) * xj;
    const int b = job / per_b, rem = job - b * per_b, j = 1 + rem / xj, y0 = (rem % xj) * d.rx;
    const int ny = min(d.rx, d.N - y0), N = d.N;
    const float *im = d.image(b);
    double *T = d.T + d.plane(b, j);
    dense_xpass(
        d, j, y0, ny, lds, [&](int y, int k) { return (double)im[y * N + k]; },
        [&](int y, int x, double v) { T[y * N + x] = v; });
}

// ---- pass B: c_j = M_j T_j ----
__device__ __forceinline__ void dense_job_b(const DenseStar &d, int job, double *lds)
{
    const int nt = d.tiles(), per_j = nt * nt, per_b = (d.J - 1) * per_j;
    const int b = job / per_b, rem = job - b * per_b, j = 1 + rem / per_j, tile = rem % per_j;
    const int y0 = (tile / nt) * kDenseTile, x0 = (tile % nt) * kDenseTile, N = d.N;
    const double *T = d.T + d.plane(b, j);
    dense_ystage(d, j, y0, x0, lds, [&](int y, int x) { return T[y * N + x]; });
    __syncthreads();
    const int ty = threadIdx.x / kDenseTile, tx = threadIdx.x % kDenseTile;
    if (threadIdx.x < kDenseTile * kDenseTile && y0 + ty < N && x0 + tx < N)
        d.C[d.plane(b, j) + (y0 + ty) * N + x0 + tx] = dense_ysum(d, j, lds, ty, tx);
}

// alpha_j at (y, k) of image b: c_j - c_{j+1} with c_0 the image, c_J = 0
__device__ __forceinline__ double dense_alpha(const DenseStar &d, int b, int j, int y, int k)
{
    const int N = d.N;
    const long long pix = (long long)y * N + k;
    const double cj = j == 0 ? (double)d.image(b)[pix] : d.C[d.plane(b, j) + pix];
    const double cn = j + 1 < d.J ? d.C[d.plane(b, j + 1) + pix] : 0.0;
    return cj - cn;
}

// z_j at (y, k): lambda W_j sgn(alpha_j) (FP32 product), or the given subgradient
__device__ __forceinline__ float dense_z(const DenseStar &d, int b, int j, int y, int k, float lam)
{
    const long long pix = (long long)y * d.N + k, NN = (long long)d.N * d.N;
    if (d.zin) return d.zin[((long long)b * d.J + j) * NN + pix];
    const float w = d.w_stride ? d.W[j * NN + pix] : d.W[j];
    return lam * w * dsgn(dense_alpha(d, b, j, y, k));
}

// ---- pass C: z, the L1 share, U_j = (D Y_j D) M_j^T ----
__device__ __forceinline__ void dense_job_c(const DenseStar &d, int job, double *lds, double *red)
{
    const int xj = d.xjobs(), per_b = d.J * xj;
    const int b = job / per_b, rem = job - b * per_b, j = rem / xj, y0 = (rem % xj) * d.rx;
    const int ny = min(d.rx, d.N - y0), N = d.N;
    const long long NN = (long long)N * N;
    const float lam = b ? d.lam1 : d.lam0;
    double l1 = 0.0;
    if (!d.zin) {
        // the level's L1 share over this job's rows
        for (int e = threadIdx.x; e < ny * N; e += blockDim.x) {
            const int y = y0 + e / N, k = e % N;
            const long long pix = (long long)y * N + k;
            const float w = d.w_stride ? d.W[j * NN + pix] : d.W[j];
            l1 += (double)lam * (double)w * fabs(dense_alpha(d, b, j, y, k));
        }
    }
    double *U = d.U + d.plane(b, j);
    if (!d.out) {
        // the loss alone: no subgradient image
    } else if (j == 0) {
        for (int e = threadIdx.x; e < ny * N; e += blockDim.x) {
            const int y = y0 + e / N, k = e % N;
            U[y * N + k] = (double)dense_z(d, b, 0, y, k, lam);
        }
    } else {
        dense_xpass(
            d, j, y0, ny, lds,
            [&](int y, int k) {
                const double yv = (double)dense_z(d, b, j, y, k, lam) - (double)dense_z(d, b, j - 1, y, k, lam);
                return dend(y, N) * dend(k, N) * yv;
            },
            [&](int y, int x, double v) { U[y * N + x] = v; });
    }
    if (d.part_l1) {
        const double s = dense_block_sum(l1, red);
        if (threadIdx.x == 0) d.part_l1[(b * d.J + j) * xj + (y0 / d.rx)] = s;
    }
}

// ---- pass D: out = U_0 + sum_j D^-1 (M_j U_j) D^-1 ----
// lds holds every level's strip at once (dense_d_lds doubles).
__device__ __forceinline__ void dense_job_d(const DenseStar &d, int job, double *lds)
{
    const int nt = d.tiles(), per_b = nt * nt;
    const int b = job / per_b, tile = job % per_b, N = d.N;
    const int y0 = (tile / nt) * kDenseTile, x0 = (tile % nt) * kDenseTile;
    // every level's strip in one batched staging pass (levels one after the other)
    int total = 0;
    for (int j = 1; j < d.J; ++j) total += (kDenseTile + 2 * d.bw(j)) * kDenseTile;
    dense_stage(lds, total, kDenseYTail, [&](int e) {
        int j = 1, off = 0;
        while (e >= off + (kDenseTile + 2 * d.bw(j)) * kDenseTile) off += (kDenseTile + 2 * d.bw(j++)) * kDenseTile;
        const double *U = d.U + d.plane(b, j);
        return dense_strip_at(d, j, y0, x0, e - off, [&](int y, int x) { return U[y * N + x]; });
    });
    __syncthreads();
    int off = 0;
    const int ty = threadIdx.x / kDenseTile, tx = threadIdx.x % kDenseTile, y = y0 + ty, x = x0 + tx;
    if (threadIdx.x >= kDenseTile * kDenseTile || y >= N || x >= N) return;
    double acc = 0.0;
    for (int j = 1; j < d.J; ++j) {
        acc += dense_ysum(d, j, lds + off, ty, tx);
        off += (kDenseTile + 2 * d.bw(j)) * kDenseTile;
    }
    const long long pix = (long long)y * N + x;
    d.out[(long long)b * N * N + pix] = (float)(d.U[d.plane(b, 0) + pix] + acc / (dend(y, N) * dend(x, N)));
}

// ---- pass D1: level j's term D^-1 (M_j U_j) D^-1 alone, into plane j of T ----
// (T_j is not needed after pass B); the subgradient image is then
// U_0 + sum_j T_j at each pixel (dense_prior_at), summed by its reader.
__device__ __forceinline__ void dense_job_d1(const DenseStar &d, int job, double *lds)
{
    const int nt = d.tiles(), per_j = nt * nt, per_b = (d.J - 1) * per_j;
    const int b = job / per_b, rem = job - b * per_b, j = 1 + rem / per_j, tile = rem % per_j;
    const int y0 = (tile / nt) * kDenseTile, x0 = (tile % nt) * kDenseTile, N = d.N;
    const double *U = d.U + d.plane(b, j);
    dense_ystage(d, j, y0, x0, lds, [&](int y, int x) { return U[y * N + x]; });
    __syncthreads();
    const int ty = threadIdx.x / kDenseTile, tx = threadIdx.x % kDenseTile, y = y0 + ty, x = x0 + tx;
    if (threadIdx.x < kDenseTile * kDenseTile && y < N && x < N)
        d.T[d.plane(b, j) + y * N + x] = dense_ysum(d, j, lds, ty, tx) / (dend(y, N) * dend(x, N));
}

// the subgradient image of image b at pixel pix after pass D1
__device__ __forceinline__ double dense_prior_at(const DenseStar &d, int b, long long pix)
{
    double v = d.U[d.plane(b, 0) + pix];
    for (int j = 1; j < d.J; ++j) v += d.T[d.plane(b, j) + pix];
    return v;
}

}  // namespace starred

namespace starred {

// One pass of the composite-filter prior carried by another launch: its work
// groups first .. first+jobs-1 run the pass's jobs (they need at least
// kDenseThreads threads and dense_piece_lds bytes of dynamic LDS).
struct DensePiece {
    DenseStar d;
    int pass = -1;  // 0..3: A..D, 4: D1; -1: none
    int first = 0;
    int jobs = 0;
};

// Runs this work group's job when it carries one; true if it did.
__device__ __forceinline__ bool dense_piece_run(const DensePiece &p, void *lds_raw, double *red)
{
    const int job = (int)blockIdx.x - p.first;
    if (p.pass < 0 || job < 0 || job >= p.jobs) return false;
    double *lds = (double *)lds_raw;
    switch (p.pass) {
    case 0: dense_job_a(p.d, job, lds); break;
    case 1: dense_job_b(p.d, job, lds); break;
    case 2: dense_job_c(p.d, job, lds, red); break;
    case 3: dense_job_d(p.d, job, lds); break;
    default: dense_job_d1(p.d, job, lds); break;
    }
    return true;
}

}  // namespace starred
