// FFT path of the deconvolution operators S_i and D (Eq. 8) and their adjoint.
//
// For a frame of fine side F = s n and kernel side K the linear 'same'
// convolution equals a circular one of size P >= F + floor(K/2) (P a multiple of
// 2s, P = 2^a 3^b 5^c). Fold the s x s block sum into the kernel
// (kb = kernel embedded at its centre and box-summed), take S''(K) = DFT_P(kb) /
// (s^2 Q^2) with Q = P/s; then the subsampled model is
//     m = IDFT_Q( sum over the s^2 aliases K = k + (a,b) Q of S''(K) F(K) ),
// where F is the spectrum of the scene. The scene spectrum is assembled from
// the spectrum of the window of h (one transform per shape class) and rank-1
// tables of the point sources and of the window indicator (Eq. 9). The adjoint
// is g = window of IDFT_P( conj(S''(K)) rho_hat(K mod Q) ), rho_hat = DFT_Q(rho).
// Transforms are unnormalised; every constant sits in S''.
//
// All 2-D transforms are row/column passes of batched 1-D Stockham FFTs
// (radices 4, 2, 3, 5) staged in LDS; each pass is one launch over every frame
// of every shape class (a table of line groups), with loads and stores that
// fuse the spectral products, the Hermitian extensions, the crops and the
// residual / chi-square epilogue.
#include "starred_fft.h"
#include "starred_finalize.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

namespace starred {

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b)  // a * conj(b)
{
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// radix-R DFT of v in place; sign -1 forward (e^{-i}), +1 inverse
template <int R>
__device__ __forceinline__ void dft_small(float2 (&v)[8], bool inv);

template <>
__device__ __forceinline__ void dft_small<2>(float2 (&v)[8], bool)
{
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <>
__device__ __forceinline__ void dft_small<4>(float2 (&v)[8], bool inv)
{
    const float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    const float2 b0 = cadd(v[1], v[3]), b1 = csub(v[1], v[3]);
    // -i * b1 (forward) or +i * b1 (inverse)
    const float2 rb1 = inv ? make_float2(-b1.y, b1.x) : make_float2(b1.y, -b1.x);
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd(a1, rb1);
    v[3] = csub(a1, rb1);
}

template <>
__device__ __forceinline__ void dft_small<3>(float2 (&v)[8], bool inv)
{
    const float c1 = -0.5f;
    const float s1 = inv ? 0.86602540378443865f : -0.86602540378443865f;
    const float2 a = v[0], b = v[1], c = v[2];
    const float2 t = cadd(b, c), d = csub(b, c);
    v[0] = cadd(a, t);
    const float2 m = make_float2(a.x + c1 * t.x, a.y + c1 * t.y);
    // s1 * i * d
    const float2 id = make_float2(-s1 * d.y, s1 * d.x);
    v[1] = cadd(m, id);
    v[2] = csub(m, id);
}

template <>
__device__ __forceinline__ void dft_small<5>(float2 (&v)[8], bool inv)
{
    const float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;
    const float sg = inv ? 1.f : -1.f;
    const float s1 = sg * 0.95105651629515357f, s2 = sg * 0.58778525229247313f;
    const float2 a = v[0];
    const float2 t1 = cadd(v[1], v[4]), d1 = csub(v[1], v[4]);
    const float2 t2 = cadd(v[2], v[3]), d2 = csub(v[2], v[3]);
    v[0] = cadd(a, cadd(t1, t2));
    const float2 m1 = make_float2(a.x + c1 * t1.x + c2 * t2.x, a.y + c1 * t1.y + c2 * t2.y);
    const float2 m2 = make_float2(a.x + c2 * t1.x + c1 * t2.x, a.y + c2 * t1.y + c1 * t2.y);
    // i*(s1 d1 + s2 d2) and i*(s2 d1 - s1 d2)
    const float2 u1 = make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y);
    const float2 u2 = make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y);
    const float2 iu1 = make_float2(-u1.y, u1.x), iu2 = make_float2(-u2.y, u2.x);
    v[1] = cadd(m1, iu1);
    v[4] = csub(m1, iu1);
    v[2] = cadd(m2, iu2);
    v[3] = csub(m2, iu2);
}

// radix 8 as two radix-4 transforms of the sums and the twiddled differences
// of the pairs (n, n+4): even outputs from the sums, odd ones from the differences
template <>
__device__ __forceinline__ void dft_small<8>(float2 (&v)[8], bool inv)
{
    const float h = 0.70710678118654752f;
    float2 e[8], o[8];
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
        e[k] = cadd(v[k], v[k + 4]);
        o[k] = csub(v[k], v[k + 4]);
    }
    // o[n] *= W8^n, W8 = e^{-i pi/4} (forward) or e^{+i pi/4} (inverse)
    const float2 b1 = o[1], b2 = o[2], b3 = o[3];
    o[1] = inv ? make_float2(h * (b1.x - b1.y), h * (b1.x + b1.y)) : make_float2(h * (b1.x + b1.y), h * (b1.y - b1.x));
    o[2] = inv ? make_float2(-b2.y, b2.x) : make_float2(b2.y, -b2.x);
    o[3] = inv ? make_float2(-h * (b3.x + b3.y), h * (b3.x - b3.y)) : make_float2(h * (b3.y - b3.x), -h * (b3.x + b3.y));
    dft_small<4>(e, inv);
    dft_small<4>(o, inv);
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[2 * k] = e[k];
        v[2 * k + 1] = o[k];
    }
}

template <int R>
__device__ __forceinline__ void stockham_stage(const float2 *__restrict__ src, float2 *__restrict__ dst,
                                               int nl, int L, int Ls, int Ns, const float2 *__restrict__ tw,
                                               bool inv)
{
    const int LR = L / R;
    const int twstep = L / (Ns * R);
    for (int b = threadIdx.x; b < nl * LR; b += blockDim.x) {
        const int l = b / LR, j = b - l * LR;
        const float2 *in = src + l * Ls;
        float2 *out = dst + l * Ls;
        const int k = j % Ns;
        float2 v[8];
        #pragma unroll
        for (int r = 0; r < R; ++r) v[r] = in[j + r * LR];
        if (Ns > 1) {
            #pragma unroll
            for (int r = 1; r < R; ++r) {
                const float2 t = tw[r * k * twstep];  // r k twstep < L
                v[r] = inv ? cmulc(v[r], t) : cmul(v[r], t);
            }
        }
        dft_small<R>(v, inv);
        const int idxD = (j / Ns) * Ns * R + k;
        #pragma unroll
        for (int r = 0; r < R; ++r) out[idxD + r * Ns] = v[r];
    }
}

// 1-D FFTs of nl lines of length f.L held in LDS buffer a with line stride
// Ls = f.L + 1 (the pad keeps column-order accesses off a single bank); b is
// scratch of the same size. Returns the buffer that holds the result.
__device__ float2 *lds_fft(float2 *a, float2 *b, int nl, const FftLen &f, const float2 *__restrict__ tw,
                           bool inv)
{
    int Ns = 1;
    const int Ls = f.L + 1;
    for (int st = 0; st < f.nst; ++st) {
        const int R = f.rad[st];
        if (R == 4) stockham_stage<4>(a, b, nl, f.L, Ls, Ns, tw, inv);
        else if (R == 2) stockham_stage<2>(a, b, nl, f.L, Ls, Ns, tw, inv);
        else if (R == 3) stockham_stage<3>(a, b, nl, f.L, Ls, Ns, tw, inv);
        else stockham_stage<5>(a, b, nl, f.L, Ls, Ns, tw, inv);
        __syncthreads();
        float2 *t = a;
        a = b;
        b = t;
        Ns *= R;
    }
    return a;
}

// Compile-time transforms for the lengths the workloads use: with L and the
// stage parameters constant, every index division becomes a multiply-shift.
constexpr int ct_nrad(int L)
{
    int n = 0;
    while (L % 8 == 0) { L /= 8; ++n; }
    while (L % 4 == 0) { L /= 4; ++n; }
    while (L % 2 == 0) { L /= 2; ++n; }
    while (L % 3 == 0) { L /= 3; ++n; }
    while (L % 5 == 0) { L /= 5; ++n; }
    return n;
}
constexpr int ct_rad(int L, int i)
{
    int k = 0;
    while (L % 8 == 0) { if (k++ == i) return 8; L /= 8; }
    while (L % 4 == 0) { if (k++ == i) return 4; L /= 4; }
    while (L % 2 == 0) { if (k++ == i) return 2; L /= 2; }
    while (L % 3 == 0) { if (k++ == i) return 3; L /= 3; }
    while (L % 5 == 0) { if (k++ == i) return 5; L /= 5; }
    return 1;
}
constexpr int ct_ns(int L, int i)
{
    int ns = 1;
    for (int k = 0; k < i; ++k) ns *= ct_rad(L, k);
    return ns;
}

template <int R, int L, int NS, bool INV>
__device__ __forceinline__ void stage_ct(const float2 *__restrict__ src, float2 *__restrict__ dst, int nl,
                                         const float2 *__restrict__ tw)
{
    constexpr int LR = L / R, Ls = L + 1, TS = L / (NS * R);
    for (int b = threadIdx.x; b < nl * LR; b += blockDim.x) {
        const int l = b / LR, j = b - l * LR;
        const float2 *in = src + l * Ls;
        float2 *out = dst + l * Ls;
        const int k = j % NS;
        float2 v[8];
        #pragma unroll
        for (int r = 0; r < R; ++r) v[r] = in[j + r * LR];
        if (NS > 1) {
            #pragma unroll
            for (int r = 1; r < R; ++r) {
                const float2 t = tw[r * k * TS];  // r k TS < L
                v[r] = INV ? cmulc(v[r], t) : cmul(v[r], t);
            }
        }
        dft_small<R>(v, INV);
        const int idxD = (j / NS) * NS * R + k;
        #pragma unroll
        for (int r = 0; r < R; ++r) out[idxD + r * NS] = v[r];
    }
}

template <int L, bool INV, int I = 0>
__device__ __forceinline__ float2 *fft_ct(float2 *a, float2 *b, int nl, const float2 *__restrict__ tw)
{
    if constexpr (I == ct_nrad(L)) {
        return a;
    } else {
        stage_ct<ct_rad(L, I), L, ct_ns(L, I), INV>(a, b, nl, tw);
        __syncthreads();
        return fft_ct<L, INV, I + 1>(b, a, nl, tw);
    }
}

// Single-plane (in-place) transforms for frames whose two planes do not fit in LDS:
// each stage reads a thread's butterflies into registers, waits for every thread,
// then writes the results over the same plane. A thread holds at most KB
// butterflies (lines at most L/2+1, blocks of kFusedThreads threads).
template <int R, int L, int NS, bool INV>
__device__ __forceinline__ void stage_ct_ip(float2 *buf, int nl, const float2 *__restrict__ tw)
{
    constexpr int LR = L / R, Ls = L + 1, TS = L / (NS * R);
    constexpr int KB = ((L / 2 + 1) * LR + kFusedThreads - 1) / kFusedThreads;
    float2 v[KB][8];
    int dst[KB];
    #pragma unroll
    for (int q = 0; q < KB; ++q) {
        const int b = threadIdx.x + q * kFusedThreads;
        dst[q] = -1;
        if (b < nl * LR) {
            const int l = b / LR, j = b - l * LR;
            const float2 *in = buf + l * Ls;
            const int k = j % NS;
            #pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = in[j + r * LR];
            if (NS > 1) {
                #pragma unroll
                for (int r = 1; r < R; ++r) {
                    const float2 t = tw[r * k * TS];  // r k TS < L
                    v[q][r] = INV ? cmulc(v[q][r], t) : cmul(v[q][r], t);
                }
            }
            dft_small<R>(v[q], INV);
            dst[q] = l * Ls + (j / NS) * NS * R + k;
        }
    }
    __syncthreads();
    #pragma unroll
    for (int q = 0; q < KB; ++q)
        if (dst[q] >= 0) {
            #pragma unroll
            for (int r = 0; r < R; ++r) buf[dst[q] + r * NS] = v[q][r];
        }
    __syncthreads();
}

template <int L, bool INV, int I = 0>
__device__ __forceinline__ void fft_ct_ip(float2 *a, int nl, const float2 *__restrict__ tw)
{
    if constexpr (I < ct_nrad(L)) {
        stage_ct_ip<ct_rad(L, I), L, ct_ns(L, I), INV>(a, nl, tw);
        fft_ct_ip<L, INV, I + 1>(a, nl, tw);
    }
}

template <bool INV>
__device__ __forceinline__ void lds_fft_ip(float2 *a, int nl, const FftLen &f, const float2 *__restrict__ tw)
{
    switch (f.L) {  // the lengths fft_ip_length admits
    case 128: fft_ct_ip<128, INV>(a, nl, tw); break;
    case 144: fft_ct_ip<144, INV>(a, nl, tw); break;
    case 160: fft_ct_ip<160, INV>(a, nl, tw); break;
    case 192: fft_ct_ip<192, INV>(a, nl, tw); break;
    default: break;
    }
}

// Transform dispatch: compile-time bodies for the common lengths, the runtime
// Stockham loop otherwise.
template <bool INV>
__device__ __forceinline__ float2 *lds_fft_any(float2 *a, float2 *b, int nl, const FftLen &f,
                                            const float2 *__restrict__ tw)
{
    switch (f.L) {
    case 48: return fft_ct<48, INV>(a, b, nl, tw);
    case 64: return fft_ct<64, INV>(a, b, nl, tw);
    case 72: return fft_ct<72, INV>(a, b, nl, tw);
    case 96: return fft_ct<96, INV>(a, b, nl, tw);
    case 128: return fft_ct<128, INV>(a, b, nl, tw);
    case 144: return fft_ct<144, INV>(a, b, nl, tw);
    case 160: return fft_ct<160, INV>(a, b, nl, tw);
    case 192: return fft_ct<192, INV>(a, b, nl, tw);
    case 256: return fft_ct<256, INV>(a, b, nl, tw);
    case 288: return fft_ct<288, INV>(a, b, nl, tw);
    case 320: return fft_ct<320, INV>(a, b, nl, tw);
    case 384: return fft_ct<384, INV>(a, b, nl, tw);
    case 576: return fft_ct<576, INV>(a, b, nl, tw);
    default: return lds_fft(a, b, nl, f, tw, INV);
    }
}

// One-launch forward: two planes (a source and a scratch plane; returns the one
// holding the result) or, when ip, one plane transformed in place.
template <bool INV>
__device__ __forceinline__ float2 *lds_fft_plane(float2 *a, float2 *b, int nl, const FftLen &f,
                                                 const float2 *__restrict__ tw, bool ip)
{
    if (ip) {
        lds_fft_ip<INV>(a, nl, f, tw);
        return a;
    }
    return lds_fft_any<INV>(a, b, nl, f, tw);
}

// --------------------------------------------------------------------------
// Generic line pass: load -> FFT -> store, for a table of line groups
// --------------------------------------------------------------------------

// Ops may carry extra work groups behind their line groups (Op::extra, run_extra)
template <class Op, class = void>
struct has_extra : std::false_type {};
template <class Op>
struct has_extra<Op, std::void_t<decltype(Op::extra)>> : std::true_type {};

template <class Op>
__global__ __launch_bounds__(kFftThreads) void k_lines(const LineItem *__restrict__ items,
                                                       const ClassFft *__restrict__ classes,
                                                       const float2 *__restrict__ tw, Op op, DensePiece dp)
{
    extern __shared__ float2 sm[];
    {
        // a starlet-prior job carried by this launch (work groups after the line groups and extras)
        __shared__ double dred[kFftThreads / 64];
        if (dense_piece_run(dp, sm, dred)) return;
    }
    if constexpr (has_extra<Op>::value) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && op.tick) *op.tick += 1;
        if ((int)blockIdx.x >= op.n_items) {
            op.run_extra(blockIdx.x - op.n_items, classes, tw);
            return;
        }
    }
    const LineItem it = items[blockIdx.x];
    const ClassFft &cl = classes[it.cls];
    const FftLen &f = op.len(cl);
    const int Ls = f.L + 1;
    float2 *a = sm;
    float2 *b = sm + it.nl * Ls;
    const int tot = it.nl * f.L;
    // column passes walk the lines fastest so that neighbouring threads touch
    // neighbouring columns of a row in global memory
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
        int l, j;
        if (Op::col) { l = e % it.nl; j = e / it.nl; }
        else { l = e / f.L; j = e - l * f.L; }
        a[l * Ls + j] = op.load(cl, it.frame, it.line0 + l, j);
    }
    __syncthreads();
    float2 *r = lds_fft_any<Op::inverse>(a, b, it.nl, f, tw + f.tw_off);
    double acc = 0.0;
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
        int l, j;
        if (Op::col) { l = e % it.nl; j = e / it.nl; }
        else { l = e / f.L; j = e - l * f.L; }
        if constexpr (Op::rowsum)
            acc += (double)op.store(cl, it.frame, it.line0 + l, j, r[l * Ls + j]);
        else
            op.store(cl, it.frame, it.line0 + l, j, r[l * Ls + j]);
    }
    if constexpr (Op::rowsum) {
        __shared__ double red[kFftThreads / 64];
        const double tot_sum = block_sum_d_fft(acc, red);
        if (threadIdx.x == 0) op.gpart[blockIdx.x] = tot_sum;
    }
}

// Half-spectrum access with Hermitian symmetry: X is [P][P/2+1]; returns X(ky, kx)
// for any kx in [0, P).
// Branch-free (selects, one unconditional load) so that the loads of several
// calls can be in flight together.
__device__ __forceinline__ float2 half_get(const float2 *__restrict__ X, int P, int ky, int kx)
{
    const int H = P / 2 + 1;
    const bool lo = kx < H;
    const int ry = lo ? ky : (ky == 0 ? 0 : P - ky);
    const int rx = lo ? kx : P - kx;
    float2 v = X[(long long)ry * H + rx];
    v.y = lo ? v.y : -v.y;
    return v;
}

// ---- pass A: rows of the h window of each class (real -> half spectrum) ----
// Its launch carries extra work groups per class (when M > 0) that compute the
// per-evaluation factor tables alongside: 16 for up to four sources,
// more with more sources (the (1 + 4M) P entries each sum 17 Gaussian samples), so
// that the tables are not the launch's longest work groups.
__host__ __device__ inline int tab_blocks(int M) { return M <= 4 ? 16 : (M >= 32 ? 128 : 4 * M); }
__device__ void tables_part(const ClassFft &c, const float2 *__restrict__ tw, const float *__restrict__ params,
                            int N, int E, int M, float sigma, float2 *__restrict__ tab, int e0, int estep);
struct OpHRows {
    const float *h;
    int N;
    float2 *Th;
    int n_items, E, M;
    float sigma;
    float2 *tab;
    int *tick;  // optimiser step counter advanced by the launch (null: none)
    static constexpr bool extra = true;
    __device__ void run_extra(int xb, const ClassFft *classes, const float2 *tw) const
    {
        const int tb = tab_blocks(M);
        tables_part(classes[xb / tb], tw, h, N, E, M, sigma, tab, threadIdx.x + (xb % tb) * blockDim.x,
                    blockDim.x * tb);
    }
    static constexpr bool col = false;
    static constexpr bool rowsum = false;
    static constexpr bool inverse = false;
    __device__ const FftLen &len(const ClassFft &c) const { return c.fP; }
    __device__ float2 load(const ClassFft &c, int, int y, int x) const
    {
        return make_float2(x < c.F ? h[(long long)(c.o + y) * N + c.o + x] : 0.f, 0.f);
    }
    __device__ void store(const ClassFft &c, int, int y, int kx, float2 v) const
    {
        const int H = c.P / 2 + 1;
        if (kx < H) Th[c.th_off + (long long)y * H + kx] = v;
    }
};

// ---- pass B: columns -> H_hat[P][P/2+1] ----
struct OpHCols {
    const float2 *Th;
    float2 *Hh;
    static constexpr bool col = true;
    static constexpr bool rowsum = false;
    static constexpr bool inverse = false;
    __device__ const FftLen &len(const ClassFft &c) const { return c.fP; }
    __device__ float2 load(const ClassFft &c, int, int kx, int y) const
    {
        const int H = c.P / 2 + 1;
        return y < c.F ? Th[c.th_off + (long long)y * H + kx] : make_float2(0.f, 0.f);
    }
    __device__ void store(const ClassFft &c, int, int kx, int ky, float2 v) const
    {
        const int H = c.P / 2 + 1;
        Hh[c.hh_off + (long long)ky * H + kx] = v;
    }
};

// ---- set_frames: kernel spectra. Rows of kb, kb(y,x) = sum_{al,be<s} kt((y+al+kap)%P, (x+be+kap)%P)
struct OpKRows {
    const FrameFft *fr;
    const float *psf;
    int s;
    float2 *TS;
    static constexpr bool col = false;
    static constexpr bool rowsum = false;
    static constexpr bool inverse = false;
    __device__ const FftLen &len(const ClassFft &c) const { return c.fP; }
    __device__ float2 load(const ClassFft &c, int i, int y, int x) const
    {
        const FrameFft &f = fr[i];
        const int P = c.P, K = c.K, kap = K / 2;
        const float *k = psf + f.kern_off;
        float acc = 0.f;
        for (int al = 0; al < s; ++al) {
            const int v = (y + al + kap) % P;
            if (v >= K) continue;
            for (int be = 0; be < s; ++be) {
                const int u = (x + be + kap) % P;
                if (u < K) acc += k[v * K + u];
            }
        }
        return make_float2(acc, 0.f);
    }
    __device__ void store(const ClassFft &c, int i, int y, int kx, float2 v) const
    {
        const int H = c.P / 2 + 1;
        if (kx < H) TS[fr[i].t3_off + (long long)y * H + kx] = v;
    }
};

struct OpKCols {
    const FrameFft *fr;
    const float2 *TS;
    float2 *S;
    static constexpr bool col = true;
    static constexpr bool rowsum = false;
    static constexpr bool inverse = false;
    __device__ const FftLen &len(const ClassFft &c) const { return c.fP; }
    __device__ float2 load(const ClassFft &c, int i, int kx, int y) const
    {
        const int H = c.P / 2 + 1;
        return TS[fr[i].t3_off + (long long)y * H + kx];
    }
    __device__ void store(const ClassFft &c, int i, int kx, int ky, float2 v) const
    {
        const int H = c.P / 2 + 1;
        S[fr[i].s_off + (long long)ky * H + kx] = cscale(v, c.sscale);
    }
};

// ---- pass D: forward spectral product + alias fold + inverse along ky ----
struct OpFwdCols {
    const FrameFft *fr;
    const float2 *S;
    const float2 *Hh;
    const float2 *tab;
    const float *params;
    int N, E, M, s;
    float2 *T;
    const float2 *scene_spec;  // per-frame scene spectra (standalone operator) or NULL
    static constexpr bool col = true;
    static constexpr bool rowsum = false;
    static constexpr bool inverse = true;
    __device__ const FftLen &len(const ClassFft &c) const { return c.fQ; }
    // scene spectrum at K (any Kx in [0,P)): Gamma w(Ky) w(Kx) + H(K) + sum_k a g_y(Ky) g_x(Kx)
    __device__ float2 scene_hat(const ClassFft &c, int i, int Ky, int Kx) const
    {
        const int P = c.P;
        if (scene_spec) return half_get(scene_spec + fr[i].t3_off, P, Ky, Kx);
        const float2 *t = tab + c.tab_off;
        float2 v = half_get(Hh + c.hh_off, P, Ky, Kx);
        const float G = params[(long long)N * N + i];
        v = cadd(v, cscale(cmul(t[Ky], t[Kx]), G));
        const float *a = params + (long long)N * N + E + (long long)i * M;
        for (int k = 0; k < M; ++k) {
            const float2 *tk = t + (long long)(1 + 4 * k) * P;  // [gx | gy | dgx | dgy]
            v = cadd(v, cscale(cmul(tk[P + Ky], tk[Kx]), a[k]));
        }
        return v;
    }
    __device__ float2 load(const ClassFft &c, int i, int kx, int ky) const
    {
        const FrameFft &f = fr[i];
        const int P = c.P, Q = c.Q;
        const float2 *Si = S + f.s_off;
        float2 acc = make_float2(0.f, 0.f);
        for (int al = 0; al < s; ++al)
            for (int be = 0; be < s; ++be) {
                const int Ky = ky + al * Q, Kx = kx + be * Q;
                acc = cadd(acc, cmul(half_get(Si, P, Ky, Kx), scene_hat(c, i, Ky, Kx)));
            }
        return acc;
    }
    __device__ void store(const ClassFft &c, int i, int kx, int y, float2 v) const
    {
        const int H = c.Q / 2 + 1;
        if (y < c.n) T[fr[i].t_off + (long long)y * H + kx] = v;
    }
};

// ---- forward spectral product: M_hat_i(k) = sum over the s^2 aliases of
// S''_i(K) F_i(K), F_i = H + Gamma_i w x w + sum_k a_ik gy_k x gx_k (Eq. 9).
// One thread per output bin of a class, looping over a chunk of its frames, so
// the shared spectra of the bin's aliases are read once per chunk. ----
// MS > 0: the point-source spectra of the bin's aliases (M <= MS) are formed once
// per work item and kept in registers; MS = 0 reads the tables for every frame.
template <int S, int MS>
__global__ __launch_bounds__(kFftThreads) void k_spec_fwd(const SpecItem *__restrict__ items,
                                                          const ClassFft *__restrict__ classes,
                                                          const FrameFft *__restrict__ fr,
                                                          const int *__restrict__ cls_frames,
                                                          const float2 *__restrict__ Sp,
                                                          const float2 *__restrict__ Hh,
                                                          const float2 *__restrict__ tab,
                                                          const float *__restrict__ params, int N, int E, int M,
                                                          float2 *__restrict__ Mh)
{
    const SpecItem it = items[blockIdx.x];
    const ClassFft &c = classes[it.cls];
    const int P = c.P, Q = c.Q, HQ = Q / 2 + 1;
    const int bin = it.bin0 + threadIdx.x;
    if (bin >= Q * HQ) return;
    const int ky = bin / HQ, kx = bin - ky * HQ;
    const float2 *t = tab + c.tab_off;
    float2 hv[S * S], wv[S * S];
    int Kys[S], Kxs[S];
    #pragma unroll
    for (int a = 0; a < S; ++a) {
        Kys[a] = ky + a * Q;
        Kxs[a] = kx + a * Q;
    }
    #pragma unroll
    for (int a = 0; a < S; ++a)
        #pragma unroll
        for (int b = 0; b < S; ++b) {
            hv[a * S + b] = half_get(Hh + c.hh_off, P, Kys[a], Kxs[b]);
            wv[a * S + b] = cmul(t[Kys[a]], t[Kxs[b]]);
        }
    constexpr int MR = MS > 0 ? MS : 1;
    float2 rk[S * S][MR];
    if (MS > 0) {
        #pragma unroll
        for (int a = 0; a < S; ++a)
            #pragma unroll
            for (int b = 0; b < S; ++b)
                #pragma unroll
                for (int k = 0; k < MR; ++k) {
                    const float2 *tk = t + (long long)(1 + 4 * k) * P;  // [gx | gy | dgx | dgy]
                    rk[a * S + b][k] = k < M ? cmul(tk[P + Kys[a]], tk[Kxs[b]]) : make_float2(0.f, 0.f);
                }
    }
    // frames in groups of kFwdFrames: every load of a group is issued before its
    // arithmetic, so one memory round trip serves several frames
    constexpr int FG = kFwdFrames;
    for (int f0 = it.f0; f0 < it.f0 + it.nf; f0 += FG) {
        const int nfg = min(FG, it.f0 + it.nf - f0);
        float2 sv[FG][S * S];
        float Gv[FG], av[FG][MR];
        long long roff[FG];
        #pragma unroll
        for (int u = 0; u < FG; ++u) {
            if (u < nfg) {
                const int i = cls_frames[c.cf_off + f0 + u];
                const FrameFft &fi = fr[i];
                roff[u] = fi.r_off;
                Gv[u] = params[(long long)N * N + i];
                const float *ai = params + (long long)N * N + E + (long long)i * M;
                #pragma unroll
                for (int k = 0; k < MR; ++k) av[u][k] = (MS > 0 && k < M) ? ai[k] : 0.f;
                #pragma unroll
                for (int a = 0; a < S; ++a)
                    #pragma unroll
                    for (int b = 0; b < S; ++b) sv[u][a * S + b] = half_get(Sp + fi.s_off, P, Kys[a], Kxs[b]);
            }
        }
        if (MS > 0) {
            #pragma unroll
            for (int u = 0; u < FG; ++u) {
                if (u < nfg) {
                    float2 acc = make_float2(0.f, 0.f);
                    #pragma unroll
                    for (int a = 0; a < S; ++a)
                        #pragma unroll
                        for (int b = 0; b < S; ++b) {
                            float2 F = cadd(hv[a * S + b], cscale(wv[a * S + b], Gv[u]));
                            #pragma unroll
                            for (int k = 0; k < MR; ++k) F = cadd(F, cscale(rk[a * S + b][k], av[u][k]));
                            acc = cadd(acc, cmul(sv[u][a * S + b], F));
                        }
                    Mh[roff[u] + bin] = acc;
                }
            }
        } else {
            // many sources: source-major over the frame group, so each source's 1-D table
            // values are loaded once per group, not once per frame and alias (the sums per
            // frame and alias keep their order: H + Gamma W, then the sources in order)
            float2 F[FG][S * S];
            const float *ai[FG];
            #pragma unroll
            for (int u = 0; u < FG; ++u) {
                const int i = cls_frames[c.cf_off + f0 + (u < nfg ? u : 0)];
                ai[u] = params + (long long)N * N + E + (long long)i * M;
                #pragma unroll
                for (int ab = 0; ab < S * S; ++ab) F[u][ab] = cadd(hv[ab], cscale(wv[ab], Gv[u < nfg ? u : 0]));
            }
            for (int k = 0; k < M; ++k) {
                const float2 *tk = t + (long long)(1 + 4 * k) * P;  // [gx | gy | dgx | dgy]
                float2 ty[S], tx[S];
                #pragma unroll
                for (int a = 0; a < S; ++a) {
                    ty[a] = tk[P + Kys[a]];
                    tx[a] = tk[Kxs[a]];
                }
                float ak[FG];
                #pragma unroll
                for (int u = 0; u < FG; ++u) ak[u] = ai[u][k];
                #pragma unroll
                for (int a = 0; a < S; ++a)
                    #pragma unroll
                    for (int b = 0; b < S; ++b) {
                        const float2 R = cmul(ty[a], tx[b]);
                        #pragma unroll
                        for (int u = 0; u < FG; ++u) F[u][a * S + b] = cadd(F[u][a * S + b], cscale(R, ak[u]));
                    }
            }
            #pragma unroll
            for (int u = 0; u < FG; ++u) {
                if (u < nfg) {
                    float2 acc = make_float2(0.f, 0.f);
                    #pragma unroll
                    for (int ab = 0; ab < S * S; ++ab) acc = cadd(acc, cmul(sv[u][ab], F[u][ab]));
                    Mh[roff[u] + bin] = acc;
                }
            }
        }
    }
}

// ---- inverse along ky of M_hat -> rows of the model spectra ----
struct OpMCols {
    const FrameFft *fr;
    const float2 *Mh;
    float2 *T;
    static constexpr bool col = true;
    static constexpr bool rowsum = false;
    static constexpr bool inverse = true;
    __device__ const FftLen &len(const ClassFft &c) const { return c.fQ; }
    __device__ float2 load(const ClassFft &c, int i, int kx, int ky) const
    {
        const int H = c.Q / 2 + 1;
        return Mh[fr[i].r_off + (long long)ky * H + kx];
    }
    __device__ void store(const ClassFft &c, int i, int kx, int y, float2 v) const
    {
        const int H = c.Q / 2 + 1;
        if (y < c.n) T[fr[i].t_off + (long long)y * H + kx] = v;
    }
};

// ---- pass F: forward along ky of the rho row spectra -> rho_hat[Q][Q/2+1] ----
struct OpRhoCols {
    const FrameFft *fr;
    const float2 *T2;
    float2 *Rh;
    static constexpr bool col = true;
    static constexpr bool rowsum = false;
    static constexpr bool inverse = false;
    __device__ const FftLen &len(const ClassFft &c) const { return c.fQ; }
    __device__ float2 load(const ClassFft &c, int i, int kx, int y) const
    {
        const int H = c.Q / 2 + 1;
        return y < c.n ? T2[fr[i].t_off + (long long)y * H + kx] : make_float2(0.f, 0.f);
    }
    __device__ void store(const ClassFft &c, int i, int kx, int ky, float2 v) const
    {
        const int H = c.Q / 2 + 1;
        Rh[fr[i].r_off + (long long)ky * H + kx] = v;
    }
};

// ---- pass G: conj(S'') * rho_hat(K mod Q), inverse along Ky, crop rows < F ----
struct OpAdjCols {
    const FrameFft *fr;
    const float2 *S;
    const float2 *Rh;
    float2 *T3;
    static constexpr bool col = true;
    static constexpr bool rowsum = false;
    static constexpr bool inverse = true;
    __device__ const FftLen &len(const ClassFft &c) const { return c.fP; }
    __device__ float2 load(const ClassFft &c, int i, int Kx, int Ky) const
    {
        const FrameFft &f = fr[i];
        const int P = c.P, Q = c.Q, HP = P / 2 + 1;
        const float2 sv = S[f.s_off + (long long)Ky * HP + Kx];
        const int ky = Ky % Q, kx = Kx % Q;
        const float2 rv = half_get(Rh + f.r_off, Q, ky, kx);
        return cmulc(rv, sv);
    }
    __device__ void store(const ClassFft &c, int i, int Kx, int y, float2 v) const
    {
        const int H = c.P / 2 + 1;
        if (y < c.F) T3[fr[i].t3_off + (long long)y * H + Kx] = v;
    }
};

// ---- pass H: rows, Hermitian extension, inverse, crop x < F -> g_i ----
struct OpAdjRows {
    const FrameFft *fr;
    const float2 *T3;
    float *g;
    double *gpart;  // one partial sum of g per work group
    static constexpr bool col = false;
    static constexpr bool rowsum = true;  // per-group sum of g: the frame sums for Gamma
    static constexpr bool inverse = true;
    __device__ const FftLen &len(const ClassFft &c) const { return c.fP; }
    __device__ float2 load(const ClassFft &c, int i, int y, int Kx) const
    {
        const int P = c.P, H = P / 2 + 1;
        const float2 *row = T3 + fr[i].t3_off + (long long)y * H;
        return Kx < H ? row[Kx] : conjf2(row[P - Kx]);
    }
    __device__ float store(const ClassFft &c, int i, int y, int x, float2 v) const
    {
        if (x >= c.F) return 0.f;
        g[fr[i].fine_off + (long long)y * c.F + x] = v.x;
        return v.x;
    }
};

// ---- standalone adjoint: rows of a given residual -> T2 ----
struct OpResidRows {
    const FrameFft *fr;
    const float *resid;
    float2 *T2;
    static constexpr bool col = false;
    static constexpr bool rowsum = false;
    static constexpr bool inverse = false;
    __device__ const FftLen &len(const ClassFft &c) const { return c.fQ; }
    __device__ float2 load(const ClassFft &c, int i, int y, int x) const
    {
        return make_float2(x < c.n ? resid[fr[i].data_off + (long long)y * c.n + x] : 0.f, 0.f);
    }
    __device__ void store(const ClassFft &c, int i, int y, int kx, float2 v) const
    {
        const int H = c.Q / 2 + 1;
        if (kx < H) T2[fr[i].t_off + (long long)y * H + kx] = v;
    }
};

// ---- standalone forward: spectrum of a given scene, rows then columns in place ----
struct OpSceneRows {
    const FrameFft *fr;
    const float *scene;
    float2 *T3;
    static constexpr bool col = false;
    static constexpr bool rowsum = false;
    static constexpr bool inverse = false;
    __device__ const FftLen &len(const ClassFft &c) const { return c.fP; }
    __device__ float2 load(const ClassFft &c, int i, int y, int x) const
    {
        return make_float2(x < c.F ? scene[fr[i].fine_off + (long long)y * c.F + x] : 0.f, 0.f);
    }
    __device__ void store(const ClassFft &c, int i, int y, int kx, float2 v) const
    {
        const int H = c.P / 2 + 1;
        if (kx < H) T3[fr[i].t3_off + (long long)y * H + kx] = v;
    }
};

struct OpSceneCols {  // every column is read and written by the same work group
    const FrameFft *fr;
    float2 *T3;
    static constexpr bool col = true;
    static constexpr bool rowsum = false;
    static constexpr bool inverse = false;
    __device__ const FftLen &len(const ClassFft &c) const { return c.fP; }
    __device__ float2 load(const ClassFft &c, int i, int kx, int y) const
    {
        const int H = c.P / 2 + 1;
        return y < c.F ? T3[fr[i].t3_off + (long long)y * H + kx] : make_float2(0.f, 0.f);
    }
    __device__ void store(const ClassFft &c, int i, int kx, int ky, float2 v) const
    {
        const int H = c.P / 2 + 1;
        T3[fr[i].t3_off + (long long)ky * H + kx] = v;
    }
};

// ---- pass E: model rows (inverse), residual and chi-square, rho rows (forward) ----
__global__ __launch_bounds__(kFftThreads) void k_fwd_rows(const LineItem *__restrict__ items,
                                                          const ClassFft *__restrict__ classes,
                                                          const FrameFft *__restrict__ fr,
                                                          const float2 *__restrict__ tw,
                                                          const float2 *__restrict__ T,
                                                          const float *__restrict__ data,
                                                          const float *__restrict__ invvar,
                                                          float2 *__restrict__ T2, float *model,
                                                          double *__restrict__ part_chi)
{
    extern __shared__ float2 sm[];
    __shared__ double red[kFftThreads / 64];
    const LineItem it = items[blockIdx.x];
    const ClassFft &c = classes[it.cls];
    const FrameFft &f = fr[it.frame];
    const FftLen &fl = c.fQ;
    const int Q = c.Q, H = Q / 2 + 1, n = c.n, Ls = Q + 1;
    // the rows are real: two of them share one complex transform (row 2p in the real
    // part, row 2p+1 in the imaginary part; a missing partner row is zero)
    const int np = (it.nl + 1) / 2;
    float2 *a = sm;
    float2 *b = sm + np * Ls;
    const int tot = np * Q;
    // the data and weights of this thread's first kRowPre residual elements, loaded
    // now so that they arrive during the inverse transform
    constexpr int kRowPre = 4;
    float pd[kRowPre][2], pw[kRowPre][2];
    #pragma unroll
    for (int k = 0; k < kRowPre; ++k) {
        const int e = threadIdx.x + k * blockDim.x;
        const int l = e / Q, x = e - l * Q;
        #pragma unroll
        for (int u = 0; u < 2; ++u) {
            // (no loads at all when only the model is written: data may be NULL then)
            const bool ok = !model && e < tot && x < n && 2 * l + u < it.nl;
            const long long idx = f.data_off + (long long)(it.line0 + 2 * l + u) * n + x;
            pd[k][u] = ok ? data[idx] : 0.f;
            pw[k][u] = ok ? invvar[idx] : 0.f;
        }
    }
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
        const int l = e / Q, kx = e - l * Q;
        const float2 *row0 = T + f.t_off + (long long)(it.line0 + 2 * l) * H;
        const float2 x0 = kx < H ? row0[kx] : conjf2(row0[Q - kx]);
        float2 x1 = make_float2(0.f, 0.f);
        if (2 * l + 1 < it.nl) {
            const float2 *row1 = row0 + H;
            x1 = kx < H ? row1[kx] : conjf2(row1[Q - kx]);
        }
        a[l * Ls + kx] = make_float2(x0.x - x1.y, x0.y + x1.x);  // X0 + i X1
    }
    __syncthreads();
    float2 *r = lds_fft_any<true>(a, b, np, fl, tw + fl.tw_off);
    float2 *o = (r == a) ? b : a;
    double chi = 0.0;
    for (int k = 0, e = threadIdx.x; e < tot; ++k, e += blockDim.x) {
        const int l = e / Q, x = e - l * Q;
        float v[2] = {0.f, 0.f};
        if (x < n) {
            const float2 z = r[l * Ls + x];
            const float mm[2] = {z.x, z.y};
            #pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (2 * l + u >= it.nl) break;
                const int y = it.line0 + 2 * l + u;
                const long long idx = f.data_off + (long long)y * n + x;
                if (model) {
                    model[idx] = mm[u];
                } else {
                    float dv = 0.f, w = 0.f;
                    #pragma unroll
                    for (int kk = 0; kk < kRowPre; ++kk)
                        if (kk == k) {
                            dv = pd[kk][u];
                            w = pw[kk][u];
                        }
                    if (k >= kRowPre) {
                        dv = data[idx];
                        w = invvar[idx];
                    }
                    const float res = mm[u] - dv;
                    v[u] = w * res;
                    chi += 0.5 * (double)w * (double)res * (double)res;
                }
            }
        }
        o[l * Ls + x] = make_float2(v[0], v[1]);
    }
    const double tchi = block_sum_d_fft(chi, red);
    if (threadIdx.x == 0 && part_chi) part_chi[blockIdx.x] = tchi;
    if (model) return;
    __syncthreads();
    float2 *q = lds_fft_any<false>(o, r, np, fl, tw + fl.tw_off);
    // split the pair's spectrum Z into the two rows' half spectra:
    // X0 = (Z(k) + conj Z(Q-k)) / 2, X1 = (Z(k) - conj Z(Q-k)) / (2i)
    const int toth = np * H;
    for (int e = threadIdx.x; e < toth; e += blockDim.x) {
        const int l = e / H, kx = e - l * H;
        const float2 zk = q[l * Ls + kx];
        const float2 zc = conjf2(q[l * Ls + (kx == 0 ? 0 : Q - kx)]);
        float2 *dst = T2 + f.t_off + (long long)(it.line0 + 2 * l) * H + kx;
        dst[0] = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y));
        if (2 * l + 1 < it.nl) dst[H] = make_float2(0.5f * (zk.y - zc.y), -0.5f * (zk.x - zc.x));
    }
}

// ---- one-launch forward of a frame whose Q-grid spectra fit in LDS ----
// A work group per frame runs the whole forward of the loss in LDS: the
// spectral product and alias fold into the Q x (Q/2+1) model spectrum (stored
// column-major), the inverse transform along ky, the Hermitian rows and the
// inverse along x (the model m, Eq. 8), the weighted residual rho and its
// chi-square partial (Eq. 10), then the forward transforms of rho along x and
// along y, and writes rho_hat [Q][Q/2+1] to memory for the adjoint. Two LDS
// planes of max(Q/2+1, (n+1)/2) lines of stride Q+1 alternate as FFT source and
// scratch; the Q-point twiddles and the class's factor tables sit behind them.
template <int S, int MS>
__global__ __launch_bounds__(kFusedThreads) void k_frame_fwd(const FusedItem *__restrict__ items,
                                                             const ClassFft *__restrict__ classes,
                                                             const float2 *__restrict__ tw,
                                                             const float2 *__restrict__ Sp,
                                                             const float2 *__restrict__ Hh,
                                                             const float2 *__restrict__ tab,
                                                             const float *__restrict__ params, int N, int E, int M,
                                                             const float *__restrict__ data,
                                                             const float *__restrict__ invvar,
                                                             float2 *__restrict__ Rh, double *__restrict__ part_chi,
                                                             DensePiece dp)
{
    extern __shared__ float2 sm[];
    __shared__ double red[kFusedThreads / 64];
    if (dense_piece_run(dp, sm, red)) return;  // a starlet-prior job carried by this launch
    const FusedItem &f = items[blockIdx.x];
    const int i = f.frame;
    const FftLen &fl = classes[f.cls].fQ;
    const float2 *twQ = tw + f.tw_off;
    const int P = f.P, Q = f.Q, HQ = Q / 2 + 1, n = f.n, Ls = Q + 1;
    const int rows = fused_plane_lines(Q, n);
    // one plane transformed in place (frames whose two planes exceed the LDS), else two
    // (not with 5-8 sources held in registers: that form keeps its registers for them)
    const bool ip = MS != 8 && f.inplace != 0;
    float2 *A = sm, *B = ip ? sm : sm + rows * Ls;
    float2 *twl = sm + (ip ? 1 : 2) * rows * Ls;
    float2 *t = twl + Q;
    {
        // the twiddles and the tables: all of a thread's loads issued before its LDS writes
        const float2 *tg = tab + f.tab_off;
        const int nt = (1 + 4 * M) * P;
        constexpr int kTabBatch = 4;
        for (int e = threadIdx.x; e < Q; e += blockDim.x) twl[e] = twQ[e];
        for (int e0 = threadIdx.x; e0 < nt; e0 += kTabBatch * kFusedThreads) {
            float2 v[kTabBatch];
            #pragma unroll
            for (int u = 0; u < kTabBatch; ++u) v[u] = tg[min(e0 + u * kFusedThreads, nt - 1)];
            #pragma unroll
            for (int u = 0; u < kTabBatch; ++u)
                if (e0 + u * kFusedThreads < nt) t[e0 + u * kFusedThreads] = v[u];
        }
    }
    twQ = twl;
    const float2 *Si = Sp + f.s_off;
    const float2 *Hc = Hh + f.hh_off;
    const float G = params[(long long)N * N + i];
    const float *ai = params + (long long)N * N + E + (long long)i * M;

    // lanes over columns kx, row groups over ky (no index divisions in the loops)
    // (threads packed over the HQ columns: column lane = tid % HQ, row group tid / HQ)
    const int RGF = kFusedThreads / HQ;
    const int Q0L = Q <= 64 ? 64 : 128;  // lanes along a row of Q values
    // this thread's data and weights for the residual (its first kPreRows row pairs),
    // loaded now so that they arrive during the transforms
    constexpr int kPreRows = S <= 2 ? 4 : 0;  // (s = 3 keeps its registers for the aliases)
    const int n2 = (n + 1) / 2;
    float pre[kPreRows > 0 ? kPreRows : 1][4];
    {
        const int x = threadIdx.x % Q0L;
        #pragma unroll
        for (int k = 0; k < kPreRows; ++k) {
            const int yp = threadIdx.x / Q0L + k * (kFusedThreads / Q0L);
            const bool va = x < n && yp < n2, vb = va && 2 * yp + 1 < n;
            const long long ia = f.data_off + (long long)(va ? 2 * yp : 0) * n + (va ? x : 0);
            const long long ib = vb ? ia + n : ia;
            pre[k][0] = data[ia];
            pre[k][1] = invvar[ia];
            pre[k][2] = data[ib];
            pre[k][3] = invvar[ib];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x % HQ, rg = threadIdx.x / HQ;
    const bool colw = rg < RGF;  // this thread works in the column-wise loops
    // model spectrum, column-major: A[kx][ky]
    // (with MS > 0 sources at most, the column factors a_k gx_k(Kx) stay in registers)
    constexpr int MR = MS > 0 ? MS : 1;
    if (colw) {
        const int kx = lane;
        const int HP = P / 2 + 1;
        float2 wxG[S], px[S][MR];
        // half-spectrum access of the column aliases Kx_b (Hermitian fold for Kx >= P/2+1)
        bool lob[S];
        int rxb[S];
        #pragma unroll
        for (int b = 0; b < S; ++b) {
            const int Kx = kx + b * Q;
            lob[b] = Kx < HP;
            rxb[b] = lob[b] ? Kx : P - Kx;
            wxG[b] = cscale(t[Kx], G);
            #pragma unroll
            for (int k = 0; k < MR; ++k)
                px[b][k] = (MS > 0 && k < M) ? cscale(t[(1 + 4 * k) * P + Kx], ai[k]) : make_float2(0.f, 0.f);
        }
        // the s^2 alias terms of the model spectrum at (kx, ky), from the loaded bins
        auto load_row = [&](int ky, float2 (&hv)[S][S], float2 (&sv)[S][S]) {
            #pragma unroll
            for (int a = 0; a < S; ++a) {
                const int Ky = ky + a * Q;
                const int rlo = Ky * HP, rhi = (Ky == 0 ? 0 : P - Ky) * HP;
                #pragma unroll
                for (int b = 0; b < S; ++b) {
                    const int hidx = (lob[b] ? rlo : rhi) + rxb[b];
                    hv[a][b] = Hc[hidx];
                    sv[a][b] = Si[hidx];
                }
            }
        };
        auto row_sum = [&](int ky, const float2 (&hv)[S][S], const float2 (&sv)[S][S]) {
            float2 acc = make_float2(0.f, 0.f);
            #pragma unroll
            for (int a = 0; a < S; ++a) {
                const int Ky = ky + a * Q;
                const float2 wy = t[Ky];
                float2 gy[MR];
                #pragma unroll
                for (int k = 0; k < MR; ++k)
                    gy[k] = (MS > 0 && k < M) ? t[(1 + 4 * k) * P + P + Ky] : make_float2(0.f, 0.f);
                #pragma unroll
                for (int b = 0; b < S; ++b) {
                    const int Kx = kx + b * Q;
                    float2 h = hv[a][b], sk = sv[a][b];
                    if (!lob[b]) {
                        h.y = -h.y;
                        sk.y = -sk.y;
                    }
                    float2 F = cadd(h, cmul(wy, wxG[b]));
                    if (MS > 0) {
                        #pragma unroll
                        for (int k = 0; k < MR; ++k) {
                            F.x = fmaf(gy[k].x, px[b][k].x, fmaf(-gy[k].y, px[b][k].y, F.x));
                            F.y = fmaf(gy[k].x, px[b][k].y, fmaf(gy[k].y, px[b][k].x, F.y));
                        }
                    } else {
                        for (int k = 0; k < M; ++k) {
                            const float2 *tk = t + (1 + 4 * k) * P;  // [gx | gy | dgx | dgy]
                            F = cadd(F, cscale(cmul(tk[P + Ky], tk[Kx]), ai[k]));
                        }
                    }
                    acc = cadd(acc, cmul(sk, F));
                }
            }
            return acc;
        };
        if (S <= 2 && MS != 8 && Q >= kProdPairQ) {
            // long columns: the loads of two rows in flight together (the loop is a chain
            // of memory round trips otherwise)
            for (int ky0 = rg; ky0 < Q; ky0 += 2 * RGF) {
                const int ky1 = ky0 + RGF;
                float2 h0[S][S], s0[S][S], h1[S][S], s1[S][S];
                load_row(ky0, h0, s0);
                load_row(ky1 < Q ? ky1 : ky0, h1, s1);  // (past the end: row ky0 again, unused)
                A[kx * Ls + ky0] = row_sum(ky0, h0, s0);
                if (ky1 < Q) A[kx * Ls + ky1] = row_sum(ky1, h1, s1);
            }
        } else {
            for (int ky = rg; ky < Q; ky += RGF) {
                float2 h0[S][S], s0[S][S];
                load_row(ky, h0, s0);
                A[kx * Ls + ky] = row_sum(ky, h0, s0);
            }
        }
    }
    __syncthreads();
    float2 *r = lds_fft_plane<true>(A, B, HQ, fl, twQ, ip);  // along ky
    float2 *o = (r == A) ? B : A;
    // Rows in pairs (two real rows per complex transform): the inverse of
    // Z = X_2p + i X_2p+1, X_y the Hermitian rows of the column results, is
    // x_2p + i x_2p+1; a missing second row (odd n) is zero.
    auto pair_in = [&](int yp, int kx) {
        const int ya = 2 * yp, yb = 2 * yp + 1;
        const bool lo = kx < HQ;
        const int col = lo ? kx : Q - kx;
        float2 xa = r[col * Ls + ya];
        float2 xb = yb < n ? r[col * Ls + yb] : make_float2(0.f, 0.f);
        if (!lo) {
            xa.y = -xa.y;
            xb.y = -xb.y;
        }
        return make_float2(xa.x - xb.y, xa.y + xb.x);  // xa + i xb
    };
    if (!ip) {
        for (int yp = threadIdx.x / Q0L; yp < n2; yp += kFusedThreads / Q0L)
            for (int kx = threadIdx.x % Q0L; kx < Q; kx += Q0L) o[yp * Ls + kx] = pair_in(yp, kx);
    } else {
        // in place: every value read before any is overwritten (Q in (64, 192]: 128
        // lanes along a row, 8 row pairs per sweep, at most 97 pairs)
        constexpr int IY = (192 / 2 + 1 + 7) / 8;
        float2 hold[IY][2];
        #pragma unroll
        for (int iy = 0; iy < IY; ++iy)
            #pragma unroll
            for (int ix = 0; ix < 2; ++ix) {
                const int yp = threadIdx.x / 128 + iy * 8, kx = threadIdx.x % 128 + ix * 128;
                hold[iy][ix] = (yp < n2 && kx < Q) ? pair_in(yp, kx) : make_float2(0.f, 0.f);
            }
        __syncthreads();
        #pragma unroll
        for (int iy = 0; iy < IY; ++iy)
            #pragma unroll
            for (int ix = 0; ix < 2; ++ix) {
                const int yp = threadIdx.x / 128 + iy * 8, kx = threadIdx.x % 128 + ix * 128;
                if (yp < n2 && kx < Q) o[yp * Ls + kx] = hold[iy][ix];
            }
    }
    __syncthreads();
    r = lds_fft_plane<true>(o, r, n2, fl, twQ, ip);  // along x: model rows 2p, 2p+1 in the real, imaginary parts
    o = (r == A) ? B : A;
    double chi = 0.0;
    for (int k = 0, yp = threadIdx.x / Q0L; yp < n2; ++k, yp += kFusedThreads / Q0L)
        for (int x = threadIdx.x % Q0L; x < Q; x += Q0L) {
            float va = 0.f, vb = 0.f;
            if (x < n) {
                const float2 mv = r[yp * Ls + x];
                const long long ia = f.data_off + (long long)(2 * yp) * n + x;
                // prefetched for the first kPreRows row pairs of the first column sweep
                const bool have = k < kPreRows && x < Q0L;
                float da = 0.f, wa = 0.f, db = 0.f, wb = 0.f;
                #pragma unroll
                for (int kk = 0; kk < kPreRows; ++kk)
                    if (kk == k) {
                        da = pre[kk][0];
                        wa = pre[kk][1];
                        db = pre[kk][2];
                        wb = pre[kk][3];
                    }
                if (!have) {
                    da = data[ia];
                    wa = invvar[ia];
                    if (2 * yp + 1 < n) {
                        db = data[ia + n];
                        wb = invvar[ia + n];
                    }
                }
                const float ra = mv.x - da;
                va = wa * ra;
                chi += 0.5 * (double)wa * (double)ra * (double)ra;
                if (2 * yp + 1 < n) {
                    const float rb = mv.y - db;
                    vb = wb * rb;
                    chi += 0.5 * (double)wb * (double)rb * (double)rb;
                }
            }
            o[yp * Ls + x] = make_float2(va, vb);  // rho rows 2p + i (2p+1)
        }
    // the frame's chi-square: wave sums in LDS across the barrier the transform needs
    // anyway, then thread 0 adds them (in wave order) while the others transform
    #pragma unroll
    for (int off = 32; off > 0; off >>= 1) chi += __shfl_xor(chi, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = chi;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tchi = 0.0;
        #pragma unroll
        for (int w = 0; w < kFusedThreads / 64; ++w) tchi += red[w];
        part_chi[blockIdx.x] = tchi;
    }
    r = lds_fft_plane<false>(o, r, n2, fl, twQ, ip);  // rho pairs along x
    o = (r == A) ? B : A;
    // split each pair's spectrum Z into the two rows' (Hermitian) spectra,
    // R_a = (Z(k) + conj Z(-k)) / 2 and R_b = (Z(k) - conj Z(-k)) / 2i, and lay the
    // half spectra out column-major with zero rows y >= n
    const int km = lane == 0 ? 0 : Q - lane;
    auto split_at = [&](int y) {
        float2 v = make_float2(0.f, 0.f);
        if (y < n) {
            const float2 z = r[(y >> 1) * Ls + lane], zm = r[(y >> 1) * Ls + km];
            v = (y & 1) ? make_float2(0.5f * (z.y + zm.y), 0.5f * (zm.x - z.x))
                        : make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
        }
        return v;
    };
    if (!ip) {
        if (colw)
            for (int y = rg; y < Q; y += RGF) o[lane * Ls + y] = split_at(y);
    } else {
        // in place: at most 192 rows over at least 10 row groups (Q/2+1 <= 97 lanes)
        constexpr int IS = (192 + 9) / 10;
        float2 hold[IS];
        #pragma unroll
        for (int i2 = 0; i2 < IS; ++i2) {
            const int y = rg + i2 * RGF;
            hold[i2] = (colw && y < Q) ? split_at(y) : make_float2(0.f, 0.f);
        }
        __syncthreads();
        #pragma unroll
        for (int i2 = 0; i2 < IS; ++i2) {
            const int y = rg + i2 * RGF;
            if (colw && y < Q) o[lane * Ls + y] = hold[i2];
        }
    }
    __syncthreads();
    r = lds_fft_plane<false>(o, r, HQ, fl, twQ, ip);  // along y
    float2 *R = Rh + f.r_off;
    if (colw)
        for (int ky = rg; ky < Q; ky += RGF) R[ky * HQ + lane] = r[lane * Ls + ky];
}

// ---- per-eval tables: window indicator and point-source factors ----
// tab[c]: [w (P) | for each source k: gx, gy, dgx, dgy (P each)], the 1-D DFTs
// over the frame of the window indicator, of g(x + o - c) (r = g(dx) g(dy),
// Eq. 9) and of g(x + o - c)(x + o - c)/sigma^2 (its derivative in c).
__device__ void tables_part(const ClassFft &c, const float2 *__restrict__ tw, const float *__restrict__ params,
                            int N, int E, int M, float sigma, float2 *__restrict__ tab, int e0, int estep)
{
    const int P = c.P;
    const float2 *twP = tw + c.fP.tw_off;
    float2 *t = tab + c.tab_off;
    const float *cc = params + (long long)N * N + E + (long long)E * M;
    const float inv2s2 = 1.0f / (2.0f * sigma * sigma), invs2 = 1.0f / (sigma * sigma);
    const float norm = 1.0f / (2.50662827463100050f * sigma);  // 1/(sqrt(2 pi) sigma)
    const int nent = (1 + 4 * M) * P;
    for (int e = e0; e < nent; e += estep) {
        const int which = e / P, K = e - which * P;
        if (which == 0) continue;  // the window factor is static, written at plan creation
        const int k = (which - 1) / 4, part = (which - 1) % 4;
        const float ctr = cc[2 * k + (part & 1)];
        const bool deriv = part >= 2;
        const int lo = max(0, (int)ceilf(ctr - c.o - kGaussRadius));
        const int hi = min(c.F - 1, (int)floorf(ctr - c.o + kGaussRadius));
        float2 acc = make_float2(0.f, 0.f);
        // twiddle index K x mod P, advanced by K per sample (K < P)
        int kx = lo <= hi ? (int)(((long long)K * lo) % P) : 0;
        for (int x = lo; x <= hi; ++x) {
            const float d = (float)(x + c.o) - ctr;
            float g = norm * expf(-d * d * inv2s2);
            if (deriv) g *= d * invs2;
            const float2 w = twP[kx];
            acc.x += g * w.x;
            acc.y += g * w.y;
            kx += K;
            if (kx >= P) kx -= P;
        }
        t[e] = acc;
    }
}

// ---- adjoint in the frequency domain ----
// For bin K of a class's half spectrum and each frame i of a chunk:
//   G_i(K) = conj(S''_i(K)) rho_hat_i(K mod Q),
// summed over the chunk (the spectrum of the chunk's contribution to dL/dh), and
// the frame's dot products <g_i, x> = sum over the full spectrum of G_i conj(X_hat)
// (Parseval; half spectrum with weight 2 off the Kx = 0 and P/2 columns) for x the
// window indicator (dGamma_i), r_k (da_ik) and r_k (X - c_k)/sigma^2 (dc_k, x and y).
// Those spectra are products ty(Ky) tx(Kx) of 1-D tables, so each dot product is
//   sum_Kx wgt(Kx) Re( conj(tx(Kx)) V_ty(Kx) ),  V_ty(Kx) = sum_Ky G(Ky, Kx) conj(ty(Ky)),
// with one column sum V per y-table (window, gy_k, dgy_k). A block takes a chunk of
// FC frames and the rows of a range of representatives y (rows congruent to y or
// -y modulo Q, see below), SB sources per pass (one when M <= 1; four, or eight with
// 2-frame chunks and more than four sources, otherwise); a thread owns columns Kx (lanes)
// and every RG-th row of the range, accumulates V over its rows, folds it with the
// x-tables, and the block reduces the dot products once per group of SB sources through
// LDS. Each pass reads the chunk's spectra again, so fewer, wider passes save reads.
// The per-block partials are summed per frame (and the chunk spectra over chunks)
// by k_adj_sums.
template <int FC, int SB>
__global__ __launch_bounds__(kFftThreads) void k_spec_adj(const AdjItem *__restrict__ items,
                                                          const float2 *__restrict__ Sp,
                                                          const float2 *__restrict__ Rh,
                                                          const float2 *__restrict__ tab, int M, int maxpb,
                                                          float2 *__restrict__ Gp, double *__restrict__ part)
{
    constexpr int NY = 1 + 2 * SB, NQ = 1 + 3 * SB;
    // rows of a thread whose loads are issued together: about 12-16 loads in flight
    constexpr int RB = FC >= 8 ? 1 : (FC >= 4 ? 2 : kAdjRB);
    static_assert(FC <= kAdjMaxFrames, "chunk larger than the work items hold");
    constexpr int kRow = kFftThreads + 8;  // padded LDS rows of per-thread partials
    // rows of per-thread partials reduced per pass (LDS kept small for occupancy)
    constexpr int NRED = FC * NQ < 32 ? FC * NQ : 32;
    static_assert(FC * NQ <= 2 * 32, "two reduction passes of 32 quantities");
    __shared__ float red[NRED * kRow];
    const AdjItem &it = items[blockIdx.x];
    const int P = it.P, Q = it.Q, HP = P / 2 + 1;
    const int y0 = it.y0, y1 = it.y1, pb = it.pb;
    // The block's rows: for each representative y in [y0, y1) (0 <= y <= Q/2) the rows
    // Ky = y + aQ and Ky = (Q - y) + aQ, a < s, i.e. every row whose rho_hat row is y or
    // its mirror Q - y; local row i: representative i / 2s, a = (i % 2s) / 2, mirrored
    // when i is odd (no mirrored rows for y = 0 and y = Q/2, which are their own
    // mirrors). So the s^2 reads of each rho_hat value fall in one block.
    const int S2 = 2 * (P / Q);
    const int nloc = S2 * (y1 - y0);
    auto row_of = [&](int li, bool &valid) {
        const int y = y0 + li / S2, j = li % S2;
        const bool mir = j & 1;
        valid = !(mir && (y == 0 || 2 * y == Q));
        return (mir && valid ? Q - y : y) + (j >> 1) * Q;
    };
    // lanes over columns, row groups over rows
    const int CX = adj_lanes(HP), RG = kFftThreads / CX;
    const int lane = threadIdx.x % CX, rg = threadIdx.x / CX;
    const float2 *t = tab + it.tab_off;
    const int Q3 = 1 + 3 * M;
    float2 *gout = Gp + it.gout;
    const int HQ = Q / 2 + 1;
    __shared__ float2 tys[NY * kAdjMaxRows];  // y-tables of the block's rows
    for (int k0 = 0; k0 < max(M, 1); k0 += SB) {
        const int nk = min(SB, M - k0);  // sources of this group (may be 0 when M = 0)
        const bool first = (k0 == 0);
        // y-tables of this group for the block's rows: window, gy_k, dgy_k
        for (int e = threadIdx.x; e < NY * nloc; e += kFftThreads) {
            const int u = e / nloc, r = e - u * nloc;
            bool valid;
            const int Ky = row_of(r, valid);
            float2 v = make_float2(0.f, 0.f);
            if (valid) {
                if (u == 0) v = t[Ky];
                else if (u <= SB) { if (u - 1 < nk) v = t[(1 + 4 * (k0 + u - 1)) * P + P + Ky]; }
                else if (u - 1 - SB < nk) v = t[(1 + 4 * (k0 + u - 1 - SB)) * P + 3 * P + Ky];
            }
            tys[u * kAdjMaxRows + r] = v;
        }
        __syncthreads();
        // spectra of the chunk's frames (a slot past the chunk's frames reads its first
        // frame again; its product is discarded)
        int fid[FC];
        long long soff[FC], roff[FC];
        #pragma unroll
        for (int f = 0; f < FC; ++f) {
            fid[f] = it.fid[f];
            soff[f] = it.soff[f];
            roff[f] = it.roff[f];
        }
        float dot[FC][NQ];
        #pragma unroll
        for (int f = 0; f < FC; ++f)
            #pragma unroll
            for (int q = 0; q < NQ; ++q) dot[f][q] = 0.f;
        for (int Kx = lane; Kx < HP; Kx += CX) {
            float2 V[FC][NY];
            #pragma unroll
            for (int f = 0; f < FC; ++f)
                #pragma unroll
                for (int u = 0; u < NY; ++u) V[f][u] = make_float2(0.f, 0.f);
            // rho_hat is indexed by K mod Q (Kx < P/2 + 1 <= 2Q, so one subtraction)
            const int kxq = Kx >= Q ? Kx - Q : Kx;
            const bool lo = kxq < HQ;
            const int rx = lo ? kxq : Q - kxq;
            const float cj = lo ? 1.f : -1.f;
            // RB rows of this thread at a time: every load of the batch is issued
            // before the first is used (a row group is whole waves, so the row tests are uniform)
            for (int ib = rg; ib < nloc; ib += RB * RG) {
                float2 sv[RB][FC], rv[RB][FC];
                int kyb[RB];
                bool okb[RB];
                #pragma unroll
                for (int b = 0; b < RB; ++b) {
                    const int li = ib + b * RG;
                    bool valid;
                    const int Ky = row_of(li < nloc ? li : ib, valid);  // (past the range: a row loaded again)
                    okb[b] = valid && li < nloc;  // (an invalid slot still names a row in range)
                    kyb[b] = Ky;
                    const int ryq = Ky % Q;
                    const long long bin = (long long)Ky * HP + Kx;
                    const int ridx = (lo ? ryq : (ryq == 0 ? 0 : Q - ryq)) * HQ + rx;
                    #pragma unroll
                    for (int f = 0; f < FC; ++f) {
                        sv[b][f] = Sp[soff[f] + bin];
                        rv[b][f] = Rh[roff[f] + ridx];
                    }
                }
                #pragma unroll
                for (int b = 0; b < RB; ++b) {
                    if (!okb[b]) continue;
                    const int Ky = kyb[b], li = ib + b * RG;
                    float2 ty[NY];
                    #pragma unroll
                    for (int u = 0; u < NY; ++u) ty[u] = tys[u * kAdjMaxRows + li];
                    float2 gsum = make_float2(0.f, 0.f);
                    #pragma unroll
                    for (int f = 0; f < FC; ++f) {
                        // a missing frame's product is replaced by zero with a select (a branch
                        // here would let the compiler sink the loads above back to their use;
                        // a product with zero would let a non-finite value through)
                        const bool on = f < it.nf;
                        const float2 z = make_float2(0.f, 0.f);
                        float2 r = on ? rv[b][f] : z;
                        r.y *= cj;
                        const float2 G = cmulc(r, on ? sv[b][f] : z);
                        gsum = cadd(gsum, G);
                        #pragma unroll
                        for (int u = 0; u < NY; ++u) V[f][u] = cadd(V[f][u], cmulc(G, ty[u]));
                    }
                    if (first) gout[(long long)Ky * HP + Kx] = gsum;
                }
            }
            // fold with the x-tables of this column
            const float wgt = (Kx == 0 || 2 * Kx == P) ? 1.f : 2.f;
            float2 tx[1 + 2 * SB];
            tx[0] = t[Kx];
            #pragma unroll
            for (int k = 0; k < SB; ++k) {
                const float2 *tk = t + (1 + 4 * (k0 + k)) * P;
                tx[1 + k] = k < nk ? tk[Kx] : make_float2(0.f, 0.f);           // gx_k
                tx[1 + SB + k] = k < nk ? tk[2 * P + Kx] : make_float2(0.f, 0.f);  // dgx_k
            }
            #pragma unroll
            for (int f = 0; f < FC; ++f) {
                // Re(conj(tx) V) = tx.x V.x + tx.y V.y
                dot[f][0] += wgt * (tx[0].x * V[f][0].x + tx[0].y * V[f][0].y);
                #pragma unroll
                for (int k = 0; k < SB; ++k) {
                    const float2 vy = V[f][1 + k], vdy = V[f][1 + SB + k];
                    dot[f][1 + k] += wgt * (tx[1 + k].x * vy.x + tx[1 + k].y * vy.y);                  // da
                    dot[f][1 + SB + k] += wgt * (tx[1 + SB + k].x * vy.x + tx[1 + SB + k].y * vy.y);   // dcx
                    dot[f][1 + 2 * SB + k] += wgt * (tx[1 + k].x * vdy.x + tx[1 + k].y * vdy.y);       // dcy
                }
            }
        }
        // block reduction of FC x NQ quantities in passes of 32 rows
        for (int p0 = 0; p0 < FC * NQ; p0 += NRED) {
            #pragma unroll
            for (int v = 0; v < FC * NQ; ++v)
                if (v >= p0 && v < p0 + NRED) red[(v - p0) * kRow + threadIdx.x] = dot[v / NQ][v % NQ];
            __syncthreads();
            const int pr = threadIdx.x >> 3, j = threadIdx.x & 7, v = p0 + pr;
            double acc = 0.0;
            if (pr < NRED && v < FC * NQ) {
                const float *rr = red + pr * kRow;
                #pragma unroll 8
                for (int u = j; u < kFftThreads; u += 8) acc += (double)rr[u];
            }
            acc += __shfl_xor(acc, 1, 8);
            acc += __shfl_xor(acc, 2, 8);
            acc += __shfl_xor(acc, 4, 8);
            if (j == 0 && pr < NRED && v < FC * NQ) {
                const int f = v / NQ, ql = v % NQ;
                // local quantity -> global index: window, da_k, dcx_k, dcy_k
                int q = -1;
                if (ql == 0) q = first ? 0 : -1;
                else if (ql <= SB) q = (ql - 1 < nk) ? 1 + k0 + (ql - 1) : -1;
                else if (ql <= 2 * SB) q = (ql - 1 - SB < nk) ? 1 + M + k0 + (ql - 1 - SB) : -1;
                else q = (ql - 1 - 2 * SB < nk) ? 1 + 2 * M + k0 + (ql - 1 - 2 * SB) : -1;
                if (f < it.nf && q >= 0) part[((long long)fid[f] * maxpb + pb) * Q3 + q] = acc;
            }
            __syncthreads();
        }
    }
}

// Two independent reductions in one launch, each in a fixed order:
//  blocks [0, gblocks): the frame-chunk spectra of each class summed into the
//    first chunk's slot: a block takes kSumBins consecutive bins and kSumParts
//    threads per bin, each summing its own run of consecutive chunks (every load
//    of the run in flight together), the runs then added in order;
//  the remaining blocks: per-frame sums of the per-block dot products,
//    fsum[i][q], one thread per (frame, quantity).
__global__ __launch_bounds__(256) void k_adj_sums(const ClassFft *__restrict__ classes, int ncls, int gblocks,
                                                  const FrameFft *__restrict__ fr, int E, int M, int maxpb,
                                                  float2 *__restrict__ Gp, const double *__restrict__ part,
                                                  double *__restrict__ fsum)
{
    static_assert(kSumBins * kSumParts == 256, "one thread per (bin, run)");
    if ((int)blockIdx.x < gblocks) {
        __shared__ float2 runs[kSumParts][kSumBins];
        const int lane = threadIdx.x % kSumBins, q = threadIdx.x / kSumBins;
        int g = blockIdx.x * kSumBins + lane;
        float2 *gp = nullptr;
        int ngch = 0;
        long long nbins = 0;
        for (int ci = 0; ci < ncls; ++ci) {
            const ClassFft &c = classes[ci];
            if (c.direct) continue;  // classes on the direct algorithm have no spectra here
            const int nb = c.P * (c.P / 2 + 1);
            if (g < nb) {
                gp = Gp + c.gp_off + g;
                ngch = c.ngch;
                nbins = nb;
                break;
            }
            g -= nb;
        }
        float2 acc = make_float2(0.f, 0.f);
        const int per = (ngch + kSumParts - 1) / kSumParts, c0 = q * per, c1 = min(ngch, c0 + per);
        for (int b0 = c0; b0 < c1; b0 += kSumBatch) {
            float2 v[kSumBatch];
            #pragma unroll
            for (int u = 0; u < kSumBatch; ++u) v[u] = gp[(long long)min(b0 + u, c1 - 1) * nbins];
            #pragma unroll
            for (int u = 0; u < kSumBatch; ++u)
                if (b0 + u < c1) acc = cadd(acc, v[u]);
        }
        runs[q][lane] = acc;
        __syncthreads();
        if (q == 0 && gp) {
            #pragma unroll
            for (int r = 1; r < kSumParts; ++r) acc = cadd(acc, runs[r][lane]);
            gp[0] = acc;
        }
        return;
    }
    const int Q3 = 1 + 3 * M;
    const int idx = (blockIdx.x - gblocks) * blockDim.x + threadIdx.x;
    if (idx >= E * Q3) return;
    const int i = idx / Q3, q = idx - i * Q3;
    if (classes[fr[i].cls].direct) return;  // its sums come from the direct path
    const int npb = classes[fr[i].cls].nrr;
    const double *pp = part + (long long)i * maxpb * Q3 + q;
    double acc = 0.0;
    #pragma unroll 8
    for (int b = 0; b < npb; ++b) acc += pp[(long long)b * Q3];
    fsum[idx] = acc;
}

// ---- dL/dh of each class: inverse columns of the summed spectra, crop rows < F ----
struct OpGCols {
    const float2 *Gp;
    float2 *Th;
    static constexpr bool col = true;
    static constexpr bool rowsum = false;
    static constexpr bool inverse = true;
    __device__ const FftLen &len(const ClassFft &c) const { return c.fP; }
    __device__ float2 load(const ClassFft &c, int, int Kx, int Ky) const
    {
        return Gp[c.gp_off + (long long)Ky * (c.P / 2 + 1) + Kx];  // chunk sum, in the first slot
    }
    __device__ void store(const ClassFft &c, int, int Kx, int y, float2 v) const
    {
        const int H = c.P / 2 + 1;
        if (y < c.F) Th[c.th_off + (long long)y * H + Kx] = v;
    }
};

struct OpGRows {
    const float2 *Th;
    float *hcls;
    static constexpr bool col = false;
    static constexpr bool rowsum = false;
    static constexpr bool inverse = true;
    __device__ const FftLen &len(const ClassFft &c) const { return c.fP; }
    __device__ float2 load(const ClassFft &c, int, int y, int Kx) const
    {
        const int P = c.P, H = P / 2 + 1;
        const float2 *row = Th + c.th_off + (long long)y * H;
        return Kx < H ? row[Kx] : conjf2(row[P - Kx]);
    }
    __device__ void store(const ClassFft &c, int, int y, int x, float2 v) const
    {
        if (x < c.F) hcls[c.hc_off + (long long)y * c.F + x] = v.x;
    }
};

// dL/dh of a single class whose window is the whole grid, written by the inverse
// rows themselves: the prior's gradient plus the row value, and the update of h
// in a step; one extra work group does the evaluation's small reductions.
struct OpGRowsFin {
    const float2 *Th;
    const float *prior;
    FinalArgs fin;
    int n_items;
    int *tick;  // the line launch's own counter hook: unused (null)
    DenseStar psum;  // with psum.U set, the prior's gradient is summed from its per-level planes here
    static constexpr bool extra = true;
    static constexpr bool col = false;
    static constexpr bool rowsum = false;
    static constexpr bool inverse = true;
    __device__ void run_extra(int xb, const ClassFft *, const float2 *) const
    {
        if (xb == 0) finalize_small_body<kFftThreads>(fin);
    }
    __device__ const FftLen &len(const ClassFft &c) const { return c.fP; }
    __device__ float2 load(const ClassFft &c, int, int y, int Kx) const
    {
        const int P = c.P, H = P / 2 + 1;
        const float2 *row = Th + c.th_off + (long long)y * H;
        return Kx < H ? row[Kx] : conjf2(row[P - Kx]);
    }
    __device__ void store(const ClassFft &c, int, int y, int x, float2 v) const
    {
        if (x >= c.F) return;
        const long long pix = (long long)y * fin.N + x;
        float bc1, bc2;
        adam_bias(fin.adam, bc1, bc2);
        const float pg = psum.U ? (float)dense_prior_at(psum, 0, pix) : (prior ? prior[pix] : 0.f);
        finalize_h_pixel(fin.adam, bc1, bc2, pix, pg + v.x, fin.grad);
    }
};

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------

// LDS bytes a carried prior pass needs
static size_t piece_lds(const DensePiece &p)
{
    if (p.pass < 0) return 0;
    if (p.pass == 0 || p.pass == 2) return dense_lds_xr(p.d.N, p.d.J, p.d.rx);
    return p.pass == 3 ? dense_lds_d(p.d.J) : dense_lds_y(p.d.J);
}

// n_main work groups of line groups (and extras), then the carried pass's jobs
template <class Op>
static hipError_t run_lines(hipStream_t st, const LinePass &lp, const ClassFft *classes, const float2 *tw,
                            const Op &op, int n_main = -1, DensePiece *piece = nullptr)
{
    if (n_main < 0) n_main = lp.n_items;
    DensePiece dp;
    size_t lds = lp.lds_bytes;
    if (piece && piece->pass >= 0) {
        dp = *piece;
        dp.first = n_main;
        lds = std::max(lds, piece_lds(dp));
    }
    const int grid = n_main + (dp.pass >= 0 ? dp.jobs : 0);
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_lines<Op>), dim3(grid), dim3(kFftThreads), lds, st, lp.items, classes, tw, op, dp);
    return hipGetLastError();
}

hipError_t fft_prep_kernels(hipStream_t st, const FftPlanDev &d, const float *psf, int s)
{
    hipError_t e = run_lines(st, d.krows, d.classes, d.tw, OpKRows{d.frames, psf, s, d.T3});
    if (e != hipSuccess) return e;
    return run_lines(st, d.kcols, d.classes, d.tw, OpKCols{d.frames, d.T3, d.S});
}

hipError_t fft_spectra(hipStream_t st, const FftPlanDev &d, const float *params, int N, int E, int M,
                       float sigma, int *tick, DensePiece *pa, DensePiece *pb)
{
    // rows of the h windows, with the factor tables in extra work groups
    const int extra = M > 0 ? d.n_classes * tab_blocks(M) : 0;
    const OpHRows op{params, N, d.Th, d.hrows.n_items, E, M, sigma, d.tab, tick};
    hipError_t e = run_lines(st, d.hrows, d.classes, d.tw, op, d.hrows.n_items + extra, pa);
    if (e != hipSuccess) return e;
    return run_lines(st, d.hcols, d.classes, d.tw, OpHCols{d.Th, d.Hh}, -1, pb);
}

hipError_t fft_spec_fwd(hipStream_t st, const FftPlanDev &d, const float *params, int N, int E, int M, int s,
                        bool lg)
{
    const int ns = lg ? d.n_spec_lg : d.n_spec;
    const SpecItem *items = lg ? d.spec_lg : d.spec;
    if (ns <= 0) return hipSuccess;
#define SPEC_FWD(SS, MS)                                                                                     \
    hipLaunchKernelGGL((k_spec_fwd<SS, MS>), dim3(ns), dim3(kFftThreads), 0, st, items, d.classes,            \
                       d.frames, d.cls_frames, d.S, d.Hh, d.tab, params, N, E, M, d.Rh)
    if (s == 1) {
        if (M <= 16) SPEC_FWD(1, 16); else SPEC_FWD(1, 0);
    } else if (s == 2) {
        if (M <= 4) SPEC_FWD(2, 4); else if (M <= 8) SPEC_FWD(2, 8); else SPEC_FWD(2, 0);
    } else {
        if (M <= 2) SPEC_FWD(3, 2); else SPEC_FWD(3, 0);
    }
#undef SPEC_FWD
    return hipGetLastError();
}

hipError_t fft_model_cols(hipStream_t st, const FftPlanDev &d)
{
    return run_lines(st, d.fcols, d.classes, d.tw, OpMCols{d.frames, d.Rh, d.T});
}

hipError_t fft_model_rows(hipStream_t st, const FftPlanDev &d, const float *data, const float *invvar,
                          double *part_chi, float *model)
{
    if (d.frows.n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fwd_rows, dim3(d.frows.n_items), dim3(kFftThreads), d.frows.lds_bytes, st, d.frows.items,
                       d.classes, d.frames, d.tw, d.T, data, invvar, d.T2, model, part_chi);
    return hipGetLastError();
}

hipError_t fft_scene_model(hipStream_t st, const FftPlanDev &d, const float *scene, int s, float *model)
{
    // the kernel spectra are indexed like the row passes over P lines
    hipError_t e = run_lines(st, d.srows, d.classes, d.tw, OpSceneRows{d.frames, scene, d.T3});
    if (e != hipSuccess) return e;
    e = run_lines(st, d.scols, d.classes, d.tw, OpSceneCols{d.frames, d.T3});
    if (e != hipSuccess) return e;
    e = run_lines(st, d.fcols, d.classes, d.tw,
                  OpFwdCols{d.frames, d.S, d.Hh, d.tab, nullptr, 0, 0, 0, s, d.T, d.T3});
    if (e != hipSuccess) return e;
    if (d.frows.n_items > 0) {
        hipLaunchKernelGGL(k_fwd_rows, dim3(d.frows.n_items), dim3(kFftThreads), d.frows.lds_bytes, st,
                           d.frows.items, d.classes, d.frames, d.tw, d.T, nullptr, nullptr, d.T2, model,
                           nullptr);
        e = hipGetLastError();
    }
    return e;
}

hipError_t fft_xf_forward(hipStream_t st, const FftPlanDev &d, const float *scene, int s, const float *data,
                          const float *invvar, double *part_chi)
{
    hipError_t e = run_lines(st, d.srows_x, d.classes, d.tw, OpSceneRows{d.frames, scene, d.T3});
    if (e != hipSuccess) return e;
    e = run_lines(st, d.scols_x, d.classes, d.tw, OpSceneCols{d.frames, d.T3});
    if (e != hipSuccess) return e;
    e = run_lines(st, d.fcols_x, d.classes, d.tw, OpFwdCols{d.frames, d.S, d.Hh, d.tab, nullptr, 0, 0, 0, s, d.T, d.T3});
    if (e != hipSuccess || d.frows_x.n_items <= 0) return e;
    hipLaunchKernelGGL(k_fwd_rows, dim3(d.frows_x.n_items), dim3(kFftThreads), d.frows_x.lds_bytes, st,
                       d.frows_x.items, d.classes, d.frames, d.tw, d.T, data, invvar, d.T2, nullptr, part_chi);
    return hipGetLastError();
}

hipError_t fft_xf_adjoint(hipStream_t st, const FftPlanDev &d, float *g)
{
    hipError_t e = run_lines(st, d.rcols_x, d.classes, d.tw, OpRhoCols{d.frames, d.T2, d.Rh});
    if (e == hipSuccess) e = run_lines(st, d.acols_x, d.classes, d.tw, OpAdjCols{d.frames, d.S, d.Rh, d.T3});
    if (e == hipSuccess) e = run_lines(st, d.arows_x, d.classes, d.tw, OpAdjRows{d.frames, d.T3, g, d.gpart_x});
    return e;
}

hipError_t fft_resid_rows(hipStream_t st, const FftPlanDev &d, const float *resid)
{
    return run_lines(st, d.rrows, d.classes, d.tw, OpResidRows{d.frames, resid, d.T2});
}

hipError_t fft_fused_fwd(hipStream_t st, const FftPlanDev &d, const float *params, int N, int E, int M, int s,
                         const float *data, const float *invvar, double *part_chi, DensePiece *pc)
{
    if (d.n_fused <= 0) return hipSuccess;
    DensePiece dp;
    size_t lds = d.fused_lds;
    if (pc && pc->pass >= 0) {
        dp = *pc;
        dp.first = d.n_fused;
        lds = std::max(lds, piece_lds(dp));
    }
    const int grid = d.n_fused + (dp.pass >= 0 ? dp.jobs : 0);
#define FUSED_FWD(SS, MS)                                                                                     \
    hipLaunchKernelGGL((k_frame_fwd<SS, MS>), dim3(grid), dim3(kFusedThreads), lds, st, d.fused, d.classes,      \
                       d.tw, d.S, d.Hh, d.tab, params, N, E, M, data, invvar, d.Rh, part_chi, dp)
#define FUSED_FWD_M(SS)                       \
    if (M <= 4) FUSED_FWD(SS, 4);             \
    else if (M <= 8) FUSED_FWD(SS, 8);        \
    else FUSED_FWD(SS, 0)
    if (s == 1) { FUSED_FWD_M(1); }
    else if (s == 2) { FUSED_FWD_M(2); }
    else { FUSED_FWD_M(3); }
#undef FUSED_FWD_M
#undef FUSED_FWD
    return hipGetLastError();
}

hipError_t fft_model_cols_lg(hipStream_t st, const FftPlanDev &d)
{
    return run_lines(st, d.fcols_lg, d.classes, d.tw, OpMCols{d.frames, d.Rh, d.T});
}

hipError_t fft_model_rows_lg(hipStream_t st, const FftPlanDev &d, const float *data, const float *invvar,
                             double *part_chi)
{
    if (d.frows_lg.n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fwd_rows, dim3(d.frows_lg.n_items), dim3(kFftThreads), d.frows_lg.lds_bytes, st,
                       d.frows_lg.items, d.classes, d.frames, d.tw, d.T, data, invvar, d.T2, nullptr, part_chi);
    return hipGetLastError();
}

hipError_t fft_rho_cols_lg(hipStream_t st, const FftPlanDev &d)
{
    return run_lines(st, d.rcols_lg, d.classes, d.tw, OpRhoCols{d.frames, d.T2, d.Rh});
}

hipError_t fft_rho_cols(hipStream_t st, const FftPlanDev &d)
{
    return run_lines(st, d.rcols, d.classes, d.tw, OpRhoCols{d.frames, d.T2, d.Rh});
}

hipError_t fft_adj_cols(hipStream_t st, const FftPlanDev &d)
{
    return run_lines(st, d.acols, d.classes, d.tw, OpAdjCols{d.frames, d.S, d.Rh, d.T3});
}

hipError_t fft_adj_rows(hipStream_t st, const FftPlanDev &d, float *g)
{
    return run_lines(st, d.arows, d.classes, d.tw, OpAdjRows{d.frames, d.T3, g, d.gpart});
}

hipError_t fft_spec_adj(hipStream_t st, const FftPlanDev &d, int M)
{
    if (d.n_aspec == 0) return hipSuccess;
    const dim3 g(d.n_aspec), b(kFftThreads);
#define SPEC_ADJ(FC, SB)                                                                               \
    hipLaunchKernelGGL((k_spec_adj<FC, SB>), g, b, 0, st, d.aspec, d.S, d.Rh, d.tab, M, d.maxpb, d.Gp, \
                       d.apart)
    if (M <= 1) {
        switch (d.adj_fc) {
        case 2: SPEC_ADJ(2, 1); break;
        case 4: SPEC_ADJ(4, 1); break;
        case 8: SPEC_ADJ(8, 1); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (d.adj_fc) {
        case 1: SPEC_ADJ(1, kAdjSBOne); break;
        case 2:
            if (M > kAdjSB)
                SPEC_ADJ(2, kAdjSBWide);
            else
                SPEC_ADJ(2, kAdjSB);
            break;
        case 4: SPEC_ADJ(4, kAdjSB); break;
        default: return hipErrorInvalidValue;
        }
    }
#undef SPEC_ADJ
    return hipGetLastError();
}

hipError_t fft_adj_sums(hipStream_t st, const FftPlanDev &d, int M, double *fsum)
{
    const int gblocks = (int)((d.total_bins + kSumBins - 1) / kSumBins);
    const int fblocks = (d.n_frames * (1 + 3 * M) + 255) / 256;
    if (gblocks + fblocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_sums, dim3(gblocks + fblocks), dim3(256), 0, st, d.classes, d.n_classes, gblocks,
                       d.frames, d.n_frames, M, d.maxpb, d.Gp, d.apart, fsum);
    return hipGetLastError();
}

hipError_t fft_grad_h_cols(hipStream_t st, const FftPlanDev &d, DensePiece *pd)
{
    return run_lines(st, d.gcols, d.classes, d.tw, OpGCols{d.Gp, d.Th}, -1, pd);
}

hipError_t fft_grad_h_rows_final(hipStream_t st, const FftPlanDev &d, const float *prior, const FinalArgs &fin,
                                 const DenseStar *psum)
{
    const OpGRowsFin op{d.Th, prior, fin, d.grows.n_items, nullptr, psum ? *psum : DenseStar()};
    return run_lines(st, d.grows, d.classes, d.tw, op, d.grows.n_items + 1);
}

hipError_t fft_grad_h_inverse(hipStream_t st, const FftPlanDev &d, DensePiece *pd)
{
    hipError_t e = run_lines(st, d.gcols, d.classes, d.tw, OpGCols{d.Gp, d.Th}, -1, pd);
    if (e != hipSuccess) return e;
    return run_lines(st, d.grows, d.classes, d.tw, OpGRows{d.Th, d.hcls});
}

hipError_t fft_adjoint(hipStream_t st, const FftPlanDev &d, float *g)
{
    hipError_t e = fft_rho_cols(st, d);
    if (e == hipSuccess) e = fft_adj_cols(st, d);
    if (e == hipSuccess) e = fft_adj_rows(st, d, g);
    return e;
}

}  // namespace starred
