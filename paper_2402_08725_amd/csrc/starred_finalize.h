// The final small reductions of a loss+gradient evaluation (chi-square and L1
// totals, dL/dGamma, dL/da, dL/dc) and the optimiser update of those parameters,
// as a work-group body shared by the launches that carry it.
#pragma once

#include "starred_internal.h"

namespace starred {

struct FinalArgs {
    int E = 0, M = 0, N = 0;
    int n_chi = 0, n_l1 = 0;
    const double *part_chi = nullptr, *part_l1 = nullptr;
    const double *fsum = nullptr;  // [E][1+3M] per-frame sums
    const float *params = nullptr;
    float *grad = nullptr;
    double *loss = nullptr;
    const int *gcsr_off = nullptr, *gcsr_item = nullptr;  // optional CSR of dL/dGamma partials
    const double *gpart = nullptr;
    int *tick = nullptr;           // step counter advanced here (null: none)
    AdamDev adam;                  // update of Gamma, a, c (params null: none)
    const double *pts = nullptr;   // point-source prior's shares (3M) or null
};

__device__ __forceinline__ void adam_bias(const AdamDev &adam, float &bc1, float &bc2)
{
    bc1 = bc2 = 1.f;
    if (adam.params) {
        const float t = (float)(*adam.d_t);
        bc1 = 1.f - powf(adam.beta1, t);
        bc2 = 1.f - powf(adam.beta2, t);
    }
}

// Deterministic sum over the work group of one double per thread (a fixed
// shuffle tree per wave, then the waves in order); every thread gets the total.
template <int NT>
__device__ __forceinline__ double group_sum(double v, double *sh)
{
    #pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();  // sh may still be read by the previous sum
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double t = 0.0;
    #pragma unroll
    for (int w = 0; w < NT / 64; ++w) t += sh[w];
    return t;
}

// One work group of NT threads. Each reduced quantity is summed by the whole group:
// thread t takes the items t, t + NT, ... (their loads independent, so they are in
// flight together), then the fixed-order group sum.
// loss[0] = sum chi partials, loss[1] = sum L1 partials, loss[2] = total.
template <int NT>
__device__ void finalize_small_body(const FinalArgs &a)
{
    __shared__ double sums[2];
    __shared__ double gsh[NT / 64];
    const int E = a.E, M = a.M;
    const long long NN = (long long)a.N * a.N;
    const int stride = 1 + 3 * M;
    if (a.tick && threadIdx.x == 0) *a.tick += 1;  // the update that follows reads it
    const float *pa = a.params + NN + E;
    for (int r = 0; r < 2; ++r) {
        double acc = 0.0;
        if (r == 0) {
            for (int i = threadIdx.x; i < a.n_chi; i += NT) acc += a.part_chi[i];
        } else {
            for (int i = threadIdx.x; i < a.n_l1; i += NT) acc += a.part_l1[i];
        }
        acc = group_sum<NT>(acc, gsh);
        if (threadIdx.x == 0) sums[r] = acc;
    }
    // dL/dc_k = sum_i a_ik <g_i, dr_k/dc> (plus the point-source prior's share pts[3k+1+axis])
    const int nq = a.grad ? 2 * M : 0;
    if (nq <= 4) {
        // few sources (and often many frames): one whole-group sum per quantity
        for (int q = 0; q < nq; ++q) {
            const int k = q >> 1, axis = q & 1;
            double acc = 0.0;
            for (int i = threadIdx.x; i < E; i += NT)
                acc += (double)pa[(long long)i * M + k] * a.fsum[(long long)i * stride + 1 + (1 + axis) * M + k];
            acc = group_sum<NT>(acc, gsh);
            if (threadIdx.x == 0) {
                if (a.pts) acc += a.pts[3 * k + 1 + axis];
                a.grad[NN + E + (long long)E * M + q] = (float)acc;
            }
        }
    } else {
        // many sources: the 2M sums side by side, L lanes per sum (each lane takes frames
        // l, l + L, ... in order, then a fixed butterfly over the L lanes), so that they
        // cost a pass or two rather than one group sum each
        int L = 64;
        while (L > 8 && L * nq > NT) L >>= 1;
        for (int q0 = 0; q0 < nq; q0 += NT / L) {
            const int q = q0 + threadIdx.x / L, l = threadIdx.x % L;
            double acc = 0.0;
            if (q < nq) {
                const int k = q >> 1, axis = q & 1;
                for (int i = l; i < E; i += L)
                    acc += (double)pa[(long long)i * M + k] * a.fsum[(long long)i * stride + 1 + (1 + axis) * M + k];
            }
            for (int off = L >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (q < nq && l == 0) {
                if (a.pts) acc += a.pts[3 * (q >> 1) + 1 + (q & 1)];
                a.grad[NN + E + (long long)E * M + q] = (float)acc;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && a.loss) {
        a.loss[0] = sums[0];
        a.loss[1] = sums[1];
        a.loss[2] = sums[0] + sums[1];
    }
    if (!a.grad) return;
    float *gG = a.grad + NN, *ga = gG + E;
    for (int i = threadIdx.x; i < E; i += NT) {
        if (a.gcsr_off) {
            double acc = 0.0;
            for (int q = a.gcsr_off[i]; q < a.gcsr_off[i + 1]; ++q) acc += a.gpart[a.gcsr_item[q]];
            gG[i] = (float)acc;
        } else {
            gG[i] = (float)a.fsum[(long long)i * stride];
        }
    }
    for (long long e = threadIdx.x; e < (long long)E * M; e += NT) {
        const long long i = e / M, k = e - i * M;
        ga[e] = (float)(a.fsum[i * stride + 1 + k] + (a.pts ? a.pts[3 * k] : 0.0));
    }
    const AdamDev &ad = a.adam;
    if (!ad.params) return;
    float bc1, bc2;
    adam_bias(ad, bc1, bc2);
    // Gamma, a and c after their gradients (written above by this group) are final;
    // the a values read for dL/dc were taken before this point
    __syncthreads();
    const long long e1 = NN + E, e2 = e1 + (long long)E * M, e3 = e2 + 2LL * M;
    for (long long e = NN + threadIdx.x; e < e3; e += NT) {
        const float lr = e < e1 ? ad.lr[1] : (e < e2 ? ad.lr[2] : ad.lr[3]);
        float pi = ad.params[e], mi = ad.m[e], vi = ad.v[e];
        adam_update(pi, mi, vi, a.grad[e], lr, ad.beta1, ad.beta2, bc1, bc2, ad.eps, ad.rule == 1, ad.eps_root);
        ad.m[e] = mi;
        ad.v[e] = vi;
        ad.params[e] = pi;
    }
}

// dL/dh at one pixel from its value and the update of h there (step mode)
__device__ __forceinline__ void finalize_h_pixel(const AdamDev &ad, float bc1, float bc2, long long pix, float g,
                                                 float *grad)
{
    grad[pix] = g;
    if (ad.params) {
        float pi = ad.params[pix], mi = ad.m[pix], vi = ad.v[pix];
        adam_update(pi, mi, vi, g, ad.lr[0], ad.beta1, ad.beta2, bc1, bc2, ad.eps, ad.rule == 1, ad.eps_root);
        ad.m[pix] = mi;
        ad.v[pix] = vi;
        ad.params[pix] = pi;
    }
}

}  // namespace starred
