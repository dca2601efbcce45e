// fft.hpp -- in-LDS complex FFTs for gfx950 workgroups.
//
// Mixed-radix (4, 2, 3) Stockham autosort: stage with radix R after sub-transforms
// of size Ns reads x[j + r*(n/R)], multiplies input r by w_n^{(j mod Ns) r n/(Ns R)},
// does an R-point DFT and writes x[(j - j mod Ns) R + (j mod Ns) + r Ns].  Each
// stage is done in place: every thread loads its butterflies into registers,
// the workgroup synchronises, then stores.  `nseq` sequences of the same length
// at stride `ld` (complex elements) are transformed together.  Twiddles come
// from a precomputed table w_n^e = e^{-2 pi i e/n} (FP64-computed, stored FP32).
// Forward = sign -1, unnormalised; inverse = sign +1, unnormalised.
#pragma once

#include <hip/hip_runtime.h>

#include "pat_internal.hpp"

namespace pat {

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b)  // a * conj(b)
{
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -i (inv = false) or +i (inv = true)
__device__ __forceinline__ float2 mul_mi(float2 a, bool inv)
{
    return inv ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// q / d and q % d for 0 <= q < 2^22 with a float reciprocal and one correction step
__device__ __forceinline__ void fdivmod(int q, int d, float rcp, int& quo, int& rem)
{
    int t = (int)((float)q * rcp);
    int r = q - t * d;
    if (r < 0) { t -= 1; r += d; }
    else if (r >= d) { t += 1; r -= d; }
    quo = t;
    rem = r;
}

template <int R>
__device__ __forceinline__ void butterfly(float2 (&v)[R], bool inv)
{
    if constexpr (R == 2) {
        float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        float2 t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        float2 m = mul_mi(t3, inv);  // -i t3 (forward)
        v[1] = cadd(t1, m);
        v[3] = csub(t1, m);
    } else {  // R == 3
        const float s3 = 0.86602540378443864676f;
        float2 s = cadd(v[1], v[2]), df = csub(v[1], v[2]);
        float2 t = make_float2(v[0].x - 0.5f * s.x, v[0].y - 0.5f * s.y);
        v[0] = cadd(v[0], s);
        float2 m = mul_mi(cscale(df, s3), inv);  // -i (sqrt3/2)(a1 - a2) (forward)
        v[1] = cadd(t, m);
        v[2] = csub(t, m);
    }
}

template <int R, int MAXB>
__device__ __forceinline__ void fft_stage(float2* x, int ld, int nseq, int n, int Ns,
                                          const float2* __restrict__ tw, bool inv)
{
    const int nb = n / R;
    const int total = nb * nseq;
    const int tstride = n / (Ns * R);
    const float rcp_nb = 1.0f / (float)nb;
    const float rcp_ns = 1.0f / (float)Ns;
    float2 v[MAXB][R];
    int dst[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int q = threadIdx.x + i * blockDim.x;
        dst[i] = -1;
        if (q < total) {
            int f, j, jq, k;
            fdivmod(q, nb, rcp_nb, f, j);
            fdivmod(j, Ns, rcp_ns, jq, k);
            const float2* xs = x + f * ld;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = xs[j + r * nb];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w = tw[k * r * tstride];
                if (inv) w.y = -w.y;
                v[i][r] = cmul(v[i][r], w);
            }
            butterfly<R>(v[i], inv);
            dst[i] = f * ld + jq * Ns * R + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        if (dst[i] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) x[dst[i] + r * Ns] = v[i][r];
        }
    }
    __syncthreads();
}

// Transform `nseq` sequences in LDS (x[f*ld .. f*ld + n)), in place.
// Requires nseq * n / radix <= blockDim.x * MAXB for every stage radix.
// Must be reached by every thread of the workgroup (contains barriers).
template <int MAXB>
__device__ void fft_lds(float2* x, int ld, int nseq, const FftDev& d, const float2* __restrict__ twall,
                        bool inv)
{
    const float2* tw = twall + d.tw;
    int Ns = 1;
    for (int s = 0; s < d.nst; ++s) {
        const int R = d.rad[s];
        if (R == 4) fft_stage<4, MAXB>(x, ld, nseq, d.n, Ns, tw, inv);
        else if (R == 2) fft_stage<2, MAXB>(x, ld, nseq, d.n, Ns, tw, inv);
        else fft_stage<3, MAXB>(x, ld, nseq, d.n, Ns, tw, inv);
        Ns *= R;
    }
}

// Largest number of butterflies one stage of length n has per sequence.
__host__ __device__ inline int fft_max_butterflies(const FftDev& d)
{
    int minr = 4;
    for (int s = 0; s < d.nst; ++s) minr = d.rad[s] < minr ? d.rad[s] : minr;
    return d.n / minr;
}

}  // namespace pat
