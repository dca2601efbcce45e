// fft.hpp -- in-LDS complex FFTs for gfx950 workgroups.
//
// Mixed-radix (8, 4, 2, 3) Stockham autosort: stage with radix R after sub-transforms
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
    } else if constexpr (R == 8) {
        // X[k] = E[k] + W8^k O[k], X[k+4] = E[k] - W8^k O[k]; E, O = 4-point DFTs of even/odd inputs
        float2 e[4] = {v[0], v[2], v[4], v[6]};
        float2 o[4] = {v[1], v[3], v[5], v[7]};
        butterfly<4>(e, inv);
        butterfly<4>(o, inv);
        const float r2 = 0.70710678118654752440f;
        // W8^1 = (1 - i)/sqrt2, W8^2 = -i, W8^3 = (-1 - i)/sqrt2 (conjugates for the inverse)
        const float2 o1 = inv ? make_float2(r2 * (o[1].x - o[1].y), r2 * (o[1].x + o[1].y))
                              : make_float2(r2 * (o[1].x + o[1].y), r2 * (o[1].y - o[1].x));
        const float2 o2 = mul_mi(o[2], inv);
        const float2 o3 = inv ? make_float2(-r2 * (o[3].x + o[3].y), r2 * (o[3].x - o[3].y))
                              : make_float2(r2 * (o[3].y - o[3].x), -r2 * (o[3].x + o[3].y));
        v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);   v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);   v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);   v[7] = csub(e[3], o3);
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

// Twiddles w_n^e = e^{-2 pi i e / n} from a two-level table in LDS:
// w^e = lo[e & 63] * hi[e >> 6] (lo: 64 entries, hi: ceil(n/64) entries).
// With sh = 1 the table of length 2n serves length n (w_n^e = w_2n^{2e}).
struct TwLds {
    const float2* lo;
    const float2* hi;
    int sh;
    __device__ __forceinline__ float2 operator()(int e) const
    {
        e <<= sh;
        return cmul(lo[e & 63], hi[e >> 6]);
    }
};

// Number of float2 slots tw_lds_build needs for length n.
__host__ __device__ inline int tw_lds_slots(int n) { return 64 + (n + 63) / 64; }

// Fill the two-level table of length d.n at `dst` from the global full table.
// Caller synchronises before use.
__device__ __forceinline__ TwLds tw_lds_build(float2* dst, const FftDev& d, const float2* __restrict__ twall)
{
    const float2* tw = twall + d.tw;
    const int nhi = (d.n + 63) / 64;
    for (int e = threadIdx.x; e < 64 + nhi; e += blockDim.x) {
        int idx = e < 64 ? e : 64 * (e - 64);
        while (idx >= d.n) idx -= d.n;
        dst[e] = tw[idx];
    }
    return TwLds{dst, dst + 64, 0};
}

// One Stockham stage of radix R on the sequence `xs` (length n), done by the
// `tps` threads with local index u (butterflies j = u, u + tps, ...).
template <int R, int MAXB>
__device__ __forceinline__ void fft_stage(float2* xs, bool active, int u, int tps, int n, int Ns,
                                          const TwLds& tw, bool inv)
{
    const int nb = n / R;
    const int tstride = n / (Ns * R);
    const float rcp_ns = 1.0f / (float)Ns;
    float2 v[MAXB][R];
    int dst[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int j = u + i * tps;
        dst[i] = -1;
        if (active && j < nb) {
            int jq, k;
            fdivmod(j, Ns, rcp_ns, jq, k);
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = xs[j + r * nb];
            if (k) {
                const int e = k * tstride;
                float2 w1 = tw(e);
                if (inv) w1.y = -w1.y;
                v[i][1] = cmul(v[i][1], w1);
                if constexpr (R >= 3) {
                    const float2 w2 = cmul(w1, w1);
                    v[i][2] = cmul(v[i][2], w2);
                    if constexpr (R >= 4) {
                        const float2 w3 = cmul(w2, w1);
                        v[i][3] = cmul(v[i][3], w3);
                        if constexpr (R == 8) {
                            float2 w4 = tw(4 * e);
                            if (inv) w4.y = -w4.y;
                            v[i][4] = cmul(v[i][4], w4);
                            v[i][5] = cmul(v[i][5], cmul(w4, w1));
                            v[i][6] = cmul(v[i][6], cmul(w4, w2));
                            v[i][7] = cmul(v[i][7], cmul(w4, w3));
                        }
                    }
                }
            }
            butterfly<R>(v[i], inv);
            dst[i] = jq * Ns * R + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        if (dst[i] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) xs[dst[i] + r * Ns] = v[i][r];
        }
    }
    __syncthreads();
}

// Transform `nseq` sequences in LDS (x[f*ld .. f*ld + n)), in place.  Thread t
// works on sequence t / tps with tps = blockDim.x / nseq threads per sequence;
// requires tps >= fft_min_tps(d) (each thread holds MAXB butterflies of a
// radix-2/3/4 stage, MAXB/2 of a radix-8 stage).  Must be reached by every
// thread of the workgroup (contains barriers).
template <int MAXB>
__device__ void fft_lds(float2* x, int ld, int nseq, const FftDev& d, const TwLds& tw, bool inv)
{
    const int tps = blockDim.x / nseq;
    const int f = threadIdx.x / tps;
    const int u = threadIdx.x - f * tps;
    const bool active = f < nseq;
    float2* xs = x + (active ? f : 0) * ld;
    int Ns = 1;
    for (int s = 0; s < d.nst; ++s) {
        const int R = d.rad[s];
        if (R == 8) fft_stage<8, (MAXB + 1) / 2>(xs, active, u, tps, d.n, Ns, tw, inv);
        else if (R == 4) fft_stage<4, MAXB>(xs, active, u, tps, d.n, Ns, tw, inv);
        else if (R == 2) fft_stage<2, MAXB>(xs, active, u, tps, d.n, Ns, tw, inv);
        else fft_stage<3, MAXB>(xs, active, u, tps, d.n, Ns, tw, inv);
        Ns *= R;
    }
}

// Threads per sequence the stages of length d.n need with `maxb` butterflies
// per thread (maxb/2 for radix 8).
__host__ __device__ inline int fft_min_tps(const FftDev& d, int maxb)
{
    int t = 1;
    for (int s = 0; s < d.nst; ++s) {
        const int R = d.rad[s];
        const int per = R == 8 ? (maxb + 1) / 2 : maxb;
        const int need = (d.n / R + per - 1) / per;
        t = need > t ? need : t;
    }
    return t;
}

}  // namespace pat
