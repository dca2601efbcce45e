// fft.hpp -- in-LDS complex FFTs for gfx950 workgroups.
//
// Mixed-radix Stockham autosort over n = 2^a 3^b with radices 2, 3, 4, 6, 8, 9
// and 16.  The pass of radix R after sub-transforms of size Ns reads
// x[j + r n/R] (r < R), multiplies input r by w^r with w = e^{-2 pi i k/(Ns R)},
// k = j mod Ns, does an R-point DFT and writes x[(j - k) R + k + r Ns].  Each
// pass is done in place: every thread loads its butterflies into registers, the
// workgroup synchronises, then stores.  `nseq` sequences of one length at
// stride `ld` (complex elements) are transformed together.
//
// Twiddles: one table per length holds, pass after pass, the base twiddle
// e^{-2 pi i k/(Ns R)} for k < Ns (FP64-computed, stored FP32; sum of the
// passes' Ns entries, n/R_last + n/(R_last R_prev) + ...).  A butterfly loads
// its base twiddle once and forms the powers w^r by products of lower powers
// (at most four products deep).  Radices 6, 9 and 16 are two-level DFTs
// (2 x 3, 3 x 3, 4 x 4) with constant inner twiddles.
//
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
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a)
{
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
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

// e^{-2 pi i m / R}: the inner twiddles of the two-level radices (m = r1 k1)
template <int R>
__device__ __forceinline__ float2 inner_tw(int m)
{
    if constexpr (R == 6) {
        constexpr float s = 0.86602540378443864676f;  // sin(pi/3)
        return m == 1 ? make_float2(0.5f, -s) : make_float2(-0.5f, -s);
    } else if constexpr (R == 9) {
        switch (m) {  // angles 40, 80 and 160 degrees
            case 1: return make_float2(0.76604444311897803520f, -0.64278760968653932632f);
            case 2: return make_float2(0.17364817766693034885f, -0.98480775301220805936f);
            default: return make_float2(-0.93969262078590838405f, -0.34202014332566873304f);
        }
    } else {
        static_assert(R == 16, "two-level radices: 6, 9, 16");
        constexpr float c = 0.92387953251128675613f, s = 0.38268343236508977173f, h = 0.70710678118654752440f;
        switch (m) {  // multiples of 22.5 degrees: 1, 2, 3, 4, 6, 9
            case 1: return make_float2(c, -s);
            case 2: return make_float2(h, -h);
            case 3: return make_float2(s, -c);
            case 4: return make_float2(0.f, -1.f);
            case 6: return make_float2(-h, -h);
            default: return make_float2(-c, s);
        }
    }
}

template <int R, bool INV>
__device__ __forceinline__ void butterfly(float2 (&v)[R]);

// R = A B point DFT: with r = r1 + A r2 and k = k1 + B k2,
//   X[k1 + B k2] = sum_r1 w_A^{r1 k2} w_R^{r1 k1} sum_r2 v[r1 + A r2] w_B^{r2 k1}.
template <int A, int B, bool INV>
__device__ __forceinline__ void butterfly_two_level(float2 (&v)[A * B])
{
    float2 y[A][B];
#pragma unroll
    for (int r1 = 0; r1 < A; ++r1) {
        float2 t[B];
#pragma unroll
        for (int r2 = 0; r2 < B; ++r2) t[r2] = v[r1 + A * r2];
        butterfly<B, INV>(t);
#pragma unroll
        for (int k1 = 0; k1 < B; ++k1) {
            if (r1 && k1) {
                float2 c = inner_tw<A * B>(r1 * k1);
                if (INV) c.y = -c.y;
                y[r1][k1] = cmul(t[k1], c);
            } else {
                y[r1][k1] = t[k1];
            }
        }
    }
#pragma unroll
    for (int k1 = 0; k1 < B; ++k1) {
        float2 t[A];
#pragma unroll
        for (int r1 = 0; r1 < A; ++r1) t[r1] = y[r1][k1];
        butterfly<A, INV>(t);
#pragma unroll
        for (int k2 = 0; k2 < A; ++k2) v[k1 + B * k2] = t[k2];
    }
}

template <int R, bool INV>
__device__ __forceinline__ void butterfly(float2 (&v)[R])
{
    if constexpr (R == 2) {
        const float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 3) {
        const float s3 = 0.86602540378443864676f;
        const float2 s = cadd(v[1], v[2]), df = csub(v[1], v[2]);
        const float2 t = make_float2(v[0].x - 0.5f * s.x, v[0].y - 0.5f * s.y);
        v[0] = cadd(v[0], s);
        const float2 m = mul_mi<INV>(cscale(df, s3));  // -i (sqrt3/2)(a1 - a2) (forward)
        v[1] = cadd(t, m);
        v[2] = csub(t, m);
    } else if constexpr (R == 4) {
        const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        const float2 t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        const float2 m = mul_mi<INV>(t3);
        v[1] = cadd(t1, m);
        v[3] = csub(t1, m);
    } else if constexpr (R == 8) {
        // X[k] = E[k] + W8^k O[k], X[k+4] = E[k] - W8^k O[k]; E, O = 4-point DFTs of even/odd inputs
        float2 e[4] = {v[0], v[2], v[4], v[6]};
        float2 o[4] = {v[1], v[3], v[5], v[7]};
        butterfly<4, INV>(e);
        butterfly<4, INV>(o);
        const float r2 = 0.70710678118654752440f;
        // W8^1 = (1 - i)/sqrt2, W8^2 = -i, W8^3 = (-1 - i)/sqrt2 (conjugates for the inverse)
        const float2 o1 = INV ? make_float2(r2 * (o[1].x - o[1].y), r2 * (o[1].x + o[1].y))
                              : make_float2(r2 * (o[1].x + o[1].y), r2 * (o[1].y - o[1].x));
        const float2 o2 = mul_mi<INV>(o[2]);
        const float2 o3 = INV ? make_float2(-r2 * (o[3].x + o[3].y), r2 * (o[3].x - o[3].y))
                              : make_float2(r2 * (o[3].y - o[3].x), -r2 * (o[3].x + o[3].y));
        v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);   v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);   v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);   v[7] = csub(e[3], o3);
    } else if constexpr (R == 6) {
        butterfly_two_level<2, 3, INV>(v);
    } else if constexpr (R == 9) {
        butterfly_two_level<3, 3, INV>(v);
    } else {
        static_assert(R == 16, "radices: 2, 3, 4, 6, 8, 9, 16");
        butterfly_two_level<4, 4, INV>(v);
    }
}

// v[r] *= w^r, r = 1 .. R-1: w^r = (w^p)^2 for r = 2p, else w^p w^{r-p} with p
// the largest power of two below r (all indices compile-time constants).
__host__ __device__ constexpr int pow2_below(int r)
{
    int p = 1;
    while (2 * p < r) p *= 2;
    return p;
}

template <int R, int r>
__device__ __forceinline__ void twiddle_powers(float2 (&pw)[R])
{
    if constexpr (r < R) {
        constexpr int p = pow2_below(r);
        pw[r] = (r == 2 * p) ? cmul(pw[p], pw[p]) : cmul(pw[p], pw[r - p]);
        twiddle_powers<R, r + 1>(pw);
    }
}

template <int R>
__device__ __forceinline__ void apply_twiddles(float2 (&v)[R], float2 w)
{
    float2 pw[R];
    pw[1] = w;
    twiddle_powers<R, 2>(pw);
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], pw[r]);
}

// One Stockham pass of radix R on the sequence `xs` (length n) by the `tps`
// threads with local index u (butterflies j = u, u + tps, ..., at most
// radix_max_butterflies(R) per thread).  `lg` = log2 Ns when Ns is a power of
// two, else -1; `tb` = this pass's base twiddles.
template <int R, bool INV, int MAXB>
__device__ __forceinline__ void fft_pass(float2* xs, bool active, int u, int tps, int n, int Ns, int lg,
                                         const float2* tb)
{
    constexpr int MB = radix_max_butterflies(R, MAXB);
    const int nb = n / R;
    // the hardware reciprocal (within 1 ulp): fdivmod's correction step makes
    // the quotient exact, so no IEEE division is needed here
    const float rcp = __builtin_amdgcn_rcpf((float)Ns);
    float2 v[MB][R];
    int dst[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int j = u + i * tps;
        dst[i] = -1;
        if (active && j < nb) {
            int jq, k;
            if (lg >= 0) {
                jq = j >> lg;
                k = j & (Ns - 1);
            } else {
                fdivmod(j, Ns, rcp, jq, k);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = xs[j + r * nb];
            if (Ns > 1) {
                float2 w = tb[k];
                if (INV) w.y = -w.y;
                apply_twiddles<R>(v[i], w);
            }
            butterfly<R, INV>(v[i]);
            dst[i] = jq * Ns * R + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        if (dst[i] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) xs[dst[i] + r * Ns] = v[i][r];
        }
    }
    __syncthreads();
}

// Copy a length's per-pass base twiddles (d.ntb entries) from the plan's table
// to LDS at `dst`.  The caller synchronises before the transform.
__device__ __forceinline__ const float2* fft_twiddles_to_lds(float2* dst, const FftDev& d,
                                                             const float2* __restrict__ tab)
{
    const float2* src = tab + d.tb;
    for (int e = threadIdx.x; e < d.ntb; e += blockDim.x) dst[e] = src[e];
    return dst;
}

// Transform `nseq` sequences in LDS (x[f*ld .. f*ld + n)), in place.  Thread t
// works on sequence t / tps with tps = blockDim.x / nseq threads per sequence;
// requires tps >= fft_min_tps(d).  `tb` = the length's base twiddles in LDS
// (fft_twiddles_to_lds).  Must be reached by every thread of the workgroup
// (contains barriers).
template <bool INV, int MAXB = kFftMaxButterflies>
__device__ __forceinline__ void fft_lds(float2* x, int ld, int nseq, const FftDev& d, const float2* tb)
{
    const int tps = blockDim.x / nseq;
    const int f = threadIdx.x / tps;
    const int u = threadIdx.x - f * tps;
    const bool active = f < nseq;
    float2* xs = x + (active ? f : 0) * ld;
    int Ns = 1;
    for (int s = 0; s < d.nst; ++s) {
        const int R = d.rad[s];
        const int lg = (Ns & (Ns - 1)) == 0 ? __builtin_ctz(Ns) : -1;
        switch (R) {
            case 2: fft_pass<2, INV, MAXB>(xs, active, u, tps, d.n, Ns, lg, tb); break;
            case 3: fft_pass<3, INV, MAXB>(xs, active, u, tps, d.n, Ns, lg, tb); break;
            case 4: fft_pass<4, INV, MAXB>(xs, active, u, tps, d.n, Ns, lg, tb); break;
            case 6: fft_pass<6, INV, MAXB>(xs, active, u, tps, d.n, Ns, lg, tb); break;
            case 8: fft_pass<8, INV, MAXB>(xs, active, u, tps, d.n, Ns, lg, tb); break;
            case 9: fft_pass<9, INV, MAXB>(xs, active, u, tps, d.n, Ns, lg, tb); break;
            default: fft_pass<16, INV, MAXB>(xs, active, u, tps, d.n, Ns, lg, tb); break;
        }
        tb += Ns;
        Ns *= R;
    }
}

// Two-level table of the twiddles w_n^e = e^{-2 pi i e / n} (used outside the
// transforms): w^e = lo[e & 63] * hi[e >> 6] (lo: 64 entries, hi: ceil(n/64)).
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

// Entry e of the two-level table of length d.n, read from the plan's table of
// w_n^e (e < n).
__device__ __forceinline__ float2 tw_lds_entry(const FftDev& d, const float2* __restrict__ twall, int e)
{
    // for e < tw_lds_slots(n) the hi entries 64 (e - 64) are below n and the lo
    // entries e < 64 wrap only when n < 64: reduce by subtraction (n is the
    // same for the whole workgroup; at most 63 / n rounds)
    const int n = max(d.n, 1);
    int idx = e < 64 ? e : 64 * (e - 64);
    while (idx >= n) idx -= n;
    return twall[d.tw + idx];
}

// The first two entries per thread of a two-level table (e = threadIdx.x and
// threadIdx.x + blockDim.x), loaded into registers so that the loads can be
// in flight together with others (indices past the table are clamped, not
// branched around); tw_lds_store writes them and the rest.
struct TwFetch {
    float2 v[2];
};

__device__ __forceinline__ TwFetch tw_lds_fetch(const FftDev& d, const float2* __restrict__ twall)
{
    const int cnt = tw_lds_slots(d.n);
    TwFetch f;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        f.v[i] = tw_lds_entry(d, twall, min((int)(threadIdx.x + i * blockDim.x), cnt - 1));
    }
    return f;
}

// Fill the two-level table of length d.n at `dst` (the fetched entries plus
// any beyond two per thread).  Caller synchronises before use.
__device__ __forceinline__ TwLds tw_lds_store(float2* dst, const FftDev& d, const float2* __restrict__ twall,
                                              const TwFetch& f)
{
    const int cnt = tw_lds_slots(d.n);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int e = threadIdx.x + i * blockDim.x;
        if (e < cnt) dst[e] = f.v[i];
    }
    for (int e = threadIdx.x + 2 * blockDim.x; e < cnt; e += blockDim.x) dst[e] = tw_lds_entry(d, twall, e);
    return TwLds{dst, dst + 64, 0};
}

__device__ __forceinline__ TwLds tw_lds_build(float2* dst, const FftDev& d, const float2* __restrict__ twall)
{
    return tw_lds_store(dst, d, twall, tw_lds_fetch(d, twall));
}

}  // namespace pat
