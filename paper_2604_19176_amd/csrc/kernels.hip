// kernels.hip -- gfx950 kernels of the PAT operator pair.
//
// Forward A (steps of the discrete operator; layouts per instance, row-major):
//   colpass_fwd : f [N][N] -> mask, deapodise, zero-pad to Ng, FFT along y of
//                 column pairs packed as complex -> X1 [Hy][N] (rows m_y = -4..Ng/2+4)
//                 + per-tile partial sums of h^2 m f (endpoint term)
//   rowpass_fwd : X1 -> FFT along x -> G [Hy][Ng]  (oversampled half spectrum)
//   ring_fwd    : per radial frequency n: ES interpolation of G at the ring's
//                 half-plane points, completion by conjugate symmetry, angular
//                 FFT, weight i^k J_k(lam_n R) W_n / Npsi(n) -> b [nlam][Kp]
//   dct         : per mode k: B_k(j) = sum_n b_k(n) cos(pi n j / M) via one
//                 complex FFT of length 2M -> Bt [T][Kp]
//   czt_fwd     : per time sample: Bluestein chirp-z over detector angles,
//                 g = Re(...) + kappa * mass -> g [D][T]
// Adjoint A* runs the exact transposes in reverse (czt_adj, dct, ring_adj,
// spread, rowpass_adj, colpass_adj).  No floating-point atomics anywhere:
// every sum has a fixed order, so results are bitwise repeatable.
#include "fft.hpp"
#include "pat_internal.hpp"

namespace pat {

constexpr int kMaxB = 8;  // butterflies per thread per FFT stage

__device__ __forceinline__ float es_weight(float t)
{
    const float z = t * (2.0f / kEsWidth);
    const float q = 1.0f - z * z;
    return q >= 0.0f ? __expf((float)kEsBeta * (__fsqrt_rn(q) - 1.0f)) : 0.0f;
}

__device__ __forceinline__ void es_weights8(float frac, float (&w)[8])
{
#pragma unroll
    for (int d = 0; d < 8; ++d) w[d] = es_weight(frac + 3.0f - (float)d);
}

__device__ __forceinline__ int fbits(float v) { return __float_as_int(v); }

// Deterministic block sum (fixed tree); every thread gets the total.
__device__ float block_sum(float v, float* scratch)
{
    const int tid = threadIdx.x;
    scratch[tid] = v;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (s < (int)blockDim.x && tid < s && tid + s < (int)blockDim.x) scratch[tid] += scratch[tid + s];
        __syncthreads();
    }
    float r = scratch[0];
    __syncthreads();
    return r;
}

struct InstPtrs {
    char* ws;         // workspace base of instance 0
    size_t stride;    // bytes per instance
};

// ---------------------------------------------------------------------------
// forward: column pass (FFT along y of real columns, packed in pairs)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_colpass_fwd(PlanDev d, WsLayout L, const float* __restrict__ f,
                                                     InstPtrs wsp, int NP)
{
    extern __shared__ float2 sm[];
    __shared__ float red_s[512];
    const int b = blockIdx.y;
    const int N = d.N, Ng = d.Ng, CT = 2 * NP;
    const float* fb = f + (size_t)b * N * N;
    char* wb = wsp.ws + (size_t)b * wsp.stride;
    float2* X1 = (float2*)(wb + L.x1);
    float* red = (float*)(wb + L.red);
    const int j0 = blockIdx.x * CT;
    for (int e = threadIdx.x; e < NP * Ng; e += blockDim.x) sm[e] = make_float2(0.f, 0.f);
    __syncthreads();
    float msum = 0.f;
    for (int e = threadIdx.x; e < N * CT; e += blockDim.x) {
        const int i = e / CT, jj = e - i * CT, j = j0 + jj;
        float v = 0.f;
        if (j < N) {
            const int2 mr = d.mask_rows[i];
            if (j >= mr.x && j < mr.y) {
                const float fv = fb[(size_t)i * N + j];
                msum += fv;
                v = fv * d.deap[i] * d.deap[j];
            }
        }
        int pos = i - N / 2;
        if (pos < 0) pos += Ng;
        float* slot = (float*)&sm[(jj >> 1) * Ng + pos];
        slot[jj & 1] = v;
    }
    const float tot = block_sum(msum, red_s);
    if (threadIdx.x == 0) red[blockIdx.x] = tot * d.h2;
    __syncthreads();
    fft_lds<kMaxB>(sm, Ng, NP, d.ffts[d.fft_grid], d.tw, false);
    for (int e = threadIdx.x; e < d.Hy * CT; e += blockDim.x) {
        const int r = e / CT, jj = e - r * CT, j = j0 + jj;
        if (j >= N) continue;
        const int m = r - 4;
        const int ip = m < 0 ? m + Ng : m;
        const int in = m > 0 ? Ng - m : -m;
        const float2 zp = sm[(jj >> 1) * Ng + ip], zn = sm[(jj >> 1) * Ng + in];
        float2 o;
        if ((jj & 1) == 0) {  // (Z(m) + conj Z(-m)) / 2
            o = make_float2(0.5f * (zp.x + zn.x), 0.5f * (zp.y - zn.y));
        } else {              // (Z(m) - conj Z(-m)) / (2i)
            o = make_float2(0.5f * (zp.y + zn.y), -0.5f * (zp.x - zn.x));
        }
        X1[(size_t)r * N + j] = o;
    }
}

// ---------------------------------------------------------------------------
// forward: row pass (FFT along x)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_rowpass_fwd(PlanDev d, WsLayout L, InstPtrs wsp, int RPB)
{
    extern __shared__ float2 sm[];
    const int b = blockIdx.y;
    const int N = d.N, Ng = d.Ng;
    char* wb = wsp.ws + (size_t)b * wsp.stride;
    const float2* X1 = (const float2*)(wb + L.x1);
    float2* G = (float2*)(wb + L.grid);
    const int r0 = blockIdx.x * RPB;
    const int nr = min(RPB, d.Hy - r0);
    for (int e = threadIdx.x; e < nr * Ng; e += blockDim.x) sm[e] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int e = threadIdx.x; e < nr * N; e += blockDim.x) {
        const int rr = e / N, j = e - rr * N;
        int pos = j - N / 2;
        if (pos < 0) pos += Ng;
        sm[rr * Ng + pos] = X1[(size_t)(r0 + rr) * N + j];
    }
    __syncthreads();
    fft_lds<kMaxB>(sm, Ng, nr, d.ffts[d.fft_grid], d.tw, false);
    for (int e = threadIdx.x; e < nr * Ng; e += blockDim.x) G[(size_t)r0 * Ng + e] = sm[e];
}

// ---------------------------------------------------------------------------
// forward: ring kernel (interpolation + angular FFT + radial weight)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_ring_fwd(PlanDev d, WsLayout L, InstPtrs wsp)
{
    extern __shared__ float2 sm[];
    const int b = blockIdx.y, n = blockIdx.x;
    char* wb = wsp.ws + (size_t)b * wsp.stride;
    const float2* __restrict__ G = (const float2*)(wb + L.grid);
    float2* bm = (float2*)(wb + L.modes);
    const int Ng = d.Ng;
    const int off = d.ring_off[n], P = d.ring_off[n + 1] - off;
    for (int l = threadIdx.x; l < P; l += blockDim.x) {
        const float4 gq = d.pt_geo[off + l];
        const int bx = fbits(gq.x), r0 = fbits(gq.y);
        float wx[8], wy[8];
        es_weights8(gq.z, wx);
        es_weights8(gq.w, wy);
        int cols[8];
#pragma unroll
        for (int dx = 0; dx < 8; ++dx) {
            int c = bx + dx;
            cols[dx] = c >= Ng ? c - Ng : c;
        }
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int dy = 0; dy < 8; ++dy) {
            const float2* row = G + (size_t)(r0 + dy) * Ng;
            float2 ra = make_float2(0.f, 0.f);
#pragma unroll
            for (int dx = 0; dx < 8; ++dx) {
                const float2 gv = row[cols[dx]];
                ra.x += wx[dx] * gv.x;
                ra.y += wx[dx] * gv.y;
            }
            acc.x += wy[dy] * ra.x;
            acc.y += wy[dy] * ra.y;
        }
        const float2 F = cmul(acc, d.pt_phase[off + l]);
        sm[l] = F;
        sm[l + P] = cconj(F);
    }
    __syncthreads();
    fft_lds<kMaxB>(sm, 2 * P, 1, d.ffts[d.ring_fft[n]], d.tw, false);
    const int Kn = d.ring_K[n], jo = d.ring_joff[n];
    for (int k = threadIdx.x; k <= Kn; k += blockDim.x) {
        const float2 v = cscale(sm[k], d.Jw[jo + k]);
        float2 o;
        switch (k & 3) {  // multiply by i^k
            case 0: o = v; break;
            case 1: o = make_float2(-v.y, v.x); break;
            case 2: o = make_float2(-v.x, -v.y); break;
            default: o = make_float2(v.y, -v.x); break;
        }
        bm[(size_t)n * d.Kp + k] = o;
    }
}

// ---------------------------------------------------------------------------
// cosine transform per mode (shared by forward and adjoint)
//   forward (adj = 0): in = b [nlam][Kp] (row n-1 = lam_n), out = Bt [T][Kp]
//   adjoint (adj = 1): in = Bt [T][Kp], out = b [nlam][Kp]
// out(q) = sum_p in(p) cos(pi p q / M) = (X[q] + X[2M - q]) / 2, X = FFT_2M(in).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_dct(PlanDev d, WsLayout L, InstPtrs wsp, int MT, int adj)
{
    extern __shared__ float2 sm[];
    const int b = blockIdx.y;
    const int twoM = 2 * d.M, Kp = d.Kp;
    char* wb = wsp.ws + (size_t)b * wsp.stride;
    const float2* in = (const float2*)(wb + (adj ? L.tmodes : L.modes));
    float2* out = (float2*)(wb + (adj ? L.modes : L.tmodes));
    const int nin = adj ? d.T : d.nlam;
    const int nout = adj ? d.nlam : d.T;
    const int k0 = blockIdx.x * MT;
    const int mt = min(MT, Kp - k0);
    for (int e = threadIdx.x; e < mt * twoM; e += blockDim.x) sm[e] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int e = threadIdx.x; e < nin * mt; e += blockDim.x) {
        const int p = e / mt, kk = e - p * mt, k = k0 + kk;   // p = row index (0-based), lambda/t index p+1
        const bool keep = adj ? true : (p >= d.mode_nmin[k]);
        if (keep) sm[kk * twoM + p + 1] = in[(size_t)p * Kp + k];
    }
    __syncthreads();
    fft_lds<kMaxB>(sm, twoM, mt, d.ffts[d.fft_dct], d.tw, false);
    for (int e = threadIdx.x; e < nout * mt; e += blockDim.x) {
        const int q = e / mt, kk = e - q * mt, k = k0 + kk;
        if (adj && q < d.mode_nmin[k]) continue;
        const int s = q + 1;
        const float2 a = sm[kk * twoM + s], c = sm[kk * twoM + (twoM - s)];
        out[(size_t)q * Kp + k] = make_float2(0.5f * (a.x + c.x), 0.5f * (a.y + c.y));
    }
}

// ---------------------------------------------------------------------------
// forward: chirp-z synthesis over detector angles, per time sample
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_czt_fwd(PlanDev d, WsLayout L, InstPtrs wsp, float* __restrict__ g,
                                                 int TT, int PAR, int n_mass)
{
    extern __shared__ float2 sm[];
    __shared__ float mass_s;
    const int b = blockIdx.y;
    const int Ln = d.L, Kp = d.Kp, D = d.D, T = d.T;
    char* wb = wsp.ws + (size_t)b * wsp.stride;
    const float2* Bt = (const float2*)(wb + L.tmodes);
    const float* red = (const float*)(wb + L.red);
    float* ot = (float*)(sm + PAR * Ln);  // [D][TT]
    float* gb = g + (size_t)b * D * T;
    if (threadIdx.x == 0) {
        float m = 0.f;
        for (int t = 0; t < n_mass; ++t) m += red[t];
        mass_s = m;
    }
    const int j0 = blockIdx.x * TT;
    const int nt = min(TT, T - j0);
    const FftDev& fd = d.ffts[d.fft_czt];
    for (int jb = 0; jb < nt; jb += PAR) {
        const int np = min(PAR, nt - jb);
        for (int e = threadIdx.x; e < np * Ln; e += blockDim.x) {
            const int p = e / Ln, q = e - p * Ln;
            float2 v = make_float2(0.f, 0.f);
            if (q < Kp) v = cmul(d.czt_pre[q], Bt[(size_t)(j0 + jb + p) * Kp + q]);
            sm[e] = v;
        }
        __syncthreads();
        fft_lds<kMaxB>(sm, Ln, np, fd, d.tw, false);
        for (int e = threadIdx.x; e < np * Ln; e += blockDim.x) {
            const int q = e % Ln;
            sm[e] = cmul(sm[e], d.czt_vhat[q]);
        }
        __syncthreads();
        fft_lds<kMaxB>(sm, Ln, np, fd, d.tw, true);
        const float km = d.kappa * mass_s;
        for (int e = threadIdx.x; e < np * D; e += blockDim.x) {
            const int p = e / D, q = e - p * D;
            const float2 s = sm[p * Ln + q], w = d.czt_post[q];
            ot[q * TT + jb + p] = (w.x * s.x - w.y * s.y) + km;
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < D * nt; e += blockDim.x) {
        const int q = e / nt, tt = e - q * nt;
        gb[(size_t)q * T + j0 + tt] = ot[q * TT + tt];
    }
}

// ---------------------------------------------------------------------------
// adjoint: chirp-z transpose, detectors -> modes, per time sample
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_czt_adj(PlanDev d, WsLayout L, InstPtrs wsp, const float* __restrict__ g,
                                                 int TT, int PAR)
{
    extern __shared__ float2 sm[];
    __shared__ float red_s[512];
    const int b = blockIdx.y;
    const int Ln = d.L, Kp = d.Kp, D = d.D, T = d.T;
    char* wb = wsp.ws + (size_t)b * wsp.stride;
    float2* Bt = (float2*)(wb + L.tmodes);
    float* red = (float*)(wb + L.red);
    float* it = (float*)(sm + PAR * Ln);  // [D][TT]
    const float* gb = g + (size_t)b * D * T;
    const int j0 = blockIdx.x * TT;
    const int nt = min(TT, T - j0);
    float ls = 0.f;
    for (int e = threadIdx.x; e < D * nt; e += blockDim.x) {
        const int q = e / nt, tt = e - q * nt;
        const float v = gb[(size_t)q * T + j0 + tt];
        it[q * TT + tt] = v;
        ls += v;
    }
    const float tot = block_sum(ls, red_s);
    if (threadIdx.x == 0) red[blockIdx.x] = tot;
    __syncthreads();
    const FftDev& fd = d.ffts[d.fft_czt];
    for (int jb = 0; jb < nt; jb += PAR) {
        const int np = min(PAR, nt - jb);
        for (int e = threadIdx.x; e < np * Ln; e += blockDim.x) {
            const int p = e / Ln, q = e - p * Ln;
            float2 v = make_float2(0.f, 0.f);
            if (q < D) v = cmulc(make_float2(it[q * TT + jb + p], 0.f), d.czt_post[q]);
            sm[e] = v;
        }
        __syncthreads();
        fft_lds<kMaxB>(sm, Ln, np, fd, d.tw, false);
        for (int e = threadIdx.x; e < np * Ln; e += blockDim.x) {
            const int q = e % Ln;
            sm[e] = cmulc(sm[e], d.czt_vhat[q]);
        }
        __syncthreads();
        fft_lds<kMaxB>(sm, Ln, np, fd, d.tw, true);
        for (int e = threadIdx.x; e < np * Kp; e += blockDim.x) {
            const int p = e / Kp, k = e - p * Kp;
            Bt[(size_t)(j0 + jb + p) * Kp + k] = cmulc(sm[p * Ln + k], d.czt_pre[k]);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// adjoint: ring kernel (conjugate weight, inverse angular FFT, fold, phase)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_ring_adj(PlanDev d, WsLayout L, InstPtrs wsp)
{
    extern __shared__ float2 sm[];
    const int b = blockIdx.y, n = blockIdx.x;
    char* wb = wsp.ws + (size_t)b * wsp.stride;
    const float2* bm = (const float2*)(wb + L.modes);
    float2* H = (float2*)(wb + L.polar);
    const int off = d.ring_off[n], P = d.ring_off[n + 1] - off, np = 2 * P;
    const int Kn = d.ring_K[n], jo = d.ring_joff[n];
    for (int e = threadIdx.x; e < np; e += blockDim.x) {
        float2 o = make_float2(0.f, 0.f);
        if (e <= Kn) {
            const float2 v = cscale(bm[(size_t)n * d.Kp + e], d.Jw[jo + e]);
            switch (e & 3) {  // multiply by (-i)^k
                case 0: o = v; break;
                case 1: o = make_float2(v.y, -v.x); break;
                case 2: o = make_float2(-v.x, -v.y); break;
                default: o = make_float2(-v.y, v.x); break;
            }
        }
        sm[e] = o;
    }
    __syncthreads();
    fft_lds<kMaxB>(sm, np, 1, d.ffts[d.ring_fft[n]], d.tw, true);
    for (int l = threadIdx.x; l < P; l += blockDim.x) {
        const float2 a = sm[l], c = sm[l + P];
        const float2 hh = make_float2(a.x + c.x, a.y - c.y);  // F~(l) + conj F~(l + P)
        H[d.perm[off + l]] = cmulc(hh, d.pt_phase[off + l]);
    }
}

// ---------------------------------------------------------------------------
// adjoint: deterministic spread of the polar half-plane values onto G~ [Hy][Ng]
// One lane owns one column; bands (footprint base rows) are swept in order and
// an 8-row register window accumulates; band points are staged in LDS with
// their ES weights.  Every output is a fixed-order sum.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_spread(PlanDev d, WsLayout L, InstPtrs wsp, int TH, int CAP)
{
    extern __shared__ float sf[];
    const int b = blockIdx.z;
    const int Ng = d.Ng, NB = d.NB, Hy = d.Hy;
    char* wb = wsp.ws + (size_t)b * wsp.stride;
    const float2* __restrict__ H = (const float2*)(wb + L.polar);
    float2* Gt = (float2*)(wb + L.grid);
    float* wxs = sf;                       // [CAP][8]
    float* wys = sf + CAP * 8;             // [CAP][8]
    float2* hs = (float2*)(sf + CAP * 16); // [CAP]
    int* bxs = (int*)(sf + CAP * 18);      // [CAP]
    const int CB = blockDim.x;
    const int C0 = blockIdx.x * CB, R0 = blockIdx.y * TH;
    const int mx = C0 + threadIdx.x;
    const bool active = mx < Ng;
    const int rend = min(R0 + TH, Hy);
    float2 acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = make_float2(0.f, 0.f);
    const int band_lo = max(0, R0 - 7), band_hi = min(NB - 1, rend - 1);
    const int lo_col = C0 - 7;
    const int hi_col = min(C0 + CB, Ng);  // exclusive
    for (int rb = band_lo; rb <= band_hi; ++rb) {
        const int* bp = d.band_ptr + (size_t)rb * (Ng + 1);
        const int aLo = lo_col < 0 ? bp[Ng + lo_col] : 0;
        const int aHi = lo_col < 0 ? bp[Ng] : 0;
        const int bLo = bp[max(lo_col, 0)], bHi = bp[hi_col];
        const int nA = aHi - aLo, ntot = nA + (bHi - bLo);
        int lo = 0, hi = 0;
        if (active) {
            const int c = mx - 7;
            lo = c < 0 ? (bp[Ng + c] - aLo) : (nA + bp[c] - bLo);
            hi = nA + bp[mx + 1] - bLo;
        }
        for (int c0 = 0; c0 < ntot; c0 += CAP) {
            const int cn = min(CAP, ntot - c0);
            for (int e = threadIdx.x; e < cn; e += blockDim.x) {
                const int idx = c0 + e;
                const int slot = idx < nA ? aLo + idx : bLo + (idx - nA);
                const float4 gq = d.bpt_geo[slot];
                float w[8];
                es_weights8(gq.z, w);
#pragma unroll
                for (int k = 0; k < 8; ++k) wxs[e * 8 + k] = w[k];
                es_weights8(gq.w, w);
#pragma unroll
                for (int k = 0; k < 8; ++k) wys[e * 8 + k] = w[k];
                hs[e] = H[slot];
                bxs[e] = fbits(gq.x);
            }
            __syncthreads();
            const int s0 = max(lo, c0), s1 = min(hi, c0 + cn);
            for (int s = s0; s < s1; ++s) {
                const int e = s - c0;
                int dx = mx - bxs[e];
                if (dx < 0) dx += Ng;
                const float w = wxs[e * 8 + dx];
                const float2 t = cscale(hs[e], w);
                const float4 wa = *(const float4*)&wys[e * 8];
                const float4 wb4 = *(const float4*)&wys[e * 8 + 4];
                acc[0].x += wa.x * t.x; acc[0].y += wa.x * t.y;
                acc[1].x += wa.y * t.x; acc[1].y += wa.y * t.y;
                acc[2].x += wa.z * t.x; acc[2].y += wa.z * t.y;
                acc[3].x += wa.w * t.x; acc[3].y += wa.w * t.y;
                acc[4].x += wb4.x * t.x; acc[4].y += wb4.x * t.y;
                acc[5].x += wb4.y * t.x; acc[5].y += wb4.y * t.y;
                acc[6].x += wb4.z * t.x; acc[6].y += wb4.z * t.y;
                acc[7].x += wb4.w * t.x; acc[7].y += wb4.w * t.y;
            }
            __syncthreads();
        }
        // row rb is complete
        if (active && rb >= R0 && rb < rend) Gt[(size_t)rb * Ng + mx] = acc[0];
#pragma unroll
        for (int k = 0; k < 7; ++k) acc[k] = acc[k + 1];
        acc[7] = make_float2(0.f, 0.f);
    }
    // rows after the last band receive no further contributions
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        const int r = band_hi + 1 + k;
        if (active && r >= R0 && r < rend) Gt[(size_t)r * Ng + mx] = acc[k];
    }
}

// ---------------------------------------------------------------------------
// adjoint: row pass (inverse FFT along x, crop to the N image columns)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_rowpass_adj(PlanDev d, WsLayout L, InstPtrs wsp, int RPB)
{
    extern __shared__ float2 sm[];
    const int b = blockIdx.y;
    const int N = d.N, Ng = d.Ng;
    char* wb = wsp.ws + (size_t)b * wsp.stride;
    const float2* Gt = (const float2*)(wb + L.grid);
    float2* X1 = (float2*)(wb + L.x1);
    const int r0 = blockIdx.x * RPB;
    const int nr = min(RPB, d.Hy - r0);
    for (int e = threadIdx.x; e < nr * Ng; e += blockDim.x) sm[e] = Gt[(size_t)r0 * Ng + e];
    __syncthreads();
    fft_lds<kMaxB>(sm, Ng, nr, d.ffts[d.fft_grid], d.tw, true);
    for (int e = threadIdx.x; e < nr * N; e += blockDim.x) {
        const int rr = e / N, j = e - rr * N;
        int pos = j - N / 2;
        if (pos < 0) pos += Ng;
        X1[(size_t)(r0 + rr) * N + j] = sm[rr * Ng + pos];
    }
}

// ---------------------------------------------------------------------------
// adjoint: column pass (Hermitian symmetrisation, inverse FFT along y, real
// parts of two columns packed as one complex transform, crop, deapodise, mask)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_colpass_adj(PlanDev d, WsLayout L, InstPtrs wsp, float* __restrict__ f,
                                                     int NP, int n_sum)
{
    extern __shared__ float2 sm[];
    __shared__ float gsum_s;
    const int b = blockIdx.y;
    const int N = d.N, Ng = d.Ng, CT = 2 * NP;
    char* wb = wsp.ws + (size_t)b * wsp.stride;
    const float2* X1 = (const float2*)(wb + L.x1);
    const float* red = (const float*)(wb + L.red);
    float* fb = f + (size_t)b * N * N;
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int t = 0; t < n_sum; ++t) s += red[t];
        gsum_s = s;
    }
    const int j0 = blockIdx.x * CT;
    const int top = Ng / 2 + 4;
    for (int e = threadIdx.x; e < NP * Ng; e += blockDim.x) {
        const int p = e / Ng, q = e - p * Ng;
        const int ja = j0 + 2 * p, jb = ja + 1;
        // stored row of residue q and of -q (or -1 if not stored)
        const int rq = q <= top ? q + 4 : (q >= Ng - 4 ? q - Ng + 4 : -1);
        const int qn = q == 0 ? 0 : Ng - q;
        const int rn = qn <= top ? qn + 4 : (qn >= Ng - 4 ? qn - Ng + 4 : -1);
        float2 ua = make_float2(0.f, 0.f), una = ua, ub = ua, unb = ua;
        if (ja < N) {
            if (rq >= 0) ua = X1[(size_t)rq * N + ja];
            if (rn >= 0) una = X1[(size_t)rn * N + ja];
        }
        if (jb < N) {
            if (rq >= 0) ub = X1[(size_t)rq * N + jb];
            if (rn >= 0) unb = X1[(size_t)rn * N + jb];
        }
        // z = (ua + conj una)/2 + i (ub + conj unb)/2
        const float2 ha = make_float2(0.5f * (ua.x + una.x), 0.5f * (ua.y - una.y));
        const float2 hb = make_float2(0.5f * (ub.x + unb.x), 0.5f * (ub.y - unb.y));
        sm[e] = make_float2(ha.x - hb.y, ha.y + hb.x);
    }
    __syncthreads();
    fft_lds<kMaxB>(sm, Ng, NP, d.ffts[d.fft_grid], d.tw, true);
    const float kt = d.kappa * d.h2 * gsum_s;
    for (int e = threadIdx.x; e < N * CT; e += blockDim.x) {
        const int i = e / CT, jj = e - i * CT, j = j0 + jj;
        if (j >= N) continue;
        int pos = i - N / 2;
        if (pos < 0) pos += Ng;
        const float2 z = sm[(jj >> 1) * Ng + pos];
        const float c = (jj & 1) ? z.y : z.x;
        const int2 mr = d.mask_rows[i];
        fb[(size_t)i * N + j] = (j >= mr.x && j < mr.y) ? d.deap[i] * d.deap[j] * c + kt : 0.f;
    }
}

// ---------------------------------------------------------------------------
// total variation (smoothed, isotropic, forward differences, Neumann boundary)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float tv_mag(const float* f, int n, int i, int j, float eps2, float& dx, float& dy)
{
    const float c = f[(size_t)i * n + j];
    dx = (j + 1 < n) ? f[(size_t)i * n + j + 1] - c : 0.f;
    dy = (i + 1 < n) ? f[(size_t)(i + 1) * n + j] - c : 0.f;
    return sqrtf(dx * dx + dy * dy + eps2);
}

__global__ __launch_bounds__(256) void k_tv_grad(const float* __restrict__ f, float* __restrict__ grad, int n,
                                                 float eps2)
{
    const int b = blockIdx.z;
    const int j = blockIdx.x * 16 + (threadIdx.x & 15);
    const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= n || j >= n) return;
    const float* fb = f + (size_t)b * n * n;
    float dx, dy;
    const float s = tv_mag(fb, n, i, j, eps2, dx, dy);
    float gval = -(dx + dy) / s;
    if (j > 0) {
        float dxl, dyl;
        const float sl = tv_mag(fb, n, i, j - 1, eps2, dxl, dyl);
        gval += dxl / sl;
    }
    if (i > 0) {
        float dxu, dyu;
        const float su = tv_mag(fb, n, i - 1, j, eps2, dxu, dyu);
        gval += dyu / su;
    }
    grad[(size_t)b * n * n + (size_t)i * n + j] = gval;
}

__global__ __launch_bounds__(1024) void k_tv_value(const float* __restrict__ f, float* __restrict__ tv, int n,
                                                   float eps2)
{
    __shared__ float red_s[1024];
    const int b = blockIdx.x;
    const float* fb = f + (size_t)b * n * n;
    float acc = 0.f;
    for (long e = threadIdx.x; e < (long)n * n; e += blockDim.x) {
        const int i = (int)(e / n), j = (int)(e - (long)i * n);
        float dx, dy;
        acc += tv_mag(fb, n, i, j, eps2, dx, dy);
    }
    const float tot = block_sum(acc, red_s);
    if (threadIdx.x == 0) tv[b] = tot;
}

__global__ __launch_bounds__(256) void k_pgd_update(float* __restrict__ f, const float* __restrict__ adj,
                                                    const float* __restrict__ tvg, long count, float tau,
                                                    float lam)
{
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x) {
        float gr = adj[e];
        if (tvg) gr += lam * tvg[e];
        const float v = f[e] - tau * gr;
        f[e] = v > 0.f ? v : 0.f;
    }
}

__global__ __launch_bounds__(256) void k_residual(float* __restrict__ g, const float* __restrict__ gm, long count)
{
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x)
        g[e] = g[e] - gm[e];
}

__global__ __launch_bounds__(1024) void k_half_sq(const float* __restrict__ g, float* __restrict__ sq, long per)
{
    __shared__ float red_s[1024];
    const int b = blockIdx.x;
    const float* gb = g + (size_t)b * per;
    float acc = 0.f;
    for (long e = threadIdx.x; e < per; e += blockDim.x) acc += gb[e] * gb[e];
    const float tot = block_sum(acc, red_s);
    if (threadIdx.x == 0) sq[b] = 0.5f * tot;
}

}  // namespace pat
