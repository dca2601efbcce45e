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

constexpr int kMaxB = 4;  // butterflies per thread per FFT stage (workgroups of up to 1024 threads)

// XCD-aware work mapping.  The hardware hands workgroup w to XCD (w mod 8);
// remap so that XCD x owns the contiguous item range [start(x), start(x+1))
// of the U work items (instance-major), keeping one instance's intermediates
// in one XCD's L2.  Returns -1 for the padding workgroups of the last round.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_item(int w, int U)
{
    const int x = w % kXcds, q = w / kXcds;
    const int Q = U / kXcds, Rm = U - Q * kXcds;
    const int cnt = Q + (x < Rm ? 1 : 0);
    if (q >= cnt) return -1;
    return x * Q + min(x, Rm) + q;
}

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

// Sum of v[0..n) in an order fixed by n alone (64 strided partial sums, then a
// fixed shuffle tree): the same bits for every workgroup size.  Must be
// reached by all threads of the first wave; the total is returned to lane 0.
__device__ __forceinline__ float wave0_fixed_sum(const float* __restrict__ v, int n)
{
    float s = 0.f;
    for (int t = threadIdx.x; t < n; t += 64) s += v[t];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    return s;
}

struct InstPtrs {
    char* ws;         // workspace base of instance 0
    size_t stride;    // bytes per instance
};

// ---------------------------------------------------------------------------
// forward: column pass (FFT along y of real columns, packed in pairs)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void colpass_fwd_tile(const PlanDev& d, const WsLayout& L, const float* __restrict__ fb,
                                                 char* wb, int tile, int NP, float2* sm, float* red_s)
{
    const int N = d.N, Ng = d.Ng, CT = 2 * NP;
    float2* X1 = (float2*)(wb + L.x1);
    float* red = (float*)(wb + L.red);
    const int j0 = tile * CT;
    const TwLds tw = tw_lds_build(sm + NP * Ng, d.ffts[d.fft_grid], d.tw);
    for (int e = threadIdx.x; e < NP * Ng; e += blockDim.x) sm[e] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int e = threadIdx.x; e < N * CT; e += blockDim.x) {
        const int i = e / CT, jj = e - i * CT, j = j0 + jj;
        float v = 0.f;
        if (j < N) {
            const int2 mr = d.mask_rows[i];
            if (j >= mr.x && j < mr.y) v = fb[(size_t)i * N + j] * d.deap[i] * d.deap[j];
        }
        int pos = i - N / 2;
        if (pos < 0) pos += Ng;
        float* slot = (float*)&sm[(jj >> 1) * Ng + pos];
        slot[jj & 1] = v;
    }
    // endpoint term: h^2 times the masked sum of each column, rows in 8 classes
    // mod 8 summed in order (independent of the workgroup size and the tiling)
    for (int t = threadIdx.x; t < 8 * CT; t += blockDim.x) {
        const int jj = t % CT, c = t / CT, j = j0 + jj;
        float sc = 0.f;
        if (j < N)
            for (int i = c; i < N; i += 8) {
                const int2 mr = d.mask_rows[i];
                if (j >= mr.x && j < mr.y) sc += fb[(size_t)i * N + j];
            }
        red_s[t] = sc;
    }
    __syncthreads();
    if ((int)threadIdx.x < CT && j0 + (int)threadIdx.x < N) {
        float sc = 0.f;
        for (int c = 0; c < 8; ++c) sc += red_s[c * CT + threadIdx.x];
        red[j0 + threadIdx.x] = sc * d.h2;
    }
    __syncthreads();
    fft_lds<kMaxB>(sm, Ng, NP, d.ffts[d.fft_grid], tw, false);
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
__device__ __forceinline__ void rowpass_fwd_tile(const PlanDev& d, const WsLayout& L, char* wb, int tile, int RPB,
                                                 float2* sm)
{
    const int N = d.N, Ng = d.Ng;
    const float2* X1 = (const float2*)(wb + L.x1);
    float2* G = (float2*)(wb + L.grid);
    const int r0 = tile * RPB;
    const int nr = min(RPB, d.Hy - r0);
    const TwLds tw = tw_lds_build(sm + RPB * Ng, d.ffts[d.fft_grid], d.tw);
    for (int e = threadIdx.x; e < nr * Ng; e += blockDim.x) sm[e] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int e = threadIdx.x; e < nr * N; e += blockDim.x) {
        const int rr = e / N, j = e - rr * N;
        int pos = j - N / 2;
        if (pos < 0) pos += Ng;
        sm[rr * Ng + pos] = X1[(size_t)(r0 + rr) * N + j];
    }
    __syncthreads();
    fft_lds<kMaxB>(sm, Ng, nr, d.ffts[d.fft_grid], tw, false);
    for (int e = threadIdx.x; e < nr * Ng; e += blockDim.x) G[(size_t)r0 * Ng + e] = sm[e];
}

// ---------------------------------------------------------------------------
// Ring kernels.  One workgroup handles RT consecutive radial frequencies
// (rings) of one instance, one ring after another:
//   forward: the ring's interpolated half-plane values (k_gather), completion
//            F(l + Npsi/2) = conj F(l), angular FFT,
//            a_k = c_k e^{i k theta_0} i^k J_k(lam_n R) W_n F_k / Npsi (k <= K_n),
//            synthesis over detectors h(d) = Re sum_k a_k e^{i k d dtheta}
//            (one inverse FFT of length P after folding k mod P when
//            dtheta = 2 pi / P, else Bluestein with two FFTs of length L),
//            -> hT[d][n]  (real; the cosine transform over n follows)
//   adjoint: the exact transpose, ending with the Hermitian fold and the
//            conjugate half-pixel phase -> H (band order) for the spread.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// forward: ES interpolation of the half spectrum at the half-plane polar
// points, in band order (points sorted by footprint base row r0, then by
// base column bx).  A workgroup owns the points with r0 in [R0, R0 + TH) and
// bx in [C0, C0 + CB); it keeps the 8 spectrum rows r0 .. r0 + 7 of columns
// C0 .. C0 + CB + 6 in an LDS ring buffer (one coalesced row load per band)
// and each thread interpolates one point from LDS.  Output Fb[slot] (band
// order) times the half-pixel phase.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void gather_tile(const PlanDev& d, const WsLayout& L, char* wb, int tile, int TH,
                                            float2* win /* [8][CB + 7] */)
{
    const int Ng = d.Ng, NB = d.NB, Hy = d.Hy;
    const int CB = blockDim.x, W = CB + 7;
    const int ncb = (Ng + CB - 1) / CB;
    const int rbk = tile / ncb, cbk = tile - rbk * ncb;
    const int C0 = cbk * CB, R0 = rbk * TH;
    const int rend = min(R0 + TH, NB);
    const int cend = min(C0 + CB, Ng);
    const float2* __restrict__ G = (const float2*)(wb + L.grid);
    float2* Fb = (float2*)(wb + L.polar);
    // rows R0 .. R0 + 6 of the window
    for (int e = threadIdx.x; e < 7 * W; e += CB) {
        const int rr = e / W, cc = e - rr * W;
        const int r = R0 + rr;
        const int c = (C0 + cc) % Ng;  // the window may wrap around the periodic grid
        win[(r & 7) * W + cc] = r < Hy ? G[(size_t)r * Ng + c] : make_float2(0.f, 0.f);
    }
    for (int rb = R0; rb < rend; ++rb) {
        {
            const int r = rb + 7;  // <= NB - 1 + 7 = Hy - 1
            for (int cc = threadIdx.x; cc < W; cc += CB) {
                const int c = (C0 + cc) % Ng;
                win[(r & 7) * W + cc] = G[(size_t)r * Ng + c];
            }
        }
        __syncthreads();
        const int* bp = d.band_ptr + (size_t)rb * (Ng + 1);
        const int lo = bp[C0], hi = bp[cend];
        for (int s = lo + threadIdx.x; s < hi; s += CB) {
            const float4 gq = d.bpt_geo[s];
            const int c0 = fbits(gq.x) - C0;
            float wx[8], wy[8];
            es_weights8(gq.z, wx);
            es_weights8(gq.w, wy);
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int dy = 0; dy < 8; ++dy) {
                const float2* row = win + ((rb + dy) & 7) * W + c0;
                float2 ra = make_float2(0.f, 0.f);
#pragma unroll
                for (int dx = 0; dx < 8; ++dx) {
                    const float2 gv = row[dx];
                    ra.x += wx[dx] * gv.x;
                    ra.y += wx[dx] * gv.y;
                }
                acc.x += wy[dy] * ra.x;
                acc.y += wy[dy] * ra.y;
            }
            Fb[s] = cmul(acc, d.bpt_phase[s]);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ float2 mul_ipow(float2 v, int k)  // v * i^k
{
    switch (k & 3) {
        case 0: return v;
        case 1: return make_float2(-v.y, v.x);
        case 2: return make_float2(-v.x, -v.y);
        default: return make_float2(v.y, -v.x);
    }
}

// Unpack one bin of a real length-2H DFT from Z = FFT_H(z), z(t) = q(2t) + i q(2t+1):
//   Q_k = (Z_k + conj Z_{H-k}) / 2 - (i/2) w_{2H}^k (Z_k - conj Z_{H-k}),  0 <= k < H.
__device__ __forceinline__ float2 real_unpack(const float2* Z, int H, int k, float2 wk)
{
    const float2 zk = Z[k];
    const float2 zc = cconj(Z[k == 0 ? 0 : H - k]);
    const float2 sm = cadd(zk, zc), df = csub(zk, zc);
    const float2 t = cmul(wk, df);
    return make_float2(0.5f * (sm.x + t.y), 0.5f * (sm.y - t.x));
}

// Layout of the ring kernels' dynamic LDS (float2 slots unless noted).
struct RingLds {
    float2 *sa, *sy, *sc, *twPs, *twNs, *twAs, *twBs;
    float* tile;  // [D][RT] floats
};

__device__ __forceinline__ RingLds ring_lds(float2* sm, const PlanDev& d, int RT)
{
    RingLds r;
    const int Pmax = d.npsi_max / 2;
    const int S = d.syn_len;
    const int B2 = S > Pmax ? S : Pmax;
    const int B3 = d.syn_half ? S / 2 : 0;
    r.sa = sm;
    r.sy = r.sa + Pmax;
    r.sc = r.sy + B2;
    r.tile = (float*)(r.sc + B3);
    r.twPs = (float2*)(r.tile + ((d.D * RT + 1) & ~1));
    r.twNs = r.twPs + tw_lds_slots(Pmax);
    r.twAs = r.twNs + tw_lds_slots(d.npsi_max);
    r.twBs = r.twAs + tw_lds_slots(S);
    return r;
}

template <int RB>
__device__ __forceinline__ void ring_fwd_tile(const PlanDev& d, const WsLayout& L, char* wb, int tile, int RT,
                                              float2* sm)
{
    const float2* __restrict__ Fp = (const float2*)(wb + L.polar);
    float* hT = (float*)(wb + L.hdet);
    const int D = d.D, S = d.syn_len;
    const RingLds R = ring_lds(sm, d, RT);
    float* ot = R.tile;
    const int n0 = tile * RT;
    const int nr = min(RT, d.nlam - n0);
    // synthesis tables: fold with even P -> FFT of P/2 (twB) + twiddles of P (twA); else FFT of S (twA)
    const TwLds twA = tw_lds_build(R.twAs, d.ffts[d.fft_syn], d.tw);
    const TwLds twB = d.syn_half ? tw_lds_build(R.twBs, d.ffts[d.fft_synh], d.tw) : twA;
    for (int r = 0; r < nr; ++r) {
        const int n = n0 + r;
        const int off = d.ring_off[n], P = d.ring_off[n + 1] - off;
        const TwLds twP = tw_lds_build(R.twPs, d.ffts[d.ring_fft[n]], d.tw);   // FFT of length P
        const TwLds twN = tw_lds_build(R.twNs, d.ffts[d.ring_twn[n]], d.tw);   // w_{2P}^k
        // q(m) = Re F + Im F (m < P), Re F - Im F (m >= P) is real; pack z(t) = q(2t) + i q(2t+1)
        for (int t = threadIdx.x; t < P; t += blockDim.x) {
            float qv[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int m = 2 * t + u;
                const bool lo = m < P;
                const float2 F = Fp[d.perm[off + (lo ? m : m - P)]];
                qv[u] = lo ? F.x + F.y : F.x - F.y;
            }
            R.sa[t] = make_float2(qv[0], qv[1]);
        }
        __syncthreads();
        fft_lds<RB>(R.sa, P, 1, d.ffts[d.ring_fft[n]], twP, false);
        const int Kn = d.ring_K[n], jo = d.ring_joff[n];
        // a_k = pre_k i^k Jw_k F_k, F_k = Q_k (k even) or i Q_k (k odd)
        auto amode = [&](int k) {
            float2 Q = real_unpack(R.sa, P, k, twN(k));
            if (k & 1) Q = make_float2(-Q.y, Q.x);
            return cmul(d.syn_pre[k], mul_ipow(cscale(Q, d.Jw[jo + k]), k));
        };
        if (d.fold_P) {
            const int Pf = d.fold_P;
            for (int sidx = threadIdx.x; sidx < Pf; sidx += blockDim.x) {
                float2 acc = make_float2(0.f, 0.f);
                for (int k = sidx; k <= Kn; k += Pf) acc = cadd(acc, amode(k));
                R.sy[sidx] = acc;
            }
            __syncthreads();
            if (d.syn_half) {
                // Re(IFFT_P(y)) as a half-length inverse FFT of the Hermitian part
                const int H2 = Pf / 2;
                for (int sidx = threadIdx.x; sidx < H2; sidx += blockDim.x) {
                    const int s1 = sidx, s2 = sidx + H2;
                    const float2 y1 = R.sy[s1], y1c = cconj(R.sy[s1 == 0 ? 0 : Pf - s1]);
                    const float2 y2 = R.sy[s2], y2c = cconj(R.sy[Pf - s2]);
                    const float2 h1 = cscale(cadd(y1, y1c), 0.5f), h2 = cscale(cadd(y2, y2c), 0.5f);
                    const float2 E = cadd(h1, h2);
                    const float2 O = cmulc(csub(h1, h2), twA(sidx));   // times e^{+2 pi i s / P}
                    R.sc[sidx] = make_float2(E.x - O.y, E.y + O.x);    // E + i O
                }
                __syncthreads();
                fft_lds<RB>(R.sc, H2, 1, d.ffts[d.fft_synh], twB, true);
                for (int q = threadIdx.x; q < D; q += blockDim.x) {
                    const float2 z = R.sc[q >> 1];
                    ot[q * RT + r] = (q & 1) ? z.y : z.x;
                }
            } else {
                fft_lds<RB>(R.sy, Pf, 1, d.ffts[d.fft_syn], twA, true);
                for (int q = threadIdx.x; q < D; q += blockDim.x) ot[q * RT + r] = R.sy[q].x;
            }
        } else {
            for (int q = threadIdx.x; q < S; q += blockDim.x) R.sy[q] = q <= Kn ? amode(q) : make_float2(0.f, 0.f);
            __syncthreads();
            fft_lds<RB>(R.sy, S, 1, d.ffts[d.fft_syn], twA, false);
            for (int q = threadIdx.x; q < S; q += blockDim.x) R.sy[q] = cmul(R.sy[q], d.czt_vhat[q]);
            __syncthreads();
            fft_lds<RB>(R.sy, S, 1, d.ffts[d.fft_syn], twA, true);
            for (int q = threadIdx.x; q < D; q += blockDim.x) {
                const float2 v = R.sy[q], w = d.czt_post[q];
                ot[q * RT + r] = w.x * v.x - w.y * v.y;
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < D * nr; e += blockDim.x) {
        const int q = e / nr, r = e - q * nr;
        hT[(size_t)q * d.nlam + n0 + r] = ot[q * RT + r];
    }
}

template <int RB>
__device__ __forceinline__ void ring_adj_tile(const PlanDev& d, const WsLayout& L, char* wb, int tile, int RT,
                                              float2* sm)
{
    const float* hT = (const float*)(wb + L.hdet);
    float2* Hb = (float2*)(wb + L.polar);
    const int D = d.D, S = d.syn_len;
    const RingLds R = ring_lds(sm, d, RT);
    float* it = R.tile;
    const int n0 = tile * RT;
    const int nr = min(RT, d.nlam - n0);
    const TwLds twA = tw_lds_build(R.twAs, d.ffts[d.fft_syn], d.tw);
    const TwLds twB = d.syn_half ? tw_lds_build(R.twBs, d.ffts[d.fft_synh], d.tw) : twA;
    for (int e = threadIdx.x; e < D * nr; e += blockDim.x) {
        const int q = e / nr, r = e - q * nr;
        it[q * RT + r] = hT[(size_t)q * d.nlam + n0 + r];
    }
    __syncthreads();
    for (int r = 0; r < nr; ++r) {
        const int n = n0 + r;
        const int off = d.ring_off[n], P = d.ring_off[n + 1] - off;
        const int Kn = d.ring_K[n], jo = d.ring_joff[n];
        const TwLds twP = tw_lds_build(R.twPs, d.ffts[d.ring_fft[n]], d.tw);
        const TwLds twN = tw_lds_build(R.twNs, d.ffts[d.ring_twn[n]], d.tw);
        // y~ = FFT of the real detector values, zero-padded to the synthesis length
        if (d.fold_P && d.syn_half) {
            const int H2 = d.fold_P / 2;
            for (int t = threadIdx.x; t < H2; t += blockDim.x) {
                const int q0 = 2 * t, q1 = 2 * t + 1;
                R.sc[t] = make_float2(q0 < D ? it[q0 * RT + r] : 0.f, q1 < D ? it[q1 * RT + r] : 0.f);
            }
            __syncthreads();
            fft_lds<RB>(R.sc, H2, 1, d.ffts[d.fft_synh], twB, false);
        } else if (d.fold_P) {
            for (int sidx = threadIdx.x; sidx < S; sidx += blockDim.x)
                R.sy[sidx] = make_float2(sidx < D ? it[sidx * RT + r] : 0.f, 0.f);
            __syncthreads();
            fft_lds<RB>(R.sy, S, 1, d.ffts[d.fft_syn], twA, false);
        } else {
            for (int q = threadIdx.x; q < S; q += blockDim.x)
                R.sy[q] = q < D ? cmulc(make_float2(it[q * RT + r], 0.f), d.czt_post[q]) : make_float2(0.f, 0.f);
            __syncthreads();
            fft_lds<RB>(R.sy, S, 1, d.ffts[d.fft_syn], twA, false);
            for (int q = threadIdx.x; q < S; q += blockDim.x) R.sy[q] = cmulc(R.sy[q], d.czt_vhat[q]);
            __syncthreads();
            fft_lds<RB>(R.sy, S, 1, d.ffts[d.fft_syn], twA, true);
        }
        // y~ at synthesis index sidx (0 <= sidx < S)
        auto ytil = [&](int sidx) {
            if (!(d.fold_P && d.syn_half)) return R.sy[sidx];
            const int Pf = d.fold_P, H2 = Pf / 2;
            if (sidx == H2) return make_float2(R.sc[0].x - R.sc[0].y, 0.f);
            const bool hi = sidx > H2;
            const int s0 = hi ? Pf - sidx : sidx;
            const float2 v = real_unpack(R.sc, H2, s0, twA(s0));
            return hi ? cconj(v) : v;
        };
        // Q~_k = F~_k (k even) or -i F~_k (k odd), F~_k = conj(pre_k i^k) Jw_k y~_{k mod P}
        for (int k = threadIdx.x; k <= Kn; k += blockDim.x) {
            int sidx = k;
            if (d.fold_P) while (sidx >= d.fold_P) sidx -= d.fold_P;
            const float2 F = cscale(mul_ipow(cmulc(ytil(sidx), d.syn_pre[k]), (4 - (k & 3)) & 3), d.Jw[jo + k]);
            R.sa[k] = (k & 1) ? make_float2(F.y, -F.x) : F;
        }
        __syncthreads();
        // Re(IFFT_{2P}(Q~)) as a half-length inverse FFT: build E + i O in place of the
        // upper part of sa (the Hermitian part of Q~ vanishes above K < P).
        // Q~_h[s] = Q~[s]/2 (0 < s <= K), Re Q~[0] (s = 0); Q~_h[s + P] = conj Q~[P - s]/2 (P - s <= K).
        for (int sidx = threadIdx.x; sidx < P; sidx += blockDim.x) {
            float2 a = make_float2(0.f, 0.f), c = a;
            if (sidx == 0) a = make_float2(R.sa[0].x, 0.f);
            else {
                if (sidx <= Kn) a = cscale(R.sa[sidx], 0.5f);
                if (P - sidx <= Kn) c = cscale(cconj(R.sa[P - sidx]), 0.5f);
            }
            const float2 E = cadd(a, c);
            const float2 O = cmulc(csub(a, c), twN(sidx));
            R.sy[sidx] = make_float2(E.x - O.y, E.y + O.x);
        }
        __syncthreads();
        fft_lds<RB>(R.sy, P, 1, d.ffts[d.ring_fft[n]], twP, true);
        // q~(m): m = 2t -> Re z_t, m = 2t + 1 -> Im z_t;  F~_h(l) = (q~(l) + q~(l+P)) + i (q~(l) - q~(l+P))
        for (int l = threadIdx.x; l < P; l += blockDim.x) {
            const float2 z1 = R.sy[l >> 1];
            const float a = (l & 1) ? z1.y : z1.x;
            const int m = l + P;
            const float2 z2 = R.sy[m >> 1];
            const float c = (m & 1) ? z2.y : z2.x;
            const float2 Fh = make_float2(a + c, a - c);
            Hb[d.perm[off + l]] = cmulc(Fh, d.pt_phase[off + l]);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Cosine transform over radial frequencies, per detector, two detectors packed
// as the real and imaginary parts of one complex sequence (the transform is
// real):  out(q) = sum_p in(p) cos(pi p q / M) = (X[q] + X[2M - q]) / 2 with
// X = FFT_2M of the zero-padded input (p, q >= 1).
//   forward: hT [D][nlam] -> g [D][T] (+ kappa * mass)
//   adjoint: g [D][T] -> hT [D][nlam] (+ per-workgroup partial sums of g)
// ---------------------------------------------------------------------------
// gout / gin point at this instance's [D][T] data.
__device__ __forceinline__ void dct_tile(const PlanDev& d, const WsLayout& L, char* wb, float* __restrict__ gout,
                                         const float* __restrict__ gin, int tile, int DP, int adj, int n_mass,
                                         float2* sm, float* red_s, float* mass_s)
{
    const int twoM = 2 * d.M, D = d.D, T = d.T, NL = d.nlam;
    float* hT = (float*)(wb + L.hdet);
    float* red = (float*)(wb + L.red);
    const int p0 = tile * DP;                        // first detector pair
    const int np = min(DP, (D + 1) / 2 - p0);
    const int nin = adj ? T : NL;
    const int nout = adj ? NL : T;
    const float* src = adj ? gin : hT;
    const int sld = adj ? T : NL;
    if (!adj && threadIdx.x < 64) {
        const float m = wave0_fixed_sum(red, n_mass);
        if (threadIdx.x == 0) *mass_s = m;
    }
    const TwLds tw = tw_lds_build(sm + DP * twoM, d.ffts[d.fft_dct], d.tw);
    for (int e = threadIdx.x; e < np * twoM; e += blockDim.x) sm[e] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int e = threadIdx.x; e < np * nin; e += blockDim.x) {
        const int p = e / nin, q = e - p * nin;
        const int d0 = 2 * (p0 + p);
        const float re = src[(size_t)d0 * sld + q];
        const float im = (d0 + 1 < D) ? src[(size_t)(d0 + 1) * sld + q] : 0.f;
        sm[p * twoM + q + 1] = make_float2(re, im);
    }
    if (adj) {
        // data sum of each detector of the tile: samples in 8 classes mod 8, summed in order
        const int nd = 2 * np;
        for (int t = threadIdx.x; t < 8 * nd; t += blockDim.x) {
            const int dd = t % nd, c = t / nd, dg = 2 * p0 + dd;
            float sc = 0.f;
            if (dg < D)
                for (int q = c; q < T; q += 8) sc += gin[(size_t)dg * T + q];
            red_s[t] = sc;
        }
        __syncthreads();
        if ((int)threadIdx.x < nd && 2 * p0 + (int)threadIdx.x < D) {
            float sc = 0.f;
            for (int c = 0; c < 8; ++c) sc += red_s[c * nd + threadIdx.x];
            red[2 * p0 + threadIdx.x] = sc;
        }
    }
    __syncthreads();
    fft_lds<kMaxB>(sm, twoM, np, d.ffts[d.fft_dct], tw, false);
    const float add = adj ? 0.f : d.kappa * *mass_s;
    float* dst = adj ? hT : gout;
    const int dld = adj ? NL : T;
    for (int e = threadIdx.x; e < np * nout; e += blockDim.x) {
        const int p = e / nout, q = e - p * nout;
        const int d0 = 2 * (p0 + p);
        const float2 a = sm[p * twoM + q + 1], c = sm[p * twoM + twoM - q - 1];
        dst[(size_t)d0 * dld + q] = 0.5f * (a.x + c.x) + add;
        if (d0 + 1 < D) dst[(size_t)(d0 + 1) * dld + q] = 0.5f * (a.y + c.y) + add;
    }
}

// ---------------------------------------------------------------------------
// adjoint: deterministic spread of the polar half-plane values onto G~ [Hy][Ng]
// One lane owns one column; bands (footprint base rows) are swept in order and
// an 8-row register window accumulates; band points are staged in LDS with
// their ES weights.  Every output is a fixed-order sum.  The next band's
// ranges and first points are fetched into registers while the current band
// is processed.
// ---------------------------------------------------------------------------
struct BandMeta {
    int aLo, nA, bLo, ntot, lo, hi;
};

__device__ __forceinline__ BandMeta band_meta(const PlanDev& d, int rb, int C0, int mx, bool active)
{
    const int Ng = d.Ng;
    const int* bp = d.band_ptr + (size_t)rb * (Ng + 1);
    const int lo_col = C0 - 7, hi_col = min(C0 + (int)blockDim.x, Ng);
    BandMeta m;
    m.aLo = lo_col < 0 ? bp[Ng + lo_col] : 0;
    const int aHi = lo_col < 0 ? bp[Ng] : 0;
    m.bLo = bp[max(lo_col, 0)];
    const int bHi = bp[hi_col];
    m.nA = aHi - m.aLo;
    m.ntot = m.nA + (bHi - m.bLo);
    m.lo = m.hi = 0;
    if (active) {
        const int c = mx - 7;
        m.lo = c < 0 ? (bp[Ng + c] - m.aLo) : (m.nA + bp[c] - m.bLo);
        m.hi = m.nA + bp[mx + 1] - m.bLo;
    }
    return m;
}

__device__ __forceinline__ int band_slot(const BandMeta& m, int idx)
{
    return idx < m.nA ? m.aLo + idx : m.bLo + (idx - m.nA);
}

__device__ __forceinline__ void spread_stage(float* wxs, float* wys, float2* hs, int* bxs, int e, float4 gq, float2 h)
{
    float w[8];
    es_weights8(gq.z, w);
#pragma unroll
    for (int k = 0; k < 8; ++k) wxs[e * 8 + k] = w[k];
    es_weights8(gq.w, w);
#pragma unroll
    for (int k = 0; k < 8; ++k) wys[e * 8 + k] = w[k];
    hs[e] = h;
    bxs[e] = fbits(gq.x);
}

__device__ __forceinline__ void spread_visit(const float* wxs, const float* wys, const float2* hs, const int* bxs,
                                             int s0, int s1, int c0, int mx, int Ng, float2 (&acc)[8])
{
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
}

// CAP must be 2 * blockDim.x (two staged points per thread per chunk).
__device__ __forceinline__ void spread_tile(const PlanDev& d, const WsLayout& L, char* wb, int tile, int TH, int CAP,
                                            float* sf /* [CAP][19] */)
{
    const int Ng = d.Ng, NB = d.NB, Hy = d.Hy;
    const int CB = blockDim.x;
    const int ncb = (Ng + CB - 1) / CB;
    const int rb_ = tile / ncb, cb_ = tile - rb_ * ncb;
    const float2* __restrict__ H = (const float2*)(wb + L.polar);
    float2* Gt = (float2*)(wb + L.grid);
    float* wxs = sf;                       // [CAP][8]
    float* wys = sf + CAP * 8;             // [CAP][8]
    float2* hs = (float2*)(sf + CAP * 16); // [CAP]
    int* bxs = (int*)(sf + CAP * 18);      // [CAP]
    const int C0 = cb_ * CB, R0 = rb_ * TH;
    const int mx = C0 + threadIdx.x;
    const bool active = mx < Ng;
    const int rend = min(R0 + TH, Hy);
    float2 acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = make_float2(0.f, 0.f);
    const int band_lo = max(0, R0 - 7), band_hi = min(NB - 1, rend - 1);
    const int e0 = threadIdx.x, e1 = threadIdx.x + CB;
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    BandMeta nm;
    float4 ng0 = zero4, ng1 = zero4;
    float2 nh0 = make_float2(0.f, 0.f), nh1 = nh0;
    if (band_lo <= band_hi) {
        nm = band_meta(d, band_lo, C0, mx, active);
        if (e0 < nm.ntot) { const int sl = band_slot(nm, e0); ng0 = d.bpt_geo[sl]; nh0 = H[sl]; }
        if (e1 < nm.ntot) { const int sl = band_slot(nm, e1); ng1 = d.bpt_geo[sl]; nh1 = H[sl]; }
    }
    for (int rb = band_lo; rb <= band_hi; ++rb) {
        const BandMeta m = nm;
        const float4 g0 = ng0, g1 = ng1;
        const float2 h0 = nh0, h1 = nh1;
        if (rb < band_hi) {  // prefetch the next band
            nm = band_meta(d, rb + 1, C0, mx, active);
            if (e0 < nm.ntot) { const int sl = band_slot(nm, e0); ng0 = d.bpt_geo[sl]; nh0 = H[sl]; }
            if (e1 < nm.ntot) { const int sl = band_slot(nm, e1); ng1 = d.bpt_geo[sl]; nh1 = H[sl]; }
        }
        // chunk 0 from registers
        if (e0 < m.ntot) spread_stage(wxs, wys, hs, bxs, e0, g0, h0);
        if (e1 < m.ntot) spread_stage(wxs, wys, hs, bxs, e1, g1, h1);
        __syncthreads();
        spread_visit(wxs, wys, hs, bxs, m.lo, min(m.hi, CAP), 0, mx, Ng, acc);
        __syncthreads();
        // further chunks (dense bands only)
        for (int c0 = CAP; c0 < m.ntot; c0 += CAP) {
            const int cn = min(CAP, m.ntot - c0);
            for (int e = threadIdx.x; e < cn; e += CB) {
                const int sl = band_slot(m, c0 + e);
                spread_stage(wxs, wys, hs, bxs, e, d.bpt_geo[sl], H[sl]);
            }
            __syncthreads();
            spread_visit(wxs, wys, hs, bxs, max(m.lo, c0), min(m.hi, c0 + cn), c0, mx, Ng, acc);
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
__device__ __forceinline__ void rowpass_adj_tile(const PlanDev& d, const WsLayout& L, char* wb, int tile, int RPB,
                                                 float2* sm)
{
    const int N = d.N, Ng = d.Ng;
    const float2* Gt = (const float2*)(wb + L.grid);
    float2* X1 = (float2*)(wb + L.x1);
    const int r0 = tile * RPB;
    const int nr = min(RPB, d.Hy - r0);
    const TwLds tw = tw_lds_build(sm + RPB * Ng, d.ffts[d.fft_grid], d.tw);
    for (int e = threadIdx.x; e < nr * Ng; e += blockDim.x) sm[e] = Gt[(size_t)r0 * Ng + e];
    __syncthreads();
    fft_lds<kMaxB>(sm, Ng, nr, d.ffts[d.fft_grid], tw, true);
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
__device__ __forceinline__ void colpass_adj_tile(const PlanDev& d, const WsLayout& L, char* wb, float* __restrict__ fb,
                                                 int tile, int NP, int n_sum, float2* sm, float* gsum_s)
{
    const int N = d.N, Ng = d.Ng, CT = 2 * NP;
    const float2* X1 = (const float2*)(wb + L.x1);
    const float* red = (const float*)(wb + L.red);
    if (threadIdx.x < 64) {
        const float s = wave0_fixed_sum(red, n_sum);
        if (threadIdx.x == 0) *gsum_s = s;
    }
    const int j0 = tile * CT;
    const int top = Ng / 2 + 4;
    const TwLds tw = tw_lds_build(sm + NP * Ng, d.ffts[d.fft_grid], d.tw);
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
    fft_lds<kMaxB>(sm, Ng, NP, d.ffts[d.fft_grid], tw, true);
    const float kt = d.kappa * d.h2 * *gsum_s;
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
// Launch wrappers.  Single-plan kernels: `batch` instances of one plan with
// instance workspaces `wsp.stride` bytes apart.  Batch kernels (suffix _b):
// one launch covers every instance of a heterogeneous batch; the workgroup's
// work item is located in the per-stage prefix table and the instance's plan
// is read from the device table.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int batch_find(const int* __restrict__ base, int count, int item)
{
    int lo = 0, hi = count;  // base[lo] <= item < base[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= item) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Locates the workgroup's instance and local tile for stage `st`; false for padding workgroups.
__device__ __forceinline__ bool batch_item(const BatchDev& bt, int st, int& inst, int& tile)
{
    const int* base = bt.base + st * (bt.count + 1);
    const int item = xcd_item(blockIdx.x, base[bt.count]);
    if (item < 0) return false;
    inst = batch_find(base, bt.count, item);
    tile = item - base[inst];
    return true;
}

__global__ __launch_bounds__(1024) void k_colpass_fwd(PlanDev d, WsLayout L, const float* __restrict__ f,
                                                     InstPtrs wsp, int NP)
{
    extern __shared__ float2 sm[];
    __shared__ float red_s[1024];
    const int b = blockIdx.y;
    colpass_fwd_tile(d, L, f + (size_t)b * d.N * d.N, wsp.ws + (size_t)b * wsp.stride, blockIdx.x, NP, sm, red_s);
}

__global__ __launch_bounds__(1024) void k_colpass_fwd_b(BatchDev bt, const float* const* __restrict__ fin, char* ws)
{
    extern __shared__ float2 sm[];
    __shared__ float red_s[1024];
    int i, tile;
    if (!batch_item(bt, kStCol, i, tile)) return;
    const BatchInst& I = bt.inst[i];
    const PlanDev d = I.d;
    colpass_fwd_tile(d, I.L, fin[i], ws + I.ws_off, tile, I.col_np, sm, red_s);
}

__global__ __launch_bounds__(1024) void k_rowpass_fwd(PlanDev d, WsLayout L, InstPtrs wsp, int RPB)
{
    extern __shared__ float2 sm[];
    rowpass_fwd_tile(d, L, wsp.ws + (size_t)blockIdx.y * wsp.stride, blockIdx.x, RPB, sm);
}

__global__ __launch_bounds__(1024) void k_rowpass_fwd_b(BatchDev bt, char* ws)
{
    extern __shared__ float2 sm[];
    int i, tile;
    if (!batch_item(bt, kStRow, i, tile)) return;
    const BatchInst& I = bt.inst[i];
    const PlanDev d = I.d;
    rowpass_fwd_tile(d, I.L, ws + I.ws_off, tile, I.row_rpb, sm);
}

__global__ __launch_bounds__(256) void k_gather(PlanDev d, WsLayout L, InstPtrs wsp, int TH, int batch)
{
    extern __shared__ float2 win[];
    const int per = ((d.Ng + (int)blockDim.x - 1) / (int)blockDim.x) * ((d.NB + TH - 1) / TH);
    const int item = xcd_item(blockIdx.x, per * batch);
    if (item < 0) return;
    const int b = item / per;
    gather_tile(d, L, wsp.ws + (size_t)b * wsp.stride, item - b * per, TH, win);
}

__global__ __launch_bounds__(256) void k_gather_b(BatchDev bt, char* ws)
{
    extern __shared__ float2 win[];
    int i, tile;
    if (!batch_item(bt, kStGather, i, tile)) return;
    const BatchInst& I = bt.inst[i];
    const PlanDev d = I.d;
    gather_tile(d, I.L, ws + I.ws_off, tile, I.gat_th, win);
}

template <int RB>
__global__ __launch_bounds__(1024) void k_ring_fwd(PlanDev d, WsLayout L, InstPtrs wsp, int RT, int batch)
{
    extern __shared__ float2 sm[];
    const int ntile = (d.nlam + RT - 1) / RT;
    const int item = xcd_item(blockIdx.x, ntile * batch);
    if (item < 0) return;
    const int b = item / ntile;
    ring_fwd_tile<RB>(d, L, wsp.ws + (size_t)b * wsp.stride, item - b * ntile, RT, sm);
}

template <int RB>
__global__ __launch_bounds__(1024) void k_ring_fwd_b(BatchDev bt, char* ws)
{
    extern __shared__ float2 sm[];
    int i, tile;
    if (!batch_item(bt, kStRing, i, tile)) return;
    const BatchInst& I = bt.inst[i];
    const PlanDev d = I.d;
    ring_fwd_tile<RB>(d, I.L, ws + I.ws_off, tile, I.ring_rt, sm);
}

template <int RB>
__global__ __launch_bounds__(1024) void k_ring_adj(PlanDev d, WsLayout L, InstPtrs wsp, int RT, int batch)
{
    extern __shared__ float2 sm[];
    const int ntile = (d.nlam + RT - 1) / RT;
    const int item = xcd_item(blockIdx.x, ntile * batch);
    if (item < 0) return;
    const int b = item / ntile;
    ring_adj_tile<RB>(d, L, wsp.ws + (size_t)b * wsp.stride, item - b * ntile, RT, sm);
}

template <int RB>
__global__ __launch_bounds__(1024) void k_ring_adj_b(BatchDev bt, char* ws)
{
    extern __shared__ float2 sm[];
    int i, tile;
    if (!batch_item(bt, kStRing, i, tile)) return;
    const BatchInst& I = bt.inst[i];
    const PlanDev d = I.d;
    ring_adj_tile<RB>(d, I.L, ws + I.ws_off, tile, I.ring_rt, sm);
}

__global__ __launch_bounds__(1024) void k_dct_det(PlanDev d, WsLayout L, InstPtrs wsp, float* __restrict__ gout,
                                                  const float* __restrict__ gin, int DP, int adj, int n_mass, int batch)
{
    extern __shared__ float2 sm[];
    __shared__ float red_s[1024];
    __shared__ float mass_s;
    const int ntile = ((d.D + 1) / 2 + DP - 1) / DP;
    const int item = xcd_item(blockIdx.x, ntile * batch);
    if (item < 0) return;
    const int b = item / ntile;
    const size_t go = (size_t)b * d.D * d.T;
    dct_tile(d, L, wsp.ws + (size_t)b * wsp.stride, adj ? nullptr : gout + go, adj ? gin + go : nullptr,
             item - b * ntile, DP, adj, n_mass, sm, red_s, &mass_s);
}

// adj = 0: out[i] receives the data of instance i; adj = 1: in[i] is read.
__global__ __launch_bounds__(1024) void k_dct_det_b(BatchDev bt, char* ws, float* const* __restrict__ out,
                                                    const float* const* __restrict__ in, int adj)
{
    extern __shared__ float2 sm[];
    __shared__ float red_s[1024];
    __shared__ float mass_s;
    int i, tile;
    if (!batch_item(bt, kStDct, i, tile)) return;
    const BatchInst& I = bt.inst[i];
    const PlanDev d = I.d;
    dct_tile(d, I.L, ws + I.ws_off, adj ? nullptr : out[i], adj ? in[i] : nullptr, tile, I.dct_dp, adj, d.N, sm,
             red_s, &mass_s);
}

__global__ __launch_bounds__(256) void k_spread(PlanDev d, WsLayout L, InstPtrs wsp, int TH, int CAP, int batch)
{
    extern __shared__ float sf[];
    const int per = ((d.Ng + (int)blockDim.x - 1) / (int)blockDim.x) * ((d.Hy + TH - 1) / TH);
    const int item = xcd_item(blockIdx.x, per * batch);
    if (item < 0) return;
    const int b = item / per;
    spread_tile(d, L, wsp.ws + (size_t)b * wsp.stride, item - b * per, TH, CAP, sf);
}

__global__ __launch_bounds__(256) void k_spread_b(BatchDev bt, char* ws)
{
    extern __shared__ float sf[];
    int i, tile;
    if (!batch_item(bt, kStSpread, i, tile)) return;
    const BatchInst& I = bt.inst[i];
    const PlanDev d = I.d;
    spread_tile(d, I.L, ws + I.ws_off, tile, I.spr_th, 2 * (int)blockDim.x, sf);
}

__global__ __launch_bounds__(1024) void k_rowpass_adj(PlanDev d, WsLayout L, InstPtrs wsp, int RPB)
{
    extern __shared__ float2 sm[];
    rowpass_adj_tile(d, L, wsp.ws + (size_t)blockIdx.y * wsp.stride, blockIdx.x, RPB, sm);
}

__global__ __launch_bounds__(1024) void k_rowpass_adj_b(BatchDev bt, char* ws)
{
    extern __shared__ float2 sm[];
    int i, tile;
    if (!batch_item(bt, kStRow, i, tile)) return;
    const BatchInst& I = bt.inst[i];
    const PlanDev d = I.d;
    rowpass_adj_tile(d, I.L, ws + I.ws_off, tile, I.row_rpb, sm);
}

__global__ __launch_bounds__(1024) void k_colpass_adj(PlanDev d, WsLayout L, InstPtrs wsp, float* __restrict__ f,
                                                     int NP, int n_sum)
{
    extern __shared__ float2 sm[];
    __shared__ float gsum_s;
    const int b = blockIdx.y;
    colpass_adj_tile(d, L, wsp.ws + (size_t)b * wsp.stride, f + (size_t)b * d.N * d.N, blockIdx.x, NP, n_sum, sm,
                     &gsum_s);
}

__global__ __launch_bounds__(1024) void k_colpass_adj_b(BatchDev bt, char* ws, float* const* __restrict__ fout)
{
    extern __shared__ float2 sm[];
    __shared__ float gsum_s;
    int i, tile;
    if (!batch_item(bt, kStCol, i, tile)) return;
    const BatchInst& I = bt.inst[i];
    const PlanDev d = I.d;
    colpass_adj_tile(d, I.L, ws + I.ws_off, fout[i], tile, I.col_np, d.D, sm, &gsum_s);
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
