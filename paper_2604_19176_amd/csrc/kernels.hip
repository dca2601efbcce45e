// kernels.hip -- gfx950 kernels of the PAT operator pair.
//
// Forward A (steps of the discrete operator; layouts per instance, row-major):
//   colpass_fwd : f [N][N] -> mask, deapodise, zero-pad to Ng, FFT along y of
//                 column pairs packed as complex -> X1 [Hy][N] (rows m_y = -4..Ng/2+4)
//                 + per-column sums of h^2 m f (endpoint term)
//   rowpass_fwd : X1 -> FFT along x -> G [Hy][Ng]  (oversampled half spectrum)
//   gather      : ES interpolation of G at the half-plane polar points, times
//                 the half-pixel phase -> F [npts] in ring order
//   ring_fwd    : per radial frequency n: angular FFT of the ring (completed by
//                 conjugate symmetry), weights c_k i^k J_k(lam_n R) W_n / Npsi(n),
//                 synthesis over the detector angles (one FFT after folding
//                 k mod P, or Bluestein) -> hT [nlam][D]
//   syn_dense   : explicit detector angles only: the synthesis as a matrix-core
//                 product of the ring's mode coefficients with a cos/sin table
//   dct         : per detector: g(d, j) = sum_n hT[n][d] cos(pi n j / M) via one
//                 complex FFT of length 2M for two detectors, + kappa * mass -> g [D][T]
// Adjoint A* runs the exact transposes in reverse (dct, ring_adj or
// syn_dense adjoint + ring_adj, spread (which applies the conjugate half-pixel
// phase as it stages each point), rowpass_adj, colpass_adj).  No
// floating-point atomics anywhere: every sum has a fixed order, so results are
// bitwise repeatable.
#include "cfft.hpp"
#include "fft.hpp"
#include "pat_internal.hpp"

namespace pat {


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

// The 8 taps of the ES kernel phi(t) = exp(beta (sqrt(1 - (2t/w)^2) - 1)) at
// t = frac + 3 - d (d = 0..7, frac in [0, 1)): z = t / 4 lies in [-1, 1], so
// 1 - z^2 only needs a clamp against rounding below 0; the hardware square
// root and base-2 exponential (about 1 ulp each) are used directly, since the
// argument of the exponential lies in [-beta log2(e), 0].  The same routine
// serves the interpolation and the spread, which keeps them exact transposes.
__device__ __forceinline__ void es_weights8(float frac, float (&w)[8])
{
    constexpr float kb = (float)(kEsBeta * 1.4426950408889634);  // beta log2(e)
    const float z0 = frac * 0.25f;
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const float z = z0 + 0.25f * (float)(3 - d);
        const float q = fmaxf(fmaf(-z, z, 1.0f), 0.0f);
        w[d] = __builtin_amdgcn_exp2f(fmaf(kb, __builtin_amdgcn_sqrtf(q), -kb));
    }
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

// Row / sample classes of the endpoint-term sums; red_s[1024] holds
// kSumClasses x (columns or detectors of a tile), so tiles have at most 32 of
// either (col_np, dct_dp <= 16).
constexpr int kSumClasses = 32;

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

// st(t, ld(t)) for t < count by the workgroup (t = t0 + threadIdx.x + j blockDim.x,
// U values of t per thread and chunk).  A chunk issues all of a thread's loads
// before its first store, and no load sits under a divergent branch (indices
// past the end are clamped to count - 1 and their values dropped), so a chunk
// waits for one memory latency instead of one per element.
template <int U, class Ld, class St>
__device__ __forceinline__ void fill_batched(int count, Ld ld, St st)
{
    const int tid = threadIdx.x, bd = blockDim.x;
    for (int t0 = 0; t0 < count; t0 += U * bd) {
        decltype(ld(0)) v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) v[j] = ld(min(t0 + tid + j * bd, count - 1));
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int t = t0 + tid + j * bd;
            if (t < count) st(t, v[j]);
        }
    }
}

struct IdxVal {
    int i;
    float2 v;
};

struct IdxF {
    int i;
    float v;
};

// ---------------------------------------------------------------------------
// The grid transforms (length Ng, `nseq` sequences at stride ld in LDS): with
// a compile-time length (plans with grid_spec) sequence s is transformed by
// threads s T .. s T + T - 1 (T = cfft_lanes(Ng), or twice that for `wide`
// tiles of one sequence: the same butterflies in the same order on more
// lanes); else by the run-time plan.
// ---------------------------------------------------------------------------
template <int NG, bool INV, int T>
__device__ __forceinline__ void grid_cfft(const PlanDev& d, float2* x, int ld, int nseq)
{
    const int sq = threadIdx.x / T;
    cfft<NG, INV, T>(x + (size_t)min(sq, nseq - 1) * ld, d.ctw + d.grid_ctw, threadIdx.x - sq * T, sq < nseq);
}

template <bool INV>
__device__ __forceinline__ void grid_fft(const PlanDev& d, float2* x, int ld, int nseq, const float2* tb, bool wide)
{
    if (d.grid_spec) {
        switch (d.Ng) {
#define PAT_GRID_CASE(NG)                                                                        \
    case NG:                                                                                     \
        if (wide) grid_cfft<NG, INV, 2 * cfft_lanes(NG)>(d, x, ld, nseq);                       \
        else grid_cfft<NG, INV, cfft_lanes(NG)>(d, x, ld, nseq);                                 \
        break;
            PAT_GRID_LENGTHS(PAT_GRID_CASE)
#undef PAT_GRID_CASE
            default: break;
        }
    } else {
        fft_lds<INV>(x, ld, nseq, d.ffts[d.fft_grid], tb);
    }
}

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
    const float2* tb = fft_twiddles_to_lds(sm + NP * Ng, d.ffts[d.fft_grid], d.tw);
    for (int e = threadIdx.x; e < NP * Ng; e += blockDim.x) sm[e] = make_float2(0.f, 0.f);
    __syncthreads();
    // the tile's columns, masked and deapodised, at rows centred in the padded
    // column (batched, branch-free loads; columns past N read as zero).
    // Endpoint term: h^2 times the masked sum of each column, rows in
    // kSumClasses classes (row i in class i mod kSumClasses), each summed in
    // order, then the classes in order (independent of the workgroup size and
    // of the tiling).  With kSumClasses x CT threads each thread's elements are
    // one column's rows of one class, in order: the class sums are taken from
    // the values loaded here; else a second loop reads the columns again.
    const float rcpCT = 1.0f / (float)CT;
    const bool own_class = (int)blockDim.x == kSumClasses * CT;
    float csum = 0.f;
    struct Elt {
        int i;
        float v, raw;
        bool in;
    };
    fill_batched<4>(
        N * CT,
        [&](int e) {
            int i, jj;
            fdivmod(e, CT, rcpCT, i, jj);
            const int j = j0 + jj, jc = min(j, N - 1);
            const int2 mr = d.mask_rows[i];
            const float fv = fb[(size_t)i * N + jc], di = d.deap[i], dj = d.deap[jc];
            const bool in = j < N && j >= mr.x && j < mr.y;
            const float v = in ? fv * di * dj : 0.f;
            int pos = i - N / 2;
            if (pos < 0) pos += Ng;
            return Elt{2 * ((jj >> 1) * Ng + pos) + (jj & 1), v, fv, in};
        },
        [&](int, Elt el) {
            ((float*)sm)[el.i] = el.v;
            csum = el.in ? csum + el.raw : csum;
        });
    if (own_class) red_s[threadIdx.x] = csum;  // class threadIdx.x / CT, column threadIdx.x % CT
    for (int t = threadIdx.x; !own_class && t < kSumClasses * CT; t += blockDim.x) {
        const int jj = t % CT, c = t / CT, j = j0 + jj, jc = min(j, N - 1);
        float sc = 0.f;
        for (int i0 = c; i0 < N; i0 += 4 * kSumClasses) {
            float v[4];
            bool in[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + u * kSumClasses, ic = min(i, N - 1);
                const int2 mr = d.mask_rows[ic];
                v[u] = fb[(size_t)ic * N + jc];
                in[u] = i < N && j < N && j >= mr.x && j < mr.y;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) sc = in[u] ? sc + v[u] : sc;
        }
        red_s[t] = sc;
    }
    __syncthreads();
    if ((int)threadIdx.x < CT && j0 + (int)threadIdx.x < N) {
        float sc = 0.f;
        for (int c = 0; c < kSumClasses; ++c) sc += red_s[c * CT + threadIdx.x];
        red[j0 + threadIdx.x] = sc * d.h2;
    }
    __syncthreads();
    grid_fft<false>(d, sm, Ng, NP, tb, NP == 1);
    fill_batched<4>(
        d.Hy * CT,
        [&](int e) {
            int r, jj;
            fdivmod(e, CT, rcpCT, r, jj);
            const int j = j0 + jj;
            const int m = r - 4;
            const int ip = m < 0 ? m + Ng : m;
            const int in = m > 0 ? Ng - m : -m;
            const float2 zp = sm[(jj >> 1) * Ng + ip], zn = sm[(jj >> 1) * Ng + in];
            // even column: (Z(m) + conj Z(-m)) / 2; odd: (Z(m) - conj Z(-m)) / (2i)
            const float2 o = (jj & 1) == 0 ? make_float2(0.5f * (zp.x + zn.x), 0.5f * (zp.y - zn.y))
                                           : make_float2(0.5f * (zp.y + zn.y), -0.5f * (zp.x - zn.x));
            return IdxVal{j < N ? r * N + j : -1, o};
        },
        [&](int, IdxVal iv) {
            if (iv.i >= 0) X1[iv.i] = iv.v;
        });
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
    const float2* tb = fft_twiddles_to_lds(sm + RPB * Ng, d.ffts[d.fft_grid], d.tw);
    for (int e = threadIdx.x; e < nr * Ng; e += blockDim.x) sm[e] = make_float2(0.f, 0.f);
    __syncthreads();
    const float rcpN = 1.0f / (float)N;
    fill_batched<4>(
        nr * N,
        [&](int e) {
            int rr, j;
            fdivmod(e, N, rcpN, rr, j);
            int pos = j - N / 2;
            if (pos < 0) pos += Ng;
            return IdxVal{rr * Ng + pos, X1[(size_t)(r0 + rr) * N + j]};
        },
        [&](int, IdxVal iv) { sm[iv.i] = iv.v; });
    __syncthreads();
    grid_fft<false>(d, sm, Ng, nr, tb, RPB == 1);
    fill_batched<4>(
        nr * Ng, [&](int e) { return sm[e]; }, [&](int e, float2 v) { G[(size_t)r0 * Ng + e] = v; });
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
//            -> hT[n][d]  (real; the cosine transform over n follows)
//   adjoint: the exact transpose, ending with the Hermitian fold -> H,
//            stored in band order for the spread, which applies the conjugate
//            half-pixel phase as it stages each point from a band-order table
//            (scattered writes here, contiguous reads there: reading
//            H through each band-order point's ring index instead makes every
//            wave-load of the spread touch tens of cache lines per instance,
//            which costs the spread more than the scatter costs here).
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// forward: ES interpolation of the half spectrum at the half-plane polar
// points.  Points are visited in band order (sorted by footprint base row r0,
// then base column bx); a tile is TH bands x CB columns: the points with r0
// in [R0, R0 + TH) and bx in [C0, C0 + CB).  The tile's whole window of the
// spectrum (rows R0 .. R0 + TH + 6, columns C0 .. C0 + CB + 6, wrapping
// around the periodic grid) is loaded into LDS once; then each band is
// handled by kGatherThreads / TH threads, one point per thread at a time.
// Output: the polar value times the half-pixel phase, stored in ring order
// (the ring-order index is the y field of the point's band-order geometry).
// ---------------------------------------------------------------------------
// IB instances of one plan share a tile (wbs[b], b < nb; b >= nb is padding):
// one window per instance, the ES weights and indexing of each point once.
template <int IB, int CB>
__device__ __forceinline__ void gather_tile(const PlanDev& d, const WsLayout& L, char* const (&wbs)[IB], int nb,
                                            int tile, int TH, float2* win)
{
    constexpr int W = CB + 7;  // compile-time row stride: the 64 taps are immediate offsets
    const int Ng = d.Ng, NB = d.NB, Hy = d.Hy;
    const int R = TH + 7, RW = R * W;
    const int ncb = (Ng + CB - 1) / CB;
    const int rbk = tile / ncb, cbk = tile - rbk * ncb;
    const int C0 = cbk * CB, R0 = rbk * TH;
    const int cend = min(C0 + CB, Ng);
    const int nbands = min(TH, NB - R0);
    int* seg_lo = (int*)(win + IB * RW);
    int* seg_hi = seg_lo + TH;
#pragma unroll
    for (int b = 0; b < IB; ++b) {
        if (b >= nb) break;
        const float2* __restrict__ G = (const float2*)(wbs[b] + L.grid);
        float2* wn = win + b * RW;
        // window rows R0 .. R0 + TH + 6 (zero past the stored rows), columns
        // C0 .. C0 + CB + 6 wrapped mod Ng (C0 + CB + 6 < 2 Ng)
        fill_batched<4>(
            RW,
            [&](int e) {
                const int rr = e / W, cc = e - rr * W;
                const int r = R0 + rr;
                int c = C0 + cc;
                c = c >= Ng ? c - Ng : c;
                const float2 v = G[(size_t)min(r, Hy - 1) * Ng + c];
                return r < Hy ? v : make_float2(0.f, 0.f);
            },
            [&](int e, float2 v) { wn[e] = v; });
    }
    if ((int)threadIdx.x < nbands) {
        const int* bp = d.band_ptr + (size_t)(R0 + threadIdx.x) * (Ng + 1);
        seg_lo[threadIdx.x] = bp[C0];
        seg_hi[threadIdx.x] = bp[cend];
    }
    __syncthreads();
    const int Q = kGatherThreads / TH;  // threads per band
    const int bnd = threadIdx.x / Q, u = threadIdx.x - bnd * Q;
    if (bnd >= nbands) return;          // no barrier follows
    const int hi = seg_hi[bnd];
    // the next point's geometry is loaded while the current one is interpolated
    // (index clamped to the segment's last point, or to point 0 for an empty
    // segment at the start: always a valid point)
    const int slast = max(hi - 1, 0);
    int s = seg_lo[bnd] + u;
    float4 ngq = d.bpt_geo[min(s, slast)];
    float2 nph = d.bpt_phase[min(s, slast)];
    for (; s < hi; s += Q) {
        const float4 gq = ngq;
        const float2 ph = nph;
        const int ri = fbits(gq.y);  // ring-order index of the point
        const int sn = min(s + Q, slast);
        ngq = d.bpt_geo[sn];
        nph = d.bpt_phase[sn];
        const int c0 = fbits(gq.x) - C0;
        float wx[8], wy[8];
        es_weights8(gq.z, wx);
        es_weights8(gq.w, wy);
#pragma unroll
        for (int b = 0; b < IB; ++b) {
            if (b >= nb) break;
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int dy = 0; dy < 8; ++dy) {
                const float2* row = win + b * RW + (bnd + dy) * W + c0;
                float2 ra = make_float2(0.f, 0.f);
#pragma unroll
                for (int dx = 0; dx < 8; ++dx) {
                    const float2 gv = row[dx];
                    ra.x = fmaf(wx[dx], gv.x, ra.x);
                    ra.y = fmaf(wx[dx], gv.y, ra.y);
                }
                acc.x = fmaf(wy[dy], ra.x, acc.x);
                acc.y = fmaf(wy[dy], ra.y, acc.y);
            }
            ((float2*)(wbs[b] + L.polar))[ri] = cmul(acc, ph);
        }
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

// Layout of the ring kernels' dynamic LDS (float2 slots, ring_lds_slots):
// sa (ring FFT; the half-length synthesis buffer sc shares it), sy
// (synthesis), and the two-level twiddles of lengths Npsi(n) (twN) and S
// (twA) used outside the transforms.  The transforms read their per-pass
// twiddles, and the mode loops the ring's coefficients, from global memory
// (tables shared by all instances of a plan, cache resident): small LDS per
// ring keeps many rings resident per CU, and nothing is held in registers
// across a transform.
struct RingLds {
    float2 *sa, *sc, *sy, *twN, *twA;
};

__device__ __forceinline__ RingLds ring_lds(float2* sm, const PlanDev& d)
{
    RingLds r;
    const int Pmax = d.npsi_max / 2;
    const int S = d.syn_len;
    const int B1 = max(Pmax, d.syn_half ? S / 2 : 0);
    const int B2 = max(S, Pmax);
    r.sa = sm;
    r.sc = sm;
    r.sy = sm + B1;
    r.twN = r.sy + B2;
    r.twA = r.twN + ring_tw_slots(d.npsi_max);
    return r;
}

__device__ __forceinline__ void ring_fwd_tile(const PlanDev& d, const WsLayout& L, char* wb, int tile, int RT,
                                              float2* sm)
{
    const float2* __restrict__ Fp = (const float2*)(wb + L.polar);
    float* hT = (float*)(wb + L.hdet);  // [nlam][D]
    const int D = d.D, S = d.syn_len;
    const int tid = threadIdx.x, bd = blockDim.x;
    const RingLds R = ring_lds(sm, d);
    const int n0 = tile * RT;
    const int nr = min(RT, d.nlam - n0);
    // synthesis: fold with even P -> transform of P/2 + twiddles of P (twA); else transform of S
    const TwLds twA = d.syn_dense ? TwLds{R.twA, R.twA, 0} : tw_lds_build(R.twA, d.ffts[d.fft_syn], d.tw);
    const FftDev& fS = d.ffts[d.fft_synh];
    const float2* __restrict__ tbS = d.tw + fS.tb;
    for (int r = 0; r < nr; ++r) {
        const int n = n0 + r;
        const int off = d.ring_off[n], P = d.ring_off[n + 1] - off;
        const int Kn = d.ring_K[n];
        const float2* __restrict__ cf = d.coef + d.ring_joff[n];
        float* hn = hT + (size_t)n * D;
        const FftDev& fR = d.ffts[d.ring_fft[n]];
        const float2* __restrict__ tbR = d.tw + fR.tb;
        const FftDev& fN = d.ffts[d.ring_twn[n]];
        // the ring's inputs, all loads in flight together: twiddles w_{2P}^k (twN)
        // and the polar values, packed as follows:
        // q(m) = Re F + Im F (m < P), Re F - Im F (m >= P) is real; z(t) = q(2t) + i q(2t+1)
        const TwFetch twf = tw_lds_fetch(fN, d.tw);
        fill_batched<kRingFillUnroll>(
            P,
            [&](int t) {
                float qv[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int m = 2 * t + u;
                    const bool lo = m < P;
                    const float2 F = Fp[off + (lo ? m : m - P)];
                    qv[u] = lo ? F.x + F.y : F.x - F.y;
                }
                return make_float2(qv[0], qv[1]);
            },
            [&](int t, float2 v) { R.sa[t] = v; });
        const TwLds twN = tw_lds_store(R.twN, fN, d.tw, twf);
        __syncthreads();
        fft_lds<false, kRingFftMaxButterflies>(R.sa, P, 1, fR, tbR);
        if (d.syn_dense) {
            // explicit detector angles: the mode coefficients a_k go to the workspace;
            // the dense product with the cos/sin table synthesises the detectors
            float2* am = (float2*)(wb + L.modes) + (size_t)n * d.Kp;
            fill_batched<kRingFillUnroll>(
                Kn + 1, [&](int k) { return cmul(cf[k], real_unpack(R.sa, P, k, twN(k))); },
                [&](int k, float2 v) { am[k] = v; });
            __syncthreads();
            continue;
        }
        // y = the a_k = coef_k Q_k (Q: the real length-2P transform of q) folded
        // mod Pf (fold) or zero-padded to S (chirp-z), summed in order of k: pass
        // 0 writes k < Pf, each further pass adds the next Pf modes
        const int Pf = d.fold_P ? d.fold_P : S;
        for (int q = tid; q < Pf; q += bd)
            if (q > Kn) R.sy[q] = make_float2(0.f, 0.f);
        for (int base = 0; base <= Kn; base += Pf) {
            if (base) __syncthreads();
            fill_batched<kRingFillUnroll>(
                min(Kn + 1 - base, Pf),
                [&](int t) {
                    const int k = base + t;
                    const float2 a = cmul(cf[k], real_unpack(R.sa, P, k, twN(k)));
                    return base ? cadd(R.sy[t], a) : a;
                },
                [&](int t, float2 v) { R.sy[t] = v; });
        }
        __syncthreads();
        if (d.fold_P) {
            if (d.syn_half) {
                // Re(IFFT_P(y)) as a half-length inverse FFT of the Hermitian part
                const int H2 = Pf / 2;
                fill_batched<kRingFillUnroll>(
                    H2,
                    [&](int sidx) {
                        const int s1 = sidx, s2 = sidx + H2;
                        const float2 y1 = R.sy[s1], y1c = cconj(R.sy[s1 == 0 ? 0 : Pf - s1]);
                        const float2 y2 = R.sy[s2], y2c = cconj(R.sy[Pf - s2]);
                        const float2 h1 = cscale(cadd(y1, y1c), 0.5f), h2 = cscale(cadd(y2, y2c), 0.5f);
                        const float2 E = cadd(h1, h2);
                        const float2 O = cmulc(csub(h1, h2), twA(sidx));  // times e^{+2 pi i s / P}
                        return make_float2(E.x - O.y, E.y + O.x);         // E + i O
                    },
                    [&](int sidx, float2 v) { R.sc[sidx] = v; });
                __syncthreads();
                fft_lds<true, kRingFftMaxButterflies>(R.sc, H2, 1, fS, tbS);
                // detector q is point s q of the P-point grid
                fill_batched<kRingFillUnroll>(
                    D,
                    [&](int q) {
                        const int j = q * d.fold_s;
                        const float2 z = R.sc[j >> 1];
                        return (j & 1) ? z.y : z.x;
                    },
                    [&](int q, float v) { hn[q] = v; });
            } else {
                fft_lds<true, kRingFftMaxButterflies>(R.sy, Pf, 1, fS, tbS);
                fill_batched<kRingFillUnroll>(
                    D, [&](int q) { return R.sy[q * d.fold_s].x; }, [&](int q, float v) { hn[q] = v; });
            }
        } else {
            fft_lds<false, kRingFftMaxButterflies>(R.sy, S, 1, fS, tbS);
            for (int q = tid; q < S; q += bd) R.sy[q] = cmul(R.sy[q], d.czt_vhat[q]);
            __syncthreads();
            fft_lds<true, kRingFftMaxButterflies>(R.sy, S, 1, fS, tbS);
            for (int q = tid; q < D; q += bd) {
                const float2 v = R.sy[q], w = d.czt_post[q];
                hn[q] = w.x * v.x - w.y * v.y;
            }
        }
        __syncthreads();
    }
}

// Value at point j of the P-point angular grid of the detector values placed
// at points s q (q < D), zero elsewhere.
__device__ __forceinline__ float grid_det(const float* hn, int j, int s, float rcp_s, int D)
{
    int q = j, rem = 0;
    if (s != 1) fdivmod(j, s, rcp_s, q, rem);
    const float v = hn[min(q, D - 1)];  // unconditional load (batched by the caller), value selected
    return (rem == 0 && q < D) ? v : 0.f;
}

__device__ __forceinline__ void ring_adj_tile(const PlanDev& d, const WsLayout& L, char* wb, int tile, int RT,
                                              float2* sm)
{
    const float* hT = (const float*)(wb + L.hdet);  // [nlam][D]
    float2* Hb = (float2*)(wb + L.polar);
    const int D = d.D, S = d.syn_len;
    const int tid = threadIdx.x, bd = blockDim.x;
    const RingLds R = ring_lds(sm, d);
    const int n0 = tile * RT;
    const int nr = min(RT, d.nlam - n0);
    const bool half = d.fold_P && d.syn_half;
    const float rcp_s = 1.0f / (float)max(d.fold_s, 1);
    const float rcp_P = __builtin_amdgcn_rcpf((float)max(d.fold_P, 1));  // fdivmod makes k mod P exact
    // the mode values Q~ go to qb, the Hermitian-part input of the ring's inverse FFT to eb
    float2* const qb = half ? R.sy : R.sa;
    float2* const eb = half ? R.sa : R.sy;
    const TwLds twA = d.syn_dense ? TwLds{R.twA, R.twA, 0} : tw_lds_build(R.twA, d.ffts[d.fft_syn], d.tw);
    const FftDev& fS = d.ffts[d.fft_synh];
    const float2* __restrict__ tbS = d.tw + fS.tb;
    for (int r = 0; r < nr; ++r) {
        const int n = n0 + r;
        const int off = d.ring_off[n], P = d.ring_off[n + 1] - off;
        const int Kn = d.ring_K[n];
        const float2* __restrict__ cf = d.coef + d.ring_joff[n];
        const float* hn = hT + (size_t)n * D;
        // explicit detector angles: y~_k from the dense product (workspace), no transform
        const float2* __restrict__ am = (const float2*)(wb + L.modes) + (size_t)n * d.Kp;
        const FftDev& fR = d.ffts[d.ring_fft[n]];
        const float2* __restrict__ tbR = d.tw + fR.tb;
        const FftDev& fN = d.ffts[d.ring_twn[n]];
        const TwFetch twf = tw_lds_fetch(fN, d.tw);
        // the ring's inputs, all loads in flight together: twiddles (twN) and the
        // detector values zero-padded to the synthesis length; then y~ = their
        // FFT.  Explicit angles: Q~ directly.
        if (d.syn_dense) {
            fill_batched<kRingFillUnroll>(
                Kn + 1, [&](int k) { return cmulc(am[k], cf[k]); }, [&](int k, float2 v) { qb[k] = v; });
            tw_lds_store(R.twN, fN, d.tw, twf);
        } else if (half) {
            const int H2 = d.fold_P / 2;
            fill_batched<kRingFillUnroll>(
                H2,
                [&](int t) {
                    return make_float2(grid_det(hn, 2 * t, d.fold_s, rcp_s, D), grid_det(hn, 2 * t + 1, d.fold_s, rcp_s, D));
                },
                [&](int t, float2 v) { R.sc[t] = v; });
            tw_lds_store(R.twN, fN, d.tw, twf);
            __syncthreads();
            fft_lds<false, kRingFftMaxButterflies>(R.sc, H2, 1, fS, tbS);
        } else if (d.fold_P) {
            fill_batched<kRingFillUnroll>(
                S, [&](int t) { return make_float2(grid_det(hn, t, d.fold_s, rcp_s, D), 0.f); },
                [&](int t, float2 v) { R.sy[t] = v; });
            tw_lds_store(R.twN, fN, d.tw, twf);
            __syncthreads();
            fft_lds<false, kRingFftMaxButterflies>(R.sy, S, 1, fS, tbS);
        } else {
            fill_batched<kRingFillUnroll>(
                S,
                [&](int q) {
                    const int qc = min(q, D - 1);
                    const float2 v = cmulc(make_float2(hn[qc], 0.f), d.czt_post[qc]);
                    return q < D ? v : make_float2(0.f, 0.f);
                },
                [&](int q, float2 v) { R.sy[q] = v; });
            tw_lds_store(R.twN, fN, d.tw, twf);
            __syncthreads();
            fft_lds<false, kRingFftMaxButterflies>(R.sy, S, 1, fS, tbS);
            for (int q = tid; q < S; q += bd) R.sy[q] = cmulc(R.sy[q], d.czt_vhat[q]);
            __syncthreads();
            fft_lds<true, kRingFftMaxButterflies>(R.sy, S, 1, fS, tbS);
        }
        const TwLds twN{R.twN, R.twN + 64, 0};
        // y~ at synthesis index sidx (0 <= sidx < S)
        auto ytil = [&](int sidx) {
            if (!half) return R.sy[sidx];
            const int Pf = d.fold_P, H2 = Pf / 2;
            if (sidx == H2) return make_float2(R.sc[0].x - R.sc[0].y, 0.f);
            const bool hi = sidx > H2;
            const int s0 = hi ? Pf - sidx : sidx;
            const float2 v = real_unpack(R.sc, H2, s0, twA(s0));
            return hi ? cconj(v) : v;
        };
        // Q~_k = conj(coef_k) y~_{k mod Pf}
        if (!d.syn_dense) {
            fill_batched<kRingFillUnroll>(
                Kn + 1,
                [&](int k) {
                    int sidx = k, fq;
                    if (d.fold_P) fdivmod(k, d.fold_P, rcp_P, fq, sidx);
                    return cmulc(ytil(sidx), cf[k]);
                },
                [&](int k, float2 v) { qb[k] = v; });
        }
        __syncthreads();
        // Re(IFFT_{2P}(Q~)) as a half-length inverse FFT: E + i O from the
        // Hermitian part of Q~ (which vanishes above K_n < P).
        // Q~_h[s] = Q~[s]/2 (0 < s <= K), Re Q~[0] (s = 0); Q~_h[s + P] = conj Q~[P - s]/2 (P - s <= K).
        fill_batched<kRingFillUnroll>(
            P,
            [&](int sidx) {
                // reads clamped into qb[0 .. Kn], values outside the mode range dropped
                const float2 q1 = qb[min(sidx, Kn)], q2 = qb[min(P - sidx, Kn)];
                const float2 zero = make_float2(0.f, 0.f);
                const float2 a = sidx == 0 ? make_float2(q1.x, 0.f) : (sidx <= Kn ? cscale(q1, 0.5f) : zero);
                const float2 c = (sidx != 0 && P - sidx <= Kn) ? cscale(cconj(q2), 0.5f) : zero;
                const float2 E = cadd(a, c);
                const float2 O = cmulc(csub(a, c), twN(sidx));
                return make_float2(E.x - O.y, E.y + O.x);
            },
            [&](int sidx, float2 v) { eb[sidx] = v; });
        __syncthreads();
        fft_lds<true, kRingFftMaxButterflies>(eb, P, 1, fR, tbR);
        // q~(m): m = 2t -> Re z_t, m = 2t + 1 -> Im z_t;  F~_h(l) = (q~(l) + q~(l+P)) + i (q~(l) - q~(l+P))
        fill_batched<kRingFillUnroll>(
            P,
            [&](int l) {
                const float2 z1 = eb[l >> 1];
                const float a = (l & 1) ? z1.y : z1.x;
                const int m = l + P;
                const float2 z2 = eb[m >> 1];
                const float c = (m & 1) ? z2.y : z2.x;
                const float2 Fh = make_float2(a + c, a - c);
                return IdxVal{d.band_of[off + l], Fh};
            },
            [&](int, IdxVal iv) { Hb[iv.i] = iv.v; });
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Ring kernels with compile-time transforms (plans with ring_spec: a uniform
// arc whose pitch is 2 pi s / P with P even, modes folded mod P, every length
// with a cfft.hpp plan).  The same operator as ring_fwd_tile /
// ring_adj_tile; lanes 0..63 of wave 0 do all the work in one LDS buffer of
// max(Npsi_max, P) / 2 complex values:
//   forward: head<Pn> (packed ring -> ring transform -> modes times their
//            coefficients, folded, straight into the half-length synthesis
//            input), synthesis transform (length P/2), tail (detectors);
//   adjoint: head (detectors -> synthesis transform), tail<Pn> (mode
//            coefficients straight into the half-length input of the ring's
//            inverse transform, transform, band-order stores).
// Each mode is evaluated once: the synthesis input at s and P/2 - s (forward),
// or the ring input at u and Pn - u (adjoint), need the same modes, so one
// lane computes both.  Twiddles come from the plan's FP64-computed tables.
// ---------------------------------------------------------------------------
struct RingSpecArgs {
    int off, Kn;
    const float2* __restrict__ cf;   // ring coefficients coef_k, k <= K_n
    const float2* __restrict__ ctwR; // ring transform table
    const float2* __restrict__ uw;   // w_{2 Pn}^k, k = 0..Pn
};

__device__ __forceinline__ RingSpecArgs ring_spec_args(const PlanDev& d, int n)
{
    RingSpecArgs a;
    a.off = d.ring_off[n];
    a.Kn = d.ring_K[n];
    a.cf = d.coef + d.ring_joff[n];
    a.ctwR = d.ctw + d.ring_ctw[n];
    a.uw = d.ctw + d.ring_uw[n];
    return a;
}

// E + i O of the real-output half-length synthesis at index s (0 <= s <= P/2)
// from y_s, y_{P-s}, y_{s+P/2}, y_{P/2-s} (y_q = a_q, q <= K_n; 0 above)
__device__ __forceinline__ float2 syn_prologue(float2 y1, float2 y1m, float2 y2, float2 y2m, float2 w)
{
    const float2 h1 = cscale(cadd(y1, cconj(y1m)), 0.5f), h2 = cscale(cadd(y2, cconj(y2m)), 0.5f);
    const float2 E = cadd(h1, h2);
    const float2 O = cmulc(csub(h1, h2), w);  // times e^{+2 pi i s / P}
    return make_float2(E.x - O.y, E.y + O.x);
}

template <int Pn, int T>
__device__ __forceinline__ void ring_fwd_spec_head(const PlanDev& d, const float2* __restrict__ Fp,
                                                   const RingSpecArgs& a, float2* buf, float2* syn)
{
    const int lane = threadIdx.x;
    const bool act = lane < T;
    // the ring's half-plane values packed as the real sequence q(m) = Re F + Im F
    // (m < Pn), Re F - Im F (m >= Pn), z(t) = q(2t) + i q(2t + 1)
    if (act) {
        constexpr int RND = (Pn + T - 1) / T;
        float2 v[RND];
#pragma unroll
        for (int i = 0; i < RND; ++i) {
            const int t = min(lane + i * T, Pn - 1);
            const int m0 = 2 * t, m1 = 2 * t + 1;
            const float2 F0 = Fp[a.off + (m0 < Pn ? m0 : m0 - Pn)];
            const float2 F1 = Fp[a.off + (m1 < Pn ? m1 : m1 - Pn)];
            v[i] = make_float2(m0 < Pn ? F0.x + F0.y : F0.x - F0.y, m1 < Pn ? F1.x + F1.y : F1.x - F1.y);
        }
#pragma unroll
        for (int i = 0; i < RND; ++i) {
            const int t = lane + i * T;
            if (Pn % T == 0 || t < Pn) buf[t] = v[i];
        }
    }
    __syncthreads();
    cfft<Pn, false, cfft_wg_lanes(Pn, T)>(buf, a.ctwR, lane, lane < cfft_wg_lanes(Pn, T));
    // a_k = coef_k Q_k for k <= K_n (zero above), in place of Z: the pair (k, Pn - k)
    // shares sm = Z_k + conj Z_{Pn-k}, df = Z_k - conj Z_{Pn-k} and t = w_{2Pn}^k df,
    //   Q_k = sm/2 - (i/2) t,  Q_{Pn-k} = conj(sm)/2 - (i/2) conj(t)
    // (w_{2Pn}^{Pn-k} = -conj w_{2Pn}^k)
    // (each lane reads and writes only its own pair's two slots)
    if (act) {
        constexpr int PAIRS = Pn / 2 + 1;  // k = 0 .. Pn/2
#pragma unroll
        for (int i = 0; i < (PAIRS + T - 1) / T; ++i) {
            const int k0 = lane + i * T;
            const int k = min(k0, PAIRS - 1);
            const int kc = k == 0 ? 0 : Pn - k;
            const float2 zk = buf[k];
            const float2 zc = cconj(buf[kc]);
            const float2 sm = cadd(zk, zc), df = csub(zk, zc);
            const float2 t = cmul(a.uw[k], df);
            const float2 Q1 = make_float2(0.5f * (sm.x + t.y), 0.5f * (sm.y - t.x));
            const float2 Q2 = make_float2(0.5f * (sm.x - t.y), 0.5f * (-sm.y - t.x));
            const float2 c1 = a.cf[min(k, a.Kn)], c2 = a.cf[min(kc, a.Kn)];
            const float2 v1 = k <= a.Kn ? cmul(c1, Q1) : make_float2(0.f, 0.f);
            const float2 v2 = kc <= a.Kn ? cmul(c2, Q2) : make_float2(0.f, 0.f);
            if (PAIRS % T == 0 || k0 < PAIRS) {
                buf[k] = v1;
                if (k != 0 && 2 * k != Pn) buf[kc] = v2;
            }
        }
    }
    __syncthreads();
    const int Pf = d.fold_P, SH = Pf >> 1;
    // y_q = sum of a_k over k = q mod Pf, k < Pn (a_k = 0 above K_n), in increasing k
    auto mode = [&](int q) {
        float2 y = q < Pn ? buf[q] : make_float2(0.f, 0.f);
        for (int k = q + Pf; k < Pn; k += Pf) y = cadd(y, buf[k]);
        return y;
    };
    const float2* __restrict__ sw = d.ctw + d.syn_sw;
    const int items = (SH + 1) >> 1;
    if (act) {
        for (int s = lane; s < items; s += T) {
            if (s == 0) {
                const float2 y0 = mode(0), yh = mode(SH), yq = mode(SH >> 1), y3 = mode(SH + (SH >> 1));
                syn[0] = syn_prologue(y0, y0, yh, yh, sw[0]);
                if ((SH & 1) == 0) syn[SH >> 1] = syn_prologue(yq, y3, y3, yq, sw[SH >> 1]);
            } else {
                const float2 ya = mode(s), yb = mode(Pf - s), yc = mode(s + SH), yd = mode(SH - s);
                syn[s] = syn_prologue(ya, yb, yc, yd, sw[s]);
                syn[SH - s] = syn_prologue(yd, yc, yb, ya, sw[SH - s]);
            }
        }
    }
    __syncthreads();
}

template <int T>
__device__ __forceinline__ void ring_fwd_spec_tail(const PlanDev& d, const float2* buf, float* hn)
{
    const int lane = threadIdx.x;
    if (lane < T) {
        // detector q is point s q of the P-point grid: Re part at even, Im at odd points
        for (int q0 = 0; q0 < d.D; q0 += 4 * T) {
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = min(q0 + lane + u * T, d.D - 1);
                const int j = q * d.fold_s;
                const float2 z = buf[j >> 1];
                v[u] = (j & 1) ? z.y : z.x;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + lane + u * T;
                if (q < d.D) hn[q] = v[u];
            }
        }
    }
    __syncthreads();
}

template <int G, int W>
__device__ __forceinline__ void ring_fwd_spec_tile(const PlanDev& d, const WsLayout& L, char* wb, int n, float2* buf)
{
    // one ring per workgroup: a loop over rings would keep every length's
    // synthesis twiddles live across it
    const float2* __restrict__ Fp = (const float2*)(wb + L.polar);
    float* hT = (float*)(wb + L.hdet);  // [nlam][D]
    float2* syn = buf + d.npsi_max / 2;  // the synthesis input after the ring buffer
    const RingSpecArgs a = ring_spec_args(d, n);
    const int Pn = d.ring_off[n + 1] - a.off;
    constexpr int T = ring_spec_threads(G, W);
    switch (Pn) {
#define PAT_RING_FWD_HEAD(LEN) \
    case LEN: ring_fwd_spec_head<LEN, T>(d, Fp, a, buf, syn); break;
        PAT_CFFT_LENGTHS_LO(PAT_RING_FWD_HEAD)
        default:
            if constexpr (G >= 1) {
                switch (Pn) {
                    PAT_CFFT_LENGTHS_HI(PAT_RING_FWD_HEAD)
                    default:
                        if constexpr (G >= 2) {
                            switch (Pn) {
                                PAT_CFFT_LENGTHS_HI2(PAT_RING_FWD_HEAD)
                                default: break;
                            }
                        }
                        break;
                }
            }
            break;
#undef PAT_RING_FWD_HEAD
    }
    cfft_run_wg<true, G, T>(syn, d.fold_P >> 1, d.ctw + d.syn_ctw);
    ring_fwd_spec_tail<T>(d, syn, hT + (size_t)n * d.D);
}

template <int T>
__device__ __forceinline__ void ring_adj_spec_head(const PlanDev& d, const float* __restrict__ hn, float2* buf)
{
    const int lane = threadIdx.x;
    const int SH = d.fold_P >> 1, fs = d.fold_s, D = d.D;
    // the detector values at points s q of the P-point grid (zero between), packed
    // as z(t) = h(2t) + i h(2t + 1)
    if (lane < T) {
        const float rcp_s = __builtin_amdgcn_rcpf((float)fs);
        for (int t0 = 0; t0 < SH; t0 += 2 * T) {
            float2 v[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int t = min(t0 + lane + u * T, SH - 1);
                float h[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int j = 2 * t + e;
                    int q = j, rem = 0;
                    if (fs != 1) fdivmod(j, fs, rcp_s, q, rem);
                    const float x = hn[min(q, D - 1)];
                    h[e] = (rem == 0 && q < D) ? x : 0.f;
                }
                v[u] = make_float2(h[0], h[1]);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int t = t0 + lane + u * T;
                if (t < SH) buf[t] = v[u];
            }
        }
    }
    __syncthreads();
}

template <int Pn, int T>
__device__ __forceinline__ void ring_adj_spec_tail(const PlanDev& d, const RingSpecArgs& a, float2* syn,
                                                   float2* buf, float2* Hb)
{
    const int lane = threadIdx.x;
    const bool act = lane < T;
    const int Pf = d.fold_P, SH = Pf >> 1;
    const float2* __restrict__ sw = d.ctw + d.syn_sw;
    // the ring points' band-order slots, for the stores at the end: loaded now,
    // in flight during the transforms
    constexpr int RO = (Pn + T - 1) / T;
    int slot[RO];
#pragma unroll
    for (int i = 0; i < RO; ++i) slot[i] = d.band_of[a.off + min(lane + i * T, Pn - 1)];
    // y~ at synthesis index q (0 <= q <= P/2) from the half-length transform Z,
    // in place of Z (slot P/2 after it): the pair (s, SH - s) shares
    // sm = Z_s + conj Z_{SH-s}, df = Z_s - conj Z_{SH-s}, t = w_P^s df,
    //   y~_s = sm/2 - (i/2) t,  y~_{SH-s} = conj(sm)/2 - (i/2) conj(t),
    // and y~_{SH} = Re Z_0 - Im Z_0; above P/2, y~_{P-q} = conj y~_q
    // (each lane reads and writes only its own pair's slots)
    float2* ys = syn;
    if (act) {
        const int PAIRS = SH / 2 + 1;  // s = 0 .. SH/2
        for (int s = lane; s < PAIRS; s += T) {
            const int sc = s == 0 ? 0 : SH - s;
            const float2 zk = ys[s];
            const float2 zc = cconj(ys[sc]);
            const float2 sm = cadd(zk, zc), df = csub(zk, zc);
            const float2 t = cmul(sw[s], df);
            ys[s] = make_float2(0.5f * (sm.x + t.y), 0.5f * (sm.y - t.x));
            if (s == 0) ys[SH] = make_float2(zc.x + zc.y, 0.f);
            else if (2 * s != SH) ys[sc] = make_float2(0.5f * (sm.x - t.y), 0.5f * (-sm.y - t.x));
        }
    }
    __syncthreads();
    // Q~_k = conj(coef_k) y~_{k mod P} for k <= K_n (0 above)
    auto qmode = [&](int k) {
        const int kc = min(k, a.Kn);
        int kf = kc;  // synthesis index k mod Pf
        while (kf >= Pf) kf -= Pf;
        const bool hi = kf > SH;
        const float2 y0 = ys[hi ? Pf - kf : kf];
        const float2 v = cmulc(hi ? cconj(y0) : y0, a.cf[kc]);
        return k <= a.Kn ? v : make_float2(0.f, 0.f);
    };
    // input of the ring's half-length inverse transform at u: E + i O from the
    // Hermitian part of Q~ (q1 = Q~_u, q2 = Q~_{Pn-u})
    auto herm = [&](int u, float2 q1, float2 q2) {
        const float2 zero = make_float2(0.f, 0.f);
        const float2 av = u == 0 ? make_float2(q1.x, 0.f) : cscale(q1, 0.5f);
        const float2 cv = u == 0 ? zero : cscale(cconj(q2), 0.5f);
        const float2 E = cadd(av, cv);
        const float2 O = cmulc(csub(av, cv), a.uw[u]);
        return make_float2(E.x - O.y, E.y + O.x);
    };
    // item u < (Pn + 1)/2 writes slots u and Pn - u; item 0 writes slot 0 and,
    // for even Pn, slot Pn/2 (one path for every lane: no branch on u, the
    // loads of all rounds can be issued together)
    constexpr int items = (Pn + 1) / 2;
    if (act) {
#pragma unroll
        for (int i = 0; i < (items + T - 1) / T; ++i) {
            const int u0 = lane + i * T;
            const bool own = items % T == 0 || u0 < items;
            const int u = min(u0, items - 1);
            const int u2 = u == 0 ? ((Pn & 1) == 0 ? Pn / 2 : 0) : Pn - u;  // the second slot
            const float2 qa = qmode(u), qb = qmode(u2);
            const float2 ha = herm(u, qa, qb), hb = herm(u2, qb, u == 0 ? qb : qa);
            if (own) {
                buf[u] = ha;
                if (u2 != 0) buf[u2] = hb;
            }
        }
    }
    __syncthreads();
    cfft<Pn, true, cfft_wg_lanes(Pn, T)>(buf, a.ctwR, lane, lane < cfft_wg_lanes(Pn, T));
    // q~(m): m = 2t -> Re z_t, m = 2t + 1 -> Im z_t;  F~_h(l) = (q~(l) + q~(l+Pn)) + i (q~(l) - q~(l+Pn)),
    // stored in band order (the spread applies the conjugate half-pixel phase)
    if (act) {
#pragma unroll
        for (int i = 0; i < RO; ++i) {
            const int l0 = lane + i * T;
            const int l = min(l0, Pn - 1);
            const float2 z1 = buf[l >> 1];
            const float av = (l & 1) ? z1.y : z1.x;
            const int m = l + Pn;
            const float2 z2 = buf[m >> 1];
            const float cv = (m & 1) ? z2.y : z2.x;
            const float2 Fh = make_float2(av + cv, av - cv);
            if (Pn % T == 0 || l0 < Pn) Hb[slot[i]] = Fh;
        }
    }
    __syncthreads();
}

template <int G, int W>
__device__ __forceinline__ void ring_adj_spec_tile(const PlanDev& d, const WsLayout& L, char* wb, int n, float2* buf)
{
    const float* hT = (const float*)(wb + L.hdet);  // [nlam][D]
    float2* Hb = (float2*)(wb + L.polar);
    float2* syn = buf + d.npsi_max / 2;  // the synthesis transform after the ring buffer
    constexpr int T = ring_spec_threads(G, W);
    ring_adj_spec_head<T>(d, hT + (size_t)n * d.D, syn);
    cfft_run_wg<false, G, T>(syn, d.fold_P >> 1, d.ctw + d.syn_ctw);
    const RingSpecArgs a = ring_spec_args(d, n);
    const int Pn = d.ring_off[n + 1] - a.off;
    switch (Pn) {
#define PAT_RING_ADJ_TAIL(LEN) \
    case LEN: ring_adj_spec_tail<LEN, T>(d, a, syn, buf, Hb); break;
        PAT_CFFT_LENGTHS_LO(PAT_RING_ADJ_TAIL)
        default:
            if constexpr (G >= 1) {
                switch (Pn) {
                    PAT_CFFT_LENGTHS_HI(PAT_RING_ADJ_TAIL)
                    default:
                        if constexpr (G >= 2) {
                            switch (Pn) {
                                PAT_CFFT_LENGTHS_HI2(PAT_RING_ADJ_TAIL)
                                default: break;
                            }
                        }
                        break;
                }
            }
            break;
#undef PAT_RING_ADJ_TAIL
    }
}

// ---------------------------------------------------------------------------
// Explicit detector angles: the angular synthesis h(n, d) = Re sum_k a_k(n)
// e^{ik theta_d} (eq. (2)) as a dense product on the matrix cores,
//   forward  H[n][d] = sum_{j < 2(K_n + 1)} A[n][j] S[j][d],
//   adjoint  A[n][j] = sum_d H[n][d] S[j][d],
// with A the mode coefficients (re, im interleaved: [nlam][2(K+1)] floats) and
// S the FP64-computed table S[2k] = cos(k theta_d), S[2k+1] = -sin(k theta_d).
// 64 x 64 output tiles, four waves of 32 x 32 each (v_mfma_f32_32x32x2f32:
// lane i holds A[i % 32][i / 32] and B[i / 32][i % 32]; accumulator r holds
// D[8 (r / 4) + 4 (i / 32) + r % 4][i % 32]); the contraction runs in chunks of
// 32 staged in LDS.  Rows are rings: a tile stops at 2 (K_n + 1) of its last
// ring (K_n grows with n), and A's entries beyond a ring's own cut-off are
// read as zero, so the product skips the modes a ring does not have.
// ---------------------------------------------------------------------------
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kSynTile = 64;     // output tile side
constexpr int kSynChunk = 32;    // contraction chunk
constexpr int kSynThreads = 256; // four waves
constexpr int kSynLd = kSynChunk + 4;                    // LDS row stride (floats) of the operand fragments
constexpr int kSynPer = kSynTile * kSynChunk / kSynThreads;  // fragment elements fetched per thread
constexpr int kSynRows = kSynThreads / kSynChunk;        // rows one fetch step covers

// Operand fragments of a chunk in LDS, [64 tile rows / columns][kSynLd]: the
// element of contraction index k (0 .. kSynChunk-1) sits in slot
// (k & 1) * kSynChunk/2 + k / 2, so that the values lane group h = lane / 32
// feeds to the MFMAs of a chunk (k = 2 i + h) are contiguous: 128-bit LDS reads.
__device__ __forceinline__ int syn_slot(int k) { return (k & 1) * (kSynChunk / 2) + (k >> 1); }

__device__ __forceinline__ void syn_mfma_chunk(const float (*Ap)[kSynLd], const float (*Bp)[kSynLd], int wm, int wn,
                                               int lane, f32x16& acc)
{
    constexpr int NV = kSynChunk / 8;  // float4 per operand and lane
    const int h = lane >> 5, rr = lane & 31;
    const float4* ar = (const float4*)&Ap[wm + rr][h * (kSynChunk / 2)];
    const float4* br = (const float4*)&Bp[wn + rr][h * (kSynChunk / 2)];
    float4 a4[NV], b4[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        a4[i] = ar[i];
        b4[i] = br[i];
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[i].x, b4[i].x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[i].y, b4[i].y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[i].z, b4[i].z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[i].w, b4[i].w, acc, 0, 0, 0);
    }
}

// Forward: each chunk, thread t holds kSynPer values of the mode block
// (ring r = t / kSynChunk + kSynRows i, index c = t % kSynChunk) and kSynPer of
// the table block (k = t / 64 + 4 i, detector c = t % 64); the next chunk is fetched into
// registers while the matrix cores work on the current one.  Loads go to
// clamped in-bounds addresses without branches and masked entries are zeroed
// afterwards, so all 16 loads of a chunk are in flight together.
__device__ __forceinline__ void syn_dense_fwd_tile(const PlanDev& d, const WsLayout& L, char* wb, int tile)
{
    __shared__ __align__(16) float Ap[kSynTile][kSynLd];  // [ring][slot]
    __shared__ __align__(16) float Bp[kSynTile][kSynLd];  // [detector][slot]
    const int J = 2 * d.Kp, D = d.D, NL = d.nlam;
    const int tq = (D + kSynTile - 1) / kSynTile;
    const int n0 = (tile / tq) * kSynTile, q0 = (tile % tq) * kSynTile;
    const float* __restrict__ A = (const float*)(wb + L.modes);
    const float* __restrict__ S = d.syn_tab;
    float* __restrict__ H = (float*)(wb + L.hdet);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    const int jmax = 2 * (d.ring_K[min(n0 + kSynTile - 1, NL - 1)] + 1);
    const int nch = (jmax + kSynChunk - 1) / kSynChunk;
    // this thread's rings: row offsets and mode limits 2 (K_n + 1) (0 past nlam)
    int aoff[kSynPer], jlim[kSynPer];
#pragma unroll
    for (int i = 0; i < kSynPer; ++i) {
        const int n = n0 + tid / kSynChunk + kSynRows * i;
        const int nc = min(n, NL - 1);
        aoff[i] = nc * J;
        jlim[i] = n < NL ? 2 * (d.ring_K[nc] + 1) : 0;
    }
    const int ca = tid % kSynChunk, cb = tid & 63;
    const int q = q0 + cb, qc = min(q, D - 1);
    float ra[kSynPer], rb[kSynPer];
    auto fetch = [&](int j0) {
        const int j = j0 + ca, jc = min(j, J - 1);
#pragma unroll
        for (int i = 0; i < kSynPer; ++i) {
            ra[i] = A[aoff[i] + jc];
            const int jb = j0 + (tid >> 6) + 4 * i;
            rb[i] = S[(size_t)min(jb, J - 1) * D + qc];
        }
#pragma unroll
        for (int i = 0; i < kSynPer; ++i) {
            if (j >= jlim[i]) ra[i] = 0.f;
            if (j0 + (tid >> 6) + 4 * i >= J || q >= D) rb[i] = 0.f;
        }
    };
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    if (nch > 0) fetch(0);
    for (int ch = 0; ch < nch; ++ch) {
#pragma unroll
        for (int i = 0; i < kSynPer; ++i) {
            Ap[tid / kSynChunk + kSynRows * i][syn_slot(ca)] = ra[i];
            Bp[cb][syn_slot((tid >> 6) + 4 * i)] = rb[i];
        }
        __syncthreads();
        if (ch + 1 < nch) fetch((ch + 1) * kSynChunk);
        syn_mfma_chunk(Ap, Bp, wm, wn, lane, acc);
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int n = n0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), qq = q0 + wn + (lane & 31);
        if (n < NL && qq < D) H[(size_t)n * D + qq] = acc[r];
    }
}

// Adjoint: both operands are read along the detector index (row
// r = t / kSynChunk + kSynRows i, detector c = t % kSynChunk), with the same
// branch-free clamped loads.
__device__ __forceinline__ void syn_dense_adj_tile(const PlanDev& d, const WsLayout& L, char* wb, int tile)
{
    __shared__ __align__(16) float Ap[kSynTile][kSynLd];  // [ring][slot]
    __shared__ __align__(16) float Bp[kSynTile][kSynLd];  // [table row j][slot]
    const int J = 2 * d.Kp, D = d.D, NL = d.nlam;
    const int tj = (J + kSynTile - 1) / kSynTile;
    const int n0 = (tile / tj) * kSynTile, j0 = (tile % tj) * kSynTile;
    // rows j >= 2 (K_n + 1) of every ring of the tile are never read: skip the tile
    if (j0 >= 2 * (d.ring_K[min(n0 + kSynTile - 1, NL - 1)] + 1)) return;
    const float* __restrict__ H = (const float*)(wb + L.hdet);
    const float* __restrict__ S = d.syn_tab;
    float* __restrict__ A = (float*)(wb + L.modes);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    const int nch = (D + kSynChunk - 1) / kSynChunk;
    const int ca = tid % kSynChunk, r0 = tid / kSynChunk;
    int hoff[kSynPer], soff[kSynPer];
    unsigned okh = 0, oks = 0;  // row i inside nlam / inside the table
#pragma unroll
    for (int i = 0; i < kSynPer; ++i) {
        const int n = n0 + r0 + kSynRows * i, j = j0 + r0 + kSynRows * i;
        hoff[i] = min(n, NL - 1) * D;
        soff[i] = min(j, J - 1) * D;
        okh |= (n < NL ? 1u : 0u) << i;
        oks |= (j < J ? 1u : 0u) << i;
    }
    float ra[kSynPer], rb[kSynPer];
    auto fetch = [&](int c0) {
        const int qv = c0 + ca, qc = min(qv, D - 1);
#pragma unroll
        for (int i = 0; i < kSynPer; ++i) {
            ra[i] = H[hoff[i] + qc];
            rb[i] = S[soff[i] + qc];
        }
#pragma unroll
        for (int i = 0; i < kSynPer; ++i) {
            if (qv >= D || !((okh >> i) & 1u)) ra[i] = 0.f;
            if (qv >= D || !((oks >> i) & 1u)) rb[i] = 0.f;
        }
    };
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    fetch(0);
    for (int ch = 0; ch < nch; ++ch) {
#pragma unroll
        for (int i = 0; i < kSynPer; ++i) {
            Ap[r0 + kSynRows * i][syn_slot(ca)] = ra[i];
            Bp[r0 + kSynRows * i][syn_slot(ca)] = rb[i];
        }
        __syncthreads();
        if (ch + 1 < nch) fetch((ch + 1) * kSynChunk);
        syn_mfma_chunk(Ap, Bp, wm, wn, lane, acc);
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int n = n0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), j = j0 + wn + (lane & 31);
        if (n < NL && j < J) A[(size_t)n * J + j] = acc[r];
    }
}

// ---------------------------------------------------------------------------
// Cosine transform over radial frequencies, per detector, two detectors packed
// as the real and imaginary parts of one complex sequence (the transform is
// real):  out(q) = sum_p in(p) cos(pi p q / M) = (X[q] + X[2M - q]) / 2 with
// X = FFT_2M of the zero-padded input (p, q >= 1).
//   forward: hT [nlam][D] -> g [D][T] (+ kappa * mass)
//   adjoint: g [D][T] -> hT [nlam][D] (+ per-detector sums of g)
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
    if (!adj && threadIdx.x < 64) {
        const float m = wave0_fixed_sum(red, n_mass);
        if (threadIdx.x == 0) *mass_s = m;
    }
    const float2* tb = fft_twiddles_to_lds(sm + DP * twoM, d.ffts[d.fft_dct], d.tw);
    for (int e = threadIdx.x; e < np * twoM; e += blockDim.x) sm[e] = make_float2(0.f, 0.f);
    __syncthreads();
    // input pairs (detector d0 real, d0 + 1 imaginary) at sm[p][q + 1]; the loads
    // of a thread are batched (fill_batched), the partner of the last odd detector is 0
    if (adj) {  // g [D][T]: contiguous along t
        const float rcp = 1.0f / (float)nin;
        fill_batched<4>(
            np * nin,
            [&](int e) {
                int p, q;
                fdivmod(e, nin, rcp, p, q);
                const int d0 = 2 * (p0 + p);
                const float re = gin[(size_t)d0 * T + q];
                const float im = gin[(size_t)min(d0 + 1, D - 1) * T + q];
                return IdxVal{p * twoM + q + 1, make_float2(re, d0 + 1 < D ? im : 0.f)};
            },
            [&](int, IdxVal iv) { sm[iv.i] = iv.v; });
    } else {    // hT [nlam][D]: the tile's detectors are contiguous within a row
        const float rcp = 1.0f / (float)np;
        fill_batched<4>(
            np * nin,
            [&](int e) {
                int q, p;
                fdivmod(e, np, rcp, q, p);
                const int d0 = 2 * (p0 + p);
                const float* row = hT + (size_t)q * D;
                const float re = row[d0];
                const float im = row[min(d0 + 1, D - 1)];
                return IdxVal{p * twoM + q + 1, make_float2(re, d0 + 1 < D ? im : 0.f)};
            },
            [&](int, IdxVal iv) { sm[iv.i] = iv.v; });
    }
    if (adj) {
        // data sum of each detector of the tile (from the copy in LDS): samples in
        // kSumClasses classes, each summed in order, then the classes in order
        __syncthreads();
        const int nd = 2 * np;
        for (int t = threadIdx.x; t < kSumClasses * nd; t += blockDim.x) {
            const int c = t % kSumClasses, dd = t / kSumClasses, dg = 2 * p0 + dd;
            const float2* col = sm + (dd >> 1) * twoM + 1;
            float sc = 0.f;
            if (dg < D) {
                if (dd & 1)
                    for (int q = c; q < T; q += kSumClasses) sc += col[q].y;
                else
                    for (int q = c; q < T; q += kSumClasses) sc += col[q].x;
            }
            red_s[t] = sc;
        }
        __syncthreads();
        if ((int)threadIdx.x < nd && 2 * p0 + (int)threadIdx.x < D) {
            float sc = 0.f;
            for (int c = 0; c < kSumClasses; ++c) sc += red_s[threadIdx.x * kSumClasses + c];
            red[2 * p0 + threadIdx.x] = sc;
        }
    }
    __syncthreads();
    fft_lds<false>(sm, twoM, np, d.ffts[d.fft_dct], tb);
    const float add = adj ? 0.f : d.kappa * *mass_s;
    // outputs X[q + 1] + X[2M - q - 1] (halved) of each pair; the LDS reads of a
    // thread are batched ahead of its stores
    if (adj) {  // -> hT [nlam][D]
        const float rcp = 1.0f / (float)np;
        fill_batched<4>(
            np * nout,
            [&](int e) {
                int q, p;
                fdivmod(e, np, rcp, q, p);
                const float2 a = sm[p * twoM + q + 1], c = sm[p * twoM + twoM - q - 1];
                return make_float2(0.5f * (a.x + c.x), 0.5f * (a.y + c.y));
            },
            [&](int e, float2 v) {
                int q, p;
                fdivmod(e, np, rcp, q, p);
                const int d0 = 2 * (p0 + p);
                float* row = hT + (size_t)q * D;
                row[d0] = v.x;
                if (d0 + 1 < D) row[d0 + 1] = v.y;
            });
    } else {    // -> g [D][T]
        const float rcp = 1.0f / (float)nout;
        fill_batched<4>(
            np * nout,
            [&](int e) {
                int p, q;
                fdivmod(e, nout, rcp, p, q);
                const float2 a = sm[p * twoM + q + 1], c = sm[p * twoM + twoM - q - 1];
                return make_float2(0.5f * (a.x + c.x) + add, 0.5f * (a.y + c.y) + add);
            },
            [&](int e, float2 v) {
                int p, q;
                fdivmod(e, nout, rcp, p, q);
                const int d0 = 2 * (p0 + p);
                gout[(size_t)d0 * T + q] = v.x;
                if (d0 + 1 < D) gout[(size_t)(d0 + 1) * T + q] = v.y;
            });
    }
}

// ---------------------------------------------------------------------------
// The cosine transform with a compile-time length N2 = 2M (plans with
// dct_spec): the same transform as dct_tile, one detector pair per sequence
// of cfft_lanes(N2) lanes, DP pairs per workgroup.  The first pass (Ns = 1,
// no twiddles) takes its inputs straight from memory, so the zero padding is
// never stored, and blocks of it are never read.  The adjoint writes hT row
// by row, the workgroup's pairs side by side.  The adjoint's per-detector data
// sums are taken from the first pass's inputs, lane by lane in order, across
// each wave's lanes by a fixed tree, then over the pair's waves in order (the
// partial sums cross the barrier that precedes the second pass): one order
// for every launch shape.
// ---------------------------------------------------------------------------
template <int N2>
__device__ __forceinline__ void dct_spec_tile(const PlanDev& d, const WsLayout& L, char* wb, float* __restrict__ gout,
                                              const float* __restrict__ gin, int tile, int DP, int adj, int n_mass,
                                              float2* sm, float* red_s, float* mass_s)
{
    constexpr int T = cfft_lanes(N2);
    constexpr CPlan P = CPlanOf<N2>::p;
    constexpr int R0 = P.rad[0], NB0 = N2 / R0, RND0 = (NB0 + T - 1) / T;
    const int D = d.D, TT = d.T, NL = d.nlam;
    float* hT = (float*)(wb + L.hdet);
    float* red = (float*)(wb + L.red);
    const int npair = (D + 1) / 2;
    const int p0 = tile * DP;               // the workgroup's first pair
    const int npw = min(DP, npair - p0);    // and its number of pairs
    const int sq = threadIdx.x / T, lane = threadIdx.x - sq * T;
    const bool active = sq < npw;
    const int d0 = 2 * min(p0 + sq, npair - 1);
    const int d1 = d0 + 1 < D ? d0 + 1 : d0;  // the partner of the last odd detector reads d0, weighted 0
    const float w1 = d0 + 1 < D ? 1.f : 0.f;
    // D even: every pair's two values sit at an 8-byte aligned address of each row
    const bool pair2 = (D & 1) == 0;
    constexpr int NP2 = cfft_padded_len(N2);  // LDS slots per pair (padded sequence)
    float2* x = sm + (size_t)min(sq, DP - 1) * NP2;
    const float2* __restrict__ tw = d.ctw + d.dct_ctw;
    if (!adj && threadIdx.x < 64) {
        const float m = wave0_fixed_sum(red, n_mass);
        if (threadIdx.x == 0) *mass_s = m;
    }
    const int nin = adj ? TT : NL;
    // input position pos (1..nin) of the pair: g(d, pos-1) (adjoint) or
    // hT[pos-1][d] (forward); zero elsewhere
    auto inp = [&](int pos) {
        const int q = min(max(pos - 1, 0), nin - 1);
        float re, im;
        if (adj) {
            re = gin[(size_t)d0 * TT + q];
            im = gin[(size_t)d1 * TT + q];
        } else if (pair2) {  // the pair's two values are adjacent in the row: one 8-byte load
            const float2 v = *(const float2*)(hT + (size_t)q * D + d0);
            re = v.x;
            im = v.y;
        } else {
            const float* row = hT + (size_t)q * D;
            re = row[d0];
            im = row[d1];
        }
        const bool in = pos >= 1 && pos <= nin;
        return make_float2(in ? re : 0.f, in ? w1 * im : 0.f);
    };
    // first pass (Ns = 1, no twiddles), fed from the inputs; inputs past
    // position nin are the zero padding: a whole block of them needs no load.
    // The adjoint's lanes sum the pair's data (for the endpoint term's
    // transpose) from the same values.
    float s0 = 0.f, s1 = 0.f;
    float2 v[RND0][R0];
    // the second pass's twiddles, in flight with the inputs
    PassTw<N2, P.rad[1], P.ns[1], T> tw1;
    pass_tw_load<N2, P.rad[1], P.ns[1], P.twoff[1], T>(tw1, tw, active, lane);
    if (active) {
#pragma unroll
        for (int i = 0; i < RND0; ++i) {
            const int j0 = lane + i * T;
            const bool own = NB0 % T == 0 || i + 1 < RND0 || j0 < NB0;
            // the last round's idle lanes work on the last butterfly (results dropped)
            const int j = own ? j0 : NB0 - 1;
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                v[i][r] = (r * NB0 <= nin) ? inp(j + r * NB0) : make_float2(0.f, 0.f);
                if (adj && own) {
                    s0 += v[i][r].x;
                    s1 += v[i][r].y;
                }
            }
            butterfly<R0, false>(v[i]);
        }
    }
    if (active) {
#pragma unroll
        for (int i = 0; i < RND0; ++i) {
            const int j = lane + i * T;
            if (NB0 % T == 0 || i + 1 < RND0 || j < NB0) {
#pragma unroll
                for (int r = 0; r < R0; ++r) x[cfft_slot<true>(j * R0 + r)] = v[i][r];
            }
        }
    }
    if (adj) {  // each wave's share of the sums, across its lanes by a fixed tree
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            s0 += __shfl_down(s0, o, 64);
            s1 += __shfl_down(s1, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            red_s[2 * (threadIdx.x >> 6)] = s0;
            red_s[2 * (threadIdx.x >> 6) + 1] = s1;
        }
    }
    __syncthreads();
    if (adj && active && lane == 0) {  // the pair's waves in order
        const int w0 = threadIdx.x >> 6;
        float t0 = 0.f, t1 = 0.f;
#pragma unroll
        for (int k = 0; k < T / 64; ++k) {
            t0 += red_s[2 * (w0 + k)];
            t1 += red_s[2 * (w0 + k) + 1];
        }
        red[d0] = t0;
        if (d0 + 1 < D) red[d0 + 1] = t1;
    }
    cfft_passes_tw<N2, false, 1, true, T>(x, tw, active, lane, tw1);
    if (adj) {
        // -> hT [nlam][D]: row by row, the workgroup's pairs side by side
        const float rcp = 1.0f / (float)npw;
        fill_batched<4>(
            NL * npw,
            [&](int e) {
                int q, p;
                fdivmod(e, npw, rcp, q, p);
                const float2 a = sm[p * NP2 + cfft_slot<true>(q + 1)], c = sm[p * NP2 + cfft_slot<true>(N2 - q - 1)];
                return make_float2(0.5f * (a.x + c.x), 0.5f * (a.y + c.y));
            },
            [&](int e, float2 o) {
                int q, p;
                fdivmod(e, npw, rcp, q, p);
                const int a = 2 * (p0 + p);
                float* row = hT + (size_t)q * D;
                if (pair2) {
                    *(float2*)(row + a) = o;
                } else {
                    row[a] = o.x;
                    if (a + 1 < D) row[a + 1] = o.y;
                }
            });
        return;
    }
    if (!active) return;  // no barrier follows
    const float add = d.kappa * *mass_s;
    // -> g [D][T]: contiguous along t
    for (int q0 = 0; q0 < TT; q0 += 2 * T) {
        float2 o[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int q = min(q0 + lane + u * T, TT - 1);
            const float2 a = x[cfft_slot<true>(q + 1)], c = x[cfft_slot<true>(N2 - q - 1)];
            o[u] = make_float2(0.5f * (a.x + c.x) + add, 0.5f * (a.y + c.y) + add);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int q = q0 + lane + u * T;
            if (q < TT) {
                gout[(size_t)d0 * TT + q] = o[u].x;
                if (d0 + 1 < D) gout[(size_t)(d0 + 1) * TT + q] = o[u].y;
            }
        }
    }
}

// Lengths 2M with a compile-time cosine transform
#define PAT_DCT_LENGTHS(X) X(256) X(512) X(1024) X(2048) X(4096) X(8192)

__device__ __forceinline__ void dct_run(const PlanDev& d, const WsLayout& L, char* wb, float* __restrict__ gout,
                                        const float* __restrict__ gin, int tile, int DP, int adj, int n_mass,
                                        float2* sm, float* red_s, float* mass_s)
{
    switch (2 * d.M) {
#define PAT_DCT_CASE(N2) \
    case N2: dct_spec_tile<N2>(d, L, wb, gout, gin, tile, DP, adj, n_mass, sm, red_s, mass_s); break;
        PAT_DCT_LENGTHS(PAT_DCT_CASE)
#undef PAT_DCT_CASE
        default: break;
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

// A band's row of the band CSR as the spread tile at columns [C0, C0 + CB)
// needs it: v[k] = band_ptr[rb][col] for col = C0 - 7 + k (k = 0 .. CB + 8),
// wrapped to col + Ng below 0 and clamped to Ng above, and v[CB + 9] =
// band_ptr[rb][Ng].  Each thread fetches entries tid and tid + CB.
__device__ __forceinline__ void band_row_fetch(const PlanDev& d, int rb, int C0, int CB, int (&v)[2])
{
    const int Ng = d.Ng;
    const int* bp = d.band_ptr + (size_t)rb * (Ng + 1);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int k = threadIdx.x + i * CB;
        v[i] = 0;
        if (k < CB + 10) {
            const int col = C0 - 7 + k;
            v[i] = k == CB + 9 ? bp[Ng] : bp[col < 0 ? col + Ng : min(col, Ng)];
        }
    }
}

__device__ __forceinline__ void band_row_store(int* row, int CB, const int (&v)[2])
{
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int k = threadIdx.x + i * CB;
        if (k < CB + 10) row[k] = v[i];
    }
}

// Staged-index ranges of a band from its CSR row in LDS: the wrapped segment
// (columns Ng-7 .. Ng-1, only for the tile at column 0) comes first, then the
// columns C0-7 .. C0+CB-1; lane's visit range is its footprint columns mx-7 .. mx.
__device__ __forceinline__ BandMeta band_meta(const int* row, int Ng, int C0, int CB, bool active)
{
    const int lo_col = C0 - 7;
    const int khi = min(C0 + CB, Ng) - lo_col;
    BandMeta m;
    m.aLo = lo_col < 0 ? row[0] : 0;
    const int aHi = lo_col < 0 ? row[CB + 9] : 0;
    m.bLo = row[lo_col < 0 ? -lo_col : 0];
    m.nA = aHi - m.aLo;
    m.ntot = m.nA + (row[khi] - m.bLo);
    m.lo = m.hi = 0;
    if (active) {
        const int t = threadIdx.x;
        m.lo = (lo_col + t < 0) ? (row[t] - m.aLo) : (m.nA + row[t] - m.bLo);
        m.hi = m.nA + row[t + 8] - m.bLo;
    }
    return m;
}

__device__ __forceinline__ int band_slot(const BandMeta& m, int idx)
{
    return idx < m.nA ? m.aLo + idx : m.bLo + (idx - m.nA);
}

// LDS of the spread (spread_lds_words): column-major so that lanes reading
// neighbouring points hit distinct banks.
template <int IB>
struct SpreadLds {
    float* wx;
    float* wy;
    int* bx;
    float2* h;
};

// staged value: the point's H times the conjugate half-pixel phase ph
template <int IB, int CAP>
__device__ __forceinline__ void spread_stage(const SpreadLds<IB>& S, int e, float4 gq, int bx_rel,
                                             const float2 (&h)[IB], float2 ph)
{
    float w[8];
    es_weights8(gq.z, w);
#pragma unroll
    for (int k = 0; k < 8; ++k) S.wx[k * CAP + e] = w[k];
    es_weights8(gq.w, w);
#pragma unroll
    for (int k = 0; k < 8; ++k) S.wy[k * CAP + e] = w[k];
    S.bx[e] = bx_rel;
    // explicit roundings: the same product in every instantiation of the tile
#pragma unroll
    for (int b = 0; b < IB; ++b)
        S.h[b * CAP + e] = make_float2(fmaf(h[b].x, ph.x, __fmul_rn(h[b].y, ph.y)),
                                       fmaf(h[b].y, ph.x, -__fmul_rn(h[b].x, ph.y)));
}

template <int IB, int CAP>
__device__ __forceinline__ void spread_visit(const SpreadLds<IB>& S, int s0, int s1, int c0, int lane7,
                                             float2 (&acc)[IB][8])
{
    if constexpr (IB == 1) {
        // one instance (small batches, where a tile's wave is often alone on
        // its SIMD): the LDS reads of the next point, and the column of the
        // one after, are issued before the current point's products (the same
        // products in the same order)
        if (s0 >= s1) return;
        const int last = s1 - 1 - c0;
        int e = s0 - c0;
        float w = S.wx[(lane7 - S.bx[e]) * CAP + e];
        float wy[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) wy[k] = S.wy[k * CAP + e];
        float2 hv = S.h[e];
        int bxn = S.bx[min(e + 1, last)];
        for (int s = s0; s < s1; ++s) {
            const int en = min(e + 1, last);
            const int bx2 = S.bx[min(e + 2, last)];
            const float wn = S.wx[(lane7 - bxn) * CAP + en];
            float wyn[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) wyn[k] = S.wy[k * CAP + en];
            const float2 hn = S.h[en];
            const float2 t = cscale(hv, w);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                acc[0][k].x = fmaf(wy[k], t.x, acc[0][k].x);
                acc[0][k].y = fmaf(wy[k], t.y, acc[0][k].y);
            }
            w = wn;
            hv = hn;
#pragma unroll
            for (int k = 0; k < 8; ++k) wy[k] = wyn[k];
            bxn = bx2;
            e = en;
        }
        return;
    }
    for (int s = s0; s < s1; ++s) {
        const int e = s - c0;
        const int dx = lane7 - S.bx[e];
        const float w = S.wx[dx * CAP + e];
        float wy[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) wy[k] = S.wy[k * CAP + e];
#pragma unroll
        for (int b = 0; b < IB; ++b) {
            const float2 t = cscale(S.h[b * CAP + e], w);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                acc[b][k].x = fmaf(wy[k], t.x, acc[b][k].x);
                acc[b][k].y = fmaf(wy[k], t.y, acc[b][k].y);
            }
        }
    }
}

// One tile of the spread for IB instances of one plan (wbs[b], b < nb, are the
// instance workspaces; instances b >= nb are padding and neither read nor
// written).  The workgroup has CB threads, one per column; CAP = 2 CB points
// are staged per chunk.  Work row wr (d.spr_row[wr]) sweeps a run of bands:
// a whole row tile rt, bands [8 rt, 8 rt + 8), writes their grid rows and
// leaves its partial sums for the 7 rows after its last band in the tail
// region unless it is the last row tile (the adjoint row pass adds them to the
// next tile's first rows); a run of a split row tile writes every row it
// touches, partial, to its rows of the slab region.  CB is a compile-time
// constant so that every LDS access of the inner loops is an immediate offset
// from one base address.
template <int IB, int CB>
__device__ __forceinline__ void spread_tile(const PlanDev& d, const WsLayout& L, char* const (&wbs)[IB], int nb,
                                            int tile, float* sf)
{
    constexpr int CAP = 2 * CB;
    const int Ng = d.Ng, NB = d.NB;
    const int ncb = (Ng + CB - 1) / CB;
    const int wr = tile / ncb, cb_ = tile - wr * ncb;
    const int4 run = d.spr_row[wr];
    const int band_lo = run.x, band_hi = run.y, rt = run.w;
    const bool to_slab = run.z >= 0;
    // the work row's output rows, from its first band on: grid or slab rows
    const float2* __restrict__ H[IB];
    float2* Ob[IB];
#pragma unroll
    for (int b = 0; b < IB; ++b) {
        H[b] = (const float2*)(wbs[b] + L.polar);
        Ob[b] = to_slab ? (float2*)(wbs[b] + L.slab) + (size_t)run.z * Ng : (float2*)(wbs[b] + L.grid) + (size_t)band_lo * Ng;
    }
    SpreadLds<IB> S;
    S.wx = sf;
    S.wy = sf + 8 * CAP;
    S.bx = (int*)(sf + 16 * CAP);
    S.h = (float2*)(sf + 17 * CAP);  // CAP is even: 8-byte aligned
    int* rows = (int*)(sf + (size_t)CAP * (17 + 2 * IB));  // [3][CB + 10]
    const int C0 = cb_ * CB;
    const int mx = C0 + threadIdx.x;
    const int lane7 = threadIdx.x + 7;
    const bool active = mx < Ng;
    float2 acc[IB][8];
#pragma unroll
    for (int b = 0; b < IB; ++b)
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[b][k] = make_float2(0.f, 0.f);
    const int e0 = threadIdx.x, e1 = threadIdx.x + CB;
    // tile-relative footprint column of a staged point: the wrapped segment
    // (columns Ng-7 .. Ng-1 seen from a tile at column 0) is shifted by -Ng
    auto rel = [&](const BandMeta& m, int idx, float4 gq) {
        return fbits(gq.x) - (idx < m.nA ? Ng : 0) - C0 + 7;
    };
    // a point's geometry, half-pixel phase and values (the phase is applied
    // when the point is staged, so that the loads stay in flight until then)
    auto fetch = [&](const BandMeta& m, int idx, float4& gq, float2& ph, float2 (&h)[IB]) {
        const int sl = band_slot(m, idx);
        gq = d.bpt_geo[sl];
        ph = d.bpt_phase[sl];
#pragma unroll
        for (int b = 0; b < IB; ++b) h[b] = b < nb ? H[b][sl] : make_float2(0.f, 0.f);
    };
    // band_lo <= band_hi always (plan.hip, spread_runs)
    // Pipeline over bands (three LDS slots of CSR rows, slot of band r = (r - band_lo) % 3):
    // in the step of band rb, the CSR row of band rb+2 (fetched in the previous
    // step) is stored, the row of band rb+3 and the points of band rb+1 are
    // fetched, and band rb (points fetched in the previous step) is staged and
    // visited.  Every global load is first waited for one step after it is issued.
    // With one instance (small batches, registers to spare) the points are
    // fetched two bands ahead instead (a second register set holds band rb+1):
    // the band's CSR row is in LDS after the barrier of the step that stores it.
    constexpr bool AHEAD2 = IB == 1;
    auto slot = [&](int r) { return rows + ((r - band_lo) % 3) * (CB + 10); };
    BandMeta nm, qm;
    float4 ng0 = make_float4(0.f, 0.f, 0.f, 0.f), ng1 = ng0, qg0 = ng0, qg1 = ng0;
    float2 np0 = make_float2(0.f, 0.f), np1 = np0, qp0 = np0, qp1 = np0;
    float2 nh0[IB], nh1[IB], qh0[IB], qh1[IB];
#pragma unroll
    for (int b = 0; b < IB; ++b) nh0[b] = nh1[b] = qh0[b] = qh1[b] = make_float2(0.f, 0.f);
    int rv[2] = {0, 0};  // CSR row in flight (band rb + 2 at the top of the step of band rb)
    {
        int v[2];
        band_row_fetch(d, band_lo, C0, CB, v);
        band_row_store(slot(band_lo), CB, v);
        if (band_lo + 1 <= band_hi) {
            band_row_fetch(d, band_lo + 1, C0, CB, v);
            band_row_store(slot(band_lo + 1), CB, v);
        }
        if (band_lo + 2 <= band_hi) band_row_fetch(d, band_lo + 2, C0, CB, rv);
    }
    __syncthreads();
    nm = band_meta(slot(band_lo), Ng, C0, CB, active);
    if (e0 < nm.ntot) fetch(nm, e0, ng0, np0, nh0);
    if (e1 < nm.ntot) fetch(nm, e1, ng1, np1, nh1);
    if (AHEAD2 && band_lo + 1 <= band_hi) {
        qm = band_meta(slot(band_lo + 1), Ng, C0, CB, active);
        if (e0 < qm.ntot) fetch(qm, e0, qg0, qp0, qh0);
        if (e1 < qm.ntot) fetch(qm, e1, qg1, qp1, qh1);
    }
    for (int rb = band_lo; rb <= band_hi; ++rb) {
        // slot of band rb+2 last held band rb-1, whose row was read two steps ago
        if (rb + 2 <= band_hi) band_row_store(slot(rb + 2), CB, rv);
        const BandMeta m = nm;
        const float4 g0 = ng0, g1 = ng1;
        const float2 p0 = np0, p1 = np1;
        float2 h0[IB], h1[IB];
#pragma unroll
        for (int b = 0; b < IB; ++b) { h0[b] = nh0[b]; h1[b] = nh1[b]; }
        // chunk 0 from registers
        if (e0 < m.ntot) spread_stage<IB, CAP>(S, e0, g0, rel(m, e0, g0), h0, p0);
        if (e1 < m.ntot) spread_stage<IB, CAP>(S, e1, g1, rel(m, e1, g1), h1, p1);
        __syncthreads();
        if constexpr (AHEAD2) {
            if (rb + 2 <= band_hi) {  // band rb+2: its CSR row was stored at the top of this step
                nm = band_meta(slot(rb + 2), Ng, C0, CB, active);
                if (e0 < nm.ntot) fetch(nm, e0, ng0, np0, nh0);
                if (e1 < nm.ntot) fetch(nm, e1, ng1, np1, nh1);
            }
        } else if (rb < band_hi) {  // band rb+1: its CSR row was stored one step ago
            nm = band_meta(slot(rb + 1), Ng, C0, CB, active);
            if (e0 < nm.ntot) fetch(nm, e0, ng0, np0, nh0);
            if (e1 < nm.ntot) fetch(nm, e1, ng1, np1, nh1);
        }
        if (rb + 3 <= band_hi) band_row_fetch(d, rb + 3, C0, CB, rv);
        spread_visit<IB, CAP>(S, m.lo, min(m.hi, CAP), 0, lane7, acc);
        __syncthreads();
        // further chunks (dense bands only)
        for (int c0 = CAP; c0 < m.ntot; c0 += CAP) {
            const int cn = min(CAP, m.ntot - c0);
            for (int e = threadIdx.x; e < cn; e += CB) {
                float4 gq;
                float2 ph, hh[IB];
                fetch(m, c0 + e, gq, ph, hh);
                spread_stage<IB, CAP>(S, e, gq, rel(m, c0 + e, gq), hh, ph);
            }
            __syncthreads();
            spread_visit<IB, CAP>(S, max(m.lo, c0), min(m.hi, c0 + cn), c0, lane7, acc);
            __syncthreads();
        }
        // row rb has all of this work row's contributions
        if (active) {
#pragma unroll
            for (int b = 0; b < IB; ++b)
                if (b < nb) Ob[b][(size_t)(rb - band_lo) * Ng + mx] = acc[b][0];
        }
#pragma unroll
        for (int b = 0; b < IB; ++b) {
#pragma unroll
            for (int k = 0; k < 7; ++k) acc[b][k] = acc[b][k + 1];
            acc[b][7] = make_float2(0.f, 0.f);
        }
        if constexpr (AHEAD2) {  // the set of band rb+1 is staged next; band rb+2's waits
            const BandMeta tm = nm;
            nm = qm;
            qm = tm;
            const float4 t0 = ng0, t1 = ng1;
            ng0 = qg0; ng1 = qg1; qg0 = t0; qg1 = t1;
            const float2 u0 = np0, u1 = np1;
            np0 = qp0; np1 = qp1; qp0 = u0; qp1 = u1;
#pragma unroll
            for (int b = 0; b < IB; ++b) {
                const float2 a0 = nh0[b], a1 = nh1[b];
                nh0[b] = qh0[b]; nh1[b] = qh1[b]; qh0[b] = a0; qh1[b] = a1;
            }
        }
    }
    // the 7 rows after the last band: complete after the plan's last band (grid
    // rows NB .. Hy - 1), partial sums for the tail region after a whole row
    // tile's, slab rows after a run's
    const bool own = to_slab || band_hi == NB - 1;
    if (active) {
#pragma unroll
        for (int k = 0; k < 7; ++k) {
#pragma unroll
            for (int b = 0; b < IB; ++b) {
                if (b >= nb) continue;
                if (own) Ob[b][(size_t)(band_hi - band_lo + 1 + k) * Ng + mx] = acc[b][k];
                else ((float2*)(wbs[b] + L.tail))[((size_t)rt * 7 + k) * Ng + mx] = acc[b][k];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// adjoint: row pass (inverse FFT along x, crop to the N image columns)
// ---------------------------------------------------------------------------
// Grid row r = 8 q + k takes row tile q's part (its grid row, or, if the tile
// was split into S runs, the slab rows of the runs that reach relative row k)
// and, for q >= 1, k < 7 and 8 q < NB (a spread row tile q exists), row tile
// q - 1's part at relative row k + 8 (its tail row, or its runs' slab rows).
// Run j of a tile split S ways (w = 8 / S bands) holds relative rows
// j w .. j w + w + 6 at slab rows s0 + 7 j + (relative row).  The terms are
// added in one fixed order: (the tile's part, its runs in order) + (the
// previous tile's part, its runs in order).

// First and last run of a tile split 2^lg ways (lg >= 1) that reach relative
// row x (0 .. 14): run j covers x when j w <= x <= j w + w + 6, w = 8 / 2^lg.
__device__ __forceinline__ int2 split_runs_at(int lg, int x)
{
    const int w = kSpreadTh >> lg, a = x - w - 6;
    return make_int2(a > 0 ? (a + w - 1) >> (3 - lg) : 0, min((1 << lg) - 1, x >> (3 - lg)));
}

__device__ __forceinline__ void rowpass_adj_tile(const PlanDev& d, const WsLayout& L, char* wb, int tile, int RPB,
                                                 float2* sm)
{
    const int N = d.N, Ng = d.Ng;
    const float2* Gt = (const float2*)(wb + L.grid);
    float2* X1 = (float2*)(wb + L.x1);
    const int r0 = tile * RPB;
    const int nr = min(RPB, d.Hy - r0);
    const float2* tb = fft_twiddles_to_lds(sm + RPB * Ng, d.ffts[d.fft_grid], d.tw);
    static_assert(kSpreadTh == 8, "the tail lookup below divides by shifting");
    const float2* Tl = (const float2*)(wb + L.tail);
    const float2* Sl = (const float2*)(wb + L.slab);
    // a row tile's split entry (log2 of its runs, first slab row): q is
    // uniform over the workgroup, so the entry is a scalar load
    auto split_of = [&](int q) {
        const unsigned e = d.spr_head[q];
        return make_int2((int)(e & 15u), (int)(e >> 4));
    };
    // row by row (the row's case is uniform): a whole tile's row plus, if any,
    // the tail row, four elements' loads per thread in flight; rows of split
    // tiles sum up to kSpreadMaxRuns slab rows per part
    constexpr int X = kSpreadMaxRuns;
    for (int rr = 0; rr < nr; ++rr) {
        const int r = r0 + rr, q = r >> 3, k = r & 7;
        const bool tail = q >= 1 && k < 7 && 8 * q < d.NB;
        const int2 so = split_of(q), st = tail ? split_of(q - 1) : make_int2(0, 0);
        float2* dst = sm + (size_t)rr * Ng;
        if (so.x == 0 && st.x == 0) {
            const float2* __restrict__ gr = Gt + (size_t)r * Ng;
            if (tail) {
                const float2* __restrict__ tr = Tl + ((size_t)(q - 1) * 7 + k) * Ng;
                fill_batched<4>(
                    Ng,
                    [&](int c) {
                        const float2 a = gr[c], t = tr[c];
                        return make_float2(a.x + t.x, a.y + t.y);
                    },
                    [&](int c, float2 v) { dst[c] = v; });
            } else {
                fill_batched<4>(Ng, [&](int c) { return gr[c]; }, [&](int c, float2 v) { dst[c] = v; });
            }
            continue;
        }
        // the parts' rows: no own rows (the grid row, or the runs 0 .. nho of a
        // split tile) and nt tail rows (the tail row, or the previous tile's runs
        // jt.x .. jt.y); unused slots repeat the first row and are not added
        const float2* po[X];
        const float2* pt[X];
        int no, nt;
        if (so.x) {
            no = split_runs_at(so.x, k).y + 1;
#pragma unroll
            for (int j = 0; j < X; ++j) po[j] = Sl + (size_t)(so.y + 7 * (j < no ? j : 0) + k) * Ng;
        } else {
            no = 1;
#pragma unroll
            for (int j = 0; j < X; ++j) po[j] = Gt + (size_t)r * Ng;
        }
        if (st.x) {
            const int2 jt = split_runs_at(st.x, k + 8);
            nt = jt.y - jt.x + 1;
#pragma unroll
            for (int j = 0; j < X; ++j) pt[j] = Sl + (size_t)(st.y + 7 * (jt.x + (j < nt ? j : 0)) + k + 8) * Ng;
        } else {
            nt = tail ? 1 : 0;
#pragma unroll
            for (int j = 0; j < X; ++j) pt[j] = tail ? Tl + ((size_t)(q - 1) * 7 + k) * Ng : po[0];
        }
        fill_batched<2>(
            Ng,
            [&](int c) {
                float2 a[X], b[X];
#pragma unroll
                for (int j = 0; j < X; ++j) {
                    a[j] = po[j][c];
                    b[j] = pt[j][c];
                }
                float2 o = a[0], t = b[0];
#pragma unroll
                for (int j = 1; j < X; ++j) {
                    if (j < no) o = make_float2(o.x + a[j].x, o.y + a[j].y);
                    if (j < nt) t = make_float2(t.x + b[j].x, t.y + b[j].y);
                }
                return nt ? make_float2(o.x + t.x, o.y + t.y) : o;
            },
            [&](int c, float2 v) { dst[c] = v; });
    }
    __syncthreads();
    grid_fft<true>(d, sm, Ng, nr, tb, RPB == 1);
    const float rcpN = 1.0f / (float)N;
    fill_batched<4>(
        nr * N,
        [&](int e) {
            int rr, j;
            fdivmod(e, N, rcpN, rr, j);
            int pos = j - N / 2;
            if (pos < 0) pos += Ng;
            return sm[rr * Ng + pos];
        },
        [&](int e, float2 v) { X1[(size_t)r0 * N + e] = v; });
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
    const float2* tb = fft_twiddles_to_lds(sm + NP * Ng, d.ffts[d.fft_grid], d.tw);
    // column pair p at residue q: batched loads with rows and columns clamped
    // into the stored range, values outside it selected as zero
    const float rcpNg = 1.0f / (float)Ng;
    fill_batched<4>(
        NP * Ng,
        [&](int e) {
            int p, q;
            fdivmod(e, Ng, rcpNg, p, q);
            const int ja = j0 + 2 * p, jb = ja + 1;
            // stored row of residue q and of -q (or -1 if not stored)
            const int rq = q <= top ? q + 4 : (q >= Ng - 4 ? q - Ng + 4 : -1);
            const int qn = q == 0 ? 0 : Ng - q;
            const int rn = qn <= top ? qn + 4 : (qn >= Ng - 4 ? qn - Ng + 4 : -1);
            const int rqc = max(rq, 0), rnc = max(rn, 0), jac = min(ja, N - 1), jbc = min(jb, N - 1);
            const float2 z0 = make_float2(0.f, 0.f);
            const float2 la = X1[(size_t)rqc * N + jac], lna = X1[(size_t)rnc * N + jac];
            const float2 lb = X1[(size_t)rqc * N + jbc], lnb = X1[(size_t)rnc * N + jbc];
            const float2 ua = (ja < N && rq >= 0) ? la : z0, una = (ja < N && rn >= 0) ? lna : z0;
            const float2 ub = (jb < N && rq >= 0) ? lb : z0, unb = (jb < N && rn >= 0) ? lnb : z0;
            // z = (ua + conj una)/2 + i (ub + conj unb)/2
            const float2 ha = make_float2(0.5f * (ua.x + una.x), 0.5f * (ua.y - una.y));
            const float2 hb = make_float2(0.5f * (ub.x + unb.x), 0.5f * (ub.y - unb.y));
            return make_float2(ha.x - hb.y, ha.y + hb.x);
        },
        [&](int e, float2 v) { sm[e] = v; });
    __syncthreads();
    grid_fft<true>(d, sm, Ng, NP, tb, NP == 1);
    const float kt = d.kappa * d.h2 * *gsum_s;
    const float rcpCT = 1.0f / (float)CT;
    fill_batched<4>(
        N * CT,
        [&](int e) {
            int i, jj;
            fdivmod(e, CT, rcpCT, i, jj);
            const int j = j0 + jj, jc = min(j, N - 1);
            int pos = i - N / 2;
            if (pos < 0) pos += Ng;
            const float2 z = sm[(jj >> 1) * Ng + pos];
            const float c = (jj & 1) ? z.y : z.x;
            const int2 mr = d.mask_rows[i];
            const float di = d.deap[i], dj = d.deap[jc];
            const float v = (j >= mr.x && j < mr.y) ? di * dj * c + kt : 0.f;
            return IdxF{j < N ? i * N + j : -1, v};
        },
        [&](int, IdxF iv) {
            if (iv.i >= 0) fb[iv.i] = iv.v;
        });
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

template <int IB, int CB>
__global__ __launch_bounds__(kGatherThreads) void k_gather(PlanDev d, WsLayout L, InstPtrs wsp, int TH, int batch)
{
    extern __shared__ float2 win[];
    const int per = ((d.Ng + CB - 1) / CB) * ((d.NB + TH - 1) / TH);
    const int ngroups = (batch + IB - 1) / IB;
    const int item = xcd_item(blockIdx.x, per * ngroups);
    if (item < 0) return;
    const int g = item / per;
    const int b0 = g * IB, nb = min(IB, batch - b0);
    char* wbs[IB];
#pragma unroll
    for (int b = 0; b < IB; ++b) wbs[b] = wsp.ws + (size_t)(b0 + (b < nb ? b : 0)) * wsp.stride;
    gather_tile<IB, CB>(d, L, wbs, nb, item - g * per, TH, win);
}

// CB is the batch-wide tile width (the instance table carries TH).
template <int CB>
__global__ __launch_bounds__(kGatherThreads) void k_gather_b(BatchDev bt, char* ws)
{
    extern __shared__ float2 win[];
    int i, tile;
    if (!batch_item(bt, kStGather, i, tile)) return;
    const BatchInst& I = bt.inst[i];
    const PlanDev d = I.d;
    char* const wbs[1] = {ws + I.ws_off};
    gather_tile<1, CB>(d, I.L, wbs, 1, tile, I.gat_th, win);
}

// Ring kernels: at most kRingMaxThreads threads (one wave for most rings).  Both
// are held to 128 VGPRs (four waves per SIMD), where the per-instance kernels
// do not spill: they are latency bound, so resident waves count more than the
// extra registers an unconstrained schedule would take.
// Ring tile order: a ring's work grows with n, so the largest rings go first
// and a launch ends on small ones.  The XCD ranges stay instance-major (an
// instance's data in one L2).  RING_MAJOR (used when every XCD owns whole
// instances, batch a multiple of 8): an XCD's tiles run ring-major across its
// instances (largest ring of each instance, then the next); else instance by
// instance.  Measured at 256^2, batch 64: the forward ring kernel is fastest
// instance by instance (a ring's polar values follow the previous ring's), the
// adjoint ring-major.
template <bool RING_MAJOR>
__device__ __forceinline__ bool ring_item(int w, int ntile, int batch, int& b, int& t)
{
    const int item = xcd_item(w, ntile * batch);
    if (item < 0) return false;
    if (RING_MAJOR && batch % kXcds == 0) {
        const int per = batch / kXcds;  // instances per XCD
        const int x = item / (per * ntile), q = item - x * per * ntile;
        const int tr = q / per;
        b = x * per + (q - tr * per);
        t = ntile - 1 - tr;
    } else {
        b = item / ntile;
        t = ntile - 1 - (item - b * ntile);
    }
    return true;
}

__global__ __launch_bounds__(kRingMaxThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_ring_fwd(PlanDev d, WsLayout L, InstPtrs wsp, int RT, int batch)
{
    extern __shared__ float2 sm[];
    int b, t;
    if (!ring_item<false>(blockIdx.x, (d.nlam + RT - 1) / RT, batch, b, t)) return;
    ring_fwd_tile(d, L, wsp.ws + (size_t)b * wsp.stride, t, RT, sm);
}

__global__ __launch_bounds__(kRingMaxThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_ring_fwd_b(BatchDev bt, char* ws)
{
    extern __shared__ float2 sm[];
    int i, tile;
    if (!batch_item(bt, kStRing, i, tile)) return;
    const BatchInst& I = bt.inst[i];
    const PlanDev d = I.d;
    if (d.ring_spec && d.ring_spec_grp == 2) ring_fwd_spec_tile<2, 1>(d, I.L, ws + I.ws_off, tile, sm);
    else if (d.ring_spec) ring_fwd_spec_tile<1, 1>(d, I.L, ws + I.ws_off, tile, sm);
    else ring_fwd_tile(d, I.L, ws + I.ws_off, tile, I.ring_rt, sm);
}

// Ring kernels of plans with compile-time transforms: one ring per workgroup
// of ring_spec_threads(G, W) threads, largest rings first.  Length group G
// (cfft.hpp): 0 up to kCfftSplit, 1 up to 1024 (one wave), 2 up to 2048 (two
// waves); W waves per ring in the one-wave groups (the same arithmetic on
// more lanes: small batches, where a ring's chain of phases is the critical
// path).
template <int G, int W>
__global__ __launch_bounds__(ring_spec_threads(G, W)) void k_ring_fwd_spec(PlanDev d, WsLayout L, InstPtrs wsp, int batch)
{
    extern __shared__ float2 sm[];
    int b, n;
    if (!ring_item<false>(blockIdx.x, d.nlam, batch, b, n)) return;
    ring_fwd_spec_tile<G, W>(d, L, wsp.ws + (size_t)b * wsp.stride, n, sm);
}

template <int G, int W>
__global__ __launch_bounds__(ring_spec_threads(G, W)) void k_ring_adj_spec(PlanDev d, WsLayout L, InstPtrs wsp, int batch)
{
    extern __shared__ float2 sm[];
    int b, n;
    if (!ring_item<true>(blockIdx.x, d.nlam, batch, b, n)) return;
    ring_adj_spec_tile<G, W>(d, L, wsp.ws + (size_t)b * wsp.stride, n, sm);
}

__global__ __launch_bounds__(kRingMaxThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_ring_adj(PlanDev d, WsLayout L, InstPtrs wsp, int RT, int batch)
{
    extern __shared__ float2 sm[];
    int b, t;
    if (!ring_item<true>(blockIdx.x, (d.nlam + RT - 1) / RT, batch, b, t)) return;
    ring_adj_tile(d, L, wsp.ws + (size_t)b * wsp.stride, t, RT, sm);
}

__global__ __launch_bounds__(kRingMaxThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_ring_adj_b(BatchDev bt, char* ws)
{
    extern __shared__ float2 sm[];
    int i, tile;
    if (!batch_item(bt, kStRing, i, tile)) return;
    const BatchInst& I = bt.inst[i];
    const PlanDev d = I.d;
    if (d.ring_spec && d.ring_spec_grp == 2) ring_adj_spec_tile<2, 1>(d, I.L, ws + I.ws_off, tile, sm);
    else if (d.ring_spec) ring_adj_spec_tile<1, 1>(d, I.L, ws + I.ws_off, tile, sm);
    else ring_adj_tile(d, I.L, ws + I.ws_off, tile, I.ring_rt, sm);
}

// Dense synthesis (explicit detector angles): `ntile` tiles per instance,
// instance-major and XCD-contiguous, so one instance's mode coefficients stay
// in one XCD's L2 while all its tiles read them; the _b forms take their
// instance and tile from the batch tables.
__global__ __launch_bounds__(kSynThreads) void k_syn_dense_fwd(PlanDev d, WsLayout L, InstPtrs wsp, int ntile,
                                                               int batch)
{
    const int item = xcd_item(blockIdx.x, ntile * batch);
    if (item < 0) return;
    const int b = item / ntile;
    syn_dense_fwd_tile(d, L, wsp.ws + (size_t)b * wsp.stride, item - b * ntile);
}

__global__ __launch_bounds__(kSynThreads) void k_syn_dense_adj(PlanDev d, WsLayout L, InstPtrs wsp, int ntile,
                                                               int batch)
{
    const int item = xcd_item(blockIdx.x, ntile * batch);
    if (item < 0) return;
    const int b = item / ntile;
    syn_dense_adj_tile(d, L, wsp.ws + (size_t)b * wsp.stride, item - b * ntile);
}

__global__ __launch_bounds__(kSynThreads) void k_syn_dense_fwd_b(BatchDev bt, char* ws)
{
    int i, tile;
    if (!batch_item(bt, kStSynFwd, i, tile)) return;
    const BatchInst& I = bt.inst[i];
    const PlanDev d = I.d;
    syn_dense_fwd_tile(d, I.L, ws + I.ws_off, tile);
}

__global__ __launch_bounds__(kSynThreads) void k_syn_dense_adj_b(BatchDev bt, char* ws)
{
    int i, tile;
    if (!batch_item(bt, kStSynAdj, i, tile)) return;
    const BatchInst& I = bt.inst[i];
    const PlanDev d = I.d;
    syn_dense_adj_tile(d, I.L, ws + I.ws_off, tile);
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

template <int N2>
__global__ __launch_bounds__(1024) void k_dct_spec(PlanDev d, WsLayout L, InstPtrs wsp, float* __restrict__ gout,
                                                   const float* __restrict__ gin, int DP, int adj, int n_mass, int batch)
{
    extern __shared__ float2 sm[];
    __shared__ float red_s[32];  // two per wave
    __shared__ float mass_s;
    const int ntile = ((d.D + 1) / 2 + DP - 1) / DP;
    const int item = xcd_item(blockIdx.x, ntile * batch);
    if (item < 0) return;
    const int b = item / ntile;
    const size_t go = (size_t)b * d.D * d.T;
    dct_spec_tile<N2>(d, L, wsp.ws + (size_t)b * wsp.stride, adj ? nullptr : gout + go, adj ? gin + go : nullptr,
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
    if (d.dct_spec)
        dct_run(d, I.L, ws + I.ws_off, adj ? nullptr : out[i], adj ? in[i] : nullptr, tile, I.dct_dp, adj, d.N, sm,
                red_s, &mass_s);
    else
        dct_tile(d, I.L, ws + I.ws_off, adj ? nullptr : out[i], adj ? in[i] : nullptr, tile, I.dct_dp, adj, d.N, sm,
                 red_s, &mass_s);
}

// IB instances per workgroup: instances g*IB .. g*IB + IB - 1 of the batch; CB threads.
// At IB = 4 the register budget is held to three waves per SIMD (168 VGPRs;
// the kernel needs 170 unconstrained).
template <int IB, int CB>
__global__ __launch_bounds__(CB) __attribute__((amdgpu_waves_per_eu(IB == 4 ? 3 : 1))) void k_spread(PlanDev d, WsLayout L, InstPtrs wsp, int batch)
{
    extern __shared__ float sf[];
    const int per = ((d.Ng + CB - 1) / CB) * d.spr_rows;
    const int ngroups = (batch + IB - 1) / IB;
    const int item = xcd_item(blockIdx.x, per * ngroups);
    if (item < 0) return;
    const int g = item / per;
    const int b0 = g * IB, nb = min(IB, batch - b0);
    char* wbs[IB];
#pragma unroll
    for (int b = 0; b < IB; ++b) wbs[b] = wsp.ws + (size_t)(b0 + (b < nb ? b : 0)) * wsp.stride;
    spread_tile<IB, CB>(d, L, wbs, nb, item - g * per, sf);
}

template <int CB>
__global__ __launch_bounds__(CB) void k_spread_b(BatchDev bt, char* ws)
{
    extern __shared__ float sf[];
    int i, tile;
    if (!batch_item(bt, kStSpread, i, tile)) return;
    const BatchInst& I = bt.inst[i];
    const PlanDev d = I.d;
    char* const wbs[1] = {ws + I.ws_off};
    spread_tile<1, CB>(d, I.L, wbs, 1, tile, sf);
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

// ---------------------------------------------------------------------------
// primal-dual TV iteration (the paper's TV baseline): dual steps for the data
// term and the isotropic TV term, primal step with the f >= 0 projection and
// the extrapolation fbar = 2 f' - f, and the relative-change norms
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pd_dual_data(float* __restrict__ y1, const float* __restrict__ ax,
                                                      const float* __restrict__ g, long count, float sigma,
                                                      float inv1s)
{
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x)
        y1[e] = (y1[e] + sigma * (ax[e] - g[e])) * inv1s;
}

// y2 [batch][n][n] float2 (x and y components), xbar [batch][n][n]
__global__ __launch_bounds__(256) void k_pd_dual_tv(float2* __restrict__ y2, const float* __restrict__ xbar, int n,
                                                    float sigma, float alpha)
{
    const int b = blockIdx.z;
    const int j = blockIdx.x * 16 + (threadIdx.x & 15);
    const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= n || j >= n) return;
    const float* xb = xbar + (size_t)b * n * n;
    const size_t e = (size_t)b * n * n + (size_t)i * n + j;
    const float c = xb[(size_t)i * n + j];
    const float dx = (j + 1 < n) ? xb[(size_t)i * n + j + 1] - c : 0.f;
    const float dy = (i + 1 < n) ? xb[(size_t)(i + 1) * n + j] - c : 0.f;
    float2 v = y2[e];
    v.x += sigma * dx;
    v.y += sigma * dy;
    const float m = sqrtf(v.x * v.x + v.y * v.y);
    const float sc = m > alpha ? alpha / m : 1.f;  // projection onto |v| <= alpha
    y2[e] = make_float2(v.x * sc, v.y * sc);
}

// f' = max(f - tau (aty + grad* y2), 0); xbar = 2 f' - f; f = f'
__global__ __launch_bounds__(256) void k_pd_primal(float* __restrict__ f, float* __restrict__ xbar,
                                                   const float* __restrict__ aty, const float2* __restrict__ y2,
                                                   int n, float tau)
{
    const int b = blockIdx.z;
    const int j = blockIdx.x * 16 + (threadIdx.x & 15);
    const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= n || j >= n) return;
    const size_t base = (size_t)b * n * n;
    const size_t e = base + (size_t)i * n + j;
    // (grad* y2)_ij: the x component enters at (i, j) with -1 (j < n-1) and at (i, j+1) with +1,
    // the y component at (i, j) with -1 (i < n-1) and at (i+1, j) with +1
    const float2 p = y2[e];
    float gs = 0.f;
    if (j + 1 < n) gs -= p.x;
    if (j > 0) gs += y2[e - 1].x;
    if (i + 1 < n) gs -= p.y;
    if (i > 0) gs += y2[e - n].y;
    const float old = f[e];
    const float fn = fmaxf(old - tau * (aty[e] + gs), 0.f);
    f[e] = fn;
    xbar[e] = 2.f * fn - old;
}

// out[b] = (sum (xbar - f)^2, sum f^2) over instance b (after k_pd_primal,
// xbar - f = f' - f_old): one workgroup per instance, fixed-order sums
__global__ __launch_bounds__(1024) void k_pd_change(const float* __restrict__ f, const float* __restrict__ xbar,
                                                    float* __restrict__ out, long per)
{
    __shared__ float red_s[1024];
    const int b = blockIdx.x;
    const float* fb = f + (size_t)b * per;
    const float* xb = xbar + (size_t)b * per;
    float sd = 0.f, sf = 0.f;
    for (long e = threadIdx.x; e < per; e += blockDim.x) {
        const float v = fb[e], dlt = xb[e] - v;
        sd += dlt * dlt;
        sf += v * v;
    }
    const float td = block_sum(sd, red_s);
    const float tf = block_sum(sf, red_s);
    if (threadIdx.x == 0) {
        out[2 * b] = td;
        out[2 * b + 1] = tf;
    }
}


// ---------------------------------------------------------------------------
// CGLS pieces (one workgroup per instance for the norms: fixed-order sums)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_cg_norm2(const float* __restrict__ x, float* __restrict__ out, long per)
{
    __shared__ float red_s[1024];
    const int b = blockIdx.x;
    const float* xb = x + (size_t)b * per;
    float acc = 0.f;
    for (long e = threadIdx.x; e < per; e += blockDim.x) acc += xb[e] * xb[e];
    const float t = block_sum(acc, red_s);
    if (threadIdx.x == 0) out[b] = t;
}

__global__ void k_cg_step_fr(float* __restrict__ f, const float* __restrict__ p, long nf, float* __restrict__ r,
                             const float* __restrict__ q, long nr, const float* __restrict__ gamma,
                             const float* __restrict__ qq)
{
    const int b = blockIdx.y;
    const float den = qq[b];
    const float alpha = den > 0.f ? gamma[b] / den : 0.f;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nf; e += stride)
        f[(size_t)b * nf + e] += alpha * p[(size_t)b * nf + e];
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nr; e += stride)
        r[(size_t)b * nr + e] -= alpha * q[(size_t)b * nr + e];
}

__global__ void k_cg_step_p(float* __restrict__ p, const float* __restrict__ s, long n,
                            const float* __restrict__ gamma_new, const float* __restrict__ gamma)
{
    const int b = blockIdx.y;
    const float den = gamma[b];
    const float beta = den > 0.f ? gamma_new[b] / den : 0.f;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
        p[(size_t)b * n + e] = s[(size_t)b * n + e] + beta * p[(size_t)b * n + e];
}


// ---------------------------------------------------------------------------
// Streaming copies: the bandwidth yardstick the roofline figures are quoted
// against, and the known-size traffic that calibrates the byte counters.
// k_stream_copy: dst = src over n4 16-byte elements, four loads in flight per
// thread before its stores.  k_scatter_copy: dst[perm[i]] = src[i] over
// 8-byte elements (the scattered-store pattern of the ring adjoint's
// band-order output).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_stream_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                     long n4)
{
    const long stride = (long)gridDim.x * 1024;
    for (long base = (long)blockIdx.x * 1024 + threadIdx.x; base < n4; base += stride) {
        float4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long e = base + u * 256;
            v[u] = src[e < n4 ? e : n4 - 1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long e = base + u * 256;
            if (e < n4) dst[e] = v[u];
        }
    }
}

__global__ __launch_bounds__(256) void k_scatter_copy(const float2* __restrict__ src, float2* __restrict__ dst,
                                                      const int* __restrict__ perm, long n)
{
    const long stride = (long)gridDim.x * 256;
    for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += stride) dst[perm[e]] = src[e];
}

}  // namespace pat
