// sim.hip -- FFT wave-propagation data simulator (gfx950 kernels and host plan).
//
// The simulation study (Sec. 2.4.1) computes its data on a finer Cartesian grid
// with an FFT-based wave propagation method.  For a constant speed of sound the
// field is p(t) = IFFT2[F cos(c|k|t)], F = FFT2 of the zero-padded fine image on
// a periodic box wide enough that no wave wraps around to a detector by the
// last sample (box rule and sampling in pat.h).
//
// Per run: F is computed once (the image rows, then every column of the box;
// rows outside the image are zero).  The data then come in pairs of time
// samples (t_a, t_b): both fields are real, so one complex inverse transform of
// F (cos(c|k|t_a) + i cos(c|k|t_b)) gives p(t_a) + i p(t_b).  Per chunk of
// pairs: the inverse transform along y with the spectrum modulated as it is
// loaded (the phase c|k|t / 2 pi reduced mod 1 in FP64, then cos(2 pi x) in
// FP32), keeping only the box rows the detectors' stencils read; the inverse
// transform along x of those rows; the Keys samples at the detectors.
#include "../../include/pat.h"
#include "fft.hpp"
#include "pat_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

namespace pat {

struct SimDev {
    int Ns, M, off;         // fine grid side, box side, box index of the image's first row / column
    int D, T;               // detectors, time samples
    int rlo, nrow;          // box rows [rlo, rlo + nrow) read by the detectors' stencils
    int CT, RPB;            // columns per column-transform workgroup, rows per row-transform workgroup
    float a_hi, a_lo;       // alpha = c dt / (M h) as an unevaluated FP32 sum (FP64 on the host): the
                            // phase c |k| j dt / (2 pi) = j alpha sqrt(mx^2 + my^2)
    const int2* mask_rows;  // [Ns]: image row i keeps columns jlo <= j < jhi (support disc)
    const int2* dix;        // [D]: box cell (x, y) of each detector's stencil sample at offset 0
    const float2* dfr;      // [D]: its fractional offsets (FP64-computed)
    const float2* tw;       // twiddle table of the length-M transform
    FftDev fm;              // the length-M transform
};

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// FFT along x of RPB image rows (masked, zero-padded into box columns) -> W [Ns][M]
__global__ __launch_bounds__(1024) void k_sim_rows_fwd(SimDev s, const float* __restrict__ f, float2* __restrict__ W)
{
    extern __shared__ float2 sm[];
    const int M = s.M, Ns = s.Ns, RPB = s.RPB;
    const int r0 = blockIdx.x * RPB, nr = min(RPB, Ns - r0);
    const float2* tb = fft_twiddles_to_lds(sm + RPB * M, s.fm, s.tw);
    for (int e = threadIdx.x; e < RPB * M; e += blockDim.x) sm[e] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int e = threadIdx.x; e < nr * Ns; e += blockDim.x) {
        const int rr = e / Ns, j = e - rr * Ns, i = r0 + rr;
        const int2 mr = s.mask_rows[i];
        const float v = (j >= mr.x && j < mr.y) ? f[(size_t)i * Ns + j] : 0.f;
        sm[rr * M + s.off + j] = make_float2(v, 0.f);
    }
    __syncthreads();
    fft_lds<false>(sm, M, RPB, s.fm, tb);
    for (int e = threadIdx.x; e < nr * M; e += blockDim.x) W[(size_t)r0 * M + e] = sm[e];
}

// FFT along y of CT box columns (rows outside the image are zero) -> F [M][M]
__global__ __launch_bounds__(1024) void k_sim_cols_fwd(SimDev s, const float2* __restrict__ W, float2* __restrict__ F)
{
    extern __shared__ float2 sm[];
    const int M = s.M, CT = s.CT;
    const int c0 = blockIdx.x * CT, nc = min(CT, M - c0);
    const float2* tb = fft_twiddles_to_lds(sm + CT * M, s.fm, s.tw);
    for (int e = threadIdx.x; e < M * CT; e += blockDim.x) {
        const int r = e / CT, cc = e - r * CT;
        const int ri = r - s.off;
        float2 v = make_float2(0.f, 0.f);
        if (cc < nc && ri >= 0 && ri < s.Ns) v = W[(size_t)ri * M + c0 + cc];
        sm[cc * M + r] = v;
    }
    __syncthreads();
    fft_lds<false>(sm, M, CT, s.fm, tb);
    for (int e = threadIdx.x; e < M * CT; e += blockDim.x) {
        const int r = e / CT, cc = e - r * CT;
        if (cc < nc) F[(size_t)r * M + c0 + cc] = sm[cc * M + r];
    }
}

// The phase j alpha sqrt(mx^2 + my^2) reduced mod 1, in FP32 arithmetic with
// error-free products (each quantity an unevaluated sum of two floats, as in
// double-float arithmetic): q = mx^2 + my^2 is exact (q_hi + q_lo), the
// square root is refined by one Newton step on its exact FMA residual, and
// the products alpha s and j u are split exactly by FMA, so the fraction
// returned is correct to about 2^-24 (a few cycles of phase would otherwise
// lose their fraction's accuracy in FP32).
__device__ __forceinline__ float sim_phase_frac(int mx, int my, int j, float a_hi, float a_lo)
{
    const unsigned q = (unsigned)(mx * mx + my * my);
    const float q_hi = (float)q;
    const float q_lo = (float)(int)(q - (unsigned)q_hi);  // exact: |q - q_hi| < 2^3 for q < 2^27
    const float s = sqrtf(q_hi);
    const float e = fmaf(-s, s, q_hi) + q_lo;             // q - s^2
    const float sc = q == 0u ? 0.f : e * __builtin_amdgcn_rcpf(2.f * s);
    // u = alpha (s + sc) = u_hi + u_lo
    const float p = a_hi * s;
    const float pe = fmaf(a_hi, s, -p);
    const float t = pe + fmaf(a_hi, sc, a_lo * s);
    const float u_hi = p + t;
    const float u_lo = t - (u_hi - p);
    // x = j u = P + L
    const float J = (float)j;
    const float P = J * u_hi;
    const float L = fmaf(J, u_hi, -P) + J * u_lo;
    float x = (P - floorf(P)) + L;
    x -= floorf(x);
    return x;
}

// Pair p of the chunk (time indices ja = 2 (pair0 + p) + 1, jb = ja + 1): the
// inverse FFT along y of CT columns of F (cos(c|k|t_a) + i cos(c|k|t_b)),
// rows [rlo, rlo + nrow) -> Wt [chunk][nrow][M]
__global__ __launch_bounds__(1024) void k_sim_cols_inv(SimDev s, const float2* __restrict__ F, float2* __restrict__ Wt,
                                                       int pair0)
{
    extern __shared__ float2 sm[];
    const int M = s.M, CT = s.CT, p = blockIdx.y;
    const int c0 = blockIdx.x * CT, nc = min(CT, M - c0);
    const int ja = 2 * (pair0 + p) + 1, jb = ja + 1;
    const bool has_b = jb <= s.T;
    const float2* tb = fft_twiddles_to_lds(sm + CT * M, s.fm, s.tw);
    for (int e = threadIdx.x; e < M * CT; e += blockDim.x) {
        const int r = e / CT, cc = e - r * CT, c = c0 + min(cc, nc - 1);
        const float2 z = F[(size_t)r * M + c];
        const int mx = c < M / 2 ? c : c - M, my = r < M / 2 ? r : r - M;
        const float xa = sim_phase_frac(mx, my, ja, s.a_hi, s.a_lo);
        const float xb = sim_phase_frac(mx, my, jb, s.a_hi, s.a_lo);
        const float ca = cospif(2.0f * xa), cb = has_b ? cospif(2.0f * xb) : 0.f;
        sm[cc * M + r] = make_float2(z.x * ca - z.y * cb, z.y * ca + z.x * cb);
    }
    __syncthreads();
    fft_lds<true>(sm, M, CT, s.fm, tb);
    float2* out = Wt + (size_t)p * s.nrow * M;
    for (int e = threadIdx.x; e < s.nrow * CT; e += blockDim.x) {
        const int rr = e / CT, cc = e - rr * CT;
        if (cc < nc) out[(size_t)rr * M + c0 + cc] = sm[cc * M + s.rlo + rr];
    }
}

// inverse FFT along x of RPB rows of pair p's band, in place
__global__ __launch_bounds__(1024) void k_sim_rows_inv(SimDev s, float2* __restrict__ Wt)
{
    extern __shared__ float2 sm[];
    const int M = s.M, RPB = s.RPB, p = blockIdx.y;
    const int r0 = blockIdx.x * RPB, nr = min(RPB, s.nrow - r0);
    float2* base = Wt + ((size_t)p * s.nrow + r0) * M;
    const float2* tb = fft_twiddles_to_lds(sm + RPB * M, s.fm, s.tw);
    for (int e = threadIdx.x; e < RPB * M; e += blockDim.x) sm[e] = e < nr * M ? base[e] : make_float2(0.f, 0.f);
    __syncthreads();
    fft_lds<true>(sm, M, RPB, s.fm, tb);
    for (int e = threadIdx.x; e < nr * M; e += blockDim.x) base[e] = sm[e];
}

// Keys cubic convolution weight (a = -1/2) at distance t (0 <= t < 2)
__device__ __forceinline__ float keys_w(float t)
{
    constexpr float a = -0.5f;
    return t <= 1.f ? ((a + 2.f) * t - (a + 3.f)) * t * t + 1.f : ((a * t - 5.f * a) * t + 8.f * a) * t - 4.f * a;
}

// Samples at the detectors: thread (d, p) -> g[d][ja - 1] and g[d][jb - 1]
__global__ __launch_bounds__(256) void k_sim_sample(SimDev s, const float2* __restrict__ Wt, float* __restrict__ g,
                                                    int pair0, int npairs)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= s.D * npairs) return;
    const int p = t / s.D, d = t - p * s.D;
    const int ja = 2 * (pair0 + p) + 1, jb = ja + 1;
    const int2 ix = s.dix[d];
    const float2 fr = s.dfr[d];
    const float wx[4] = {keys_w(1.f + fr.x), keys_w(fr.x), keys_w(1.f - fr.x), keys_w(2.f - fr.x)};
    const float wy[4] = {keys_w(1.f + fr.y), keys_w(fr.y), keys_w(1.f - fr.y), keys_w(2.f - fr.y)};
    const float2* base = Wt + (size_t)p * s.nrow * s.M;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const float2* row = base + (size_t)(ix.y - 1 + a - s.rlo) * s.M + (ix.x - 1);
        float2 ra = make_float2(0.f, 0.f);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            ra.x = fmaf(wx[b], row[b].x, ra.x);
            ra.y = fmaf(wx[b], row[b].y, ra.y);
        }
        acc.x = fmaf(wy[a], ra.x, acc.x);
        acc.y = fmaf(wy[a], ra.y, acc.y);
    }
    const float scale = 1.0f / ((float)s.M * (float)s.M);
    g[(size_t)d * s.T + ja - 1] = acc.x * scale;
    if (jb <= s.T) g[(size_t)d * s.T + jb - 1] = acc.y * scale;
}

}  // namespace pat

// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------

using pat::SimDev;

struct pat_sim {
    SimDev dev;
    void* table_mem;
    int device;
    int thr_col, thr_row;       // workgroup sizes of the column and row transforms
    size_t lds_col, lds_row;    // their dynamic LDS
    int npairs, chunk;          // time-sample pairs, pairs per chunk
    size_t off_F, off_W, off_Wt, ws_bytes;
};

namespace {

constexpr int kSimMaxBox = 8192;
constexpr int kSimChunk = 16;
constexpr size_t kSimLdsMax = 160 * 1024;

long smooth_2a3b(long m)
{
    long best = -1;
    for (long p2 = 1; p2 < 2 * m + 2; p2 *= 2)
        for (long p = p2; p < 2 * m + 2; p *= 3)
            if (p >= m && (best < 0 || p < best)) best = p;
    return best;
}

// box side per the rule in pat.h
long sim_box_side(int ns, double det_r, double support_r, double c, double t_last)
{
    const double h = 2.0 / ns;
    const double half = std::max((det_r + support_r + c * t_last) / 2.0, det_r + 3.0 * h) + h;
    long m = std::max((long)std::ceil(2.0 * half / h), (long)ns);
    for (;;) {
        m = smooth_2a3b(m);
        if (m % 2 == 0 && (m - ns) % 2 == 0) return m;
        ++m;
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" int pat_sim_create(const pat_plan_desc* desc, pat_sim** out)
{
    if (!desc || !out) return PAT_ERR_ARG;
    const int Ns = desc->n, D = desc->n_det, T = desc->n_t;
    if (Ns < 8 || D < 1 || T < 1 || !(desc->dt > 0.0) || !(desc->c > 0.0) || !(desc->det_r > 0.0) ||
        !(desc->support_r > 0.0))
        return PAT_ERR_ARG;
    const double h = 2.0 / Ns;
    const long Ml = sim_box_side(Ns, desc->det_r, desc->support_r, desc->c, T * desc->dt);
    if (Ml > kSimMaxBox) return PAT_ERR_UNSUPPORTED;
    const int M = (int)Ml;

    pat_sim* s = new (std::nothrow) pat_sim;
    if (!s) return PAT_ERR_ALLOC;
    std::memset(s, 0, sizeof(*s));
    SimDev& d = s->dev;
    d.Ns = Ns;
    d.M = M;
    d.off = (M - Ns) / 2;
    d.D = D;
    d.T = T;
    {
        const double alpha = desc->c * desc->dt / (M * h);
        d.a_hi = (float)alpha;
        d.a_lo = (float)(alpha - (double)d.a_hi);
    }

    // support mask per image row (FP64, as the reference decides it)
    std::vector<int2> mrows(Ns);
    for (int i = 0; i < Ns; ++i) {
        const double y = -1.0 + (i + 0.5) * h;
        int lo = Ns, hi = 0;
        for (int j = 0; j < Ns; ++j) {
            const double x = -1.0 + (j + 0.5) * h;
            if (x * x + y * y < desc->support_r * desc->support_r) {
                lo = std::min(lo, j);
                hi = j + 1;
            }
        }
        mrows[i] = make_int2(lo < hi ? lo : 0, lo < hi ? hi : 0);
    }
    // detectors: stencil cells and fractional offsets in box index units
    std::vector<int2> dix(D);
    std::vector<float2> dfr(D);
    int ylo = M, yhi = -1;
    for (int q = 0; q < D; ++q) {
        const double th = desc->det_theta ? desc->det_theta[q]
                                          : desc->arc_center - desc->arc_span / 2 + (q + 0.5) * desc->arc_span / D;
        const double gx = desc->det_r * std::cos(th) / h + M / 2.0 - 0.5;
        const double gy = desc->det_r * std::sin(th) / h + M / 2.0 - 0.5;
        const int ix = (int)std::floor(gx), iy = (int)std::floor(gy);
        if (ix - 1 < 0 || ix + 2 >= M || iy - 1 < 0 || iy + 2 >= M) {
            delete s;
            return PAT_ERR_UNSUPPORTED;
        }
        dix[q] = make_int2(ix, iy);
        dfr[q] = make_float2((float)(gx - ix), (float)(gy - iy));
        ylo = std::min(ylo, iy - 1);
        yhi = std::max(yhi, iy + 3);
    }
    d.rlo = ylo;
    d.nrow = yhi - ylo;

    std::vector<float2> tw;
    const int tps = pat::fixed_fft_for(M, &d.fm, tw);
    if (!tps) {
        delete s;
        return PAT_ERR_UNSUPPORTED;
    }
    // workgroup shapes: the most columns / rows per workgroup (8, 4, 2, 1) whose
    // threads and LDS fit
    auto shape = [&](int& n_out, int& thr_out, size_t& lds_out) {
        for (int n = 8; n >= 1; n /= 2) {
            const int thr = pat::fft_workgroup_threads(n, d.fm);
            const size_t lds = sizeof(float2) * ((size_t)n * M + (size_t)d.fm.ntb);
            if (thr <= 1024 && lds <= kSimLdsMax / 2) {
                n_out = n;
                thr_out = thr;
                lds_out = lds;
                return true;
            }
        }
        return false;
    };
    if (!shape(d.CT, s->thr_col, s->lds_col) || !shape(d.RPB, s->thr_row, s->lds_row)) {
        delete s;
        return PAT_ERR_UNSUPPORTED;
    }

    // device tables
    size_t o_mask = 0, o_dix = align256(o_mask + sizeof(int2) * Ns), o_dfr = align256(o_dix + sizeof(int2) * D),
           o_tw = align256(o_dfr + sizeof(float2) * D), bytes = o_tw + sizeof(float2) * tw.size();
    std::vector<unsigned char> host(bytes, 0);
    std::memcpy(host.data() + o_mask, mrows.data(), sizeof(int2) * Ns);
    std::memcpy(host.data() + o_dix, dix.data(), sizeof(int2) * D);
    std::memcpy(host.data() + o_dfr, dfr.data(), sizeof(float2) * D);
    std::memcpy(host.data() + o_tw, tw.data(), sizeof(float2) * tw.size());
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return PAT_ERR_HIP;
    }
    if (hipMalloc(&s->table_mem, bytes) != hipSuccess) {
        delete s;
        return PAT_ERR_ALLOC;
    }
    if (hipMemcpy(s->table_mem, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(s->table_mem);
        delete s;
        return PAT_ERR_HIP;
    }
    char* base = (char*)s->table_mem;
    d.mask_rows = (const int2*)(base + o_mask);
    d.dix = (const int2*)(base + o_dix);
    d.dfr = (const float2*)(base + o_dfr);
    d.tw = (const float2*)(base + o_tw);

    // workspace: F [M][M], W [Ns][M], Wt [chunk][nrow][M]
    s->npairs = (T + 1) / 2;
    s->chunk = std::min(s->npairs, kSimChunk);
    s->off_F = 0;
    s->off_W = align256(sizeof(float2) * (size_t)M * M);
    s->off_Wt = s->off_W + align256(sizeof(float2) * (size_t)Ns * M);
    s->ws_bytes = s->off_Wt + align256(sizeof(float2) * (size_t)s->chunk * d.nrow * M);
    *out = s;
    return PAT_OK;
}

extern "C" int pat_sim_query(const pat_sim* s, int* box_side, size_t* workspace_bytes)
{
    if (!s) return PAT_ERR_ARG;
    if (box_side) *box_side = s->dev.M;
    if (workspace_bytes) *workspace_bytes = s->ws_bytes;
    return PAT_OK;
}

extern "C" int pat_sim_run(const pat_sim* s, const float* f, float* g, void* ws, size_t ws_bytes, void* stream)
{
    if (!s || !f || !g) return PAT_ERR_ARG;
    if (!ws || ws_bytes < s->ws_bytes) return PAT_ERR_WORKSPACE;
    const SimDev& d = s->dev;
    hipStream_t st = (hipStream_t)stream;
    char* w = (char*)ws;
    float2* F = (float2*)(w + s->off_F);
    float2* W = (float2*)(w + s->off_W);
    float2* Wt = (float2*)(w + s->off_Wt);
    hipLaunchKernelGGL(pat::k_sim_rows_fwd, dim3((d.Ns + d.RPB - 1) / d.RPB), dim3(s->thr_row), s->lds_row, st, d, f,
                       W);
    if (hipGetLastError() != hipSuccess) return PAT_ERR_HIP;
    hipLaunchKernelGGL(pat::k_sim_cols_fwd, dim3((d.M + d.CT - 1) / d.CT), dim3(s->thr_col), s->lds_col, st, d,
                       (const float2*)W, F);
    if (hipGetLastError() != hipSuccess) return PAT_ERR_HIP;
    for (int p0 = 0; p0 < s->npairs; p0 += s->chunk) {
        const int np = std::min(s->chunk, s->npairs - p0);
        hipLaunchKernelGGL(pat::k_sim_cols_inv, dim3((d.M + d.CT - 1) / d.CT, np), dim3(s->thr_col), s->lds_col, st, d,
                           (const float2*)F, Wt, p0);
        if (hipGetLastError() != hipSuccess) return PAT_ERR_HIP;
        hipLaunchKernelGGL(pat::k_sim_rows_inv, dim3((d.nrow + d.RPB - 1) / d.RPB, np), dim3(s->thr_row), s->lds_row,
                           st, d, Wt);
        if (hipGetLastError() != hipSuccess) return PAT_ERR_HIP;
        hipLaunchKernelGGL(pat::k_sim_sample, dim3((d.D * np + 255) / 256), dim3(256), 0, st, d, (const float2*)Wt, g,
                           p0, np);
        if (hipGetLastError() != hipSuccess) return PAT_ERR_HIP;
    }
    return PAT_OK;
}

extern "C" void pat_sim_destroy(pat_sim* s)
{
    if (!s) return;
    if (s->table_mem) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) cur = s->device;
        (void)hipSetDevice(s->device);
        (void)hipFree(s->table_mem);
        (void)hipSetDevice(cur);
    }
    delete s;
}
