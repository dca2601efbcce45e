// cfft.hpp -- complex FFTs of compile-time length, run by one wavefront.
//
// Stockham autosort passes as in fft.hpp (the pass of radix R after
// sub-transforms of size Ns reads x[j + r n/R], multiplies input r by
// w^{r k} with w = e^{-2 pi i / (Ns R)}, k = j mod Ns, does an R-point DFT and
// writes x[(j - k) R + k + r Ns]), but with the length, the radix sequence and
// every pass's Ns fixed at compile time: the loads and stores of a pass are
// immediate offsets from one lane address, j mod Ns is a shift or a constant
// multiply, and each butterfly reads its R - 1 twiddles w^{r k} from a table
// (FP64-computed, stored FP32) instead of forming powers.  The 64 lanes of
// wave 0 of the workgroup do the work; other waves of the workgroup only pass
// the barriers, so the result is the same for any workgroup size.
//
// The radix sequence depends on the length alone (make_cplan): the plan
// builder lays out the twiddle tables with the same function.
#pragma once

#include <hip/hip_runtime.h>

#include "fft.hpp"

namespace pat {

constexpr int kCfftLanes = 64;   // lanes of a one-wave transform
constexpr int kCfftMax = 8192;   // longest compile-time length
constexpr int kCfftMaxPasses = 12;

// Lanes that transform one sequence of length n: one wave up to 1024, then
// one more wave per doubling (workgroup-wide barriers between passes), 16
// elements per lane at 2048 .. 8192.
__host__ __device__ constexpr int cfft_lanes(int n)
{
    return n <= 1024 ? kCfftLanes : (n <= 2048 ? 2 * kCfftLanes : (n <= 4096 ? 4 * kCfftLanes : 8 * kCfftLanes));
}

struct CPlan {
    int np;                       // passes (0: no plan)
    int rad[kCfftMaxPasses];      // radix of each pass, in execution order
    int ns[kCfftMaxPasses];       // sub-transform size before each pass
    int twoff[kCfftMaxPasses + 1];  // table offset of each pass; twoff[np] = table entries
};

// Estimated VALU instructions of one radix-R butterfly (fft.hpp's DFTs)
__host__ __device__ constexpr int cbf_valu(int R)
{
    return R == 2 ? 4 : R == 3 ? 12 : R == 4 ? 16 : R == 6 ? 44 : R == 8 ? 60 : R == 9 ? 88 : 158;
}

// Cost of a pass of radix R over length n at cfft_lanes(n) lanes: rounds of
// butterflies (arithmetic, twiddle products, address work, LDS issue) plus a
// fixed cost per pass (two barriers and an LDS round trip).
__host__ __device__ constexpr int cpass_cost(int n, int R, bool twiddled)
{
    const int rounds = (n / R + cfft_lanes(n) - 1) / cfft_lanes(n);
    return rounds * (cbf_valu(R) + (twiddled ? 4 * (R - 1) : 0) + 8 + R) + 40;
}

// Radix sequence of length n = 2^a 3^b (2 <= n <= kCfftMax): the multiset of
// radices {16, 9, 8, 6, 4, 3, 2} of least modelled cost (dynamic programming
// over the remaining powers of 2 and 3), at most 32 complex values per lane
// and pass, ordered largest first (the first pass multiplies by no twiddle).
__host__ __device__ constexpr CPlan make_cplan(int n)
{
    CPlan p{};
    p.np = 0;
    if (n < 2 || n > kCfftMax) return p;
    const int RS[7] = {16, 9, 8, 6, 4, 3, 2};
    const int A[7] = {4, 0, 3, 1, 2, 0, 1};
    const int B[7] = {0, 2, 0, 1, 0, 1, 0};
    int x = 0, y = 0, m = n;
    while (m % 2 == 0) { m /= 2; ++x; }
    while (m % 3 == 0) { m /= 3; ++y; }
    if (m != 1) return p;
    int best[14][9] = {};
    int choice[14][9] = {};
    for (int i = 0; i <= x; ++i)
        for (int j = 0; j <= y; ++j) {
            choice[i][j] = -1;
            if (i == 0 && j == 0) { best[i][j] = 0; continue; }
            best[i][j] = 1 << 30;
            for (int c = 0; c < 7; ++c) {
                if (A[c] > i || B[c] > j) continue;
                const int R = RS[c];
                if (((n / R + cfft_lanes(n) - 1) / cfft_lanes(n)) * R > 32) continue;
                if (best[i - A[c]][j - B[c]] >= (1 << 30)) continue;
                const int v = best[i - A[c]][j - B[c]] + cpass_cost(n, R, true);
                if (v < best[i][j]) { best[i][j] = v; choice[i][j] = c; }
            }
        }
    int i = x, j = y;
    while (i > 0 || j > 0) {
        const int c = choice[i][j];
        if (c < 0 || p.np >= kCfftMaxPasses) { p.np = 0; return p; }
        p.rad[p.np++] = RS[c];
        i -= A[c];
        j -= B[c];
    }
    for (int a = 0; a < p.np; ++a)
        for (int b = a + 1; b < p.np; ++b)
            if (p.rad[b] > p.rad[a]) { const int t = p.rad[a]; p.rad[a] = p.rad[b]; p.rad[b] = t; }
    int ns = 1, off = 0;
    for (int s = 0; s < p.np; ++s) {
        p.ns[s] = ns;
        p.twoff[s] = off;
        if (ns > 1) off += ns * (p.rad[s] - 1);
        ns *= p.rad[s];
    }
    p.twoff[p.np] = off;
    return p;
}

// One-wave lengths with a compile-time transform (the switch in cfft_run and
// in the ring kernels), in two groups: the ring kernels are built once for the
// lengths up to kCfftSplit and once for all of them, so that plans whose ring
// and synthesis lengths are all short get the register budget of short ones.
constexpr int kCfftSplit = 512;
#define PAT_CFFT_LENGTHS_LO(X)                                                                                \
    X(2) X(3) X(4) X(6) X(8) X(9) X(12) X(16) X(18) X(24) X(27) X(32) X(36) X(48) X(54) X(64) X(72) X(81) \
    X(96) X(108) X(128) X(144) X(162) X(192) X(216) X(243) X(256) X(288) X(324) X(384) X(432) X(486) X(512)
#define PAT_CFFT_LENGTHS_HI(X) X(576) X(648) X(729) X(768) X(864) X(972) X(1024)
#define PAT_CFFT_LENGTHS(X) PAT_CFFT_LENGTHS_LO(X) PAT_CFFT_LENGTHS_HI(X)
// Two-wave lengths of the ring kernels (length group 2)
#define PAT_CFFT_LENGTHS_HI2(X) X(1152) X(1296) X(1458) X(1536) X(1728) X(1944) X(2048)

// Threads of a ring workgroup of length group G (0: lengths up to kCfftSplit,
// 1: up to 1024, 2: up to 2048), W waves per ring in the one-wave groups
__host__ __device__ constexpr int ring_spec_threads(int G, int W = 1) { return G == 2 ? 2 * kCfftLanes : W * kCfftLanes; }

// Grid sides Ng with a compile-time transform (2D-FFT passes)
#define PAT_GRID_LENGTHS(X) X(128) X(256) X(512) X(1024) X(2048)

__host__ __device__ constexpr bool grid_len_ok(int n)
{
    return n == 128 || n == 256 || n == 512 || n == 1024 || n == 2048;
}

__host__ __device__ constexpr bool cfft_len_ok(int n)
{
#define PAT_CFFT_CASE_OK(L) if (n == L) return true;
    PAT_CFFT_LENGTHS(PAT_CFFT_CASE_OK)
#undef PAT_CFFT_CASE_OK
    return false;
}

// A length of the ring kernels' two-wave group
__host__ __device__ constexpr bool cfft_len2_ok(int n)
{
#define PAT_CFFT_CASE_OK(L) if (n == L) return true;
    PAT_CFFT_LENGTHS_HI2(PAT_CFFT_CASE_OK)
#undef PAT_CFFT_CASE_OK
    return false;
}

// Table entries of length n's transform: for each pass s with Ns > 1, Ns rows
// of R - 1 twiddles e^{-2 pi i k r / (Ns R)}, r = 1..R-1 (row k at
// twoff[s] + k (R - 1)).
__host__ __device__ constexpr int cfft_table_size(int n) { return make_cplan(n).twoff[make_cplan(n).np]; }

template <int N>
struct CPlanOf {
    static constexpr CPlan p = make_cplan(N);
};

// LDS slot of element i of a sequence: with PAD, one spare slot after every 16
// elements, so that the stores of a radix-16 pass (stride 16 elements) and the
// power-of-two strides of later passes fall on different banks.  A padded
// sequence of length N takes cfft_padded_len(N) slots.
template <bool PAD>
__device__ __forceinline__ constexpr int cfft_slot(int i)
{
    return PAD ? i + (i >> 4) : i;
}
__host__ __device__ constexpr int cfft_padded_len(int n) { return n + n / 16; }

// The twiddles of one pass for a lane's RND butterflies: w^{r k}, r = 1..R-1,
// k = j mod NS (empty for the pass with NS = 1).
template <int N, int R, int NS, int T>
struct PassTw {
    static constexpr int RND = (N / R + T - 1) / T;
    float2 w[NS > 1 ? RND : 1][R - 1];
};

template <int N, int R, int NS, int TWOFF, int T>
__device__ __forceinline__ void pass_tw_load(PassTw<N, R, NS, T>& pt, const float2* __restrict__ tw, bool active, int lane)
{
    constexpr int NB = N / R;
    constexpr int RND = PassTw<N, R, NS, T>::RND;
    if constexpr (NS > 1) {
        if (active) {
#pragma unroll
            for (int i = 0; i < RND; ++i) {
                const int j0 = lane + i * T;
                const int j = (NB % T == 0 || i + 1 < RND) ? j0 : min(j0, NB - 1);
                const float2* tp = tw + TWOFF + (j % NS) * (R - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) pt.w[i][r - 1] = tp[r - 1];
            }
        }
    }
}

// Passes S, S+1, ... of the length's plan.  A pass's butterflies read their
// inputs from LDS (one lane address plus immediate offsets), multiply by the
// twiddles `cur` (loaded during the previous pass), and, before the barrier
// that precedes their stores, the lane loads the next pass's twiddles, so
// that their global-memory latency overlaps the store phase.  `active` lanes
// (lane = 0 .. T - 1 of the sequence, T >= cfft_lanes(N)) compute, every
// thread of the workgroup passes the barriers; more lanes run the same
// butterflies in the same order (the plan, and so every result, depends on N
// only).
template <int N, bool INV, int S, bool PAD, int T>
__device__ __forceinline__ void cfft_passes_tw(float2* __restrict__ x, const float2* __restrict__ tw, bool active,
                                               int lane, const PassTw<N, CPlanOf<N>::p.rad[S], CPlanOf<N>::p.ns[S], T>& cur)
{
    constexpr CPlan P = CPlanOf<N>::p;
    constexpr int R = P.rad[S], NS = P.ns[S];
    constexpr int NB = N / R;
    constexpr int RND = (NB + T - 1) / T;
    float2 v[RND][R];
    if (active) {
#pragma unroll
        for (int i = 0; i < RND; ++i) {
            const int j0 = lane + i * T;
            // the last round's idle lanes work on the last butterfly (results dropped)
            const int j = (NB % T == 0 || i + 1 < RND) ? j0 : min(j0, NB - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = x[cfft_slot<PAD>(j + r * NB)];
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r)
                    v[i][r] = INV ? cmulc(v[i][r], cur.w[i][r - 1]) : cmul(v[i][r], cur.w[i][r - 1]);
            }
            butterfly<R, INV>(v[i]);
        }
    }
    if constexpr (S + 1 < P.np) {
        PassTw<N, P.rad[S + 1], P.ns[S + 1], T> nxt;
        pass_tw_load<N, P.rad[S + 1], P.ns[S + 1], P.twoff[S + 1], T>(nxt, tw, active, lane);
        __syncthreads();
        if (active) {
#pragma unroll
            for (int i = 0; i < RND; ++i) {
                const int j = lane + i * T;
                if (NB % T == 0 || i + 1 < RND || j < NB) {
                    const int k = j % NS;
                    const int dst = (j - k) * R + k;
#pragma unroll
                    for (int r = 0; r < R; ++r) x[cfft_slot<PAD>(dst + r * NS)] = v[i][r];
                }
            }
        }
        __syncthreads();
        cfft_passes_tw<N, INV, S + 1, PAD, T>(x, tw, active, lane, nxt);
    } else {
        __syncthreads();
        if (active) {
#pragma unroll
            for (int i = 0; i < RND; ++i) {
                const int j = lane + i * T;
                if (NB % T == 0 || i + 1 < RND || j < NB) {
                    const int k = j % NS;
                    const int dst = (j - k) * R + k;
#pragma unroll
                    for (int r = 0; r < R; ++r) x[cfft_slot<PAD>(dst + r * NS)] = v[i][r];
                }
            }
        }
        __syncthreads();
    }
}

// Passes S, S+1, ... of the length's plan (the twiddles of pass S loaded here)
template <int N, bool INV, int S, bool PAD = false, int T = cfft_lanes(N)>
__device__ __forceinline__ void cfft_passes(float2* x, const float2* __restrict__ tw, bool active, int lane)
{
    constexpr CPlan P = CPlanOf<N>::p;
    if constexpr (S < P.np) {
        PassTw<N, P.rad[S], P.ns[S], T> cur;
        pass_tw_load<N, P.rad[S], P.ns[S], P.twoff[S], T>(cur, tw, active, lane);
        cfft_passes_tw<N, INV, S, PAD, T>(x, tw, active, lane, cur);
    }
}

// In-place transform of x[0..N) in LDS (forward: e^{-2 pi i jk/N}, inverse:
// e^{+2 pi i jk/N}, unnormalised); `tw` = the length's table.  Every thread of
// the workgroup calls it (barriers); `active` threads, lanes 0 .. T - 1 of
// the sequence (T >= cfft_lanes(N)), compute.
template <int N, bool INV, int T = cfft_lanes(N)>
__device__ __forceinline__ void cfft(float2* x, const float2* __restrict__ tw, int lane, bool active)
{
    static_assert(CPlanOf<N>::p.np > 0, "no compile-time plan for this length");
    static_assert(T >= cfft_lanes(N), "at least the length's lanes");
    cfft_passes<N, INV, 0, false, T>(x, tw, active, lane);
}

// One-wave lengths, computed by lanes 0..63 of wave 0.
template <int N, bool INV>
__device__ __forceinline__ void cfft(float2* x, const float2* __restrict__ tw)
{
    static_assert(cfft_lanes(N) == kCfftLanes, "one-wave lengths only");
    const int lane = threadIdx.x;
    cfft<N, INV>(x, tw, lane, lane < kCfftLanes);
}

// Lanes that transform a sequence of length n in a workgroup of T threads
__host__ __device__ constexpr int cfft_wg_lanes(int n, int T) { return T > cfft_lanes(n) ? T : cfft_lanes(n); }

// Run-time length of ring length group G in a workgroup of T threads, every
// thread calling (cfft_wg_lanes(n, T) lanes compute).
template <bool INV, int G, int T>
__device__ __forceinline__ void cfft_run_wg(float2* x, int n, const float2* __restrict__ tw)
{
    const int lane = threadIdx.x;
    switch (n) {
#define PAT_CFFT_CASE_WG(L) \
    case L: cfft<L, INV, cfft_wg_lanes(L, T)>(x, tw, lane, lane < cfft_wg_lanes(L, T)); break;
        PAT_CFFT_LENGTHS_LO(PAT_CFFT_CASE_WG)
        default:
            if constexpr (G >= 1) {
                switch (n) {
                    PAT_CFFT_LENGTHS_HI(PAT_CFFT_CASE_WG)
                    default:
                        if constexpr (G >= 2) {
                            switch (n) {
                                PAT_CFFT_LENGTHS_HI2(PAT_CFFT_CASE_WG)
                                default: break;
                            }
                        }
                        break;
                }
            }
            break;
#undef PAT_CFFT_CASE_WG
    }
}

}  // namespace pat
