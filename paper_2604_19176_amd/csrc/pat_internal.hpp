// pat_internal.hpp -- plan layout shared by the host plan builder and the gfx950 kernels.
//
// A plan's device tables are FP32 (or int) copies of quantities computed in FP64
// on the host at plan creation.  Kernels receive a PlanDev by value.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "../../include/pat.h"

namespace pat {

// ES ("exponential of semicircle") interpolation kernel of the polar
// interpolation: phi(t) = exp(beta (sqrt(1 - (2t/w)^2) - 1)) for |t| <= w/2.
constexpr int kEsWidth = 8;
constexpr double kEsBeta = 2.30 * kEsWidth;

constexpr int kMaxStages = 16;

// Default for pat_plan_set_split: calls of at least this many instances run
// as two half-batches on two streams, so that each half's kernels fill the
// other's partly occupied last waves (below it the fork and join cost more
// than that gains at 256^2; the autotuner measures it per plan and batch).
constexpr int kSplitMinBatch = 64;

// One complex FFT length n = 2^a 3^b: Stockham passes of radix 2, 3, 4, 6, 8, 9 or 16.
struct FftDev {
    int n;
    int nst;                       // number of passes
    int tw;                        // offset of this length's twiddles e^{-2 pi i e/n}, e = 0..n-1
    int tb;                        // offset of the per-pass base twiddles e^{-2 pi i k/(Ns R)}, k < Ns
    int ntb;                       // their count: the sum of the passes' Ns
    int pad[3];
    unsigned char rad[kMaxStages]; // radix of each pass
};

// Butterflies one thread holds in a pass of radix R: at most 32 complex values
// and at most `maxb` butterflies (kFftMaxButterflies for the fixed-length
// transforms, kRingFftMaxButterflies in the ring kernels, whose other live
// state leaves fewer registers).
constexpr int kFftMaxButterflies = 4;
constexpr int kRingFftMaxButterflies = 2;
__host__ __device__ constexpr int radix_max_butterflies(int R, int maxb = kFftMaxButterflies)
{
    return (R <= 4 ? 4 : (R <= 9 ? 2 : 1)) < maxb ? (R <= 4 ? 4 : (R <= 9 ? 2 : 1)) : maxb;
}

// Threads per sequence the passes of `d` need (at most `maxb` butterflies per thread).
// Host helpers of the plan builder for other modules (plan.hip):
// fixed_fft_for plans a fixed-length transform of length n (twiddles appended
// to tw; returns the threads per sequence, 0 if none fits);
// fft_workgroup_threads gives the threads of a workgroup transforming `nseq`
// sequences of that length.
int fixed_fft_for(long n, FftDev* out, std::vector<float2>& tw);
int fft_workgroup_threads(int nseq, const FftDev& fd);

__host__ __device__ inline int fft_min_tps(const FftDev& d, int maxb = kFftMaxButterflies)
{
    int t = 1;
    for (int s = 0; s < d.nst; ++s) {
        const int R = d.rad[s], per = radix_max_butterflies(R, maxb);
        const int need = (d.n / R + per - 1) / per;
        t = need > t ? need : t;
    }
    return t;
}

// Only the first kSpreadSplitTiles spread row tiles (around the spectrum's
// origin, where the polar points crowd) may be split, into at most
// kSpreadMaxRuns runs (see kSpreadTh below).
constexpr int kSpreadSplitTiles = 16;
constexpr int kSpreadMaxRuns = 4;

struct PlanDev {
    // sizes
    int N;         // image side
    int Ng;        // oversampled spectral grid side (even, 2^a3^b >= 2N)
    int Hy;        // stored half-spectrum rows: m_y = -4 .. Ng/2+4  (Ng/2 + 9 rows)
    int nlam;      // radial frequencies
    int K;         // highest angular mode
    int Kp;        // K + 1 (row stride of mode arrays)
    int M;         // cosine grid: FFT length 2M
    int T;         // time samples
    int D;         // detectors
    int L;         // chirp-z FFT length
    int npts;      // half-plane polar points (sum over rings of Npsi(n)/2)
    int NB;        // interpolation bands (rows of footprint bases): Ng/2 + 2
    float kappa;   // endpoint term coefficient
    float h2;      // h^2
    // image-side tables
    const float* deap;      // [N]: h / phihat(k - N/2), k = 0..N-1 (one factor per axis)
    const int2* mask_rows;  // [N]: row i keeps columns jlo <= j < jhi
    // polar points, ring order (ring n = 1..nlam occupies [ring_off[n-1], ring_off[n]))
    const int* ring_off;    // [nlam + 1]
    const int* ring_K;      // [nlam]   K_n: modes kept on ring n
    const int* ring_fft;    // [nlam]   FFT descriptor of Npsi(n)/2 (the ring's real transform)
    const int* ring_twn;    // [nlam]   descriptor whose twiddles are those of length Npsi(n)
    const int* ring_joff;   // [nlam]   offset of ring n in Jw
    const float2* coef;     // ragged [ring_joff[n] + k], k = 0..K_n: pre_k i^k J_k(lam_n R) W_n / Npsi(n) (i for odd k)
    // polar points, band order (sorted by footprint base row r0 = by + 4, then bx)
    // for the interpolation and the deterministic spread
    const int* band_of;     // [npts]   ring-order index -> band-order slot
    const float4* bpt_geo;  // [npts]   (bx mod Ng as int bits, ring-order index as int bits, fx, fy)
    const float2* bpt_phase;// [npts]   e^{-i pi (s_x + s_y)/Ng} (half-pixel shift of cell-centred pixels)
    const int* band_ptr;    // [NB][Ng + 1] CSR: first band-order slot with (r0, bx' >= bx)
    // spread work rows (spread_runs): a row tile is swept whole, or as S runs of
    // kSpreadTh / S bands each that write partial rows to the slab region
    int spr_rows;           // work rows: the sum over row tiles of their runs
    int slab_rows;          // rows of the slab region
    const int4* spr_row;    // [spr_rows] (first band, last band, first slab row or -1 if whole, row tile)
    // per row tile t (and zero for every t the adjoint row pass can name past
    // the last): (first slab row of run 0) << 4 | log2 S, or 0 if swept whole
    const unsigned* spr_head;
    // synthesis over detector angles theta_d = theta_0 + d dtheta
    int fold_P;             // P if dtheta = 2 pi s / P (P = 2^a3^b, gcd(s, P) = 1): fold k mod P, one FFT; else 0
    int fold_s;             // s: detector d is point s d of the P-point angular grid (s (D - 1) < P)
    int syn_len;            // P (fold) or the chirp-z FFT length L >= K + D (Bluestein)
    int syn_half;           // 1: fold with even P, synthesis as a real-output FFT of length P/2
    int fft_synh;           // descriptor of length P/2 (syn_half only)
    // (the synthesis factor pre_k = c_k e^{i k theta_0} (fold) or c_k e^{i k theta_0} w^{k^2} (Bluestein),
    //  c_0 = 1, c_k = 2, is part of coef)
    const float2* czt_post; // [D]   w^{d^2}, w = e^{i dtheta/2} (Bluestein only)
    const float2* czt_vhat; // [L]   FFT_L of the chirp filter w^{-m^2}, divided by L (Bluestein only)
    int syn_dense;          // 1: explicit detector angles, synthesis by the dense product with syn_tab
    const float* syn_tab;   // [2(K+1)][D] cos(k theta_d), -sin(k theta_d) (syn_dense only)
    int npsi_max;           // largest per-ring angular grid
    // FFTs
    const FftDev* ffts;
    const float2* tw;
    int fft_grid;  // length Ng
    int fft_dct;   // length 2M
    int fft_syn;   // length syn_len
    // ring kernels with compile-time transforms (cfft.hpp): every ring length
    // Npsi(n)/2 and the half-length synthesis P/2 have one (folded synthesis
    // of even length P, no explicit angles)
    int ring_spec;
    int ring_spec_grp;      // length group of the ring and synthesis lengths (cfft.hpp, ring_spec_threads)
    int syn_ctw;            // offset in ctw of the synthesis transform's table (length P/2)
    int syn_sw;             // offset in ctw of w_P^s = e^{-2 pi i s/P}, s = 0..P/2
    int dct_spec;           // 1: cosine transform of compile-time length 2M (cfft.hpp)
    int dct_ctw;            // offset in ctw of its table
    int grid_spec;          // 1: 2D-FFT passes of compile-time length Ng (cfft.hpp)
    int grid_ctw;           // offset in ctw of its table
    const int* ring_ctw;    // [nlam] offset in ctw of ring n's transform table (length Npsi(n)/2)
    const int* ring_uw;     // [nlam] offset in ctw of w_{Npsi(n)}^k, k = 0..Npsi(n)/2
    const float2* ctw;      // the tables (FP64-computed, FP32)
};

// Launch shapes chosen at plan creation (the autotuner may overwrite them).
struct LaunchCfg {
    int col_np;      // packed column pairs per column-pass workgroup
    int row_rpb;     // rows per row-pass workgroup
    int ring_rt;     // rings per ring-kernel workgroup
    int dct_dp;      // detector pairs per cosine-transform workgroup
    int gat_cb;      // interpolation: columns per tile (32, 64, 128 or 256)
    int gat_th;      // interpolation: bands per tile (power of two, 1..64)
    int spr_cb;      // spread: columns per workgroup (multiple of 64)
    int spr_th;      // spread: rows per workgroup (always kSpreadTh)
    int gat_ib;      // interpolation: instances per tile (1, 2 or 4)
    int spr_ib;      // spread: instances per tile (1, 2 or 4)
    int spr_cap;     // spread: points staged in LDS per chunk
};

// Interpolation tiles: kGatherThreads threads; window of (TH + 7) x (CB + 7)
// spectrum values plus two ints per band.
constexpr int kGatherThreads = 256;
__host__ __device__ constexpr size_t gather_lds_bytes(int CB, int TH, int IB)
{
    return sizeof(float2) * (size_t)IB * (TH + 7) * (CB + 7) + sizeof(int) * 2 * (size_t)TH;
}
// Spread tiles for CAP = 2 CB staged points and IB instances:
//   wx [8][CAP], wy [8][CAP] (ES weights), bx [CAP] (footprint column relative
//   to the tile: lane + 7 - bx is the tap), h [IB][CAP] (complex), and three
//   slots of CB + 10 ints holding bands' rows of the band CSR (pipeline).
__host__ __device__ constexpr size_t spread_lds_words(int CAP, int IB)
{
    return (size_t)CAP * (17 + 2 * IB) + 3 * (size_t)(CAP / 2 + 10);
}

// Ring kernels: a ring workgroup has at least (K + 1) / kRingModesPerThread
// threads; its fills of ring inputs issue kRingFillUnroll loads per thread
// and input at a time (more would cost the transforms registers).
constexpr int kRingModesPerThread = 8;
constexpr int kRingFillUnroll = 4;
constexpr int kRingMaxThreads = 256;
// Their LDS in float2 slots: ring buffer (aliased by the half-length
// synthesis buffer), synthesis buffer, two-level twiddle tables of lengths
// Npsi_max and S.
__host__ __device__ constexpr int ring_tw_slots(int n) { return 64 + (n + 63) / 64; }
// With compile-time transforms: the ring buffer (Npsi_max/2 values), then the
// synthesis transform's P/2 and one more slot (the adjoint's value at P/2).
__host__ __device__ constexpr size_t ring_spec_lds_slots(int npsi_max, int S)
{
    return (size_t)(npsi_max / 2) + (size_t)(S / 2) + 1;
}
__host__ __device__ constexpr size_t ring_lds_slots(int npsi_max, int S, int syn_half)
{
    return (size_t)((npsi_max / 2 > (syn_half ? S / 2 : 0)) ? npsi_max / 2 : S / 2) +
           (size_t)(S > npsi_max / 2 ? S : npsi_max / 2) + (size_t)ring_tw_slots(npsi_max) +
           (size_t)ring_tw_slots(S);
}

// Tile-shape limits of the interpolation and the spread.
inline bool ib_ok(int ib) { return ib == 1 || ib == 2 || ib == 4; }
inline bool gather_shape_ok(int cb, int th, int ib)
{
    return (cb == 32 || cb == 64 || cb == 128 || cb == 256) && th >= 1 && th <= 64 && (th & (th - 1)) == 0 &&
           ib_ok(ib) && gather_lds_bytes(cb, th, ib) <= 64 * 1024;
}
// Spread row tiles: kSpreadTh consecutive bands each (ceil(NB / kSpreadTh)
// tiles), every band swept by one tile only.  A band's footprint reaches the 7
// rows after it, so a tile's contributions to the 7 rows after its last band
// are partial sums: unless the tile is the last one, it leaves them in the
// workspace's tail region and the adjoint row pass adds them to the next
// tile's first 7 rows.  Every grid row is thus the sum of its bands from the
// same 8-row block, then plus the sum of its bands from the block before: one
// fixed order for every launch shape and batch.
//
// Near the spectrum's origin the polar points crowd, and a row tile's longest
// lane (the visits of one column over its bands) is up to three times the
// typical one; such row tiles are split into S = 2 or 4 runs of
// kSpreadTh / S consecutive bands, each swept by its own workgroup, which
// writes the kSpreadTh / S + 7 rows it touches to the slab region.  The
// adjoint row pass then forms such a tile's rows as the sum of its runs'
// partial rows, run by run in band order.  Which tiles are split, and into how
// many runs, depends on the plan's points only (spread_runs in plan.hip), so
// the order is still the same for every launch shape and batch.
constexpr int kSpreadTh = 8;
__host__ __device__ inline int spread_row_tiles(int NB) { return (NB + kSpreadTh - 1) / kSpreadTh; }
// slab rows of one run of a row tile split into S runs
__host__ __device__ inline int spread_run_rows(int S) { return kSpreadTh / S + 7; }
inline bool spread_shape_ok(int cb, int th, int ib)
{
    return cb >= 64 && cb <= 256 && cb % 64 == 0 && th == kSpreadTh && ib_ok(ib);
}
// Instances per tile for a call on `batch` instances of one plan: the largest
// of 4, 2, 1 that is at most the configured count and the batch.
inline int tile_ib(int cfg_ib, int batch)
{
    const int m = cfg_ib < batch ? cfg_ib : batch;
    return m >= 4 ? 4 : (m >= 2 ? 2 : 1);
}

// Per-instance workspace layout (byte offsets; all 256-byte aligned).
struct WsLayout {
    size_t x1;       // [Hy][N]   float2   column-pass output / row-pass-adjoint output
    size_t grid;     // [Hy][Ng]  float2   spectrum / spread target
    size_t hdet;     // [nlam][D] float    ring output (synthesised at the detectors) / cosine-adjoint output
    size_t polar;    // [npts]    float2   polar values: ring order (interpolation output), band order (spread input)
    size_t modes;    // [nlam][K+1] float2 mode coefficients (explicit detector angles only)
    size_t tail;     // [ceil(NB/8)][7][Ng] float2  spread: partial sums after each row tile's last band
    size_t slab;     // [slab_rows][Ng] float2  spread: partial rows of the runs of split row tiles
    size_t red;      // small FP32 partial sums (mass / data sum)
    int n_red;       // number of partial sums
    size_t bytes;    // total per instance
};

// Work-item classes of the stage kernels; a heterogeneous batch launches each
// class once over all of its instances.
enum BatchStage {
    kStCol = 0,   // column passes: ceil(N / (2 col_np)) tiles
    kStRow,       // row passes: ceil(Hy / row_rpb) tiles
    kStGather,    // interpolation: ceil(Ng / gat_cb) x ceil(NB / gat_th) tiles
    kStRing,      // ring kernels: ceil(nlam / ring_rt) tiles
    kStDct,       // cosine transforms: ceil(ceil(D / 2) / dct_dp) tiles
    kStSpread,    // spread: ceil(Ng / spr_cb) x spr_rows tiles
    kStSynFwd,    // dense synthesis (explicit angles): ceil(nlam / 64) x ceil(D / 64) tiles, else 0
    kStSynAdj,    // its transpose: ceil(nlam / 64) x ceil(2 (K + 1) / 64) tiles, else 0
    kNumStages
};

// One instance of a heterogeneous batch (device table entry).  Tile shapes
// that fix a workgroup's size (gat_cb, spr_cb) are common to the batch; the
// others are per instance.
struct BatchInst {
    PlanDev d;
    WsLayout L;
    size_t ws_off;    // byte offset of the instance's workspace in the batch workspace
    int col_np, row_rpb, ring_rt, dct_dp, gat_th;
    int n_col_tiles, n_pair_tiles;
};

struct BatchDev {
    const BatchInst* inst;  // [count]
    const int* base;        // [kNumStages][count + 1]: first work item of each instance, per stage
    int count;
};

}  // namespace pat

struct pat_plan {
    pat_plan_desc desc;     // as given at creation
    pat::PlanDev dev;
    pat::LaunchCfg cfg;
    pat::WsLayout ws;
    pat::FftDev h_fft_grid, h_fft_dct;  // host copies of two FFT descriptors (launch checks)
    int device;
    int max_batch;
    int n_psi_uniform;
    int M;
    double dlam;
    double kappa;
    int n_psi_max;
    int n_ring_modes;
    size_t table_bytes;
    void* table_mem;        // one device allocation holding every table
    int n_col_tiles;        // column-pass tiles (mass partials)
    int n_pair_tiles;       // cosine-transform tiles (data-sum partials)
    int thr_col, thr_row, thr_ring, thr_dct;  // workgroup sizes of the FFT kernels
    size_t lds_ring;        // dynamic LDS of the ring kernels
    double* det_theta;      // copy of the explicit detector angles (NULL for a uniform arc)
    // optional per-kernel timing (pat_profile_enable): events around each launch
    int prof;
    hipEvent_t ev[2][8];
    int ev_count[2];
    // two-stream calls (pat_plan_set_split): calls of at least split_min
    // instances run their second half on `side`, forked from and joined to the
    // caller's stream by ev_fork / ev_join; split_mu keeps one call's
    // fork-launch-join sequence together when several host threads share the plan
    int split_min;
    hipStream_t side;
    hipEvent_t ev_fork, ev_join;
    std::mutex* split_mu;
};

namespace pat {
// Threads of a 2D-FFT pass workgroup over `nseq` sequences of the plan's grid side.
int grid_threads(const pat_plan* p, int nseq);
}  // namespace pat

// A heterogeneous batch (pat_batch_create).
struct pat_batch {
    int count = 0;
    int device = 0;
    std::vector<pat_plan*> plans;
    std::vector<pat::BatchInst> inst;  // host copy of the device table
    std::vector<int> base;             // [kNumStages][count + 1]
    void* table = nullptr;             // device: BatchInst[count], then base
    size_t base_off = 0;
    size_t ws_bytes = 0;
    int gat_cb = 64, gat_th = 8, spr_cb = 64, spr_th = pat::kSpreadTh;
    // per-stage workgroup size and dynamic LDS (maxima over the instances)
    unsigned thr_col = 0, thr_row = 0, thr_ring = 0, thr_dct = 0;
    size_t lds_col = 0, lds_row = 0, lds_ring = 0, lds_dct = 0;
};
