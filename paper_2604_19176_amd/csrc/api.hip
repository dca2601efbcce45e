// api.hip -- C-ABI entry points: argument checks on the host, then stream-ordered launches.
//
// The kernels live in kernels.hip, compiled into this translation unit so the
// launches need no relocatable device code.
#include "../../include/pat.h"
#include "kernels.hip"

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>



using namespace pat;


static unsigned xcd_grid(int items) { return (unsigned)(((items + kXcds - 1) / kXcds) * kXcds); }

// Dynamic LDS of the interpolation ([8][cb + 7] float2 window) and of the
// spread (2 cb staged points x 19 words).
static size_t spread_lds(int cb, int ib) { return sizeof(float) * spread_lds_words(2 * cb, ib); }

// Launches of the interpolation and spread instantiations (tile width and
// instances per tile are template parameters of the kernels).
template <int IB>
static void gather_launch_ib(int cb, dim3 grid, size_t lds, hipStream_t st, const PlanDev& d, const WsLayout& L,
                             InstPtrs wsp, int th, int batch)
{
    const dim3 blk(kGatherThreads);
    switch (cb) {
        case 32: hipLaunchKernelGGL((k_gather<IB, 32>), grid, blk, lds, st, d, L, wsp, th, batch); break;
        case 64: hipLaunchKernelGGL((k_gather<IB, 64>), grid, blk, lds, st, d, L, wsp, th, batch); break;
        case 128: hipLaunchKernelGGL((k_gather<IB, 128>), grid, blk, lds, st, d, L, wsp, th, batch); break;
        default: hipLaunchKernelGGL((k_gather<IB, 256>), grid, blk, lds, st, d, L, wsp, th, batch); break;
    }
}

template <int IB>
static void spread_launch_ib(int cb, dim3 grid, size_t lds, hipStream_t st, const PlanDev& d, const WsLayout& L,
                             InstPtrs wsp, int batch)
{
    switch (cb) {
        case 64: hipLaunchKernelGGL((k_spread<IB, 64>), grid, dim3(64), lds, st, d, L, wsp, batch); break;
        case 128: hipLaunchKernelGGL((k_spread<IB, 128>), grid, dim3(128), lds, st, d, L, wsp, batch); break;
        case 192: hipLaunchKernelGGL((k_spread<IB, 192>), grid, dim3(192), lds, st, d, L, wsp, batch); break;
        default: hipLaunchKernelGGL((k_spread<IB, 256>), grid, dim3(256), lds, st, d, L, wsp, batch); break;
    }
}
// LDS of an FFT tile: nseq sequences of the length plus its per-pass twiddles
static size_t fft_tile_lds(int nseq, const FftDev& f) { return sizeof(float2) * ((size_t)nseq * f.n + f.ntb); }

// Output tiles of the dense synthesis (explicit detector angles) per instance
static int syn_fwd_tiles(const PlanDev& d)
{
    return ((d.nlam + kSynTile - 1) / kSynTile) * ((d.D + kSynTile - 1) / kSynTile);
}
static int syn_adj_tiles(const PlanDev& d)
{
    return ((d.nlam + kSynTile - 1) / kSynTile) * ((2 * d.Kp + kSynTile - 1) / kSynTile);
}

// LDS of a cosine-transform tile (compile-time length: no twiddles in LDS)
static size_t dct_tile_lds(const pat_plan* p, int dp)
{
    if (p->dev.dct_spec) return sizeof(float2) * (size_t)dp * cfft_padded_len(2 * p->dev.M);
    return fft_tile_lds(dp, p->h_fft_dct);
}

static void dct_launch(const pat_plan* p, hipStream_t st, const InstPtrs& wsp, float* gout, const float* gin, int adj,
                       int n_mass, int batch)
{
    const PlanDev& d = p->dev;
    const int dp = p->cfg.dct_dp;
    const dim3 grid(xcd_grid(p->n_pair_tiles * batch)), blk(p->thr_dct);
    const size_t lds = dct_tile_lds(p, dp);
    if (!d.dct_spec) {
        hipLaunchKernelGGL(k_dct_det, grid, blk, lds, st, d, p->ws, wsp, gout, gin, dp, adj, n_mass, batch);
        return;
    }
    switch (2 * d.M) {
#define PAT_DCT_LAUNCH(N2) \
    case N2: hipLaunchKernelGGL(k_dct_spec<N2>, grid, blk, lds, st, d, p->ws, wsp, gout, gin, dp, adj, n_mass, batch); break;
        PAT_DCT_LENGTHS(PAT_DCT_LAUNCH)
#undef PAT_DCT_LAUNCH
        default: break;
    }
}

static int check_launch()
{
    return hipGetLastError() == hipSuccess ? PAT_OK : PAT_ERR_HIP;
}

// Per-kernel timing: event q is recorded before launch q, event q+1 after it.
static inline void prof_mark(const pat_plan* p, int dir, int q, hipStream_t st)
{
    if (p->prof) (void)hipEventRecord(p->ev[dir][q], st);
}

static int validate(const pat_plan* p, const void* in, const void* out, int batch, const void* ws,
                    size_t ws_bytes)
{
    if (!p || !in || !out) return PAT_ERR_ARG;
    if (p->thr_col <= 0 || p->thr_row <= 0 || p->thr_dct <= 0 || p->thr_ring <= 0) return PAT_ERR_ARG;
    if (batch < 1 || batch > p->max_batch) return PAT_ERR_ARG;
    if (!ws || ((uintptr_t)ws & 255)) return PAT_ERR_WORKSPACE;
    if (ws_bytes < pat_workspace_size(p, batch)) return PAT_ERR_WORKSPACE;
    return PAT_OK;
}

// The forward's launches for `batch` instances on stream st (arguments checked)
static int forward_run(const pat_plan* p, const float* f, float* g, int batch, void* ws, hipStream_t st)
{
    int rc = PAT_OK;
    const PlanDev& d = p->dev;
    const LaunchCfg& c = p->cfg;
    const InstPtrs wsp{(char*)ws, p->ws.bytes};
    prof_mark(p, 0, 0, st);
    hipLaunchKernelGGL(k_colpass_fwd, dim3(p->n_col_tiles, batch), dim3(p->thr_col), fft_tile_lds(c.col_np, p->h_fft_grid), st,
                       d, p->ws, f, wsp, c.col_np);
    if ((rc = check_launch())) return rc;
    prof_mark(p, 0, 1, st);
    hipLaunchKernelGGL(k_rowpass_fwd, dim3((d.Hy + c.row_rpb - 1) / c.row_rpb, batch), dim3(p->thr_row),
                       fft_tile_lds(c.row_rpb, p->h_fft_grid), st, d, p->ws, wsp, c.row_rpb);
    if ((rc = check_launch())) return rc;
    prof_mark(p, 0, 2, st);
    {
        const int cb = c.gat_cb, th = c.gat_th, ib = tile_ib(c.gat_ib, batch);
        const int items = ((d.Ng + cb - 1) / cb) * ((d.NB + th - 1) / th) * ((batch + ib - 1) / ib);
        const dim3 grid(xcd_grid(items));
        const size_t lds = gather_lds_bytes(cb, th, ib);
        if (ib == 4) gather_launch_ib<4>(cb, grid, lds, st, d, p->ws, wsp, th, batch);
        else if (ib == 2) gather_launch_ib<2>(cb, grid, lds, st, d, p->ws, wsp, th, batch);
        else gather_launch_ib<1>(cb, grid, lds, st, d, p->ws, wsp, th, batch);
    }
    if ((rc = check_launch())) return rc;
    prof_mark(p, 0, 3, st);
    {
        const int rt = d.ring_spec ? 1 : c.ring_rt;  // compile-time ring kernels: one ring per workgroup
        const dim3 grid(xcd_grid((d.nlam + rt - 1) / rt * batch)), blk(p->thr_ring);
        if (d.ring_spec && d.ring_spec_grp == 2)
            hipLaunchKernelGGL((k_ring_fwd_spec<2, 1>), grid, blk, p->lds_ring, st, d, p->ws, wsp, batch);
        else if (d.ring_spec && d.ring_spec_grp == 1)
            hipLaunchKernelGGL((k_ring_fwd_spec<1, 1>), grid, blk, p->lds_ring, st, d, p->ws, wsp, batch);
        else if (d.ring_spec && p->thr_ring == ring_spec_threads(0, 2))
            hipLaunchKernelGGL((k_ring_fwd_spec<0, 2>), grid, blk, p->lds_ring, st, d, p->ws, wsp, batch);
        else if (d.ring_spec)
            hipLaunchKernelGGL((k_ring_fwd_spec<0, 1>), grid, blk, p->lds_ring, st, d, p->ws, wsp, batch);
        else hipLaunchKernelGGL(k_ring_fwd, grid, blk, p->lds_ring, st, d, p->ws, wsp, c.ring_rt, batch);
    }
    if ((rc = check_launch())) return rc;
    prof_mark(p, 0, 4, st);
    const int qd = d.syn_dense ? 5 : 4;  // event index after the synthesis
    if (d.syn_dense) {  // explicit detector angles: synthesis on the matrix cores
        const int nt = syn_fwd_tiles(d);
        hipLaunchKernelGGL(k_syn_dense_fwd, dim3(xcd_grid(nt * batch)), dim3(kSynThreads), 0, st, d, p->ws, wsp, nt,
                           batch);
        if ((rc = check_launch())) return rc;
        prof_mark(p, 0, qd, st);
    }
    dct_launch(p, st, wsp, g, nullptr, 0, d.N, batch);
    if ((rc = check_launch())) return rc;
    prof_mark(p, 0, qd + 1, st);
    return PAT_OK;
}

// The adjoint's launches for `batch` instances on stream st (arguments checked)
static int adjoint_run(const pat_plan* p, const float* g, float* f, int batch, void* ws, hipStream_t st)
{
    int rc = PAT_OK;
    const PlanDev& d = p->dev;
    const LaunchCfg& c = p->cfg;
    const InstPtrs wsp{(char*)ws, p->ws.bytes};
    prof_mark(p, 1, 0, st);
    dct_launch(p, st, wsp, nullptr, g, 1, 0, batch);
    if ((rc = check_launch())) return rc;
    prof_mark(p, 1, 1, st);
    const int qa = d.syn_dense ? 1 : 0;  // event offset after the transposed synthesis
    if (d.syn_dense) {  // explicit detector angles: the transposed synthesis on the matrix cores
        const int nt = syn_adj_tiles(d);
        hipLaunchKernelGGL(k_syn_dense_adj, dim3(xcd_grid(nt * batch)), dim3(kSynThreads), 0, st, d, p->ws, wsp, nt,
                           batch);
        if ((rc = check_launch())) return rc;
        prof_mark(p, 1, 2, st);
    }
    {
        const int rt = d.ring_spec ? 1 : c.ring_rt;
        const dim3 grid(xcd_grid((d.nlam + rt - 1) / rt * batch)), blk(p->thr_ring);
        if (d.ring_spec && d.ring_spec_grp == 2)
            hipLaunchKernelGGL((k_ring_adj_spec<2, 1>), grid, blk, p->lds_ring, st, d, p->ws, wsp, batch);
        else if (d.ring_spec && d.ring_spec_grp == 1)
            hipLaunchKernelGGL((k_ring_adj_spec<1, 1>), grid, blk, p->lds_ring, st, d, p->ws, wsp, batch);
        else if (d.ring_spec && p->thr_ring == ring_spec_threads(0, 2))
            hipLaunchKernelGGL((k_ring_adj_spec<0, 2>), grid, blk, p->lds_ring, st, d, p->ws, wsp, batch);
        else if (d.ring_spec)
            hipLaunchKernelGGL((k_ring_adj_spec<0, 1>), grid, blk, p->lds_ring, st, d, p->ws, wsp, batch);
        else hipLaunchKernelGGL(k_ring_adj, grid, blk, p->lds_ring, st, d, p->ws, wsp, c.ring_rt, batch);
    }
    if ((rc = check_launch())) return rc;
    prof_mark(p, 1, 2 + qa, st);
    {
        const int cb = c.spr_cb, ib = tile_ib(c.spr_ib, batch);
        const int items = ((d.Ng + cb - 1) / cb) * d.spr_rows * ((batch + ib - 1) / ib);
        const dim3 grid(xcd_grid(items));
        const size_t lds = spread_lds(cb, ib);
        if (ib == 4) spread_launch_ib<4>(cb, grid, lds, st, d, p->ws, wsp, batch);
        else if (ib == 2) spread_launch_ib<2>(cb, grid, lds, st, d, p->ws, wsp, batch);
        else spread_launch_ib<1>(cb, grid, lds, st, d, p->ws, wsp, batch);
    }
    if ((rc = check_launch())) return rc;
    prof_mark(p, 1, 3 + qa, st);
    hipLaunchKernelGGL(k_rowpass_adj, dim3((d.Hy + c.row_rpb - 1) / c.row_rpb, batch), dim3(p->thr_row),
                       fft_tile_lds(c.row_rpb, p->h_fft_grid), st, d, p->ws, wsp, c.row_rpb);
    if ((rc = check_launch())) return rc;
    prof_mark(p, 1, 4 + qa, st);
    hipLaunchKernelGGL(k_colpass_adj, dim3(p->n_col_tiles, batch), dim3(p->thr_col), fft_tile_lds(c.col_np, p->h_fft_grid), st,
                       d, p->ws, wsp, f, c.col_np, d.D);
    if ((rc = check_launch())) return rc;
    prof_mark(p, 1, 5 + qa, st);
    return PAT_OK;
}

// ---------------------------------------------------------------------------
// Two-stream calls.  A call of at least p->split_min instances (and not under
// per-kernel timing, whose events time one stream's launches) runs instances
// [0, h) on the caller's stream and [h, batch) on the plan's side stream,
// h = batch / 2: the side stream waits for an event recorded on the caller's
// stream, and the caller's stream waits for one recorded on the side stream
// after its launches, so the call is ordered on the caller's stream as a
// one-stream call is, and a graph captured from the caller's stream holds both
// halves.  Each instance is computed by the same kernels with the same tiles
// whichever half it is in, so the results are bitwise those of one stream.
// ---------------------------------------------------------------------------
template <class Run>
static int split_run(const pat_plan* p, int batch, hipStream_t st, size_t in_each, size_t out_each, const float* in,
                     float* out, void* ws, Run run)
{
    if (p->prof || p->split_min < 2 || batch < p->split_min || !p->side) return run(in, out, batch, ws, st);
    const int h = batch / 2;
    std::lock_guard<std::mutex> lk(*p->split_mu);
    if (hipEventRecord(p->ev_fork, st) != hipSuccess || hipStreamWaitEvent(p->side, p->ev_fork, 0) != hipSuccess)
        return PAT_ERR_HIP;
    int rc = run(in + (size_t)h * in_each, out + (size_t)h * out_each, batch - h,
                 (char*)ws + (size_t)h * p->ws.bytes, p->side);
    if (rc == PAT_OK) rc = run(in, out, h, ws, st);
    // the join is enqueued whatever the halves returned: the side stream
    // never stays forked from the caller's (nor out of a capture)
    const bool joined = hipEventRecord(p->ev_join, p->side) == hipSuccess &&
                        hipStreamWaitEvent(st, p->ev_join, 0) == hipSuccess;
    if (rc == PAT_OK && !joined) rc = PAT_ERR_HIP;
    return rc;
}

extern "C" int pat_forward(const pat_plan* p, const float* f, float* g, int batch, void* ws, size_t ws_bytes,
                           void* stream)
{
    const int rc = validate(p, f, g, batch, ws, ws_bytes);
    if (rc != PAT_OK) return rc;
    const PlanDev& d = p->dev;
    return split_run(p, batch, (hipStream_t)stream, (size_t)d.N * d.N, (size_t)d.D * d.T, f, g, ws,
                     [&](const float* fi, float* go, int nb, void* wsi, hipStream_t s) {
                         return forward_run(p, fi, go, nb, wsi, s);
                     });
}

extern "C" int pat_adjoint(const pat_plan* p, const float* g, float* f, int batch, void* ws, size_t ws_bytes,
                           void* stream)
{
    const int rc = validate(p, g, f, batch, ws, ws_bytes);
    if (rc != PAT_OK) return rc;
    const PlanDev& d = p->dev;
    return split_run(p, batch, (hipStream_t)stream, (size_t)d.D * d.T, (size_t)d.N * d.N, g, f, ws,
                     [&](const float* gi, float* fo, int nb, void* wsi, hipStream_t s) {
                         return adjoint_run(p, gi, fo, nb, wsi, s);
                     });
}

extern "C" int pat_plan_set_split(pat_plan* p, int min_batch)
{
    if (!p || min_batch < 0) return PAT_ERR_ARG;
    p->split_min = min_batch;
    return PAT_OK;
}

extern "C" int pat_plan_get_split(const pat_plan* p, int* min_batch)
{
    if (!p || !min_batch) return PAT_ERR_ARG;
    *min_batch = p->split_min;
    return PAT_OK;
}

// ---------------------------------------------------------------------------
// pat_forward_noalloc: pat_forward with the library's own workspace, a
// file-scope device array (one per GPU, held until the process ends).  On the
// host the array's name only stands for the symbol; its device address is
// looked up once per device (hipGetSymbolAddress) and kept in
// g_scratch_ptr.  Calls on one device share the array: calls that overlap
// on a device race.  The forward kernels write every workspace word they
// read, so nothing needs clearing between calls.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[PAT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

static int scratch_for_device(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxDevices) return PAT_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;  // the caller's current device is `dev`
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PAT_ERR_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PAT_OK;
}

extern "C" int pat_forward_noalloc(const pat_plan* p, const float* f, float* g, int batch, void* stream)
{
    if (!p || !f || !g || batch < 1 || batch > p->max_batch) return PAT_ERR_ARG;
    if (pat_workspace_size(p, batch) > (size_t)PAT_NOALLOC_SCRATCH_BYTES) return PAT_ERR_WORKSPACE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return PAT_ERR_HIP;
    if (dev != p->device) return PAT_ERR_ARG;
    void* ws = nullptr;
    const int rc = scratch_for_device(dev, &ws);
    if (rc != PAT_OK) return rc;
    return pat_forward(p, f, g, batch, ws, (size_t)PAT_NOALLOC_SCRATCH_BYTES, stream);
}

extern "C" int pat_tv_grad(const float* f, float* grad, float* tv, int n, int batch, float eps, void* stream)
{
    if (!f || !grad || n < 2 || batch < 1 || !(eps > 0.f)) return PAT_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    dim3 grid((n + 15) / 16, (n + 15) / 16, batch);
    hipLaunchKernelGGL(k_tv_grad, grid, dim3(256), 0, st, f, grad, n, eps * eps);
    int rc = check_launch();
    if (rc || !tv) return rc;
    hipLaunchKernelGGL(k_tv_value, dim3(batch), dim3(1024), 0, st, f, tv, n, eps * eps);
    return check_launch();
}

extern "C" int pat_pgd_update(float* f, const float* adj, const float* tvgrad, long count, float tau, float lambda,
                              void* stream)
{
    if (!f || !adj || count < 1) return PAT_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    long blocks = std::min<long>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pgd_update, dim3((unsigned)blocks), dim3(256), 0, st, f, adj, tvgrad, count, tau, lambda);
    return check_launch();
}

extern "C" int pat_residual(float* g, const float* g_meas, float* sq, long count_per, int batch, void* stream)
{
    if (!g || !g_meas || count_per < 1 || batch < 1) return PAT_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const long count = count_per * batch;
    long blocks = std::min<long>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_residual, dim3((unsigned)blocks), dim3(256), 0, st, g, g_meas, count);
    int rc = check_launch();
    if (rc || !sq) return rc;
    hipLaunchKernelGGL(k_half_sq, dim3(batch), dim3(1024), 0, st, g, sq, count_per);
    return check_launch();
}

extern "C" int pat_pd_dual_data(float* y1, const float* ax, const float* g, long count, float sigma, void* stream)
{
    if (!y1 || !ax || !g || count < 1 || !(sigma > 0.f)) return PAT_ERR_ARG;
    const long blocks = std::min<long>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pd_dual_data, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, y1, ax, g, count,
                       sigma, 1.f / (1.f + sigma));
    return check_launch();
}

extern "C" int pat_pd_dual_tv(float* y2, const float* xbar, int n, int batch, float sigma, float alpha, void* stream)
{
    if (!y2 || !xbar || n < 2 || batch < 1 || !(sigma > 0.f) || !(alpha >= 0.f)) return PAT_ERR_ARG;
    const dim3 grid((n + 15) / 16, (n + 15) / 16, batch);
    hipLaunchKernelGGL(k_pd_dual_tv, grid, dim3(256), 0, (hipStream_t)stream, (float2*)y2, xbar, n, sigma, alpha);
    return check_launch();
}

extern "C" int pat_pd_primal(float* f, float* xbar, const float* aty, const float* y2, int n, int batch, float tau,
                             void* stream)
{
    if (!f || !xbar || !aty || !y2 || n < 2 || batch < 1 || !(tau > 0.f)) return PAT_ERR_ARG;
    const dim3 grid((n + 15) / 16, (n + 15) / 16, batch);
    hipLaunchKernelGGL(k_pd_primal, grid, dim3(256), 0, (hipStream_t)stream, f, xbar, aty, (const float2*)y2, n,
                       tau);
    return check_launch();
}

extern "C" int pat_pd_change(const float* f, const float* xbar, float* out, int n, int batch, void* stream)
{
    if (!f || !xbar || !out || n < 1 || batch < 1) return PAT_ERR_ARG;
    hipLaunchKernelGGL(k_pd_change, dim3(batch), dim3(1024), 0, (hipStream_t)stream, f, xbar, out, (long)n * n);
    return check_launch();
}

static dim3 elementwise_grid(long n, int batch)
{
    long blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    return dim3((unsigned)(blocks < 1 ? 1 : blocks), (unsigned)batch);
}

extern "C" int pat_cg_norm2(const float* x, float* out, long count, int batch, void* stream)
{
    if (!x || !out || count < 1 || batch < 1) return PAT_ERR_ARG;
    hipLaunchKernelGGL(k_cg_norm2, dim3(batch), dim3(1024), 0, (hipStream_t)stream, x, out, count);
    return check_launch();
}

extern "C" int pat_cg_step_fr(float* f, const float* p, long nf, float* r, const float* q, long nr,
                              const float* gamma, const float* qq, int batch, void* stream)
{
    if (!f || !p || !r || !q || !gamma || !qq || nf < 1 || nr < 1 || batch < 1) return PAT_ERR_ARG;
    hipLaunchKernelGGL(k_cg_step_fr, elementwise_grid(nf > nr ? nf : nr, batch), dim3(256), 0, (hipStream_t)stream,
                       f, p, nf, r, q, nr, gamma, qq);
    return check_launch();
}

extern "C" int pat_cg_step_p(float* p, const float* s, long n, const float* gamma_new, const float* gamma, int batch,
                             void* stream)
{
    if (!p || !s || !gamma_new || !gamma || n < 1 || batch < 1) return PAT_ERR_ARG;
    hipLaunchKernelGGL(k_cg_step_p, elementwise_grid(n, batch), dim3(256), 0, (hipStream_t)stream, p, s, n,
                       gamma_new, gamma);
    return check_launch();
}

extern "C" int pat_stream_copy(const void* src, void* dst, size_t bytes, const int* perm, void* stream)
{
    if (!src || !dst || bytes == 0) return PAT_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (!perm) {
        if ((bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return PAT_ERR_ARG;
        const long n4 = (long)(bytes / 16);
        const long blocks = std::min<long>((n4 + 1023) / 1024, 256L * 32);
        hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, st, (const float4*)src,
                           (float4*)dst, n4);
    } else {
        if ((bytes & 7) || ((uintptr_t)src & 7) || ((uintptr_t)dst & 7) || bytes / 8 > 0x7fffffffUL)
            return PAT_ERR_ARG;
        const long n = (long)(bytes / 8);
        const long blocks = std::min<long>((n + 255) / 256, 256L * 64);
        hipLaunchKernelGGL(k_scatter_copy, dim3((unsigned)blocks), dim3(256), 0, st, (const float2*)src,
                           (float2*)dst, perm, n);
    }
    return check_launch();
}

extern "C" int pat_profile_enable(pat_plan* p, int enable)
{
    if (!p) return PAT_ERR_ARG;
    if (enable && !p->prof) {
        for (int dir = 0; dir < 2; ++dir)
            for (int q = 0; q < 8; ++q)
                if (hipEventCreate(&p->ev[dir][q]) != hipSuccess) return PAT_ERR_HIP;
        // 5 kernels per direction, 6 with the dense synthesis (explicit angles)
        p->ev_count[0] = p->ev_count[1] = p->dev.syn_dense ? 7 : 6;
        p->prof = 1;
    } else if (!enable && p->prof) {
        for (int dir = 0; dir < 2; ++dir)
            for (int q = 0; q < 8; ++q) (void)hipEventDestroy(p->ev[dir][q]);
        p->prof = 0;
    }
    return PAT_OK;
}

extern "C" int pat_profile_read(const pat_plan* p, int which, float* ms, int max_kernels, int* count)
{
    if (!p || !ms || !count || (which != 0 && which != 1)) return PAT_ERR_ARG;
    if (!p->prof) return PAT_ERR_ARG;
    const int nk = p->ev_count[which] - 1;
    if (max_kernels < nk) return PAT_ERR_ARG;
    if (hipEventSynchronize(p->ev[which][nk]) != hipSuccess) return PAT_ERR_HIP;
    for (int q = 0; q < nk; ++q)
        if (hipEventElapsedTime(&ms[q], p->ev[which][q], p->ev[which][q + 1]) != hipSuccess) return PAT_ERR_HIP;
    *count = nk;
    return PAT_OK;
}

extern "C" const char* pat_status_string(int s)
{
    switch (s) {
        case PAT_OK: return "ok";
        case PAT_ERR_ARG: return "invalid argument";
        case PAT_ERR_UNSUPPORTED: return "unsupported geometry";
        case PAT_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
        case PAT_ERR_HIP: return "HIP runtime error";
        case PAT_ERR_ALLOC: return "device allocation failed";
        default: return "unknown status";
    }
}

// ---------------------------------------------------------------------------
// launch shapes
// ---------------------------------------------------------------------------
namespace pat {
int apply_launch(pat_plan* p, const LaunchCfg& c);
}

static void launch_to_public(const LaunchCfg& c, pat_launch* o)
{
    o->col_np = c.col_np;
    o->row_rpb = c.row_rpb;
    o->ring_rt = c.ring_rt;
    o->dct_dp = c.dct_dp;
    o->gat_cb = c.gat_cb;
    o->gat_th = c.gat_th;
    o->spr_cb = c.spr_cb;
    o->spr_th = c.spr_th;
    o->gat_ib = c.gat_ib;
    o->spr_ib = c.spr_ib;
}

extern "C" int pat_plan_get_launch(const pat_plan* p, pat_launch* out)
{
    if (!p || !out) return PAT_ERR_ARG;
    launch_to_public(p->cfg, out);
    return PAT_OK;
}

extern "C" int pat_plan_set_launch(pat_plan* p, const pat_launch* in)
{
    if (!p || !in) return PAT_ERR_ARG;
    LaunchCfg c = p->cfg;
    c.col_np = in->col_np;
    c.row_rpb = in->row_rpb;
    c.ring_rt = in->ring_rt;
    c.dct_dp = in->dct_dp;
    c.gat_cb = in->gat_cb;
    c.gat_th = in->gat_th;
    c.spr_cb = in->spr_cb;
    c.spr_th = in->spr_th;
    c.gat_ib = in->gat_ib;
    c.spr_ib = in->spr_ib;
    return apply_launch(p, c);  // leaves the plan unchanged on error
}

// ---------------------------------------------------------------------------
// heterogeneous batches: one launch per stage over every instance
// ---------------------------------------------------------------------------

static bool batch_shape_ok(const pat_launch& c)
{
    return gather_shape_ok(c.gat_cb, c.gat_th, 1) && spread_shape_ok(c.spr_cb, c.spr_th, 1);
}

// Per-stage work-item prefix sums for the current batch-wide shapes, and the
// per-stage launch maxima.
static void batch_layout(pat_batch* b)
{
    const int n = b->count;
    b->base.assign((size_t)kNumStages * (n + 1), 0);
    b->thr_col = b->thr_row = b->thr_ring = b->thr_dct = 0;
    b->lds_col = b->lds_row = b->lds_ring = b->lds_dct = 0;
    for (int i = 0; i < n; ++i) {
        BatchInst& I = b->inst[i];
        const pat_plan* p = b->plans[i];
        const PlanDev& d = I.d;
        I.gat_th = b->gat_th;
        int items[kNumStages];
        items[kStCol] = I.n_col_tiles;
        items[kStRow] = (d.Hy + I.row_rpb - 1) / I.row_rpb;
        items[kStGather] = ((d.Ng + b->gat_cb - 1) / b->gat_cb) * ((d.NB + b->gat_th - 1) / b->gat_th);
        items[kStRing] = d.ring_spec ? d.nlam : (d.nlam + I.ring_rt - 1) / I.ring_rt;
        items[kStDct] = I.n_pair_tiles;
        items[kStSynFwd] = d.syn_dense ? syn_fwd_tiles(d) : 0;
        items[kStSynAdj] = d.syn_dense ? syn_adj_tiles(d) : 0;
        items[kStSpread] = ((d.Ng + b->spr_cb - 1) / b->spr_cb) * d.spr_rows;
        for (int s = 0; s < kNumStages; ++s)
            b->base[(size_t)s * (n + 1) + i + 1] = b->base[(size_t)s * (n + 1) + i] + items[s];
        // workgroup sizes from the tile shapes copied into the instance (a later
        // set_launch or autotune of the plan does not change this batch)
        b->thr_col = std::max<unsigned>(b->thr_col, grid_threads(p, I.col_np));
        b->thr_row = std::max<unsigned>(b->thr_row, grid_threads(p, I.row_rpb));
        b->thr_ring = std::max<unsigned>(b->thr_ring, p->thr_ring);
        b->thr_dct = std::max<unsigned>(b->thr_dct, d.dct_spec ? I.dct_dp * cfft_lanes(2 * d.M)
                                                               : fft_workgroup_threads(I.dct_dp, p->h_fft_dct));
        b->lds_col = std::max(b->lds_col, fft_tile_lds(I.col_np, p->h_fft_grid));
        b->lds_row = std::max(b->lds_row, fft_tile_lds(I.row_rpb, p->h_fft_grid));
        b->lds_ring = std::max(b->lds_ring, p->lds_ring);
        b->lds_dct = std::max(b->lds_dct, dct_tile_lds(p, I.dct_dp));
    }
}

static int batch_upload(pat_batch* b)
{
    const size_t ti = sizeof(BatchInst) * (size_t)b->count;
    if (hipMemcpy(b->table, b->inst.data(), ti, hipMemcpyHostToDevice) != hipSuccess) return PAT_ERR_HIP;
    if (hipMemcpy((char*)b->table + b->base_off, b->base.data(), sizeof(int) * b->base.size(),
                  hipMemcpyHostToDevice) != hipSuccess)
        return PAT_ERR_HIP;
    return PAT_OK;
}

extern "C" void pat_batch_destroy(pat_batch* b)
{
    if (!b) return;
    if (b->table) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) cur = b->device;
        (void)hipSetDevice(b->device);
        (void)hipFree(b->table);
        (void)hipSetDevice(cur);
    }
    delete b;
}

extern "C" int pat_batch_create(pat_plan* const* plans, int count, pat_batch** out)
{
    if (!plans || !out || count < 1 || count > 65536) return PAT_ERR_ARG;
    for (int i = 0; i < count; ++i)
        if (!plans[i] || plans[i]->device != plans[0]->device) return PAT_ERR_ARG;
    pat_batch* b = new (std::nothrow) pat_batch;
    if (!b) return PAT_ERR_ALLOC;
    b->count = count;
    b->device = plans[0]->device;
    b->plans.assign(plans, plans + count);
    b->inst.resize(count);
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        const pat_plan* p = plans[i];
        BatchInst& I = b->inst[i];
        std::memset(&I, 0, sizeof(I));
        I.d = p->dev;
        I.L = p->ws;
        I.ws_off = off;
        off += (p->ws.bytes + 255) & ~(size_t)255;
        I.col_np = p->cfg.col_np;
        I.row_rpb = p->cfg.row_rpb;
        I.ring_rt = p->cfg.ring_rt;
        I.dct_dp = p->cfg.dct_dp;
        I.n_col_tiles = p->n_col_tiles;
        I.n_pair_tiles = p->n_pair_tiles;
    }
    b->ws_bytes = off;
    // wide interpolation and spread tiles unless the batch is small
    long cells = 0;
    for (int i = 0; i < count; ++i) cells += (long)b->inst[i].d.Ng * b->inst[i].d.Hy;
    b->gat_cb = 64;
    b->gat_th = 8;
    if (cells >= 8L * 512 * 265) { b->gat_cb = 128; b->gat_th = 16; b->spr_cb = 256; }
    batch_layout(b);
    b->base_off = (sizeof(BatchInst) * (size_t)count + 255) & ~(size_t)255;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != b->device) { delete b; return PAT_ERR_ARG; }
    if (hipMalloc(&b->table, b->base_off + sizeof(int) * b->base.size()) != hipSuccess) {
        b->table = nullptr;
        delete b;
        return PAT_ERR_ALLOC;
    }
    const int rc = batch_upload(b);
    if (rc != PAT_OK) { pat_batch_destroy(b); return rc; }
    *out = b;
    return PAT_OK;
}

extern "C" size_t pat_batch_workspace_size(const pat_batch* b) { return b ? b->ws_bytes : 0; }

extern "C" int pat_batch_get_launch(const pat_batch* b, pat_launch* out)
{
    if (!b || !out) return PAT_ERR_ARG;
    std::memset(out, 0, sizeof(*out));
    out->gat_cb = b->gat_cb;
    out->gat_th = b->gat_th;
    out->spr_cb = b->spr_cb;
    out->spr_th = b->spr_th;
    return PAT_OK;
}

extern "C" int pat_batch_set_launch(pat_batch* b, const pat_launch* c)
{
    if (!b || !c || !batch_shape_ok(*c)) return PAT_ERR_ARG;
    if (hipDeviceSynchronize() != hipSuccess) return PAT_ERR_HIP;
    b->gat_cb = c->gat_cb;
    b->gat_th = c->gat_th;
    b->spr_cb = c->spr_cb;
    b->spr_th = c->spr_th;
    batch_layout(b);
    return batch_upload(b);
}

static int batch_validate(const pat_batch* b, const void* a, const void* c, const void* ws, size_t ws_bytes)
{
    if (!b || !a || !c) return PAT_ERR_ARG;
    if (!ws || ((uintptr_t)ws & 255) || ws_bytes < b->ws_bytes) return PAT_ERR_WORKSPACE;
    return PAT_OK;
}

static inline BatchDev batch_dev(const pat_batch* b)
{
    return BatchDev{(const BatchInst*)b->table, (const int*)((const char*)b->table + b->base_off), b->count};
}

static inline int batch_items(const pat_batch* b, int st) { return b->base[(size_t)st * (b->count + 1) + b->count]; }

extern "C" int pat_batch_forward(const pat_batch* b, const float* const* f_ptrs, float* const* g_ptrs, void* ws,
                                 size_t ws_bytes, void* stream)
{
    int rc = batch_validate(b, f_ptrs, g_ptrs, ws, ws_bytes);
    if (rc != PAT_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const BatchDev bt = batch_dev(b);
    char* w = (char*)ws;
    hipLaunchKernelGGL(k_colpass_fwd_b, dim3(xcd_grid(batch_items(b, kStCol))), dim3(b->thr_col), b->lds_col, st, bt,
                       f_ptrs, w);
    if ((rc = check_launch())) return rc;
    hipLaunchKernelGGL(k_rowpass_fwd_b, dim3(xcd_grid(batch_items(b, kStRow))), dim3(b->thr_row), b->lds_row, st, bt,
                       w);
    if ((rc = check_launch())) return rc;
    {
        const dim3 grid(xcd_grid(batch_items(b, kStGather))), blk(kGatherThreads);
        const size_t lds = gather_lds_bytes(b->gat_cb, b->gat_th, 1);
        switch (b->gat_cb) {
            case 32: hipLaunchKernelGGL(k_gather_b<32>, grid, blk, lds, st, bt, w); break;
            case 64: hipLaunchKernelGGL(k_gather_b<64>, grid, blk, lds, st, bt, w); break;
            case 128: hipLaunchKernelGGL(k_gather_b<128>, grid, blk, lds, st, bt, w); break;
            default: hipLaunchKernelGGL(k_gather_b<256>, grid, blk, lds, st, bt, w); break;
        }
    }
    if ((rc = check_launch())) return rc;
    hipLaunchKernelGGL(k_ring_fwd_b, dim3(xcd_grid(batch_items(b, kStRing))), dim3(b->thr_ring), b->lds_ring, st,
                       bt, w);
    if ((rc = check_launch())) return rc;
    if (batch_items(b, kStSynFwd) > 0) {
        hipLaunchKernelGGL(k_syn_dense_fwd_b, dim3(xcd_grid(batch_items(b, kStSynFwd))), dim3(kSynThreads), 0, st,
                           bt, w);
        if ((rc = check_launch())) return rc;
    }
    hipLaunchKernelGGL(k_dct_det_b, dim3(xcd_grid(batch_items(b, kStDct))), dim3(b->thr_dct), b->lds_dct, st, bt, w,
                       g_ptrs, (const float* const*)nullptr, 0);
    return check_launch();
}

extern "C" int pat_batch_adjoint(const pat_batch* b, const float* const* g_ptrs, float* const* f_ptrs, void* ws,
                                 size_t ws_bytes, void* stream)
{
    int rc = batch_validate(b, g_ptrs, f_ptrs, ws, ws_bytes);
    if (rc != PAT_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const BatchDev bt = batch_dev(b);
    char* w = (char*)ws;
    hipLaunchKernelGGL(k_dct_det_b, dim3(xcd_grid(batch_items(b, kStDct))), dim3(b->thr_dct), b->lds_dct, st, bt, w,
                       (float* const*)nullptr, g_ptrs, 1);
    if ((rc = check_launch())) return rc;
    if (batch_items(b, kStSynAdj) > 0) {
        hipLaunchKernelGGL(k_syn_dense_adj_b, dim3(xcd_grid(batch_items(b, kStSynAdj))), dim3(kSynThreads), 0, st,
                           bt, w);
        if ((rc = check_launch())) return rc;
    }
    hipLaunchKernelGGL(k_ring_adj_b, dim3(xcd_grid(batch_items(b, kStRing))), dim3(b->thr_ring), b->lds_ring, st,
                       bt, w);
    if ((rc = check_launch())) return rc;
    {
        const dim3 grid(xcd_grid(batch_items(b, kStSpread)));
        const size_t lds = spread_lds(b->spr_cb, 1);
        switch (b->spr_cb) {
            case 64: hipLaunchKernelGGL(k_spread_b<64>, grid, dim3(64), lds, st, bt, w); break;
            case 128: hipLaunchKernelGGL(k_spread_b<128>, grid, dim3(128), lds, st, bt, w); break;
            case 192: hipLaunchKernelGGL(k_spread_b<192>, grid, dim3(192), lds, st, bt, w); break;
            default: hipLaunchKernelGGL(k_spread_b<256>, grid, dim3(256), lds, st, bt, w); break;
        }
    }
    if ((rc = check_launch())) return rc;
    hipLaunchKernelGGL(k_rowpass_adj_b, dim3(xcd_grid(batch_items(b, kStRow))), dim3(b->thr_row), b->lds_row, st, bt,
                       w);
    if ((rc = check_launch())) return rc;
    hipLaunchKernelGGL(k_colpass_adj_b, dim3(xcd_grid(batch_items(b, kStCol))), dim3(b->thr_col), b->lds_col, st, bt,
                       w, f_ptrs);
    return check_launch();
}
