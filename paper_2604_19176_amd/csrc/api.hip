// api.hip -- C-ABI entry points: argument checks on the host, then stream-ordered launches.
//
// The kernels live in kernels.hip, compiled into this translation unit so the
// launches need no relocatable device code.
#include "../../include/pat.h"
#include "kernels.hip"

#include <algorithm>



using namespace pat;

static size_t twb(int n) { return sizeof(float2) * (size_t)tw_lds_slots(n); }

static unsigned xcd_grid(int items) { return (unsigned)(((items + kXcds - 1) / kXcds) * kXcds); }

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

extern "C" int pat_forward(const pat_plan* p, const float* f, float* g, int batch, void* ws, size_t ws_bytes,
                           void* stream)
{
    int rc = validate(p, f, g, batch, ws, ws_bytes);
    if (rc != PAT_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const PlanDev& d = p->dev;
    const LaunchCfg& c = p->cfg;
    const InstPtrs wsp{(char*)ws, p->ws.bytes};
    prof_mark(p, 0, 0, st);
    hipLaunchKernelGGL(k_colpass_fwd, dim3(p->n_col_tiles, batch), dim3(p->thr_col), sizeof(float2) * c.col_np * d.Ng + twb(d.Ng),
                       st, d, p->ws, f, wsp, c.col_np);
    if ((rc = check_launch())) return rc;
    prof_mark(p, 0, 1, st);
    hipLaunchKernelGGL(k_rowpass_fwd, dim3((d.Hy + c.row_rpb - 1) / c.row_rpb, batch), dim3(p->thr_row),
                       sizeof(float2) * c.row_rpb * d.Ng + twb(d.Ng), st, d, p->ws, wsp, c.row_rpb);
    if ((rc = check_launch())) return rc;
    prof_mark(p, 0, 2, st);
    {
        int cb = c.gat_cb, th = c.gat_th;
        const long wide = (long)((d.Ng + 255) / 256) * ((d.NB + 31) / 32) * batch;
        if (wide >= 512) { cb = 256; th = 32; }
        const int items = ((d.Ng + cb - 1) / cb) * ((d.NB + th - 1) / th) * batch;
        hipLaunchKernelGGL(k_gather, dim3(xcd_grid(items)), dim3(cb), sizeof(float2) * 8 * (cb + 7), st, d, p->ws, wsp,
                           th, batch);
    }
    if ((rc = check_launch())) return rc;
    prof_mark(p, 0, 3, st);
    {
        const dim3 grid(xcd_grid((d.nlam + c.ring_rt - 1) / c.ring_rt * batch)), blk(p->thr_ring);
        hipLaunchKernelGGL(k_ring_fwd<4>, grid, blk, p->lds_ring, st, d, p->ws, wsp, c.ring_rt, batch);
    }
    if ((rc = check_launch())) return rc;
    prof_mark(p, 0, 4, st);
    hipLaunchKernelGGL(k_dct_det, dim3(xcd_grid(p->n_pair_tiles * batch)), dim3(p->thr_dct),
                       sizeof(float2) * c.dct_dp * 2 * d.M + twb(2 * d.M), st, d, p->ws, wsp, g, (const float*)nullptr, c.dct_dp, 0,
                       p->n_col_tiles, batch);
    if ((rc = check_launch())) return rc;
    prof_mark(p, 0, 5, st);
    return PAT_OK;
}

extern "C" int pat_adjoint(const pat_plan* p, const float* g, float* f, int batch, void* ws, size_t ws_bytes,
                           void* stream)
{
    int rc = validate(p, g, f, batch, ws, ws_bytes);
    if (rc != PAT_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const PlanDev& d = p->dev;
    const LaunchCfg& c = p->cfg;
    const InstPtrs wsp{(char*)ws, p->ws.bytes};
    prof_mark(p, 1, 0, st);
    hipLaunchKernelGGL(k_dct_det, dim3(xcd_grid(p->n_pair_tiles * batch)), dim3(p->thr_dct),
                       sizeof(float2) * c.dct_dp * 2 * d.M + twb(2 * d.M), st, d, p->ws, wsp, (float*)nullptr, g, c.dct_dp, 1, 0,
                       batch);
    if ((rc = check_launch())) return rc;
    prof_mark(p, 1, 1, st);
    {
        const dim3 grid(xcd_grid((d.nlam + c.ring_rt - 1) / c.ring_rt * batch)), blk(p->thr_ring);
        hipLaunchKernelGGL(k_ring_adj<4>, grid, blk, p->lds_ring, st, d, p->ws, wsp, c.ring_rt, batch);
    }
    if ((rc = check_launch())) return rc;
    prof_mark(p, 1, 2, st);
    {
        // wide tiles amortise the per-band weight evaluation; narrow ones keep small batches parallel
        int cb = c.spr_cb, th = c.spr_th;
        const long wide = (long)((d.Ng + 255) / 256) * ((d.Hy + 15) / 16) * batch;
        if (wide >= 1024) { cb = 256; th = 16; }
        const int items = ((d.Ng + cb - 1) / cb) * ((d.Hy + th - 1) / th) * batch;
        hipLaunchKernelGGL(k_spread, dim3(xcd_grid(items)), dim3(cb), sizeof(float) * 19 * 2 * cb, st, d, p->ws, wsp,
                           th, 2 * cb, batch);
    }
    if ((rc = check_launch())) return rc;
    prof_mark(p, 1, 3, st);
    hipLaunchKernelGGL(k_rowpass_adj, dim3((d.Hy + c.row_rpb - 1) / c.row_rpb, batch), dim3(p->thr_row),
                       sizeof(float2) * c.row_rpb * d.Ng + twb(d.Ng), st, d, p->ws, wsp, c.row_rpb);
    if ((rc = check_launch())) return rc;
    prof_mark(p, 1, 4, st);
    hipLaunchKernelGGL(k_colpass_adj, dim3(p->n_col_tiles, batch), dim3(p->thr_col), sizeof(float2) * c.col_np * d.Ng + twb(d.Ng),
                       st, d, p->ws, wsp, f, c.col_np, p->n_pair_tiles);
    if ((rc = check_launch())) return rc;
    prof_mark(p, 1, 5, st);
    return PAT_OK;
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

extern "C" int pat_profile_enable(pat_plan* p, int enable)
{
    if (!p) return PAT_ERR_ARG;
    if (enable && !p->prof) {
        for (int dir = 0; dir < 2; ++dir)
            for (int q = 0; q < 8; ++q)
                if (hipEventCreate(&p->ev[dir][q]) != hipSuccess) return PAT_ERR_HIP;
        p->ev_count[0] = 6;  // 5 forward kernels
        p->ev_count[1] = 6;  // 5 adjoint kernels
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
