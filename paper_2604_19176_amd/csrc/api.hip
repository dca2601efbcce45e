// api.hip -- C-ABI entry points: argument checks on the host, then stream-ordered launches.
//
// The kernels live in kernels.hip, compiled into this translation unit so the
// launches need no relocatable device code.
#include "../../include/pat.h"
#include "kernels.hip"

#include <algorithm>



using namespace pat;

static int check_launch()
{
    return hipGetLastError() == hipSuccess ? PAT_OK : PAT_ERR_HIP;
}

static int validate(const pat_plan* p, const void* in, const void* out, int batch, const void* ws,
                    size_t ws_bytes)
{
    if (!p || !in || !out) return PAT_ERR_ARG;
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
    // column pass
    {
        dim3 grid(p->n_col_tiles, batch);
        hipLaunchKernelGGL(k_colpass_fwd, grid, dim3(p->thr_col), sizeof(float2) * c.col_np * d.Ng, st, d, p->ws,
                           f, wsp, c.col_np);
        if ((rc = check_launch())) return rc;
    }
    {
        dim3 grid((d.Hy + c.row_rpb - 1) / c.row_rpb, batch);
        hipLaunchKernelGGL(k_rowpass_fwd, grid, dim3(p->thr_row), sizeof(float2) * c.row_rpb * d.Ng, st, d, p->ws,
                           wsp, c.row_rpb);
        if ((rc = check_launch())) return rc;
    }
    {
        dim3 grid(d.nlam, batch);
        hipLaunchKernelGGL(k_ring_fwd, grid, dim3(p->thr_ring), sizeof(float2) * p->n_psi_max, st, d, p->ws, wsp);
        if ((rc = check_launch())) return rc;
    }
    {
        dim3 grid((d.Kp + c.dct_mt - 1) / c.dct_mt, batch);
        hipLaunchKernelGGL(k_dct, grid, dim3(p->thr_dct), sizeof(float2) * c.dct_mt * 2 * d.M, st, d, p->ws, wsp,
                           c.dct_mt, 0);
        if ((rc = check_launch())) return rc;
    }
    {
        dim3 grid(p->n_time_tiles, batch);
        size_t lds = sizeof(float2) * c.czt_par * d.L + sizeof(float) * d.D * c.czt_tt;
        hipLaunchKernelGGL(k_czt_fwd, grid, dim3(p->thr_czt), lds, st, d, p->ws, wsp, g, c.czt_tt, c.czt_par,
                           p->n_col_tiles);
        if ((rc = check_launch())) return rc;
    }
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
    {
        dim3 grid(p->n_time_tiles, batch);
        size_t lds = sizeof(float2) * c.czt_par * d.L + sizeof(float) * d.D * c.czt_tt;
        hipLaunchKernelGGL(k_czt_adj, grid, dim3(p->thr_czt), lds, st, d, p->ws, wsp, g, c.czt_tt, c.czt_par);
        if ((rc = check_launch())) return rc;
    }
    {
        dim3 grid((d.Kp + c.dct_mt - 1) / c.dct_mt, batch);
        hipLaunchKernelGGL(k_dct, grid, dim3(p->thr_dct), sizeof(float2) * c.dct_mt * 2 * d.M, st, d, p->ws, wsp,
                           c.dct_mt, 1);
        if ((rc = check_launch())) return rc;
    }
    {
        dim3 grid(d.nlam, batch);
        hipLaunchKernelGGL(k_ring_adj, grid, dim3(p->thr_ring), sizeof(float2) * p->n_psi_max, st, d, p->ws, wsp);
        if ((rc = check_launch())) return rc;
    }
    {
        dim3 grid((d.Ng + c.spr_cb - 1) / c.spr_cb, (d.Hy + c.spr_th - 1) / c.spr_th, batch);
        size_t lds = sizeof(float) * 19 * c.spr_cap;
        hipLaunchKernelGGL(k_spread, grid, dim3(c.spr_cb), lds, st, d, p->ws, wsp, c.spr_th, c.spr_cap);
        if ((rc = check_launch())) return rc;
    }
    {
        dim3 grid((d.Hy + c.row_rpb - 1) / c.row_rpb, batch);
        hipLaunchKernelGGL(k_rowpass_adj, grid, dim3(p->thr_row), sizeof(float2) * c.row_rpb * d.Ng, st, d, p->ws,
                           wsp, c.row_rpb);
        if ((rc = check_launch())) return rc;
    }
    {
        dim3 grid(p->n_col_tiles, batch);
        hipLaunchKernelGGL(k_colpass_adj, grid, dim3(p->thr_col), sizeof(float2) * c.col_np * d.Ng, st, d, p->ws,
                           wsp, f, c.col_np, p->n_time_tiles);
        if ((rc = check_launch())) return rc;
    }
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
