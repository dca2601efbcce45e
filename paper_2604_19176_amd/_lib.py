"""ctypes binding of libpat.so (include/pat.h).  Argument marshalling only.

Every function here has the name of the C entry point it calls.  The library
is the in-tree build (paper_2604_19176_amd/libpat.so); if it is missing the
import fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpat.so")
HEADER = os.path.join(HERE, "..", "include", "pat.h")

PAT_OK = 0
PAT_ERR_ARG = -1
PAT_ERR_UNSUPPORTED = -2
PAT_ERR_WORKSPACE = -3
PAT_ERR_HIP = -4
PAT_ERR_ALLOC = -5
# device bytes of the workspace array pat_forward_noalloc uses (include/pat.h)
PAT_NOALLOC_SCRATCH_BYTES = 128 * 1024 * 1024


class PatError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s failed: %s (%d)" % (where, pat_status_string(status), status))


class pat_plan_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("support_r", ctypes.c_double), ("det_r", ctypes.c_double),
                ("n_det", ctypes.c_int), ("arc_center", ctypes.c_double), ("arc_span", ctypes.c_double),
                ("n_t", ctypes.c_int), ("dt", ctypes.c_double), ("c", ctypes.c_double),
                ("lambda_oversample", ctypes.c_double), ("em_correction", ctypes.c_int),
                ("max_batch", ctypes.c_int), ("det_theta", ctypes.POINTER(ctypes.c_double))]


class pat_plan_info(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("dlam", ctypes.c_double), ("n_lam", ctypes.c_int),
                ("K", ctypes.c_int), ("n_psi", ctypes.c_int), ("kappa", ctypes.c_double),
                ("n_grid", ctypes.c_int), ("n_points", ctypes.c_int), ("len_czt", ctypes.c_int),
                ("syn_stride", ctypes.c_int), ("syn_dense", ctypes.c_int), ("n_ring_modes", ctypes.c_int),
                ("workspace_per_instance", ctypes.c_size_t), ("table_bytes", ctypes.c_size_t)]


class pat_launch(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in ("col_np", "row_rpb", "ring_rt", "dct_dp", "gat_cb", "gat_th",
                                             "spr_cb", "spr_th", "gat_ib", "spr_ib")]

    def asdict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


_lib = None


def load():
    """Load libpat.so once; raise ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libpat.so not built at %s; run __graft_entry__.build() or "
                          "python paper_2604_19176_amd/build.py" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, ci, cf, cl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_float, ctypes.c_long
    P = ctypes.POINTER
    sig = {
        "pat_plan_create": (ci, [P(pat_plan_desc), P(vp)]),
        "pat_plan_query": (ci, [vp, P(pat_plan_info)]),
        "pat_plan_destroy": (None, [vp]),
        "pat_workspace_size": (sz, [vp, ci]),
        "pat_forward": (ci, [vp, vp, vp, ci, vp, sz, vp]),
        "pat_adjoint": (ci, [vp, vp, vp, ci, vp, sz, vp]),
        "pat_forward_noalloc": (ci, [vp, vp, vp, ci, vp]),
        "pat_tv_grad": (ci, [vp, vp, vp, ci, ci, cf, vp]),
        "pat_pgd_update": (ci, [vp, vp, vp, cl, cf, cf, vp]),
        "pat_residual": (ci, [vp, vp, vp, cl, ci, vp]),
        "pat_profile_enable": (ci, [vp, ci]),
        "pat_stream_copy": (ci, [vp, vp, sz, vp, vp]),
        "pat_profile_read": (ci, [vp, ci, P(ctypes.c_float), ci, P(ci)]),
        "pat_plan_derive": (ci, [P(pat_plan_desc), P(pat_plan_info)]),
        "pat_bessel_jn_table": (ci, [ci, ctypes.c_double, P(ctypes.c_double)]),
        "pat_status_string": (ctypes.c_char_p, [ci]),
        "pat_plan_get_launch": (ci, [vp, P(pat_launch)]),
        "pat_plan_set_launch": (ci, [vp, P(pat_launch)]),
        "pat_plan_set_split": (ci, [vp, ci]),
        "pat_plan_get_split": (ci, [vp, P(ci)]),
        "pat_batch_create": (ci, [P(vp), ci, P(vp)]),
        "pat_batch_destroy": (None, [vp]),
        "pat_batch_workspace_size": (sz, [vp]),
        "pat_batch_forward": (ci, [vp, vp, vp, vp, sz, vp]),
        "pat_batch_adjoint": (ci, [vp, vp, vp, vp, sz, vp]),
        "pat_batch_get_launch": (ci, [vp, P(pat_launch)]),
        "pat_batch_set_launch": (ci, [vp, P(pat_launch)]),
        "pat_autotune_plan": (ci, [vp, ci, ctypes.c_char_p]),
        "pat_autotune_batch": (ci, [vp, ctypes.c_char_p]),
        "pat_pd_dual_data": (ci, [vp, vp, vp, cl, cf, vp]),
        "pat_pd_dual_tv": (ci, [vp, vp, ci, ci, cf, cf, vp]),
        "pat_pd_primal": (ci, [vp, vp, vp, vp, ci, ci, cf, vp]),
        "pat_pd_change": (ci, [vp, vp, vp, ci, ci, vp]),
        "pat_cg_norm2": (ci, [vp, vp, cl, ci, vp]),
        "pat_cg_step_fr": (ci, [vp, vp, cl, vp, vp, cl, vp, vp, ci, vp]),
        "pat_cg_step_p": (ci, [vp, vp, cl, vp, vp, ci, vp]),
        "pat_sim_create": (ci, [P(pat_plan_desc), P(vp)]),
        "pat_sim_query": (ci, [vp, P(ci), P(sz)]),
        "pat_sim_run": (ci, [vp, vp, vp, vp, sz, vp]),
        "pat_sim_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def declared_functions():
    """Names of the functions include/pat.h declares (for the export test)."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pat_[a-z0-9_]+)\s*\(", text)))


def _check(rc, where):
    if rc != PAT_OK:
        raise PatError(rc, where)


# -- thin wrappers with the C names -------------------------------------------

def pat_status_string(status: int) -> str:
    return load().pat_status_string(int(status)).decode()


def pat_plan_derive(desc: pat_plan_desc) -> pat_plan_info:
    info = pat_plan_info()
    _check(load().pat_plan_derive(ctypes.byref(desc), ctypes.byref(info)), "pat_plan_derive")
    return info


def pat_bessel_jn_table(kmax: int, x: float):
    out = (ctypes.c_double * (kmax + 1))()
    _check(load().pat_bessel_jn_table(int(kmax), float(x), out), "pat_bessel_jn_table")
    return list(out)


def pat_plan_create(desc: pat_plan_desc) -> int:
    h = ctypes.c_void_p()
    _check(load().pat_plan_create(ctypes.byref(desc), ctypes.byref(h)), "pat_plan_create")
    return h.value


def pat_plan_query(plan: int) -> pat_plan_info:
    info = pat_plan_info()
    _check(load().pat_plan_query(plan, ctypes.byref(info)), "pat_plan_query")
    return info


def pat_plan_destroy(plan: int) -> None:
    load().pat_plan_destroy(plan)


def pat_workspace_size(plan: int, batch: int) -> int:
    return int(load().pat_workspace_size(plan, int(batch)))


def pat_forward(plan, f_ptr, g_ptr, batch, ws_ptr, ws_bytes, stream) -> None:
    _check(load().pat_forward(plan, f_ptr, g_ptr, int(batch), ws_ptr, int(ws_bytes), stream), "pat_forward")


def pat_forward_noalloc(plan, f_ptr, g_ptr, batch, stream) -> None:
    _check(load().pat_forward_noalloc(plan, f_ptr, g_ptr, int(batch), stream), "pat_forward_noalloc")


def pat_stream_copy(src_ptr, dst_ptr, nbytes, perm_ptr, stream) -> None:
    _check(load().pat_stream_copy(src_ptr, dst_ptr, int(nbytes), perm_ptr, stream), "pat_stream_copy")


def pat_adjoint(plan, g_ptr, f_ptr, batch, ws_ptr, ws_bytes, stream) -> None:
    _check(load().pat_adjoint(plan, g_ptr, f_ptr, int(batch), ws_ptr, int(ws_bytes), stream), "pat_adjoint")


def pat_profile_enable(plan, enable: bool) -> None:
    _check(load().pat_profile_enable(plan, 1 if enable else 0), "pat_profile_enable")


def pat_profile_read(plan, which: int):
    ms = (ctypes.c_float * 8)()
    cnt = ctypes.c_int()
    _check(load().pat_profile_read(plan, int(which), ms, 8, ctypes.byref(cnt)), "pat_profile_read")
    return [float(ms[i]) for i in range(cnt.value)]


def pat_tv_grad(f_ptr, grad_ptr, tv_ptr, n, batch, eps, stream) -> None:
    _check(load().pat_tv_grad(f_ptr, grad_ptr, tv_ptr, int(n), int(batch), float(eps), stream), "pat_tv_grad")


def pat_pgd_update(f_ptr, adj_ptr, tvg_ptr, count, tau, lam, stream) -> None:
    _check(load().pat_pgd_update(f_ptr, adj_ptr, tvg_ptr, int(count), float(tau), float(lam), stream),
           "pat_pgd_update")


def pat_residual(g_ptr, gm_ptr, sq_ptr, count_per, batch, stream) -> None:
    _check(load().pat_residual(g_ptr, gm_ptr, sq_ptr, int(count_per), int(batch), stream), "pat_residual")


def pat_plan_get_launch(plan) -> pat_launch:
    c = pat_launch()
    _check(load().pat_plan_get_launch(plan, ctypes.byref(c)), "pat_plan_get_launch")
    return c


def pat_plan_set_launch(plan, cfg: pat_launch) -> None:
    _check(load().pat_plan_set_launch(plan, ctypes.byref(cfg)), "pat_plan_set_launch")


def pat_plan_set_split(plan, min_batch: int) -> None:
    _check(load().pat_plan_set_split(plan, int(min_batch)), "pat_plan_set_split")


def pat_plan_get_split(plan) -> int:
    v = ctypes.c_int()
    _check(load().pat_plan_get_split(plan, ctypes.byref(v)), "pat_plan_get_split")
    return v.value


def pat_batch_create(plans) -> int:
    arr = (ctypes.c_void_p * len(plans))(*plans)
    h = ctypes.c_void_p()
    _check(load().pat_batch_create(arr, len(plans), ctypes.byref(h)), "pat_batch_create")
    return h.value


def pat_batch_destroy(batch) -> None:
    load().pat_batch_destroy(batch)


def pat_batch_workspace_size(batch) -> int:
    return int(load().pat_batch_workspace_size(batch))


def pat_batch_forward(batch, f_ptrs, g_ptrs, ws_ptr, ws_bytes, stream) -> None:
    _check(load().pat_batch_forward(batch, f_ptrs, g_ptrs, ws_ptr, int(ws_bytes), stream), "pat_batch_forward")


def pat_batch_adjoint(batch, g_ptrs, f_ptrs, ws_ptr, ws_bytes, stream) -> None:
    _check(load().pat_batch_adjoint(batch, g_ptrs, f_ptrs, ws_ptr, int(ws_bytes), stream), "pat_batch_adjoint")


def pat_batch_get_launch(batch) -> pat_launch:
    c = pat_launch()
    _check(load().pat_batch_get_launch(batch, ctypes.byref(c)), "pat_batch_get_launch")
    return c


def pat_batch_set_launch(batch, cfg: pat_launch) -> None:
    _check(load().pat_batch_set_launch(batch, ctypes.byref(cfg)), "pat_batch_set_launch")


def pat_autotune_plan(plan, batch: int, cache_path) -> None:
    cp = None if cache_path is None else os.fsencode(cache_path)
    _check(load().pat_autotune_plan(plan, int(batch), cp), "pat_autotune_plan")


def pat_autotune_batch(batch, cache_path) -> None:
    cp = None if cache_path is None else os.fsencode(cache_path)
    _check(load().pat_autotune_batch(batch, cp), "pat_autotune_batch")


def pat_pd_dual_data(y1_ptr, ax_ptr, g_ptr, count, sigma, stream) -> None:
    _check(load().pat_pd_dual_data(y1_ptr, ax_ptr, g_ptr, int(count), float(sigma), stream), "pat_pd_dual_data")


def pat_pd_dual_tv(y2_ptr, xbar_ptr, n, batch, sigma, alpha, stream) -> None:
    _check(load().pat_pd_dual_tv(y2_ptr, xbar_ptr, int(n), int(batch), float(sigma), float(alpha), stream),
           "pat_pd_dual_tv")


def pat_pd_primal(f_ptr, xbar_ptr, aty_ptr, y2_ptr, n, batch, tau, stream) -> None:
    _check(load().pat_pd_primal(f_ptr, xbar_ptr, aty_ptr, y2_ptr, int(n), int(batch), float(tau), stream),
           "pat_pd_primal")


def pat_pd_change(f_ptr, xbar_ptr, out_ptr, n, batch, stream) -> None:
    _check(load().pat_pd_change(f_ptr, xbar_ptr, out_ptr, int(n), int(batch), stream), "pat_pd_change")


def pat_cg_norm2(x_ptr, out_ptr, count, batch, stream) -> None:
    _check(load().pat_cg_norm2(x_ptr, out_ptr, int(count), int(batch), stream), "pat_cg_norm2")


def pat_cg_step_fr(f_ptr, p_ptr, nf, r_ptr, q_ptr, nr, gamma_ptr, qq_ptr, batch, stream) -> None:
    _check(load().pat_cg_step_fr(f_ptr, p_ptr, int(nf), r_ptr, q_ptr, int(nr), gamma_ptr, qq_ptr, int(batch),
                                 stream), "pat_cg_step_fr")


def pat_cg_step_p(p_ptr, s_ptr, n, gnew_ptr, gamma_ptr, batch, stream) -> None:
    _check(load().pat_cg_step_p(p_ptr, s_ptr, int(n), gnew_ptr, gamma_ptr, int(batch), stream), "pat_cg_step_p")


def pat_sim_create(desc: pat_plan_desc) -> int:
    h = ctypes.c_void_p()
    _check(load().pat_sim_create(ctypes.byref(desc), ctypes.byref(h)), "pat_sim_create")
    return h.value


def pat_sim_query(sim: int):
    m, ws = ctypes.c_int(), ctypes.c_size_t()
    _check(load().pat_sim_query(sim, ctypes.byref(m), ctypes.byref(ws)), "pat_sim_query")
    return m.value, ws.value


def pat_sim_run(sim, f_ptr, g_ptr, ws_ptr, ws_bytes, stream) -> None:
    _check(load().pat_sim_run(sim, f_ptr, g_ptr, ws_ptr, int(ws_bytes), stream), "pat_sim_run")


def pat_sim_destroy(sim: int) -> None:
    load().pat_sim_destroy(sim)
