"""FP64 CPU oracle for the PAT operator pair (A, A*) -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the CPU-baseline leg of bench.py may import
this package.  It is a plain direct-sum implementation (pat_oracle.c) of the
discrete operator read from eq. (1)-(3) (Sec. 2.1) and Sec. 2.4.1; it shares
no code with the GPU library.  `reference` holds closed forms from physics and
special functions used to pin the oracle itself.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pat_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libpat_oracle.so")
_lib = None


def compile_source(src: str, out: str) -> str:
    """gcc (FP64, OpenMP) build of an oracle source file into a shared library."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-mavx2", "-mfma", "-fopenmp", "-fPIC", "-shared", "-std=c99",
           "-Wall", "-I", _HERE, "-o", tmp, src, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile pat_oracle.c into libpat_oracle.so (next to this file)."""
    if force or not os.path.exists(_LIB_PATH):
        compile_source(_SRC, _LIB_PATH)
    return _LIB_PATH


class _Geom(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("support_r", ctypes.c_double), ("det_r", ctypes.c_double),
                ("n_det", ctypes.c_int), ("arc_center", ctypes.c_double),
                ("arc_span", ctypes.c_double), ("n_t", ctypes.c_int), ("dt", ctypes.c_double),
                ("c", ctypes.c_double), ("lambda_oversample", ctypes.c_double),
                ("em_correction", ctypes.c_int), ("det_theta", ctypes.POINTER(ctypes.c_double))]


class _Sizes(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("dlam", ctypes.c_double), ("n_lam", ctypes.c_int),
                ("K", ctypes.c_int), ("n_psi", ctypes.c_int), ("kappa", ctypes.c_double)]


def _bind(lib):
    P = ctypes.POINTER
    dp = P(ctypes.c_double)
    lib.oracle_derive.argtypes = [P(_Geom), P(_Sizes)]
    lib.oracle_derive.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_get_threads.restype = ctypes.c_int
    lib.oracle_polar_spectrum.argtypes = [P(_Geom), dp, dp]
    lib.oracle_polar_to_data.argtypes = [P(_Geom), dp, ctypes.c_double, dp]
    lib.oracle_data_to_polar.argtypes = [P(_Geom), dp, dp]
    lib.oracle_polar_to_image.argtypes = [P(_Geom), dp, ctypes.c_double, dp]
    lib.oracle_forward.argtypes = [P(_Geom), dp, dp]
    lib.oracle_forward.restype = ctypes.c_int
    lib.oracle_adjoint.argtypes = [P(_Geom), dp, dp]
    lib.oracle_adjoint.restype = ctypes.c_int
    lib.oracle_adjoint_pixels.argtypes = [P(_Geom), dp, ctypes.c_int, P(ctypes.c_int), dp]
    lib.oracle_adjoint_pixels.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def use_library(path):
    """Point this wrapper at another build of pat_oracle.c (used by the
    mutation test, which compiles deliberately broken copies); returns the
    previous library handle so it can be restored with `restore_library`."""
    global _lib
    prev = _load()
    _lib = _bind(ctypes.CDLL(path))
    return prev


def restore_library(handle):
    global _lib
    _lib = handle


def _g(geom) -> _Geom:
    th = getattr(geom, "det_theta", None)
    g = _Geom(int(geom.n), float(geom.support_r), float(geom.det_r), int(geom.n_det),
              float(geom.arc_center), float(geom.arc_span), int(geom.n_t), float(geom.dt),
              float(geom.c), float(geom.lambda_oversample), int(geom.em_correction), None)
    if th is not None:
        arr = np.ascontiguousarray(th, dtype=np.float64)
        if arr.shape != (int(geom.n_det),):
            raise ValueError("det_theta needs n_det angles")
        g.det_theta = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        g._keep = arr  # the array outlives the call through the structure
    return g


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _arr(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (shape, a.shape))
    return a


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def sizes(geom) -> dict:
    s = _Sizes()
    if _load().oracle_derive(ctypes.byref(_g(geom)), ctypes.byref(s)) != 0:
        raise ValueError("invalid geometry")
    return dict(M=s.M, dlam=s.dlam, n_lam=s.n_lam, K=s.K, n_psi=s.n_psi, kappa=s.kappa)


def forward(geom, f) -> np.ndarray:
    """g = A f: f (N, N) float64 -> g (D, T) float64."""
    f = _arr(f, (geom.n, geom.n))
    out = np.empty((geom.n_det, geom.n_t))
    if _load().oracle_forward(ctypes.byref(_g(geom)), _dp(f), _dp(out)) != 0:
        raise ValueError("invalid geometry")
    return out


def adjoint(geom, g) -> np.ndarray:
    """f = A* g: g (D, T) float64 -> f (N, N) float64 (plain transpose)."""
    g = _arr(g, (geom.n_det, geom.n_t))
    out = np.empty((geom.n, geom.n))
    if _load().oracle_adjoint(ctypes.byref(_g(geom)), _dp(g), _dp(out)) != 0:
        raise ValueError("invalid geometry")
    return out


def adjoint_pixels(geom, g, flat_idx) -> np.ndarray:
    """A* g evaluated at the pixels with flat index i*N + j."""
    g = _arr(g, (geom.n_det, geom.n_t))
    idx = np.ascontiguousarray(flat_idx, dtype=np.int32)
    out = np.empty(idx.shape[0])
    rc = _load().oracle_adjoint_pixels(ctypes.byref(_g(geom)), _dp(g), int(idx.shape[0]),
                                       idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(out))
    if rc != 0:
        raise ValueError("invalid geometry")
    return out


def polar_spectrum(geom, f) -> np.ndarray:
    """Step 1 alone: F (n_lam, n_psi) complex128, row n-1 is lam_n = n dlam."""
    s = sizes(geom)
    f = _arr(f, (geom.n, geom.n))
    F = np.empty((s["n_lam"], s["n_psi"], 2))
    _load().oracle_polar_spectrum(ctypes.byref(_g(geom)), _dp(f), _dp(F))
    return F[..., 0] + 1j * F[..., 1]


def polar_to_data(geom, F, mass: float) -> np.ndarray:
    s = sizes(geom)
    Fr = np.ascontiguousarray(np.stack([F.real, F.imag], axis=-1), dtype=np.float64)
    assert Fr.shape == (s["n_lam"], s["n_psi"], 2)
    out = np.empty((geom.n_det, geom.n_t))
    _load().oracle_polar_to_data(ctypes.byref(_g(geom)), _dp(Fr), float(mass), _dp(out))
    return out


def data_to_polar(geom, g) -> np.ndarray:
    s = sizes(geom)
    g = _arr(g, (geom.n_det, geom.n_t))
    Ft = np.empty((s["n_lam"], s["n_psi"], 2))
    _load().oracle_data_to_polar(ctypes.byref(_g(geom)), _dp(g), _dp(Ft))
    return Ft[..., 0] + 1j * Ft[..., 1]


def polar_to_image(geom, Ft, data_sum: float) -> np.ndarray:
    s = sizes(geom)
    Fr = np.ascontiguousarray(np.stack([Ft.real, Ft.imag], axis=-1), dtype=np.float64)
    assert Fr.shape == (s["n_lam"], s["n_psi"], 2)
    out = np.empty((geom.n, geom.n))
    _load().oracle_polar_to_image(ctypes.byref(_g(geom)), _dp(Fr), float(data_sum), _dp(out))
    return out
