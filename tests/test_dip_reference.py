"""Pin of the FP64 deep-image-prior objective (oracle/dip.py), CPU only:
its gradient equals central finite differences of the objective (FP64, at
pixels inside and outside the support, with and without TV), which fixes the
factor 2, the sign and the transpose of the data term."""
import numpy as np

from pat_inputs import config_geometry, make_phantom


def test_dip_gradient_equals_finite_differences(oracle_mod):
    from oracle import dip
    geom = config_geometry("gradcheck")
    rng = np.random.default_rng(5)
    f = make_phantom(geom.n, 3, 1, 0, 6) + 0.05 * rng.random((geom.n, geom.n))
    g = dip.forward(geom, make_phantom(geom.n, 4, 1, 1, 7))
    for lam in (0.0, 0.3):
        grad = dip.gradient(geom, f, g, lam, 1e-2)
        for (i, j) in [(16, 16), (3, 20), (0, 0), (31, 7)]:
            h = 1e-5
            fp, fm = f.copy(), f.copy()
            fp[i, j] += h
            fm[i, j] -= h
            fd = (dip.objective(geom, fp, g, lam, 1e-2) - dip.objective(geom, fm, g, lam, 1e-2)) / (2 * h)
            assert abs(fd - grad[i, j]) <= 1e-6 * max(1.0, abs(fd)), (lam, i, j, fd, grad[i, j])
