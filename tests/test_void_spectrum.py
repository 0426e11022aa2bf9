"""Why the 1e-8 void cells stall: the spectrum of the linear part F_u of the
Lippmann-Schwinger map (Algorithm 1; Sec. 3) on compatible fields, computed
without the oracle from the explicit compatible basis (tests/closed_forms.py).
With equal Poisson ratios and the reference medium at the matrix modulus,
F_u = I - G0^-1 K on compatible fields (K, G0 the Galerkin stiffness of the cell
and of C0), so its eigenvalues are 1 - mu with mu the generalized eigenvalues
of (K, G0), which lie in [E_void/E0, 1].  The eigenvalues within 1e-4 of 1 that
carry part of the initial error are the modes a fixed point cannot damp and RPM
must hold in its basis; their number grows quickly with the resolution of a
single void (every staircase surface voxel adds some), so a basis of 32 columns
cannot reach 1e-6 on cells with hundreds of voids."""
import numpy as np
import pytest
import scipy.linalg as sl

import closed_forms as CF


def one_void(n, r_frac=0.3):
    z, y, x = np.meshgrid(*(np.arange(n) + 0.5,) * 3, indexing="ij")
    c = n / 2
    return (((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2) < (r_frac * n) ** 2).astype(np.uint8)


def spectrum(n):
    ph = one_void(n)
    V = CF.compatible_basis(ph.shape)
    lt = [CF.lame(1.0, 0.3), CF.lame(1e-8, 0.3)]
    K = V.T @ CF._apply_C(ph, lt, V)
    G0 = V.T @ CF._apply_C(np.zeros_like(ph), [CF.lame(1.0, 0.3)], V)
    mu, X = sl.eigh(K, G0)
    # the initial error E - eps* in the basis, its weight in each mode of the
    # weak residual
    E = np.array([0, 0, 0.01, 0, 0, 0.0])
    Em = np.repeat(E * CF.MANDEL_W, ph.size)
    a = np.linalg.solve(K, -(V.T @ CF._apply_C(ph, lt, Em[:, None]))[:, 0])
    c = X.T @ (G0 @ (-a))
    return 1.0 - mu, (c * mu) ** 2


@pytest.mark.slow
def test_slow_modes_of_a_void_multiply_with_resolution():
    lam8, w8 = spectrum(8)
    lam12, w12 = spectrum(12)
    for lam in (lam8, lam12):
        assert lam.min() > -1e-9 and lam.max() < 1.0  # [0, 1 - E_void/E0]
    live8 = np.sum((lam8 > 1 - 1e-4) & (w8 > 1e-24 * w8.sum()))
    live12 = np.sum((lam12 > 1 - 1e-4) & (w12 > 1e-24 * w12.sum()))
    assert live8 <= 4 and live12 >= 10 * max(live8, 1), (live8, live12)

    # even a deflation that removed the 32 slowest carrying modes exactly would
    # leave the weak residual above 1e-6 of its start after 1e4 fixed-point steps
    live = w12 > 1e-24 * w12.sum()
    order = np.argsort(-lam12 * live)
    keep = order[32:]
    r = np.sqrt(np.sum(w12[keep] * lam12[keep] ** 20000)) / np.sqrt(w12.sum())
    assert r > 1e-6, r
