"""The polarization iteration (Algorithm 3 / Sec. 5.5; Accelerated FFT for
alpha = beta = 2) and RPM around it: the HIP path through the C ABI against the
FP64 oracle.  Bars as for the Lippmann-Schwinger map: FP64 map applications
within 1e-12 and solves within 1e-10 relative; FP32 map applications within
3e-5 of the field scale; the oracle's growth decisions are replayed."""
import numpy as np
import pytest

import oracle as O
from paper_2003_07720_amd import microstructure as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch

    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2003_07720_amd import binding

    return binding


def dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    return t.to(dtype) if dtype is not None else t


PHASES = [(1.0, 0.3), (40.0, 0.25), (0.5, 0.4)]
E6 = np.array([0.01, -0.004, 0.002, 0.003, -0.002, 0.005])
GRIDS = [(1, 32, 32), (1, 6, 8), (4, 6, 8), (9, 3, 6), (3, 9, 27), (12, 16, 6), (1, 16, 128), (128, 4, 6),
         (6, 4, 128), (16, 128, 6)]


def _gl(B, phases):
    return np.array([B.lame_from_young(*p) for p in phases])


@pytest.mark.parametrize("shape", GRIDS, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ab", [(2.0, 2.0), (1.5, 1.0)], ids=["accelerated", "a1.5b1"])
def test_polarization_map_parity(B, shape, prec, ab):
    import torch

    print(f"polarization map parity {shape} {prec} {ab}", flush=True)
    ph = M.random_phases(shape, 3, seed=3 + sum(shape))
    eps = M.random_field(shape, seed=11 + sum(shape), scale=0.01)
    E = E6.copy()
    if shape[0] == 1:
        E[2] = E[3] = E[4] = 0.0
    l0 = O.lame(np.sqrt(0.5 * 40.0), 0.3)
    ref, ref_err, ref_sav, _ = O.fmap(ph, O.lame_table(PHASES), l0, E, eps, map="polarization", alpha=ab[0],
                                      beta=ab[1])
    dt = torch.float64 if prec == "fp64" else torch.float32
    opts = B.make_options(precision=prec, scheme="basic", map="polarization", alpha=ab[0], beta=ab[1])
    xi, err, sav = B.fft_apply(dev(ph), _gl(B, PHASES), B.lame_from_young(np.sqrt(20.0), 0.3), E, dev(eps, dt),
                               opts)
    xi = xi.double().cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 3e-5
    assert np.abs(xi - ref).max() <= tol * np.abs(ref).max()
    assert abs(err - ref_err) <= (1e-11 if prec == "fp64" else 3e-4) * ref_err


def test_polarization_homogeneous_one_step(B):
    ph = np.zeros((4, 6, 8), np.uint8)
    E = E6.copy()
    eps0 = M.random_field(ph.shape, seed=3, scale=0.01) + E[:, None, None, None]
    lt = _gl(B, [(3.0, 0.3)])
    g = B.fft_solve(dev(ph), lt, B.lame_from_young(3.0, 0.3), E,
                    B.make_options(scheme="basic", map="polarization", tol=1e-12), eps0=dev(eps0))
    assert g["status"] == "RPM_OK" and g["iterations"] == 2
    np.testing.assert_allclose(g["eps"].cpu().numpy(), np.broadcast_to(E[:, None, None, None], eps0.shape),
                               rtol=0, atol=1e-16)


def _case():
    shape = (6, 8, 12)
    ph = M.random_phases(shape, 3, seed=21)
    return ph, np.sqrt(0.5 * 40.0)


@pytest.mark.parametrize("scheme", ["basic", "rpm"])
def test_polarization_solve_parity_fp64(B, scheme):
    """Contrast 80 with the reference at the geometric mean of the extreme moduli, where the
    Lippmann-Schwinger map with the same reference diverges."""
    ph, e0 = _case()
    kw = dict(scheme=scheme, tol=1e-10, max_iter=3000, n_max=6, p_max=16)
    ref = O.solve(ph, O.lame_table(PHASES), O.lame(e0, 0.3), E6, map="polarization", **kw)
    assert ref["status"] == "converged"
    g = B.fft_solve(dev(ph), _gl(B, PHASES), B.lame_from_young(e0, 0.3), E6,
                    B.make_options(map="polarization", replay=list(ref["decisions"]), **kw))
    assert g["status"] == "RPM_OK"
    assert g["iterations"] == ref["iterations"] and g["basis_dim"] == ref["p"]
    eps = g["eps"].cpu().numpy()
    assert np.abs(eps - ref["eps"]).max() <= 1e-10 * np.abs(ref["eps"]).max()
    np.testing.assert_allclose(g["history"], ref["history"], rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(g["sig_avg"], ref["sig_avg"], rtol=0, atol=1e-10 * np.abs(ref["sig_avg"]).max())
    cl = B.fft_solve(dev(ph), _gl(B, PHASES), B.lame_from_young(e0, 0.3), E6,
                     B.make_options(scheme="basic", tol=1e-10, max_iter=400))
    assert cl["status"] == "RPM_DIVERGED"


def test_polarization_rpm_disk32_fp64(B):
    w = M.workload_disk32()
    lt = O.lame_table(w["phases"])
    e0 = np.sqrt(1.0 * 10.0)
    kw = dict(scheme="rpm", tol=1e-10, max_iter=3000, n_max=10, p_max=32)
    ref = O.solve(w["phase"], lt, O.lame(e0, 0.3), w["E"], map="polarization", **kw)
    assert ref["status"] == "converged"
    g = B.fft_solve(dev(w["phase"]), _gl(B, w["phases"]), B.lame_from_young(e0, 0.3), w["E"],
                    B.make_options(map="polarization", replay=list(ref["decisions"]), **kw))
    assert g["status"] == "RPM_OK" and g["iterations"] == ref["iterations"]
    eps = g["eps"].cpu().numpy()
    assert np.abs(eps - ref["eps"]).max() <= 1e-10 * np.abs(ref["eps"]).max()


def test_polarization_fp32_refined(B):
    """FP32 fields with FP64 certification and refinement reach an FP64-verified 1e-10."""
    ph, e0 = _case()
    ref = O.solve(ph, O.lame_table(PHASES), O.lame(e0, 0.3), E6, scheme="rpm", tol=1e-11, max_iter=3000,
                  n_max=6, p_max=16, map="polarization")
    g = B.fft_solve(dev(ph), _gl(B, PHASES), B.lame_from_young(e0, 0.3), E6,
                    B.make_options(precision="fp32", scheme="rpm", tol=1e-10, max_iter=3000, n_max=6, p_max=16,
                                   map="polarization", refine=6))
    assert g["status"] == "RPM_OK" and g["residual_fp64"] <= 1e-10
    eps = g["eps"].double().cpu().numpy()
    assert np.abs(eps - ref["eps"]).max() <= 1e-6 * np.abs(ref["eps"]).max()
