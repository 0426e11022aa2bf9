"""FP32 fields with FP64 RPM steps: certification of the converged field in FP64
and iterative refinement (correction solves d = F_u d + g in FP32, g the FP64
fixed-point residual) against the FP64 oracle."""
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


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_fp32_refined_reaches_fp64_tolerance_disk32(B):
    w = M.workload_disk32()
    ref = O.solve(w["phase"], O.lame_table(w["phases"]), O.lame(*w["ref"]), w["E"], scheme="rpm", tol=1e-11,
                  max_iter=3000)
    lt = np.array([B.lame_from_young(*p) for p in w["phases"]])
    l0 = B.lame_from_young(*w["ref"])
    g = B.fft_solve(dev(w["phase"]), lt, l0, w["E"],
                    B.make_options(precision="fp32", tol=1e-10, max_iter=3000, refine=6))
    assert g["status"] == "RPM_OK"
    assert g["refinements"] >= 1 and g["residual_fp64"] <= 1e-10
    eps = g["eps"].double().cpu().numpy()
    # the refined FP64 field rounded to float: within a few float ulps of the oracle
    assert np.abs(eps - ref["eps"]).max() <= 1e-6 * np.abs(ref["eps"]).max()
    # an equilibrium error of 1e-10 leaves <sigma> accurate to ~1e-9 relative
    np.testing.assert_allclose(g["sig_avg"], ref["sig_avg"], rtol=0, atol=1e-8 * np.abs(ref["sig_avg"]).max())


def test_fp32_certify_only(B):
    w = M.workload_disk32()
    lt = np.array([B.lame_from_young(*p) for p in w["phases"]])
    g = B.fft_solve(dev(w["phase"]), lt, B.lame_from_young(*w["ref"]), w["E"],
                    B.make_options(precision="fp32", tol=1e-6, refine=0))
    assert g["status"] == "RPM_OK" and g["refinements"] == 0
    # the FP64 evaluation of the FP32 solution agrees with the FP32 error to float accuracy
    assert abs(g["residual_fp64"] - g["residual"]) <= 1e-6 + 0.1 * g["residual"]


def test_fp32_refined_effective_tensor_3d(B):
    """The FP32-refined 6x6 effective stiffness within 1e-6 of the FP64 oracle."""
    ph, info = M.rsa_spheres(16, 2.0, 3.0, 0.1, seed=9)
    phases = [(1.0, 0.3), (20.0, 0.3)]
    l0 = (10.5, 0.3)
    kw = dict(scheme="rpm", tol=1e-10, max_iter=3000, n_max=10, p_max=32)
    Cref, _ = O.effective_tensor(ph, O.lame_table(phases), O.lame(*l0), **kw)
    lt = np.array([B.lame_from_young(*p) for p in phases])
    C, stats, st = B.effective_tensor(dev(ph), lt, B.lame_from_young(*l0),
                                      B.make_options(precision="fp32", refine=6, **kw))
    assert st == "RPM_OK"
    assert all(s["residual_fp64"] <= 1e-10 for s in stats)
    assert np.abs(C - Cref).max() <= 1e-6 * np.abs(Cref).max()
