"""Load cases solved together (rpm_options.batch_cases): one pass over the
shared basis serves every unit load case of the effective tensor per step.
The converged fields are unique, so the batched C_eff must equal the oracle's
case-by-case C_eff to the solve tolerance, whatever basis each side grew."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2003_07720_amd import microstructure as M

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ceff_32cube.json")


@pytest.fixture(scope="module")
def B():
    import torch

    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2003_07720_amd import binding

    return binding


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("case", ["3d_16", "2d_disk32", "3d_ragged"])
def test_batched_effective_tensor_fp64_matches_oracle(B, case):
    if case == "3d_16":
        ph, _ = M.rsa_spheres(16, 2.0, 3.0, 0.1, seed=9)
        phases, ref = [(1.0, 0.3), (20.0, 0.3)], (10.5, 0.3)
    elif case == "2d_disk32":
        w = M.workload_disk32()
        ph, phases, ref = w["phase"], w["phases"], w["ref"]
    else:
        ph = M.random_phases((6, 8, 12), 2, 11)
        phases, ref = [(1.0, 0.3), (5.0, 0.25)], (3.0, 0.3)
    kw = dict(scheme="rpm", tol=1e-10, max_iter=3000, n_max=10, p_max=32)
    Cref, _ = O.effective_tensor(ph, O.lame_table(phases), O.lame(*ref), **kw)
    lt = np.array([B.lame_from_young(*p) for p in phases])
    opts = B.make_options(precision="fp64", batch_cases=1, **kw)
    C, stats, st = B.effective_tensor(dev(ph), lt, B.lame_from_young(*ref), opts)
    print(case, st, [(s["iterations"], s["residual"]) for s in stats], flush=True)
    assert st == "RPM_OK"
    assert all(s["residual"] <= 1e-10 for s in stats)
    err = np.abs(C - Cref).max() / np.abs(Cref).max()
    assert err <= 1e-8, err
    # the same call case by case on the GPU agrees too
    C1, _, st1 = B.effective_tensor(dev(ph), lt, B.lame_from_young(*ref), B.make_options(precision="fp64", **kw))
    assert st1 == "RPM_OK" and np.abs(C1 - C).max() <= 1e-8 * np.abs(Cref).max()


def test_batched_fp32_refined_spheres_contrast_1000(B):
    """FP32 fields, batched, refined to an FP64-certified 1e-6: C_eff within 1e-6
    of the oracle's (tol 1e-8) on the 32^3 stiff-sphere cell."""
    with open(GOLDEN) as fh:
        c = json.load(fh)["cells"]["spheres32_contrast1000"]
    gen = c["generator"]
    ph, _ = M.rsa_spheres(gen["n"], gen["r_min"], gen["r_max"], gen["vf"], gen["seed"])
    lt = np.array([B.lame_from_young(*p) for p in c["phases"]])
    opts = B.make_options(precision="fp32", tol=1e-6, max_iter=20000, refine=6, check_every=32, batch_cases=1)
    C, stats, st = B.effective_tensor(dev(ph), lt, B.lame_from_young(*c["ref"]), opts)
    Cref = np.array(c["C_eff"])
    err = np.abs(C - Cref).max() / np.abs(Cref).max()
    print("batched fp32:", st, [(s["iterations"], s["refinements"], s["residual_fp64"]) for s in stats],
          f"C_eff rel err {err:.3e}", flush=True)
    assert st == "RPM_OK" and all(s["residual_fp64"] <= 1e-6 for s in stats)
    assert err <= 1e-6, err
