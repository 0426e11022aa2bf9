"""FP32 fields with the RPM steps in FP64 (precision policy): the Jacobian-vector
products that form H = Z^T F_u Z and the compatible projection of new basis
columns run in FP64 on the exact values of the stored FP32 columns, a stalled
FP32 stage hands its field to FP64 refinement, and the refined results match
the FP64 oracle at high contrast and on void cells (Algorithm 2; Sec. 3)."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2003_07720_amd import microstructure as M

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ceff_32cube.json")
EZZ = np.array([0, 0, 0.01, 0, 0, 0.0])


@pytest.fixture(scope="module")
def B():
    import torch

    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2003_07720_amd import binding

    return binding


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _golden(name):
    with open(GOLDEN) as fh:
        g = json.load(fh)
    c = g["cells"][name]
    gen = c["generator"]
    ph, _ = M.rsa_spheres(gen["n"], gen["r_min"], gen["r_max"], gen["vf"], gen["seed"])
    return ph, [tuple(p) for p in c["phases"]], tuple(c["ref"]), np.array(c["C_eff"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_seeded_h_matches_oracle_at_contrast_1000(B, prec):
    """H of a seeded basis on a stiff-sphere cell (contrast 1000): FP64 fields to
    rounding; FP32 fields differ only by the rounding of the stored columns
    (FP32 map applications would be off by ~1e-4 here)."""
    import torch

    ph, _ = M.rsa_spheres(16, 2.0, 3.0, 0.2, 2000)
    phases = [(1.0, 0.3), (1000.0, 0.25)]
    ref = (1000.0, 0.3)
    # the seeds are float values, so both sides start from the same numbers
    V = np.stack([M.random_field(ph.shape, 40 + k) for k in range(10)]).astype(np.float32).astype(np.float64)
    bas = O.Basis(ph.shape, 16)
    O.seed_basis(ph, O.lame_table(phases), O.lame(*ref), V, bas)
    lt = np.array([B.lame_from_young(*p) for p in phases])
    opts = B.make_options(precision=prec, p_max=16)
    ws = B.make_workspace(ph.shape, opts)
    dt = torch.float64 if prec == "fp64" else torch.float32
    p = B.seed_basis(dev(ph), lt, B.lame_from_young(*ref), dev(V).to(dt).contiguous(), opts, ws)
    assert p == bas.p == 10
    H = B.workspace_h(ws)
    Hr = bas.H[:10, :10]
    err = np.abs(H - Hr).max() / np.abs(Hr).max()
    print(f"H parity {prec}: {err:.3e}", flush=True)
    assert err <= (1e-12 if prec == "fp64" else 1e-6), err


def test_fp32_stall_hands_over_to_refinement_effective_tensor(B):
    """32^3 stiff spheres at contrast 1000 (E0 = the stiff modulus): the FP32 stage
    stalls above its target, refinement takes every load case to an
    FP64-certified 1e-6, and C_eff matches the oracle's (tol 1e-8) within 1e-6."""
    ph, phases, ref, Cref = _golden("spheres32_contrast1000")
    lt = np.array([B.lame_from_young(*p) for p in phases])
    opts = B.make_options(precision="fp32", tol=1e-6, max_iter=20000, refine=6, check_every=32)
    C, stats, st = B.effective_tensor(dev(ph), lt, B.lame_from_young(*ref), opts)
    print("stall hand-over:", st, [(s["iterations"], s["refinements"], s["residual"], s["residual_fp64"])
                                   for s in stats], flush=True)
    assert st == "RPM_OK"
    assert all(s["residual_fp64"] <= 1e-6 for s in stats)
    err = np.abs(C - Cref).max() / np.abs(Cref).max()
    print(f"C_eff rel err {err:.3e}", flush=True)
    assert err <= 1e-6, err


def test_fp32_void_cell_to_1e6_against_oracle(B):
    """32^3 void cell (30 % spherical pores, radii 1.5-3, stiffness 1e-3 of the
    matrix, E0 = the matrix modulus), uniaxial eps_zz: FP32 fields refined to an
    FP64-certified 1e-6 against the oracle's solve to 1e-7 -- stress field and
    <sigma> -- and the effective tensor against the oracle's."""
    ph, phases, ref, Cref = _golden("voids32_contrast1e-3")
    lt_o = O.lame_table(phases)
    r = O.solve(ph, lt_o, O.lame(*ref), EZZ, scheme="rpm", tol=1e-7, max_iter=20000, n_max=10, p_max=32)
    assert r["status"] == "converged"
    sig_ref = O.stress(ph, lt_o, r["eps"])
    lt = np.array([B.lame_from_young(*p) for p in phases])
    l0 = B.lame_from_young(*ref)
    opts = B.make_options(precision="fp32", tol=1e-6, max_iter=20000, refine=6, check_every=32)
    g = B.fft_solve(dev(ph), lt, l0, EZZ, opts, want_sig=True)
    print("void cell:", g["status"], g["iterations"], g["refinements"], g["residual_fp64"], flush=True)
    assert g["status"] == "RPM_OK" and g["residual_fp64"] <= 1e-6
    sig = g["sig"].double().cpu().numpy()
    ferr = np.abs(sig - sig_ref).max() / np.abs(sig_ref).max()
    aerr = np.abs(g["sig_avg"] - r["sig_avg"]).max() / np.abs(r["sig_avg"]).max()
    print(f"sigma field {ferr:.3e}, <sigma> {aerr:.3e}", flush=True)
    assert aerr <= 1e-6, aerr
    assert ferr <= 1e-4, ferr
    C, stats, st = B.effective_tensor(dev(ph), lt, l0, opts)
    assert st == "RPM_OK" and all(s["residual_fp64"] <= 1e-6 for s in stats)
    err = np.abs(C - Cref).max() / np.abs(Cref).max()
    print(f"void C_eff rel err {err:.3e}", flush=True)
    assert err <= 1e-6, err
