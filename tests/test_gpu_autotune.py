"""The tile autotuner of the pencil passes (rpm_fft_autotune) and the launch
shapes it returns (rpm_options.tuning).

A launch shape only regroups work: every element of every pass is computed
with the same arithmetic, so fields must come out bitwise equal to the
default shape's, on the uneven grids of the benchmark families (48^3, a
mixed 32 x 48 x 64 box) as on a power-of-two one; only the equilibrium
error, a sum of per-block partials whose grouping follows the gamma grid,
may differ in its last bits.  The y transforms held in registers (y_regs)
factor the transform differently, so they are compared with the oracle and
with the default passes to FP32 rounding instead.
"""
import numpy as np
import pytest

from paper_2003_07720_amd import microstructure as M

pytestmark = pytest.mark.gpu

PHASES = [(1.0, 0.3), (50.0, 0.3)]
E = np.array([0.0, 0.0, 0.01, 0.0, 0.0, 0.0])


@pytest.fixture(scope="module")
def B():
    import torch

    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2003_07720_amd import binding

    return binding


def _cell(B, shape, seed):
    import torch

    ph = M.random_phases(shape, 2, seed=seed)
    lt = np.array([B.lame_from_young(*p) for p in PHASES])
    l0 = B.lame_from_young(25.5, 0.3)
    return torch.from_numpy(ph).to("cuda"), lt, l0


def _fixed_steps(B, ph, lt, l0, prec, tuning):
    # a tolerance no step reaches: every run does the same 40 iterations
    opts = B.make_options(scheme="rpm", precision=prec, tol=1e-14, max_iter=40, n_max=5, p_max=8, refine=0,
                          tuning=tuning)
    return B.fft_solve(ph, lt, l0, E, opts)


@pytest.mark.parametrize("shape,prec", [((48, 48, 48), "fp32"), ((32, 48, 64), "fp64"), ((64, 64, 64), "fp32")],
                         ids=["48cube-fp32", "32x48x64-fp64", "64cube-fp32"])
def test_autotuned_shape_gives_the_default_fields(B, shape, prec):
    print(f"autotune {shape} {prec}", flush=True)
    ph, lt, l0 = _cell(B, shape, 5)
    opts = B.make_options(scheme="rpm", precision=prec, p_max=8)
    t = B.autotune(ph, lt, l0, opts, reps=5)
    print(f"tuning {t['tuning'].as_dict()} {t['ms']:.4f} ms/map, {t['candidates']} candidates", flush=True)
    assert t["candidates"] >= 1 and t["ms"] > 0
    tn = t["tuning"]
    nz = shape[0]
    assert tn.y_cols == 0 or nz % tn.y_cols == 0
    assert tn.y_blocks >= 0 and tn.gamma_blocks >= 0
    a = _fixed_steps(B, ph, lt, l0, prec, None)
    b = _fixed_steps(B, ph, lt, l0, prec, tn)
    assert a["iterations"] == b["iterations"] == 40 and a["basis_dim"] == b["basis_dim"]
    import torch

    assert torch.equal(a["eps"], b["eps"])
    np.testing.assert_allclose(b["history"], a["history"], rtol=1e-12 if prec == "fp64" else 1e-6, atol=0)


@pytest.mark.parametrize("tuning", [dict(y_cols=4, y_blocks=256, gamma_blocks=256),
                                    dict(y_cols=1, y_blocks=0, gamma_blocks=512),
                                    dict(y_cols=0, y_blocks=1536, gamma_blocks=0)],
                         ids=["cols4-256-256", "cols1-gamma512", "yblocks1536"])
def test_explicit_shapes_apply_the_same_map(B, tuning):
    import torch

    print(f"explicit tuning {tuning}", flush=True)
    ph, lt, l0 = _cell(B, (32, 32, 32), 6)
    opts = B.make_options(precision="fp32")
    eps = (torch.from_numpy(M.random_field((32, 32, 32), seed=8, scale=0.003)).float().to("cuda")
           + torch.tensor(E, dtype=torch.float32, device="cuda").view(6, 1, 1, 1)).contiguous()
    xa, ea, sa = B.fft_apply(ph, lt, l0, E, eps, opts)
    xb, eb, sb = B.fft_apply(ph, lt, l0, E, eps, B.make_options(precision="fp32", tuning=tuning))
    assert torch.equal(xa, xb)
    assert abs(ea - eb) <= 1e-6 * ea
    np.testing.assert_array_equal(sa, sb)


@pytest.mark.parametrize("shape", [(16, 128, 8), (32, 128, 6)], ids=["16x128x8", "32x128x6"])
def test_register_y_transforms_match_the_oracle(B, shape):
    """y_regs = 1 (128-point y transforms in registers, rows exchanged across
    lanes by DPP moves) applies the map of the oracle to the FP32 bar, and the
    LDS passes' result to FP32 rounding."""
    import torch

    import oracle as O

    print(f"register y transforms {shape}", flush=True)
    ph, lt, l0 = _cell(B, shape, 9)
    eps_np = M.random_field(shape, seed=10, scale=0.003) + np.asarray(E)[:, None, None, None]
    eps = torch.from_numpy(eps_np).float().to("cuda").contiguous()
    xa, ea, _ = B.fft_apply(ph, lt, l0, E, eps, B.make_options(precision="fp32"))
    xb, eb, _ = B.fft_apply(ph, lt, l0, E, eps, B.make_options(precision="fp32", tuning=dict(y_regs=1)))
    scale = float(xa.abs().max())
    assert float((xa - xb).abs().max()) <= 2e-6 * scale
    assert abs(ea - eb) <= 1e-5 * ea
    ref_xi, ref_err, _, _ = O.fmap(ph.cpu().numpy(), O.lame_table(PHASES), O.lame(25.5, 0.3), E, eps_np)
    assert np.abs(xb.double().cpu().numpy() - ref_xi).max() <= 2e-5 * np.abs(ref_xi).max()
    assert abs(eb - ref_err) <= 2e-4 * ref_err


def test_inapplicable_shape_is_rejected(B):
    ph, lt, l0 = _cell(B, (48, 48, 48), 7)
    with pytest.raises(B.RpmError) as ex:
        B.fft_solve(ph, lt, l0, E, B.make_options(tuning=dict(y_cols=5, y_blocks=0, gamma_blocks=0)))
    assert ex.value.code == -1
