"""The allocation-free map application (rpm_fft_apply_static, for callers that
cannot allocate device memory) against the workspace entry point rpm_fft_apply:
same kernels and launch shapes, so the outputs must agree bit for bit.  Two
calls in a row share the library's static scratch, the second on a smaller
grid, in FP64 and FP32, 3-D and 2-D."""
import numpy as np
import pytest
import torch

from paper_2003_07720_amd import binding as B
from paper_2003_07720_amd import microstructure as M

pytestmark = pytest.mark.gpu

CASES = [
    # (first grid, second smaller grid) as (nz, ny, nx)
    ((24, 36, 48), (8, 12, 16)),
    ((1, 64, 96), (1, 18, 24)),
]


def _inputs(shape, prec, seed):
    ph = M.random_phases(shape, 3, seed)
    lt = np.array([B.lame_from_young(E, nu) for E, nu in ((1.0, 0.3), (7.0, 0.25), (0.2, 0.35))])
    l0 = B.lame_from_young(3.0, 0.3)
    dt = torch.float64 if prec == "fp64" else torch.float32
    eps = torch.from_numpy(M.random_field(shape, seed + 1, 0.01)).to("cuda", dt).contiguous()
    E = np.array([0.01, -0.002, 0.003, 0.001, 0.0, 0.002])
    return torch.from_numpy(ph).to("cuda"), lt, l0, E, eps


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shapes", CASES, ids=["3d", "2d"])
def test_static_apply_matches_workspace_apply(prec, shapes):
    opts = B.make_options(precision=prec)
    for k, shape in enumerate(shapes):
        print(f"no_alloc: {prec} call {k} shape {shape}", flush=True)
        ph, lt, l0, E, eps = _inputs(shape, prec, 100 + 7 * k)
        xi_w, err_w, sav_w = B.fft_apply(ph, lt, l0, E, eps, opts)
        xi_s = torch.full_like(eps, float("nan"))
        xi_s, err_s, sav_s = B.fft_apply_static(ph, lt, l0, E, eps, opts, xi=xi_s)
        torch.cuda.synchronize()
        assert torch.equal(xi_s, xi_w), (shape, (xi_s - xi_w).abs().max().item())
        assert err_s == err_w and np.array_equal(sav_s, sav_w)
        assert np.isfinite(err_s) and err_s > 0


def test_static_apply_headline_grid_fp32_and_refusal():
    """The 128^3 FP32 void cell fits the static scratch (second call on a
    smaller grid after it); 128^3 FP64 is refused with RPM_E_SCRATCH."""
    w = M.workload_voids128(seed=3000, n=128)
    ph = torch.from_numpy(w["phase"]).to("cuda")
    lt = np.array([B.lame_from_young(*p) for p in w["phases"]])
    l0 = B.lame_from_young(0.5 * (1.0 + 1e-8), 0.3)
    opts = B.make_options(precision="fp32")
    eps = torch.from_numpy(M.random_field((128, 128, 128), 5, 0.01)).to("cuda", torch.float32).contiguous()
    print("no_alloc: 128^3 fp32", flush=True)
    xi_w, err_w, sav_w = B.fft_apply(ph, lt, l0, w["E"], eps, opts)
    xi_s, err_s, sav_s = B.fft_apply_static(ph, lt, l0, w["E"], eps, opts)
    assert torch.equal(xi_s, xi_w) and err_s == err_w and np.array_equal(sav_s, sav_w)
    del xi_w, xi_s
    ph2 = ph[:64, :64, :64].contiguous()
    eps2 = eps[:, :64, :64, :64].contiguous()
    print("no_alloc: 64^3 fp32 after 128^3", flush=True)
    a = B.fft_apply(ph2, lt, l0, w["E"], eps2, opts)
    b = B.fft_apply_static(ph2, lt, l0, w["E"], eps2, opts)
    assert torch.equal(a[0], b[0]) and a[1] == b[1]
    with pytest.raises(B.RpmError) as ei:
        B.fft_apply_static(ph, lt, l0, w["E"], eps.double(), B.make_options(precision="fp64"))
    assert ei.value.code == -6
