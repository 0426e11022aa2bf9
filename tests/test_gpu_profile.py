"""Per-class HIP-event timing (rpm_options.profile): every class of a
steady-state RPM step is timed, profile_classes restricts the classes and
profile_every samples one launch in every N of a class (the N-th, 2N-th, ...),
with the algorithmic bytes of exactly the sampled launches; timing never
changes the results."""
import numpy as np
import pytest

from paper_2003_07720_amd import microstructure as M

pytestmark = pytest.mark.gpu

PHASES = [(1.0, 0.3), (20.0, 0.3)]
E = np.array([0.0, 0.0, 0.01, 0.0, 0.0, 0.0])


@pytest.fixture(scope="module")
def B():
    import torch

    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2003_07720_amd import binding

    return binding


@pytest.mark.parametrize("shape,prec", [((16, 16, 16), "fp32"), ((4, 8, 128), "fp32"), ((4, 8, 128), "fp64")],
                         ids=["16cube-fp32", "4x8x128-fp32", "4x8x128-fp64"])
def test_sampled_events_and_results(B, shape, prec):
    import torch

    print(f"profile sampling {shape} {prec}", flush=True)
    ph = torch.from_numpy(M.random_phases(shape, 2, seed=4)).to("cuda")
    lt = np.array([B.lame_from_young(*p) for p in PHASES])
    l0 = B.lame_from_young(10.5, 0.3)
    common = dict(scheme="rpm", precision=prec, tol=1e-15, n_max=6, p_max=8, refine=0, check_every=8)
    ws = B.make_workspace(shape, B.make_options(max_iter=200, **common))
    # build the basis to p_max, then time steady-state windows that carry it
    B.fft_solve(ph, lt, l0, E, B.make_options(max_iter=60, **common), workspace=ws, want_eps=False)
    steady = dict(common, reuse_basis=1)
    ref = B.fft_solve(ph, lt, l0, E, B.make_options(max_iter=40, **steady), workspace=ws)
    B.fft_solve(ph, lt, l0, E, B.make_options(max_iter=60, **common), workspace=ws, want_eps=False)
    full = B.fft_solve(ph, lt, l0, E, B.make_options(max_iter=40, profile=1, **steady), workspace=ws)
    B.fft_solve(ph, lt, l0, E, B.make_options(max_iter=60, **common), workspace=ws, want_eps=False)
    k = B.KERNEL_NAMES.index("xfwd")
    samp = B.fft_solve(ph, lt, l0, E, B.make_options(max_iter=40, profile=1, profile_classes=1 << k,
                                                       profile_every=10, **steady), workspace=ws)
    for r in (full, samp):
        assert r["iterations"] == ref["iterations"] == 40
        assert torch.equal(r["eps"], ref["eps"])
    n_x = full["kernel_launches"]["xfwd"]
    assert n_x == 40 and full["kernel_launches"]["yfwd"] == 40 and full["kernel_launches"]["finalize"] >= 40
    assert all(full["kernel_ms"][c] > 0 for c in ("xfwd", "yfwd", "gamma", "yinv", "xinv", "project"))
    # one launch in ten of the x-forward class, nothing else
    assert samp["kernel_launches"]["xfwd"] == 4
    assert all(samp["kernel_launches"][c] == 0 for c in B.KERNEL_NAMES if c != "xfwd")
    # the sampled launches are steady-state ones (launches 10, 20, 30, 40); where the x pass carries the
    # recombination (FP64, nx = 128) the first launch of a window maps the uniform start without it and
    # moves fewer bytes than the others, so the sampled average is at least the full one
    per = samp["kernel_bytes"]["xfwd"] / 4
    avg = full["kernel_bytes"]["xfwd"] / 40
    assert per >= avg * (1 - 1e-12)
    if shape[2] == 128 and prec == "fp64":
        assert per > avg
    else:
        assert full["kernel_launches"]["recombine"] == 39
    assert per == pytest.approx(avg, rel=0.1)
