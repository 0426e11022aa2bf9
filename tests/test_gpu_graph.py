"""Main-loop iterations replayed from captured HIP graphs (rpm_options.graph):
the same kernels in the same order as the kernel-by-kernel launch, so every
solve must match it bit for bit -- iterates, error history, iteration count and
basis -- over several solves in a row on one stream, with the host's own
synchronisations and basis growth between the replays."""
import numpy as np
import pytest

from paper_2003_07720_amd import microstructure as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch

    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2003_07720_amd import binding

    return binding


CASES = {
    "disk32_rpm_fp64": dict(prec="fp64", scheme="rpm"),
    "disk32_basic_fp64": dict(prec="fp64", scheme="basic"),
    "spheres16_rpm_fp32_refined": dict(prec="fp32", scheme="rpm"),
}


@pytest.mark.parametrize("case", list(CASES))
def test_graph_replay_matches_eager(B, case):
    import torch

    cfg = CASES[case]
    if case.startswith("disk32"):
        w = M.workload_disk32()
        ph, phases, ref, E, tol = w["phase"], w["phases"], w["ref"], w["E"], 1e-8
    else:
        ph, _ = M.rsa_spheres(16, 2.0, 3.0, 0.2, 2000)
        phases, ref, E, tol = [(1.0, 0.3), (1000.0, 0.25)], (1000.0, 0.3), np.array([0, 0, 0.01, 0, 0, 0.0]), 1e-6
    lt = np.array([B.lame_from_young(*p) for p in phases])
    l0 = B.lame_from_young(*ref)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        phd = torch.from_numpy(np.ascontiguousarray(ph)).to("cuda")
        runs = {}
        for graph in (0, 1, 1, 0, 1):
            o = B.make_options(precision=cfg["prec"], scheme=cfg["scheme"], tol=tol, max_iter=5000, check_every=16,
                               graph=graph)
            r = B.fft_solve(phd, lt, l0, E, o)
            runs.setdefault(graph, []).append(r)
        s.synchronize()
    ref_run = runs[0][0]
    assert ref_run["status"] == "RPM_OK"
    for graph, rs in runs.items():
        for r in rs:
            assert r["status"] == ref_run["status"] and r["iterations"] == ref_run["iterations"]
            assert r["basis_dim"] == ref_run["basis_dim"] and list(r["decisions"]) == list(ref_run["decisions"])
            assert np.array_equal(r["history"], ref_run["history"])
            assert torch.equal(r["eps"], ref_run["eps"]), (graph, (r["eps"] - ref_run["eps"]).abs().max().item())
            assert np.array_equal(r["sig_avg"], ref_run["sig_avg"])
