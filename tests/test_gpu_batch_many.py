"""Many independent cells solved concurrently (batch.effective_many): worker
threads with a stream each must give exactly the results of one worker (the
per-cell arithmetic does not depend on what else runs on the GPU), and a
tuned launch shape per grid the same tensors up to the solver tolerance."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KW = dict(scheme="rpm", precision="fp32", tol=1e-6, refine=4, p_max=16, max_iter=5000, check_every=32)


@pytest.fixture(scope="module")
def batch():
    import torch

    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2003_07720_amd import batch as bt

    return bt


@pytest.fixture(scope="module")
def cells(batch):
    return batch.random_cells(6, grids=(16, 24, 32), seed0=7, contrast=(1e-2, 1e2))


def test_concurrent_workers_match_one_worker(batch, cells):
    print("effective_many workers 1 and 3", flush=True)
    r1, w1 = batch.effective_many(cells, KW, workers=1)
    r3, w3 = batch.effective_many(cells, KW, workers=3)
    print(f"wall {w1:.3f} s (1 worker), {w3:.3f} s (3 workers)", flush=True)
    assert len({r["worker"] for r in r3}) > 1
    for a, b in zip(r1, r3):
        assert a["status"] == b["status"] == "RPM_OK"
        assert a["iterations"] == b["iterations"]
        np.testing.assert_array_equal(a["C"], b["C"])
        assert a["residual_fp64"] <= 1e-6
        C = a["C"]
        assert np.abs(C - C.T).max() <= 1e-6 * np.abs(C).max()
        assert np.linalg.eigvalsh(0.5 * (C + C.T)).min() > 0


def test_tuned_shapes_give_the_same_tensors(batch, cells):
    print("effective_many with tuned shapes", flush=True)
    tunings = batch.tune_grids(cells, KW, reps=3)
    assert set(tunings) == {tuple(c["phase"].shape) for c in cells}
    r0, _ = batch.effective_many(cells, KW, workers=2)
    rt, _ = batch.effective_many(cells, KW, workers=2, tunings=tunings)
    for a, b in zip(r0, rt):
        assert b["status"] == "RPM_OK"
        np.testing.assert_allclose(b["C"], a["C"], rtol=1e-5, atol=1e-9 * np.abs(a["C"]).max())
