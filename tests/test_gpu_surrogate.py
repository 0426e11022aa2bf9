"""The learned warm start end to end on the GPU: training data made by the
solver (six unit load cases per seeded cell), training with the library's own
forward/backward/Adam kernels (deterministic: fixed seeds, fixed-order
reductions), then what the trained network gains over plain RPM: its
prediction of the held-out cells' strain fluctuation beats the uniform start
(relative error below 1), and on the void cell of the headline workload
(30 % voids of stiffness 1e-8, here at 64^3, FP32 fields) RPM started from it
reaches the equilibrium error 3e-3 in fewer iterations than from the uniform
start."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_trained_warm_start_gains_over_plain_rpm():
    import torch

    from paper_2003_07720_amd import binding as B
    from paper_2003_07720_amd import microstructure as M
    from paper_2003_07720_amd import surrogate as S

    assert torch.cuda.is_available()
    n = 24
    X, Y, _ = S.make_dataset(n, 48, 0)
    Xv, Yv, _ = S.make_dataset(n, 6, 100000)
    cfg = B.fno_config(2, 36, 32, 4, 12)
    params, hist = S.train(cfg, X, Y, steps=400, batch=4, lr=3e-3, seed=1, log_every=100)
    assert np.isfinite(hist).all() and np.mean(hist[-50:]) < np.mean(hist[:50])
    err = S.relative_error(cfg, params, Xv, Yv)
    print(f"held-out relative error {err:.3f}", flush=True)
    assert err < 1.0  # the uniform start predicts zero fluctuation: relative error 1
    w = M.workload_voids128(seed=3000, n=64)
    c = S.compare_warm_start(cfg, params, w["phase"], w["phases"], w["E"], 3e-3, precision="fp32",
                             ref=(0.5 * (1 + 1e-8), 0.3), max_iter=4000)
    print("voids 64^3 to 3e-3:", c, flush=True)
    assert c["plain"]["status"] == "RPM_OK" and c["warm"]["status"] == "RPM_OK"
    assert c["warm"]["iterations"] < c["plain"]["iterations"]
