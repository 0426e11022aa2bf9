"""Training and use of the learned warm start (include/rpmfno.h).

The training data are made by the solver itself: for each seeded cell the six
unit load cases are solved (Algorithm 2, FP64 fields) and the strain
fluctuations eps^(j) - E^(j) become the 36 target channels; the features are
the cell's stiffness and Poisson fields (rpm_fno_features).  Training runs the
library's forward, backward and Adam kernels (rpm_fno_train_step); this module
only draws batches and calls them.  A warm start is rpm_fno_warm_start's
E + predicted fluctuation, handed to rpm_fft_solve as eps0: the solve still
iterates to its own tolerance, so the network can only save iterations.
"""
from __future__ import annotations

import sys
import time

import numpy as np
import torch

from . import binding as B
from . import microstructure as M

VOIGT_UNIT = [(0, 1.0), (1, 1.0), (2, 1.0), (3, 0.5), (4, 0.5), (5, 0.5)]


def random_cell(n, seed, contrast_range=(1e-3, 1e3), vf_range=(0.1, 0.35), r_frac=(0.06, 0.16)):
    """A two-phase cell of seeded random spheres: radii uniform in r_frac * n,
    volume fraction and inclusion/matrix modulus ratio (log-uniform) drawn from
    the ranges; matrix E = 1, nu = 0.3, inclusions nu = 0.3."""
    r = np.random.Generator(np.random.PCG64(10_000 + seed))
    vf = r.uniform(*vf_range)
    K = float(np.exp(r.uniform(np.log(contrast_range[0]), np.log(contrast_range[1]))))
    ph, info = M.rsa_spheres(n, r_frac[0] * n, r_frac[1] * n, vf, seed)
    return ph, [(1.0, 0.3), (K, 0.3)], info


def reference_medium(phases):
    """E0 at the stiffest phase (the classical map then has its spectrum in
    [0, 1), which also keeps FP32 rounding out of undamped modes)."""
    return (max(E for E, _ in phases), 0.3)


def solve_targets(ph, phases, tol=1e-6, max_iter=20000, p_max=64):
    """Features (2, nz, ny, nx) and the 36-channel target of one cell."""
    dph = torch.from_numpy(np.ascontiguousarray(ph)).to("cuda")
    lt = np.array([B.lame_from_young(*p) for p in phases])
    l0 = B.lame_from_young(*reference_medium(phases))
    opts = B.make_options(precision="fp64", tol=tol, max_iter=max_iter, p_max=p_max, check_every=32)
    ws = B.make_workspace(tuple(ph.shape), opts)
    y = torch.empty((36,) + tuple(ph.shape), dtype=torch.float32, device="cuda")
    its = []
    for j, (c, val) in enumerate(VOIGT_UNIT):
        E = np.zeros(6)
        E[c] = val
        r = B.fft_solve(dph, lt, l0, E, opts, workspace=ws)
        its.append(r["iterations"])
        eps = r["eps"]
        for comp in range(6):
            y[6 * j + comp] = (eps[comp] - E[comp]).float()
    x = B.fno_features(dph, lt)
    return x, y, its


def make_dataset(n, count, seed0=0, log_every=16, **kw):
    """Features and targets of `count` seeded cells (progress on stderr every
    log_every cells; 0 = quiet)."""
    xs, ys, info = [], [], []
    t0 = time.perf_counter()
    for k, s in enumerate(range(seed0, seed0 + count)):
        ph, phases, inf = random_cell(n, s, **kw)
        x, y, its = solve_targets(ph, phases)
        xs.append(x)
        ys.append(y)
        info.append(dict(seed=s, contrast=phases[1][0], vf=inf["vf"], iterations=its))
        if log_every and (k + 1) % log_every == 0:
            print(f"fno data: {k + 1}/{count} cells ({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    return torch.stack(xs), torch.stack(ys), info


def train(cfg, X, Y, steps=400, batch=4, lr=2e-3, seed=0, log_every=50):
    """Adam on mini-batches drawn (seeded) from the dataset; returns the
    parameters and the loss history."""
    n_cells = X.shape[0]
    shape = tuple(X.shape[2:])
    params = B.fno_init(cfg, seed)
    grad = torch.zeros_like(params)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    ws = B.fno_workspace(cfg, shape, batch)
    rng = np.random.Generator(np.random.PCG64(seed))
    hist = []
    t0 = time.perf_counter()
    for step in range(1, steps + 1):
        idx = torch.from_numpy(rng.choice(n_cells, batch, replace=n_cells < batch)).to("cuda")
        xb = X.index_select(0, idx).contiguous()
        yb = Y.index_select(0, idx).contiguous()
        # cosine decay of the learning rate
        lr_t = lr * 0.5 * (1 + np.cos(np.pi * (step - 1) / steps))
        loss = B.fno_train_step(cfg, params, grad, m, v, step, float(max(lr_t, 1e-5)), xb, yb, ws)
        hist.append(loss)
        if log_every and step % log_every == 0:
            print(f"fno train: step {step} loss {loss:.4e} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr,
                  flush=True)
    return params, hist


def relative_error(cfg, params, X, Y):
    """|y - target| / |target| over a dataset, one cell at a time."""
    num = den = 0.0
    ws = B.fno_workspace(cfg, tuple(X.shape[2:]), 1)
    for i in range(X.shape[0]):
        y, _ = B.fno_forward(cfg, params, X[i:i + 1].contiguous(), ws)
        num += float(((y[0] - Y[i]) ** 2).sum())
        den += float((Y[i] ** 2).sum())
    return (num / den) ** 0.5


def compare_warm_start(cfg, params, ph, phases, E, tol, precision="fp64", p_max=32, max_iter=20000, ref=None,
                       seeded=False):
    """Iterations and seconds of plain RPM against RPM from the network's warm
    start (network evaluation included in the time), each after an untimed run.
    seeded: also the warm start with the basis seeded by the network's six
    predicted unit-case fluctuations (rpm_fft_seed_basis, then reuse_basis)."""
    dph = torch.from_numpy(np.ascontiguousarray(ph)).to("cuda")
    lt = np.array([B.lame_from_young(*p) for p in phases])
    l0 = B.lame_from_young(*(ref or reference_medium(phases)))
    kw = dict(precision=precision, tol=tol, max_iter=max_iter, p_max=p_max, check_every=32)
    opts = B.make_options(**kw)
    ws = B.make_workspace(tuple(ph.shape), opts)
    fws = B.fno_workspace(cfg, tuple(ph.shape), 1)
    dt = torch.float64 if precision == "fp64" else torch.float32
    out = {}
    for mode in ("plain", "warm") + (("warm_seeded",) if seeded else ()):
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            eps0 = B.fno_warm_start(cfg, params, dph, lt, l0, E, precision, fws) if mode != "plain" else None
            o = opts
            if mode == "warm_seeded":
                x = B.fno_features(dph, lt)
                y, _ = B.fno_forward(cfg, params, x[None].contiguous(), fws)
                V = y[0].view(6, 6, *dph.shape).to(dt).contiguous()
                B.seed_basis(dph, lt, l0, V, opts, ws)
                o = B.make_options(reuse_basis=1, **kw)
            r = B.fft_solve(dph, lt, l0, E, o, eps0=eps0, workspace=ws, want_eps=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        out[mode] = dict(status=r["status"], iterations=r["iterations"], jvps=r["jvps"], seconds=round(el, 4),
                         initial_error=float(r["history"][0]) if r["history"] is not None and len(r["history"]) else None,
                         residual=r["residual_fp64"])
    return out
