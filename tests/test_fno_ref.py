"""Pins of the FP64 CPU reference of the warm-start network (oracle/fno_ref.py):
its gradient against central finite differences of its own forward pass, and
its spectral layer against numpy's FFT (a low-pass of the retained frequencies
when R(k) is the identity)."""
import numpy as np
import pytest
from scipy.stats import norm

from oracle import fno_ref as F

CFG = (2, 3, 4, 2, 4)  # c_in, c_out, width, layers, modes


def rand_params(cfg, seed):
    r = np.random.default_rng(seed)
    cin, cout, C, L, m = cfg
    d = {"lift_w": r.normal(size=(C, cin)) / np.sqrt(cin), "lift_b": 0.1 * r.normal(size=C)}
    for l in range(L):
        d[f"w{l}"] = r.normal(size=(C, C)) / np.sqrt(C)
        d[f"b{l}"] = 0.1 * r.normal(size=C)
        d[f"rre{l}"] = r.normal(size=(m ** 3, C, C)) / C
        d[f"rim{l}"] = r.normal(size=(m ** 3, C, C)) / C
    d["proj_w"] = r.normal(size=(cout, C)) / np.sqrt(C)
    d["proj_b"] = 0.1 * r.normal(size=cout)
    return F.pack(d, cfg)


def test_gelu_is_t_times_normal_cdf():
    t = np.linspace(-6, 6, 101)
    assert np.allclose(F.gelu(t), t * norm.cdf(t), atol=1e-15)
    h = 1e-6
    assert np.allclose(F.gelu_grad(t), (F.gelu(t + h) - F.gelu(t - h)) / (2 * h), atol=1e-8)


def test_spectral_layer_is_fft_lowpass_with_identity_weights():
    """L = 1, W = 0, b = 0, R(k) = I, lift = identity, projection = identity: the
    output is gelu of the real part of the inverse FFT of the input restricted to
    the retained frequencies {-m/2 .. m/2-1}^3."""
    cfg = (3, 3, 3, 1, 4)
    shape = (6, 8, 5)
    d = {"lift_w": np.eye(3), "lift_b": np.zeros(3), "w0": np.zeros((3, 3)), "b0": np.zeros(3),
         "rre0": np.tile(np.eye(3), (64, 1, 1)), "rim0": np.zeros((64, 3, 3)), "proj_w": np.eye(3),
         "proj_b": np.zeros(3)}
    p = F.pack(d, cfg)
    x = np.random.default_rng(3).normal(size=(1, 3) + shape)
    y, _ = F.forward(p, cfg, x)
    ref = np.empty_like(x)
    for c in range(3):
        X = np.fft.fftn(x[0, c])
        mask = np.zeros(shape, dtype=bool)
        ks = np.arange(4) - 2
        for kz in ks:
            for ky in ks:
                for kx in ks:
                    mask[kz % shape[0], ky % shape[1], kx % shape[2]] = True
        ref[0, c] = F.gelu(np.real(np.fft.ifftn(np.where(mask, X, 0))))
    assert np.abs(y - ref).max() < 1e-13


def test_gradient_matches_finite_differences():
    cfg = CFG
    shape = (4, 6, 5)
    p = rand_params(cfg, 1)
    r = np.random.default_rng(2)
    x = r.normal(size=(2, cfg[0]) + shape)
    dy = r.normal(size=(2, cfg[1]) + shape)
    y, cache = F.forward(p, cfg, x)
    g, dx = F.backward(p, cfg, cache, dy)

    def L(pp, xx):
        return float(np.sum(dy * F.forward(pp, cfg, xx)[0]))

    h = 1e-6
    idx = r.choice(p.size, 60, replace=False)
    for i in idx:
        e = np.zeros(p.size)
        e[i] = h
        fd = (L(p + e, x) - L(p - e, x)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    for _ in range(20):
        j = tuple(r.integers(0, s) for s in x.shape)
        e = np.zeros_like(x)
        e[j] = h
        fd = (L(p, x + e) - L(p, x - e)) / (2 * h)
        assert abs(fd - dx[j]) <= 1e-6 * max(1.0, abs(fd))
