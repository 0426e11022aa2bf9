"""FP64 CPU reference of the warm-start network (TEST INFRASTRUCTURE ONLY).

Only tests may import this module.  It evaluates, in plain numpy FP64 and
written from the definition rather than from the GPU's axis-by-axis GEMM
stages, the network of include/rpmfno.h and the gradient of a scalar
sum(dy * y) with respect to its parameters and its input:

  h_0     = W_lift x + b_lift
  h_{l+1} = gelu(W_l h_l + b_l + K_l h_l)
  y       = W_proj h_L + b_proj
  K_l h   = (1/N) Re sum_{k in M} e^{+2 pi i k.x/n} R_l(k) hhat(k),
  hhat(k) = sum_x e^{-2 pi i k.x/n} h(x),
  M = {-m/2, ..., m/2 - 1}^3, gelu(t) = t Phi(t) with the normal cdf Phi.

The retained transform is a dense matrix E[k, x] = exp(-2 pi i k.x / n) built
outright (tiny grids), so the spectral layer is one matrix product each way.
The gradient is the chain rule written out layer by layer; finite differences
of the forward pass pin it in the CPU tests.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf


def unpack(params, cfg):
    """Split the flat parameter vector (layout of include/rpmfno.h)."""
    cin, cout, C, L, m = cfg
    m3 = m ** 3
    p = np.asarray(params, dtype=np.float64)
    out, off = {}, 0

    def take(name, shape):
        nonlocal off
        n = int(np.prod(shape))
        out[name] = p[off:off + n].reshape(shape)
        off += n

    take("lift_w", (C, cin))
    take("lift_b", (C,))
    for l in range(L):
        take(f"w{l}", (C, C))
        take(f"b{l}", (C,))
        take(f"rre{l}", (m3, C, C))
        take(f"rim{l}", (m3, C, C))
    take("proj_w", (cout, C))
    take("proj_b", (cout,))
    assert off == p.size
    return out


def pack(d, cfg):
    cin, cout, C, L, m = cfg
    parts = [d["lift_w"], d["lift_b"]]
    for l in range(L):
        parts += [d[f"w{l}"], d[f"b{l}"], d[f"rre{l}"], d[f"rim{l}"]]
    parts += [d["proj_w"], d["proj_b"]]
    return np.concatenate([np.ravel(a) for a in parts])


def dft_matrix(shape, m):
    """E[k, x] = exp(-2 pi i sum_a k_a x_a / n_a) for the m^3 retained signed
    frequencies (kz, ky, kx order, each k = kk - m/2) and the voxels x
    (z, y, x order, x fastest)."""
    nz, ny, nx = shape
    ks = np.arange(m) - m // 2
    kz, ky, kx = np.meshgrid(ks, ks, ks, indexing="ij")
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ph = (np.outer(kz.ravel(), z.ravel()) / nz + np.outer(ky.ravel(), y.ravel()) / ny
          + np.outer(kx.ravel(), x.ravel()) / nx)
    return np.exp(-2j * np.pi * ph)


def gelu(t):
    return 0.5 * t * (1.0 + erf(t / np.sqrt(2.0)))


def gelu_grad(t):
    return 0.5 * (1.0 + erf(t / np.sqrt(2.0))) + t * np.exp(-0.5 * t * t) / np.sqrt(2.0 * np.pi)


def forward(params, cfg, x):
    """x: (B, c_in, nz, ny, nx).  Returns y (B, c_out, nz, ny, nx) and the cache."""
    cin, cout, C, L, m = cfg
    P = unpack(params, cfg)
    B = x.shape[0]
    shape = x.shape[2:]
    N = int(np.prod(shape))
    Emat = dft_matrix(shape, m)                      # (m3, N)
    xf = np.asarray(x, dtype=np.float64).reshape(B, cin, N)
    h = np.einsum("oi,biv->bov", P["lift_w"], xf) + P["lift_b"][None, :, None]
    cache = {"x": xf, "h": [h], "pre": [], "xhat": [], "E": Emat, "N": N, "shape": shape}
    for l in range(L):
        R = P[f"rre{l}"] + 1j * P[f"rim{l}"]         # (m3, C, C)
        xh = np.einsum("kv,biv->bik", Emat, h)       # hhat
        yh = np.einsum("koi,bik->bok", R, xh)
        kh = np.real(np.einsum("kv,bok->bov", np.conj(Emat), yh)) / N
        pre = np.einsum("oi,biv->bov", P[f"w{l}"], h) + P[f"b{l}"][None, :, None] + kh
        cache["xhat"].append(xh)
        cache["pre"].append(pre)
        h = gelu(pre)
        cache["h"].append(h)
    y = np.einsum("oi,biv->bov", P["proj_w"], h) + P["proj_b"][None, :, None]
    return y.reshape((B, cout) + tuple(shape)), cache


def backward(params, cfg, cache, dy):
    """Gradient of sum(dy * y): (flat parameter gradient, input gradient)."""
    cin, cout, C, L, m = cfg
    P = unpack(params, cfg)
    N = cache["N"]
    Emat = cache["E"]
    B = dy.shape[0]
    d = np.asarray(dy, dtype=np.float64).reshape(B, cout, N)
    g = {}
    hL = cache["h"][L]
    g["proj_w"] = np.einsum("bov,biv->oi", d, hL)
    g["proj_b"] = d.sum(axis=(0, 2))
    dh = np.einsum("oi,bov->biv", P["proj_w"], d)
    for l in reversed(range(L)):
        h = cache["h"][l]
        dpre = dh * gelu_grad(cache["pre"][l])
        g[f"w{l}"] = np.einsum("bov,biv->oi", dpre, h)
        g[f"b{l}"] = dpre.sum(axis=(0, 2))
        # Kh = (1/N) Re(E^H R E h): dR(k)[o][i] = (1/N) sum_b D_b[o] conj(X_b[i]) with D = E dpre
        D = np.einsum("kv,bov->bok", Emat, dpre)
        X = cache["xhat"][l]
        dR = np.einsum("bok,bik->koi", D, np.conj(X)) / N
        g[f"rre{l}"] = dR.real
        g[f"rim{l}"] = dR.imag
        R = P[f"rre{l}"] + 1j * P[f"rim{l}"]
        RhD = np.einsum("koi,bok->bik", np.conj(R), D)
        dh = np.einsum("oi,bov->biv", P[f"w{l}"], dpre) + np.real(np.einsum("kv,bik->biv", np.conj(Emat), RhD)) / N
    g["lift_w"] = np.einsum("bov,biv->oi", dh, cache["x"])
    g["lift_b"] = dh.sum(axis=(0, 2))
    dx = np.einsum("oi,bov->biv", P["lift_w"], dh)
    return pack(g, cfg), dx.reshape((B, cin) + tuple(cache["shape"]))
