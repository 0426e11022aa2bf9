"""Seeded synthetic microstructures (inputs only; none of the solver's arithmetic).

The paper's workloads are synthetic cells: a circular fibre centred in a square
periodic cell (Sec. 5, the canonical problem), and its variants with larger
volume fractions and several fibres (Secs. 5.3, 5.4).  The generators below
produce the same kinds of cells on voxel grids:

* :func:`disk_2d` -- one centred circular inclusion (2-D, ``nz == 1``);
* :func:`rsa_spheres` -- random sequential addition of non-overlapping
  spheres (periodic), radii uniform in ``[r_min, r_max]``, stopped at the first
  voxelised volume fraction at or above the target;
* :func:`laminate` -- layers normal to one axis with a given phase sequence;
* :func:`random_phases` -- i.i.d. phase labels (for operator tests);
* :func:`random_field` -- a seeded Gaussian strain field [6, nz, ny, nx].

A voxel belongs to an inclusion iff its centre ``(i + 1/2, ...)`` lies strictly
inside it, with periodic minimum-image distances.  Phase maps are ``uint8``
arrays of shape ``(nz, ny, nx)``; x is the fastest axis.  Random numbers come
from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def disk_2d(n, radius_frac=0.25):
    """n x n x 1 phase map: 1 inside the centred disk of radius radius_frac * n, else 0."""
    c = (np.arange(n) + 0.5) - n / 2.0
    yy, xx = np.meshgrid(c, c, indexing="ij")
    r = radius_frac * n
    ph = (xx * xx + yy * yy < r * r).astype(np.uint8)
    return ph.reshape(1, n, n)


def workload_fibre(K, n=128, radius_frac=0.25):
    """The circular-fibre cell of Sec. 5 as used for the contrast sweep of Sec. 5.5
    (Table 1, whose grid and fibre size are not stated): n x n plane strain, a
    centred stiff fibre (radius radius_frac * n) of modulus K in a matrix of
    modulus 1, nu = 0.25 in both, mean shear strain eps_12 = 0.5 % (tensor
    component), reference medium at the geometric mean of the two moduli,
    tolerance 1e-4."""
    E = np.zeros(6)
    E[5] = 0.005
    return dict(phase=disk_2d(n, radius_frac), phases=[(1.0, 0.25), (float(K), 0.25)], E=E,
                ref=(float(np.sqrt(K)), 0.25), tol=1e-4)


def rsa_spheres(n, r_min, r_max, vf_target, seed, gap=1.0, max_tries=200000):
    """Periodic n^3 phase map with non-overlapping spheres (phase 1) in phase 0.

    Centres are uniform in the cell, radii uniform in [r_min, r_max]; a sphere is
    accepted iff its centre distance to every accepted sphere is at least
    r1 + r2 + gap (periodic).  Stops at the first voxelised volume fraction
    >= vf_target.  Returns (phase, info) with info = dict(vf, n_spheres, centres, radii)."""
    rng = _rng(seed)
    ph = np.zeros((n, n, n), dtype=np.uint8)
    c1 = np.arange(n) + 0.5
    centres, radii = [], []
    tries = 0
    vf = 0.0
    C = np.zeros((0, 3))
    Rr = np.zeros(0)
    while vf < vf_target and tries < max_tries:
        tries += 1
        ctr = rng.uniform(0.0, n, size=3)
        rad = rng.uniform(r_min, r_max)
        if Rr.size:
            d = C - ctr
            d -= n * np.round(d / n)
            if np.any(np.sqrt((d * d).sum(axis=1)) < rad + Rr + gap):
                continue
        centres.append(ctr)
        radii.append(rad)
        C = np.vstack([C, ctr[None, :]])
        Rr = np.append(Rr, rad)
        # voxelise with periodic minimum image, on a bounding box only
        lo = np.floor(ctr - rad - 1).astype(int)
        hi = np.ceil(ctr + rad + 1).astype(int)
        idx = [np.arange(lo[a], hi[a] + 1) for a in range(3)]
        d = [(c1[np.mod(idx[a], n)] - ctr[a]) for a in range(3)]
        d = [x - n * np.round(x / n) for x in d]
        dx, dy, dz = np.meshgrid(d[0], d[1], d[2], indexing="ij")
        inside = dx * dx + dy * dy + dz * dz < rad * rad
        ix, iy, iz = np.meshgrid(np.mod(idx[0], n), np.mod(idx[1], n), np.mod(idx[2], n), indexing="ij")
        ph[iz[inside], iy[inside], ix[inside]] = 1
        vf = float(ph.mean())
    return ph, dict(vf=vf, n_spheres=len(radii), centres=np.array(centres), radii=np.array(radii))


def laminate(n, layers, axis=2):
    """Phase map of shape n = (nx, ny, nz) whose phase depends only on the index along
    `axis` (0 = x, 1 = y, 2 = z): layers[i] is the phase of voxel layer i."""
    nx, ny, nz = n
    layers = np.asarray(layers, dtype=np.uint8)
    assert layers.size == n[axis]
    ph = np.zeros((nz, ny, nx), dtype=np.uint8)
    if axis == 0:
        ph[:, :, :] = layers[None, None, :]
    elif axis == 1:
        ph[:, :, :] = layers[None, :, None]
    else:
        ph[:, :, :] = layers[:, None, None]
    return ph


def random_phases(shape, n_phases, seed):
    """i.i.d. uniform phase labels in [0, n_phases) of shape (nz, ny, nx)."""
    return _rng(seed).integers(0, n_phases, size=shape, dtype=np.uint8)


def random_field(shape, seed, scale=1.0):
    """Gaussian field of shape (6, nz, ny, nx), float64."""
    return scale * _rng(seed).standard_normal((6,) + tuple(shape))


def random_unit_vectors(count, seed):
    return _rng(seed).standard_normal((count, 3))


# --- named workloads -------------------------------------------------------

def workload_disk32():
    """2-D plane strain 32 x 32: centred disk of radius 0.25 L (phase 1, E=10, nu=0.3)
    in a matrix (phase 0, E=1, nu=0.3); mean strain eps_xx = 0.01; reference medium at
    the arithmetic mean of the phase moduli."""
    ph = disk_2d(32, 0.25)
    phases = [(1.0, 0.3), (10.0, 0.3)]
    ref = (0.5 * (1.0 + 10.0), 0.3)
    E = np.array([0.01, 0, 0, 0, 0, 0], dtype=np.float64)
    return dict(phase=ph, phases=phases, ref=ref, E=E, tol=1e-8)


def workload_spheres64(seed=2000, ref_index=4):
    """64^3 random non-overlapping spheres (radii 4-8 voxels, 20 % volume fraction):
    matrix E=1, nu=0.3 (phase 0); inclusions E=1000, nu=0.25 (phase 1).  Reference
    medium E0 from the 5-point linear sweep between the phase moduli, nu0 = 0.3."""
    ph, info = rsa_spheres(64, 4.0, 8.0, 0.20, seed)
    phases = [(1.0, 0.3), (1000.0, 0.25)]
    sweep = np.linspace(1.0, 1000.0, 5)
    ref = (float(sweep[ref_index]), 0.3)
    return dict(phase=ph, phases=phases, ref=ref, info=info, sweep=sweep)


def workload_voids128(seed=3000, n=128):
    """n^3 random spherical voids (radii 6-12 voxels at n = 128, scaled with n; 30 %
    volume fraction) with stiffness 1e-8 E_matrix (phase 1) in a matrix E=1, nu=0.3
    (phase 0); uniaxial mean strain eps_zz = 0.01; tolerance 1e-6."""
    s = n / 128.0
    ph, info = rsa_spheres(n, 6.0 * s, 12.0 * s, 0.30, seed)
    phases = [(1.0, 0.3), (1e-8, 0.3)]
    E = np.array([0, 0, 0.01, 0, 0, 0], dtype=np.float64)
    return dict(phase=ph, phases=phases, info=info, E=E, tol=1e-6)
