"""Independent closed forms that pin the oracle (numpy only; no FFT, no Green operator).

* :func:`galerkin_solution` -- the exact discrete solution of the periodic cell
  problem (Sec. 2: div sigma = 0, sigma = C(x) eps, mean strain E) obtained by a
  dense direct solve over an explicit basis of compatible strain fields
  sym(k(m) (x) e_j) exp(2 pi i m.x/n); the fixed point of the map F lies in the
  same space, so any converged iteration must reproduce it.
* :func:`laminate_solution` -- the exact solution for a cell whose stiffness
  varies along one axis only (traction continuity across layers).
* :func:`voigt_bound`, :func:`reuss_bound` -- arithmetic and harmonic means of
  the stiffness (Loewner bounds on the effective tensor).
* :func:`acoustic_green_apply` -- the Green operator written through the inverse
  acoustic tensor (n . C0 . n)^-1, a different derivation from the fourth-order
  formula used by the oracle.

All fields use the [6][nz][ny][nx] layout, components xx, yy, zz, yz, xz, xy
(tensor shear).  Internally Mandel vectors (shear * sqrt 2) make the Euclidean
product equal the Frobenius one.
"""
from __future__ import annotations

import numpy as np

SQ2 = np.sqrt(2.0)
MANDEL_W = np.array([1.0, 1.0, 1.0, SQ2, SQ2, SQ2])
PAIRS = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def lame(E, nu):
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


def iso_mandel(lam, mu):
    """6x6 Mandel matrix of lam 1(x)1 + 2 mu I."""
    C = 2.0 * mu * np.eye(6)
    C[:3, :3] += lam
    return C


def tensor_of(v6):
    """6 tensor components -> 3x3 symmetric matrix (works on leading axis)."""
    t = np.empty((3, 3) + np.shape(v6)[1:], dtype=np.result_type(v6, np.float64))
    for c, (i, j) in enumerate(PAIRS):
        t[i, j] = v6[c]
        t[j, i] = v6[c]
    return t


def comps_of(t):
    return np.array([t[i, j] for (i, j) in PAIRS])


def wavevector(n, m):
    """Wave vector (rad/voxel) of index m on grid n; Nyquist components take -pi times the
    sign of the first non-Nyquist non-zero component in the order z, y, x (else -pi)."""
    nx = list(n)
    s = 1.0
    signed = []
    nyq = []
    for a in range(3):
        mm = m[a] if m[a] < (nx[a] + 1) // 2 else m[a] - nx[a]
        signed.append(mm)
        nyq.append(nx[a] % 2 == 0 and m[a] == nx[a] // 2)
    for a in (2, 1, 0):
        if not nyq[a] and signed[a] != 0:
            s = 1.0 if signed[a] > 0 else -1.0
            break
    return np.array([(-np.pi * s) if nyq[a] else 2 * np.pi * signed[a] / nx[a] for a in range(3)])


def compatible_basis(shape):
    """Orthonormal (Frobenius) basis of zero-mean compatible strain fields on the grid,
    as a (6N, dim) matrix of Mandel vectors, voxel-major within each component."""
    nz, ny, nx = shape
    N = nx * ny * nz
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cols = []
    seen = set()
    for mz in range(nz):
        for my in range(ny):
            for mx in range(nx):
                if mx == 0 and my == 0 and mz == 0:
                    continue
                key = (mx, my, mz)
                neg = ((-mx) % nx, (-my) % ny, (-mz) % nz)
                if neg in seen:
                    continue
                seen.add(key)
                k = wavevector((nx, ny, nz), key)
                phase = np.exp(2j * np.pi * (mx * x / nx + my * y / ny + mz * z / nz)).ravel()
                block = []
                for j in range(3):
                    e = np.zeros(3)
                    e[j] = 1.0
                    S = 0.5 * (np.outer(k, e) + np.outer(e, k))
                    v = np.array([S[i, jj] for (i, jj) in PAIRS]) * MANDEL_W
                    f = (v[:, None] * phase[None, :]).ravel()
                    block.append(f.real)
                    block.append(f.imag)
                B = np.array(block).T
                U, s, _ = np.linalg.svd(B, full_matrices=False)
                keep = s > 1e-10 * s.max()
                cols.append(U[:, keep])
    return np.concatenate(cols, axis=1)


def _mandel_field(f):
    return (np.asarray(f).reshape(6, -1) * MANDEL_W[:, None]).ravel()


def _tensor_field(v, shape):
    return (v.reshape(6, -1) / MANDEL_W[:, None]).reshape((6,) + tuple(shape))


def _apply_C(phase, lame_tab, v):
    """Mandel stiffness applied voxel by voxel to a (6N, k) block."""
    ph = phase.ravel()
    N = ph.size
    V = v.reshape(6, N, -1)
    out = np.empty_like(V)
    for p, (lam, mu) in enumerate(lame_tab):
        sel = ph == p
        Cm = iso_mandel(lam, mu)
        out[:, sel, :] = np.einsum("ab,bnk->ank", Cm, V[:, sel, :])
    return out.reshape(v.shape)


def galerkin_solution(phase, lame_tab, E):
    """Exact discrete solution (strain field, <sigma>) by a dense direct solve."""
    phase = np.asarray(phase)
    shape = phase.shape
    N = phase.size
    Vb = compatible_basis(shape)
    Emand = np.repeat(E * MANDEL_W, N)
    CV = _apply_C(phase, lame_tab, Vb)
    A = Vb.T @ CV
    rhs = -(Vb.T @ _apply_C(phase, lame_tab, Emand[:, None]))[:, 0]
    a = np.linalg.solve(A, rhs)
    eps_m = Emand + Vb @ a
    eps = _tensor_field(eps_m, shape)
    sig_m = _apply_C(phase, lame_tab, eps_m[:, None])[:, 0]
    sig_avg = sig_m.reshape(6, N).mean(axis=1) / MANDEL_W
    return eps, sig_avg


def laminate_solution(phase, lame_tab, E, axis):
    """Exact solution for layers normal to `axis` (0 = x, 1 = y, 2 = z).

    Traction continuity: sigma n = t is uniform; with K = n.C.n and b = (C:E) n the
    jump a(x) = K^-1 (t - b) gives eps = E + sym(n (x) a) and <a> = 0 fixes
    t = <K^-1>^-1 <K^-1 b>."""
    phase = np.asarray(phase)
    nvec = np.zeros(3)
    nvec[axis] = 1.0
    Et = tensor_of(np.asarray(E, dtype=np.float64))
    Kinv_sum = np.zeros((3, 3))
    Kinvb_sum = np.zeros(3)
    per_phase = {}
    for p, (lam, mu) in enumerate(lame_tab):
        K = mu * np.eye(3) + (lam + mu) * np.outer(nvec, nvec)
        sigE = lam * np.trace(Et) * np.eye(3) + 2 * mu * Et
        b = sigE @ nvec
        per_phase[p] = (np.linalg.inv(K), b, lam, mu)
    counts = np.bincount(phase.ravel(), minlength=len(lame_tab)) / phase.size
    for p, frac in enumerate(counts):
        Ki, b, _, _ = per_phase[p]
        Kinv_sum += frac * Ki
        Kinvb_sum += frac * (Ki @ b)
    t = np.linalg.solve(Kinv_sum, Kinvb_sum)
    eps = np.empty((6,) + phase.shape)
    sig_avg = np.zeros(6)
    for p, frac in enumerate(counts):
        Ki, b, lam, mu = per_phase[p]
        a = Ki @ (t - b)
        et = Et + 0.5 * (np.outer(nvec, a) + np.outer(a, nvec))
        st = lam * np.trace(et) * np.eye(3) + 2 * mu * et
        sel = phase == p
        for c, (i, j) in enumerate(PAIRS):
            eps[c][sel] = et[i, j]
        sig_avg += frac * np.array([st[i, j] for (i, j) in PAIRS])
    return eps, sig_avg


def voigt_to_mandel(Cv):
    """Voigt stiffness (engineering shear strain) -> Mandel matrix."""
    n = Cv.shape[0]
    w = MANDEL_W if n == 6 else np.array([1.0, 1.0, SQ2])
    return Cv * np.outer(w, w)


def phase_fractions(phase, n_phases):
    return np.bincount(np.asarray(phase).ravel(), minlength=n_phases) / np.asarray(phase).size


def voigt_bound(phase, lame_tab, two_d=False):
    f = phase_fractions(phase, len(lame_tab))
    C = sum(fi * iso_mandel(*lt) for fi, lt in zip(f, lame_tab))
    return C[np.ix_([0, 1, 5], [0, 1, 5])] if two_d else C


def reuss_bound(phase, lame_tab, two_d=False):
    f = phase_fractions(phase, len(lame_tab))
    if two_d:
        # plane strain: the in-plane block of the compliance of the constrained material
        S = sum(fi * np.linalg.inv(iso_mandel(*lt)[np.ix_([0, 1, 5], [0, 1, 5])]) for fi, lt in zip(f, lame_tab))
        return np.linalg.inv(S)
    S = sum(fi * np.linalg.inv(iso_mandel(*lt)) for fi, lt in zip(f, lame_tab))
    return np.linalg.inv(S)


def acoustic_green_apply(k, lame0, s6):
    """sym(n (x) K(n)^-1 (s n)) with the acoustic tensor K(n) = n . C0 . n."""
    lam0, mu0 = lame0
    kk = np.linalg.norm(k)
    if kk == 0:
        return np.zeros(6, dtype=complex)
    n = np.asarray(k) / kk
    C0 = np.zeros((3, 3, 3, 3))
    d = np.eye(3)
    for i in range(3):
        for j in range(3):
            for a in range(3):
                for b in range(3):
                    C0[i, j, a, b] = lam0 * d[i, j] * d[a, b] + mu0 * (d[i, a] * d[j, b] + d[i, b] * d[j, a])
    K = np.einsum("i,ijab,b->ja", n, C0, n)
    S = tensor_of(np.asarray(s6, dtype=complex))
    u = np.linalg.solve(K, S @ n)
    G = 0.5 * (np.outer(n, u) + np.outer(u, n))
    return np.array([G[i, j] for (i, j) in PAIRS])


def hashin_shtrikman(k1, m1, k2, m2, f1):
    """HS bounds on bulk and shear moduli, phase 1 stiffer in both (3-D)."""
    f2 = 1.0 - f1
    kL = k2 + f1 / (1.0 / (k1 - k2) + 3.0 * f2 / (3.0 * k2 + 4.0 * m2))
    kU = k1 + f2 / (1.0 / (k2 - k1) + 3.0 * f1 / (3.0 * k1 + 4.0 * m1))
    mL = m2 + f1 / (1.0 / (m1 - m2) + 6.0 * f2 * (k2 + 2.0 * m2) / (5.0 * m2 * (3.0 * k2 + 4.0 * m2)))
    mU = m1 + f2 / (1.0 / (m2 - m1) + 6.0 * f1 * (k1 + 2.0 * m1) / (5.0 * m1 * (3.0 * k1 + 4.0 * m1)))
    return (kL, kU), (mL, mU)


def iso_projection(Cv):
    """Bulk and shear modulus of the isotropic projection of a Voigt stiffness."""
    iijj = Cv[:3, :3].sum()
    ijij = np.trace(Cv[:3, :3]) + 2.0 * np.trace(Cv[3:, 3:])
    return iijj / 9.0, (ijij - iijj / 3.0) / 10.0


# ---------------------------------------------------------------------------
# Growth pin: a two-phase laminate along z whose iterate error lies in two known
# eigenvectors of the linear part of the map.
#
# With layers normal to n = e_z, a compatible zero-mean field that depends on z
# only and has the single shear component eps_xz = a(z)/2 is mapped by F_u to
# the field of the same kind with a -> (1 - m) a + <m a>, m = mu(z)/mu0 (the
# Green operator at k parallel to e_z takes the traction mu a).  A profile a
# supported on the layers of one phase with zero mean there is therefore an
# eigenvector with eigenvalue 1 - m of that phase.  Starting from
# eps* + c1 v1 + c2 v2 (v1 in phase A, v2 in phase B), the fixed point gives
# xi^(j) = eps* + sum_i c_i lam_i^(j+1) v_i, so the two differences of q that
# feed the growth after n_max + 1 steps are known in closed form.

def laminate_growth_case(n_xy=4, nz=8, n_a=3, lam=(0.9, -0.5), mu0=1.0, nu=0.3):
    """Phase map (nz, n_xy, n_xy) with phase 0 on the first n_a layers, Lame table
    whose shear moduli give F_u the eigenvalues lam on the two profiles, the
    reference medium, and the unit-norm (Frobenius) eigenvector fields v1, v2."""
    ph = np.ones((nz, n_xy, n_xy), dtype=np.uint8)
    ph[:n_a] = 0
    E0 = 2.0 * (1.0 + nu) * mu0
    phases = [(E0 * (1.0 - l), nu) for l in lam]  # mu_i / mu0 = 1 - lam_i (equal nu)
    lame_tab = [lame(E, nu) for E, nu in phases]
    prof_a = np.zeros(nz)
    prof_a[0], prof_a[1] = 1.0, -1.0              # zero mean over phase 0's layers
    prof_b = np.zeros(nz)
    prof_b[n_a], prof_b[n_a + 2], prof_b[nz - 1] = 2.0, -1.0, -1.0  # zero mean over phase 1's layers
    vs = []
    for prof in (prof_a, prof_b):
        v = np.zeros((6, nz, n_xy, n_xy))
        v[4] = 0.5 * prof[:, None, None]          # eps_xz = a/2
        vs.append(v / np.sqrt(frob(v, v)))
    return ph, lame_tab, lame(E0, nu), vs[0], vs[1]


def frob(a, b):
    """Frobenius inner product of two [6][...] tensor fields (shear weighted 2)."""
    w = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])
    return float(np.sum(w[:, None] * a.reshape(6, -1) * b.reshape(6, -1)))


def growth_ratio(c, lam, n_max):
    """T22 / T11 of the QR of [dq^(n), dq^(n-1)], n = n_max, for the iterate error
    c1 v1 + c2 v2 (unit, orthogonal v_i): dq^(n) = sum c_i lam_i^n (lam_i - 1) v_i,
    dq^(n-1) = sum c_i lam_i^(n-1) (lam_i - 1) v_i."""
    a = np.array([ci * li ** n_max * (li - 1.0) for ci, li in zip(c, lam)])
    b = a / np.array(lam)
    T11 = np.linalg.norm(a)
    T22 = abs(a[0] * b[1] - a[1] * b[0]) / T11
    return T22 / T11


def coefficient_for_ratio(rho, lam, n_max, c1=1.0):
    """c2 such that growth_ratio((c1, c2)) = rho (the smaller root)."""
    g = abs(1.0 / lam[1] - 1.0 / lam[0])
    # rho = g x / (1 + x^2), x = a2 / a1
    x = (g - np.sqrt(g * g - 4.0 * rho * rho)) / (2.0 * rho)
    a1 = c1 * lam[0] ** n_max * (lam[0] - 1.0)
    return x * a1 / (lam[1] ** n_max * (lam[1] - 1.0))
