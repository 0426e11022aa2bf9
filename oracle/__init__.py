"""FP64 CPU oracle for the RPM-FFT method (Peng, Nepal & Dayal, CMAME 2020).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the product path never does.  The
arithmetic lives in ``oracle.c`` (plain C, FP64, compiled with
``-ffp-contract=off``); this module only marshals numpy arrays.

Each wrapper names the passage of the paper it follows:

* :func:`fmap` -- the Lippmann-Schwinger fixed-point map (the iteration body
  of Algorithm 1) and the operator F defined in Sec. 3, in the literal form that
  transforms both strain and stress;
* :func:`solve` -- Algorithm 1 (``scheme="basic"``) or Algorithm 2
  (``scheme="rpm"``) for one mean strain E (Sec. 2: the average strain is
  given);
* :func:`effective_tensor` -- the effective response (title; Sec. 1: given
  the average strain, the fields in the cell) as one solve per unit load case;
* ``map="polarization"`` in :func:`fmap` / :func:`solve` -- the polarization
  iteration of Algorithm 3 (Accelerated FFT for alpha = beta = 2, Sec. 5.5) in
  place of F, with the sign of the C0 term of s_b corrected (s_b = alpha sigma
  - beta C0:eps); :func:`polarization_reduced` -- the form it takes on
  compatible fields of mean E, eps + alpha (C + C0)^{-1} C0 (F(eps) - eps).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_CMD = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-o", _LIB, _SRC, "-lm"]

STATUS = {0: "converged", 1: "not_converged", 2: "diverged", 3: "singular"}
VOIGT_PAIRS = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (building the checker is not using it)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.run(GCC_CMD, check=True)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i = ctypes.c_int
        d = ctypes.c_double
        lib.orc_dft_naive.argtypes = [dp, dp, i, i]
        lib.orc_fft1.argtypes = [dp, dp, i, i]
        lib.orc_fft3.argtypes = [dp, i, i, i, i]
        lib.orc_wavevector.argtypes = [i, i, i, i, i, i, dp]
        lib.orc_gamma_apply.argtypes = [dp, d, d, dp, dp]
        lib.orc_stress.argtypes = [ctypes.c_long, u8p, dp, dp, dp]
        lib.orc_project_compatible.argtypes = [i, i, i, d, d, dp]
        lib.orc_fmap.argtypes = [i, i, i, u8p, dp, d, d, dp, dp, dp, dp, dp, i, d, d]
        lib.orc_fmap.restype = d
        lib.orc_polarization_reduced.argtypes = [i, i, i, u8p, dp, d, d, dp, dp, d, dp]
        lib.orc_solve.argtypes = [i, i, i, u8p, dp, d, d, dp, i, d, i, i, i, d, ip, i, dp, dp, dp, dp, ip,
                                  dp, dp, ip, dp, dp, i, ip, i, i, d, d]
        lib.orc_solve.restype = i
        lib.orc_seed_basis.argtypes = [i, i, i, u8p, dp, d, d, dp, i, i, dp, dp, dp, ip, i, d, d]
        lib.orc_seed_basis.restype = i
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if a is not None else None


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def lame(E, nu):
    """Lame constants of an isotropic phase from Young's modulus and Poisson's ratio."""
    E = float(E)
    nu = float(nu)
    return E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))


def lame_table(phases):
    """[(E, nu), ...] -> float64 array [n_phases, 2] of (lambda, mu)."""
    return np.array([lame(E, nu) for (E, nu) in phases], dtype=np.float64).reshape(-1, 2)


# --------------------------------------------------------------------------
# transforms and operators
# --------------------------------------------------------------------------

def dft_naive(x, sign=-1):
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    _load().orc_dft_naive(_dp(x.view(np.float64)), _dp(y.view(np.float64)), x.size, sign)
    return y


def fft1(x, sign=-1):
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    _load().orc_fft1(_dp(x.view(np.float64)), _dp(y.view(np.float64)), x.size, sign)
    return y


def fft3(a, sign=-1):
    """3-D transform of a complex array of shape (nz, ny, nx)."""
    a = np.array(a, dtype=np.complex128, order="C", copy=True)
    nz, ny, nx = a.shape
    _load().orc_fft3(_dp(a.view(np.float64)), nx, ny, nz, sign)
    return a


def wavevector(n, m):
    """Wave vector (rad/voxel) of DFT index m = (mx, my, mz) on grid n = (nx, ny, nz)."""
    k = np.zeros(3)
    _load().orc_wavevector(n[0], n[1], n[2], m[0], m[1], m[2], _dp(k))
    return k


def gamma_apply(k, lame0, s6):
    """Green operator of the reference medium applied to 6 complex components."""
    k = np.ascontiguousarray(k, dtype=np.float64)
    s = np.ascontiguousarray(s6, dtype=np.complex128)
    o = np.empty(6, dtype=np.complex128)
    _load().orc_gamma_apply(_dp(k), float(lame0[0]), float(lame0[1]), _dp(s.view(np.float64)),
                            _dp(o.view(np.float64)))
    return o


def stress(phase, lame_tab, eps):
    phase = np.ascontiguousarray(phase, dtype=np.uint8)
    lt = np.ascontiguousarray(lame_tab, dtype=np.float64)
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    sig = np.empty_like(eps)
    _load().orc_stress(phase.size, _u8(phase), _dp(lt), _dp(eps), _dp(sig))
    return sig


def project_compatible(v, lame0):
    """Projection Gamma0 C0 of a field (6, nz, ny, nx) onto zero-mean compatible fields."""
    v = np.array(v, dtype=np.float64, order="C", copy=True)
    _, nz, ny, nx = v.shape
    _load().orc_project_compatible(nx, ny, nz, float(lame0[0]), float(lame0[1]), _dp(v))
    return v


MAPS = {"classical": 0, "polarization": 1}


def fmap(phase, lame_tab, lame0, E, eps, map="classical", alpha=2.0, beta=2.0):
    """One application of F (or of the polarization iteration): returns (xi,
    error of eps, <sigma>, max imaginary residue).

    phase: uint8 (nz, ny, nx); eps: float64 (6, nz, ny, nx)."""
    phase = np.ascontiguousarray(phase, dtype=np.uint8)
    nz, ny, nx = phase.shape
    lt = np.ascontiguousarray(lame_tab, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    eps = np.ascontiguousarray(eps, dtype=np.float64).reshape(6, nz, ny, nx)
    xi = np.empty_like(eps)
    err = np.zeros(1)
    sav = np.zeros(6)
    im = _load().orc_fmap(nx, ny, nz, _u8(phase), _dp(lt), float(lame0[0]), float(lame0[1]), _dp(E), _dp(eps),
                          _dp(xi), _dp(err), _dp(sav), MAPS[map], float(alpha), float(beta))
    return xi, float(err[0]), sav, float(im)


def polarization_reduced(phase, lame_tab, lame0, E, eps, alpha=2.0):
    """eps + alpha (C(x) + C0)^{-1} C0 : (F(eps) - eps)."""
    phase = np.ascontiguousarray(phase, dtype=np.uint8)
    nz, ny, nx = phase.shape
    lt = np.ascontiguousarray(lame_tab, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    eps = np.ascontiguousarray(eps, dtype=np.float64).reshape(6, nz, ny, nx)
    out = np.empty_like(eps)
    _load().orc_polarization_reduced(nx, ny, nz, _u8(phase), _dp(lt), float(lame0[0]), float(lame0[1]), _dp(E),
                                     _dp(eps), float(alpha), _dp(out))
    return out


class Basis:
    """Unstable-subspace basis Z, W = F_u Z and H = Z^T W carried between solves."""

    def __init__(self, shape, p_max):
        nz, ny, nx = shape
        self.p_max = int(p_max)
        L = 6 * nx * ny * nz
        self.Z = np.zeros((max(self.p_max, 1), L))
        self.W = np.zeros((max(self.p_max, 1), L))
        self.H = np.zeros((max(self.p_max, 1), max(self.p_max, 1)))
        self.p = 0


def solve(phase, lame_tab, lame0, E, scheme="rpm", tol=1e-8, max_iter=10000, n_max=10, p_max=32, kappa=0.1,
          replay=None, eps_init=None, basis=None, hist_cap=100000, map="classical", alpha=2.0, beta=2.0):
    """Algorithm 1 (scheme='basic') or Algorithm 2 (scheme='rpm') for mean strain E
    (map='polarization': the fixed-point operation is Algorithm 3's iteration).

    Returns a dict with eps (6, nz, ny, nx), sig_avg, status, iterations (main
    F calls incl. the initial one), jvps, growth, p, residual, history,
    decisions, max_imag and the basis object (reusable across load cases)."""
    phase = np.ascontiguousarray(phase, dtype=np.uint8)
    nz, ny, nx = phase.shape
    lt = np.ascontiguousarray(lame_tab, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    sch = {"basic": 0, "rpm": 1}[scheme]
    if basis is None:
        basis = Basis(phase.shape, p_max if sch == 1 else 0)
    eps = np.empty((6, nz, ny, nx))
    sav = np.zeros(6)
    counters = np.zeros(4, dtype=np.int32)
    res = np.zeros(2)
    hist = np.zeros(hist_cap)
    dec = np.zeros(1024, dtype=np.int32)
    p_io = np.array([basis.p], dtype=np.int32)
    rp = None if replay is None else np.ascontiguousarray(replay, dtype=np.int32)
    ei = None if eps_init is None else np.ascontiguousarray(eps_init, dtype=np.float64)
    st = _load().orc_solve(nx, ny, nz, _u8(phase), _dp(lt), float(lame0[0]), float(lame0[1]), _dp(E), sch,
                           float(tol), int(max_iter), int(n_max), int(basis.p_max if sch == 1 else 0),
                           float(kappa), _ip(rp), 0 if rp is None else rp.size, _dp(ei), _dp(basis.Z),
                           _dp(basis.W), _dp(basis.H), _ip(p_io), _dp(eps), _dp(sav), _ip(counters), _dp(res),
                           _dp(hist), hist_cap, _ip(dec), dec.size, MAPS[map], float(alpha), float(beta))
    if sch == 1:
        basis.p = int(p_io[0])
    it = int(counters[0])
    return dict(eps=eps, sig_avg=sav, status=STATUS[st], iterations=it, jvps=int(counters[1]),
                growth=int(counters[2]), p=int(counters[3]), residual=float(res[0]), max_imag=float(res[1]),
                history=hist[:min(it, hist_cap)].copy(), decisions=dec[:int(counters[2])].copy(), basis=basis)


def solve_stress(phase, lame_tab, lame0, Sigma, **kw):
    """Prescribed mean stress Sigma (Sec. 2: the average strain or stress is given).
    The problem is linear: the mean strain E solves C_eff E = Sigma (Voigt with
    engineering shear; 2-D plane strain over 11, 22, 12), C_eff from one solve per
    unit mean strain; then the strain-controlled solve for E.  Returns the final
    solve's dict with E and C_eff added."""
    phase = np.ascontiguousarray(phase, dtype=np.uint8)
    two_d = phase.shape[0] == 1
    idx = [0, 1, 5] if two_d else list(range(6))
    C, _ = effective_tensor(phase, lame_tab, lame0, **kw)
    g = np.linalg.solve(C, np.asarray(Sigma, dtype=np.float64)[idx])
    E = np.zeros(6)
    for r, i in enumerate(idx):
        E[i] = g[r] if i < 3 else 0.5 * g[r]
    out = solve(phase, lame_tab, lame0, E, **kw)
    out.update(E=E, C_eff=C)
    return out


def seed_basis(phase, lame_tab, lame0, V, basis, map="classical", alpha=2.0, beta=2.0):
    """Append the vectors V (k, 6, nz, ny, nx) to the basis the way growth adds a
    difference of iterates (normalise, compatible projection for the classical
    map, two Gram-Schmidt passes, drop below 1e-10), with their W = F_u z columns
    and H borders.  Returns the number of columns added; basis.p is updated."""
    phase = np.ascontiguousarray(phase, dtype=np.uint8)
    nz, ny, nx = phase.shape
    lt = np.ascontiguousarray(lame_tab, dtype=np.float64)
    V = np.ascontiguousarray(np.asarray(V, dtype=np.float64).reshape(-1, 6 * nx * ny * nz))
    p_io = np.array([basis.p], dtype=np.int32)
    added = _load().orc_seed_basis(nx, ny, nz, _u8(phase), _dp(lt), float(lame0[0]), float(lame0[1]), _dp(V),
                                   V.shape[0], basis.p_max, _dp(basis.Z), _dp(basis.W), _dp(basis.H), _ip(p_io),
                                   MAPS[map], float(alpha), float(beta))
    basis.p = int(p_io[0])
    return int(added)


def unit_load(j):
    """Unit macroscopic strain of Voigt column j (11, 22, 33, 23, 13, 12) in tensor
    components: a shear load carries eps_ab = eps_ba = 1/2 (engineering strain 1)."""
    E = np.zeros(6)
    E[j] = 1.0 if j < 3 else 0.5
    return E


def effective_tensor(phase, lame_tab, lame0, scheme="rpm", reuse_basis=True, **kw):
    """Effective stiffness (Voigt matrix, engineering shear) from one solve per unit
    load case: column j is <sigma> for E = e_j.  In 2-D (nz == 1) only the in-plane
    cases 11, 22, 12 are solved (3 x 3 result, plane strain)."""
    phase = np.ascontiguousarray(phase, dtype=np.uint8)
    two_d = phase.shape[0] == 1
    cases = [0, 1, 5] if two_d else list(range(6))
    C = np.zeros((len(cases), len(cases)))
    basis = None
    runs = []
    for col, j in enumerate(cases):
        r = solve(phase, lame_tab, lame0, unit_load(j), scheme=scheme,
                  basis=basis if reuse_basis else None, **kw)
        if reuse_basis and scheme == "rpm":
            basis = r["basis"]
        C[:, col] = r["sig_avg"][cases]
        runs.append(r)
    return C, runs
