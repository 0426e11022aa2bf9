"""ctypes binding of librpmfft.so (argument marshalling only).

Every function here forwards to the C ABI declared in include/rpmfft.h; all
arithmetic runs in the HIP kernels of the library.  Device buffers are torch
tensors on the current HIP device (PyTorch provides memory and the stream);
small arrays are host numpy arrays.  If the library is missing the import
fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loads the HIP runtime first so the library shares it

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librpmfft.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc --offload-arch=gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

RPM_NKERNEL = 10
KERNEL_NAMES = ["xfwd", "yfwd", "gamma", "yinv", "xinv", "reduce", "finalize", "growth", "project", "recombine"]
STATUS = {0: "RPM_OK", 1: "RPM_NOT_CONVERGED", 2: "RPM_DIVERGED", 3: "RPM_SINGULAR", -1: "RPM_E_INVALID",
          -2: "RPM_E_UNSUPPORTED_SIZE", -3: "RPM_E_WORKSPACE", -5: "RPM_E_HIP", -6: "RPM_E_SCRATCH"}
SCHEME = {"basic": 0, "rpm": 1}
MAP = {"classical": 0, "polarization": 1}
PRECISION = {"fp64": 0, "fp32": 1}


class RpmProblem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("phase", ctypes.c_void_p), ("n_phases", ctypes.c_int32),
                ("lame", ctypes.POINTER(ctypes.c_double)), ("lame0", ctypes.c_double * 2)]


class RpmTuning(ctypes.Structure):
    _fields_ = [("y_cols", ctypes.c_int32), ("y_blocks", ctypes.c_int32), ("gamma_blocks", ctypes.c_int32),
                ("y_regs", ctypes.c_int32)]

    def as_dict(self):
        return dict(y_cols=self.y_cols, y_blocks=self.y_blocks, gamma_blocks=self.gamma_blocks, y_regs=self.y_regs)


class RpmOptions(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("n_max", ctypes.c_int32),
                ("p_max", ctypes.c_int32), ("kappa", ctypes.c_double), ("scheme", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("reuse_basis", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("replay", ctypes.POINTER(ctypes.c_int32)), ("replay_len", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("refine", ctypes.c_int32), ("refine_tol", ctypes.c_double),
                ("map", ctypes.c_int32), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("profile_classes", ctypes.c_int32), ("stall_window", ctypes.c_int32),
                ("batch_cases", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("profile_every", ctypes.c_int32), ("tuning", ctypes.POINTER(RpmTuning))]


class RpmStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("jvps", ctypes.c_int32), ("basis_dim", ctypes.c_int32),
                ("growth_events", ctypes.c_int32), ("residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int32),
                ("decisions", ctypes.POINTER(ctypes.c_int32)), ("decisions_cap", ctypes.c_int32),
                ("kernel_ms", ctypes.c_double * RPM_NKERNEL), ("kernel_launches", ctypes.c_int32 * RPM_NKERNEL),
                ("kernel_bytes", ctypes.c_double * RPM_NKERNEL), ("residual_fp64", ctypes.c_double),
                ("refinements", ctypes.c_int32)]


_P = ctypes.POINTER
_vp = ctypes.c_void_p
_dp = _P(ctypes.c_double)
_lib.rpm_default_options.argtypes = [_P(RpmOptions)]
_lib.rpm_default_options.restype = None
_lib.rpm_lame_from_young.argtypes = [ctypes.c_double, ctypes.c_double, _dp, _dp]
_lib.rpm_workspace_size.argtypes = [_P(ctypes.c_int32), _P(RpmOptions), _P(ctypes.c_size_t)]
_lib.rpm_fft_apply.argtypes = [_P(RpmProblem), _dp, _P(RpmOptions), _vp, _vp, _dp, _dp, _vp, ctypes.c_size_t, _vp]
_lib.rpm_fft_apply_static.argtypes = [_P(RpmProblem), _dp, _P(RpmOptions), _vp, _vp, _dp, _dp, _vp]
_lib.rpm_fft_solve.argtypes = [_P(RpmProblem), _dp, _P(RpmOptions), _vp, _vp, _vp, _dp, _P(RpmStats), _vp,
                               ctypes.c_size_t, _vp]
_lib.rpm_fft_effective_tensor.argtypes = [_P(RpmProblem), _P(RpmOptions), _dp, _P(RpmStats), _vp, ctypes.c_size_t,
                                          _vp]
_lib.rpm_workspace_basis_dim.argtypes = [_vp, ctypes.c_size_t, _P(ctypes.c_int32), _vp]
_lib.rpm_fft_solve_stress.argtypes = [_P(RpmProblem), _dp, _P(RpmOptions), _vp, _vp, _dp, _dp, _P(RpmStats), _vp,
                                      ctypes.c_size_t, _vp]
_lib.rpm_fft_seed_basis.argtypes = [_P(RpmProblem), _P(RpmOptions), _vp, ctypes.c_int32, _P(ctypes.c_int32), _vp,
                                    ctypes.c_size_t, _vp]
_lib.rpm_workspace_h.argtypes = [_vp, ctypes.c_size_t, _dp, ctypes.c_int32, _P(ctypes.c_int32), _vp]
_lib.rpm_fft_autotune.argtypes = [_P(RpmProblem), _P(RpmOptions), ctypes.c_int32, _P(RpmTuning), _dp,
                                  _P(ctypes.c_int32), _vp, ctypes.c_size_t, _vp]
_lib.rpm_status_string.argtypes = [ctypes.c_int]
_lib.rpm_status_string.restype = ctypes.c_char_p
for _f in ("rpm_lame_from_young", "rpm_workspace_size", "rpm_fft_apply", "rpm_fft_apply_static", "rpm_fft_solve", "rpm_fft_effective_tensor",
           "rpm_workspace_basis_dim", "rpm_fft_seed_basis", "rpm_fft_solve_stress", "rpm_workspace_h",
           "rpm_fft_autotune"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTED_FNO = ["rpm_gemm_bf16", "rpm_fno_param_count", "rpm_fno_workspace_size", "rpm_fno_init", "rpm_fno_forward",
                "rpm_fno_backward", "rpm_fno_train_step", "rpm_fno_features", "rpm_fno_warm_start"]

EXPORTED = ["rpm_default_options", "rpm_lame_from_young", "rpm_workspace_size", "rpm_fft_apply",
            "rpm_fft_apply_static", "rpm_fft_solve",
            "rpm_fft_effective_tensor", "rpm_fft_solve_stress", "rpm_fft_seed_basis", "rpm_workspace_basis_dim",
            "rpm_workspace_h", "rpm_status_string", "rpm_fft_autotune"]


class RpmError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {status_string(code)} ({code})")
        self.code = code


def status_string(code):
    return _lib.rpm_status_string(int(code)).decode()


def lame_from_young(E, nu):
    lam = ctypes.c_double()
    mu = ctypes.c_double()
    rc = _lib.rpm_lame_from_young(float(E), float(nu), ctypes.byref(lam), ctypes.byref(mu))
    if rc != 0:
        raise RpmError(rc, "rpm_lame_from_young")
    return lam.value, mu.value


def make_options(**kw):
    o = RpmOptions()
    _lib.rpm_default_options(ctypes.byref(o))
    replay = kw.pop("replay", None)
    tuning = kw.pop("tuning", None)
    for k, v in kw.items():
        if k == "scheme" and isinstance(v, str):
            v = SCHEME[v]
        if k == "precision" and isinstance(v, str):
            v = PRECISION[v]
        if k == "map" and isinstance(v, str):
            v = MAP[v]
        setattr(o, k, v)
    keep = None
    if replay is not None and len(replay) > 0:
        keep = (ctypes.c_int32 * len(replay))(*[int(x) for x in replay])
        o.replay = ctypes.cast(keep, _P(ctypes.c_int32))
        o.replay_len = len(replay)
    o._keep = keep  # keep the replay array alive with the options
    if tuning is not None:
        t = tuning if isinstance(tuning, RpmTuning) else RpmTuning(**tuning)
        o.tuning = ctypes.pointer(t)
        o._keep_tuning = t
    return o


def field_dtype(opts):
    return torch.float64 if opts.precision == 0 else torch.float32


def _problem(phase, lame_tab, lame0):
    if not (isinstance(phase, torch.Tensor) and phase.is_cuda and phase.dtype == torch.uint8 and phase.dim() == 3):
        raise ValueError("phase must be a uint8 device tensor of shape (nz, ny, nx)")
    if not phase.is_contiguous():
        raise ValueError("phase must be contiguous")
    lt = np.ascontiguousarray(np.asarray(lame_tab, dtype=np.float64).reshape(-1, 2))
    pr = RpmProblem()
    nz, ny, nx = phase.shape
    pr.n[0], pr.n[1], pr.n[2] = nx, ny, nz
    pr.phase = phase.data_ptr()
    pr.n_phases = lt.shape[0]
    pr.lame = lt.ctypes.data_as(_dp)
    pr.lame0[0], pr.lame0[1] = float(lame0[0]), float(lame0[1])
    pr._keep = lt
    return pr


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def workspace_size(shape, opts):
    nz, ny, nx = shape
    n = (ctypes.c_int32 * 3)(nx, ny, nz)
    b = ctypes.c_size_t()
    rc = _lib.rpm_workspace_size(n, ctypes.byref(opts), ctypes.byref(b))
    if rc != 0:
        raise RpmError(rc, "rpm_workspace_size")
    return b.value


def make_workspace(shape, opts, device="cuda"):
    return torch.empty(workspace_size(shape, opts), dtype=torch.uint8, device=device)


def _check_field(t, shape, dtype, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} device tensor")
    if tuple(t.shape) != (6,) + tuple(shape):
        raise ValueError(f"{name} must have shape {(6,) + tuple(shape)}")


def fft_apply(phase, lame_tab, lame0, E, eps, opts=None, workspace=None):
    """xi = F(eps; E) (Algorithm 1, one map application), its error and <sigma>."""
    opts = opts or make_options()
    shape = tuple(phase.shape)
    _check_field(eps, shape, field_dtype(opts), "eps")
    ws = workspace if workspace is not None else make_workspace(shape, opts)
    xi = torch.empty_like(eps)
    pr = _problem(phase, lame_tab, lame0)
    Ea = (ctypes.c_double * 6)(*[float(x) for x in E])
    err = ctypes.c_double()
    sav = (ctypes.c_double * 6)()
    rc = _lib.rpm_fft_apply(ctypes.byref(pr), Ea, ctypes.byref(opts), eps.data_ptr(), xi.data_ptr(),
                            ctypes.byref(err), sav, ws.data_ptr(), ws.numel(), _stream())
    if rc != 0:
        raise RpmError(rc, "rpm_fft_apply")
    return xi, err.value, np.array(sav[:])


def autotune(phase, lame_tab, lame0, opts=None, reps=10, workspace=None):
    """Launch shape of the pencil passes that maps fastest on this grid
    (rpm_fft_autotune): dict(tuning=RpmTuning, ms=time per map, candidates=n)."""
    opts = opts or make_options()
    shape = tuple(phase.shape)
    ws = workspace if workspace is not None else make_workspace(shape, opts)
    pr = _problem(phase, lame_tab, lame0)
    best = RpmTuning()
    ms = ctypes.c_double()
    nc = ctypes.c_int32()
    rc = _lib.rpm_fft_autotune(ctypes.byref(pr), ctypes.byref(opts), int(reps), ctypes.byref(best), ctypes.byref(ms),
                               ctypes.byref(nc), ws.data_ptr(), ws.numel(), _stream())
    if rc != 0:
        raise RpmError(rc, "rpm_fft_autotune")
    return dict(tuning=best, ms=ms.value, candidates=nc.value)


def fft_apply_static(phase, lame_tab, lame0, E, eps, opts=None, xi=None):
    """fft_apply without a workspace: the library's static device scratch serves
    the call (rpm_fft_apply_static).  xi (nullable) is the caller's output."""
    opts = opts or make_options()
    shape = tuple(phase.shape)
    _check_field(eps, shape, field_dtype(opts), "eps")
    if xi is None:
        xi = torch.empty_like(eps)
    _check_field(xi, shape, field_dtype(opts), "xi")
    pr = _problem(phase, lame_tab, lame0)
    Ea = (ctypes.c_double * 6)(*[float(x) for x in E])
    err = ctypes.c_double()
    sav = (ctypes.c_double * 6)()
    rc = _lib.rpm_fft_apply_static(ctypes.byref(pr), Ea, ctypes.byref(opts), eps.data_ptr(), xi.data_ptr(),
                                   ctypes.byref(err), sav, _stream())
    if rc != 0:
        raise RpmError(rc, "rpm_fft_apply_static")
    return xi, err.value, np.array(sav[:])


def _stats_dict(st, hist, dec):
    it = st.iterations
    return dict(iterations=it, jvps=st.jvps, basis_dim=st.basis_dim, growth_events=st.growth_events,
                residual=st.residual, residual_fp64=st.residual_fp64, refinements=st.refinements,
                seconds=st.seconds,
                history=hist[:min(it, hist.size)].copy() if hist is not None else None,
                decisions=dec[:min(st.growth_events, dec.size)].copy() if dec is not None else None,
                kernel_ms={KERNEL_NAMES[k]: st.kernel_ms[k] for k in range(RPM_NKERNEL)},
                kernel_launches={KERNEL_NAMES[k]: st.kernel_launches[k] for k in range(RPM_NKERNEL)},
                kernel_bytes={KERNEL_NAMES[k]: st.kernel_bytes[k] for k in range(RPM_NKERNEL)})


def _new_stats(hist_cap):
    st = RpmStats()
    hist = np.zeros(max(hist_cap, 1))
    dec = np.zeros(4096, dtype=np.int32)
    st.history = hist.ctypes.data_as(_dp)
    st.history_cap = hist_cap
    st.decisions = dec.ctypes.data_as(_P(ctypes.c_int32))
    st.decisions_cap = dec.size
    return st, hist, dec


def fft_solve(phase, lame_tab, lame0, E, opts=None, eps0=None, workspace=None, want_eps=True, want_sig=False,
              history_cap=100000, check=True):
    """Solve for mean strain E (Algorithm 1 or 2).  Returns a dict with status, eps,
    sig (optional), sig_avg and the statistics."""
    opts = opts or make_options()
    shape = tuple(phase.shape)
    dt = field_dtype(opts)
    ws = workspace if workspace is not None else make_workspace(shape, opts)
    if eps0 is not None:
        _check_field(eps0, shape, dt, "eps0")
    eps = torch.empty((6,) + shape, dtype=dt, device=phase.device) if want_eps else None
    sig = torch.empty((6,) + shape, dtype=dt, device=phase.device) if want_sig else None
    pr = _problem(phase, lame_tab, lame0)
    Ea = (ctypes.c_double * 6)(*[float(x) for x in E])
    sav = (ctypes.c_double * 6)()
    st, hist, dec = _new_stats(history_cap)
    rc = _lib.rpm_fft_solve(ctypes.byref(pr), Ea, ctypes.byref(opts), eps0.data_ptr() if eps0 is not None else None,
                            eps.data_ptr() if eps is not None else None, sig.data_ptr() if sig is not None else None,
                            sav, ctypes.byref(st), ws.data_ptr(), ws.numel(), _stream())
    if rc < 0 and check:
        raise RpmError(rc, "rpm_fft_solve")
    out = _stats_dict(st, hist, dec)
    out.update(status=status_string(rc), code=rc, eps=eps, sig=sig, sig_avg=np.array(sav[:]), workspace=ws)
    return out


def effective_tensor(phase, lame_tab, lame0, opts=None, workspace=None, history_cap=100000):
    """Effective stiffness (Voigt, engineering shear); 6x6 in 3-D, 3x3 (11, 22, 12) in 2-D."""
    opts = opts or make_options()
    shape = tuple(phase.shape)
    two_d = shape[0] == 1
    nc = 3 if two_d else 6
    ws = workspace if workspace is not None else make_workspace(shape, opts)
    pr = _problem(phase, lame_tab, lame0)
    C = (ctypes.c_double * (nc * nc))()
    sts = (RpmStats * nc)()
    keep = []
    for i in range(nc):
        hist = np.zeros(history_cap)
        dec = np.zeros(4096, dtype=np.int32)
        sts[i].history = hist.ctypes.data_as(_dp)
        sts[i].history_cap = history_cap
        sts[i].decisions = dec.ctypes.data_as(_P(ctypes.c_int32))
        sts[i].decisions_cap = dec.size
        keep.append((hist, dec))
    rc = _lib.rpm_fft_effective_tensor(ctypes.byref(pr), ctypes.byref(opts), C, sts, ws.data_ptr(), ws.numel(),
                                       _stream())
    if rc < 0:
        raise RpmError(rc, "rpm_fft_effective_tensor")
    stats = [_stats_dict(sts[i], keep[i][0], keep[i][1]) for i in range(nc)]
    return np.array(C[:]).reshape(nc, nc), stats, status_string(rc)


def fft_solve_stress(phase, lame_tab, lame0, Sigma, opts=None, workspace=None, want_eps=True, want_sig=False,
                     history_cap=100000):
    """Solve for a prescribed mean stress Sigma (rpm_fft_solve_stress).  Returns a
    dict with status, eps, sig (optional), sig_avg, E (the mean strain found) and
    the statistics of the unit load cases and of the final solve."""
    opts = opts or make_options()
    shape = tuple(phase.shape)
    dt = field_dtype(opts)
    ws = workspace if workspace is not None else make_workspace(shape, opts)
    eps = torch.empty((6,) + shape, dtype=dt, device=phase.device) if want_eps else None
    sig = torch.empty((6,) + shape, dtype=dt, device=phase.device) if want_sig else None
    pr = _problem(phase, lame_tab, lame0)
    Sa = (ctypes.c_double * 6)(*[float(x) for x in Sigma])
    sav = (ctypes.c_double * 6)()
    Eo = (ctypes.c_double * 6)()
    ns = 4 if shape[0] == 1 else 7
    sts = (RpmStats * ns)()
    keep = []
    for i in range(ns):
        hist = np.zeros(history_cap)
        dec = np.zeros(4096, dtype=np.int32)
        sts[i].history = hist.ctypes.data_as(_dp)
        sts[i].history_cap = history_cap
        sts[i].decisions = dec.ctypes.data_as(_P(ctypes.c_int32))
        sts[i].decisions_cap = dec.size
        keep.append((hist, dec))
    rc = _lib.rpm_fft_solve_stress(ctypes.byref(pr), Sa, ctypes.byref(opts),
                                   eps.data_ptr() if eps is not None else None,
                                   sig.data_ptr() if sig is not None else None, sav, Eo, sts, ws.data_ptr(),
                                   ws.numel(), _stream())
    if rc < 0:
        raise RpmError(rc, "rpm_fft_solve_stress")
    stats = [_stats_dict(sts[i], keep[i][0], keep[i][1]) for i in range(ns)]
    return dict(status=status_string(rc), code=rc, eps=eps, sig=sig, sig_avg=np.array(sav[:]), E=np.array(Eo[:]),
                cases=stats[:-1], final=stats[-1], workspace=ws)


def seed_basis(phase, lame_tab, lame0, V, opts, workspace):
    """Append the fields V (k, 6, nz, ny, nx; device, field dtype) to the workspace's
    basis (rpm_fft_seed_basis; opts.reuse_basis keeps the basis already held).
    Returns the basis dimension afterwards."""
    shape = tuple(phase.shape)
    dt = field_dtype(opts)
    if not (isinstance(V, torch.Tensor) and V.is_cuda and V.dtype == dt and V.is_contiguous()
            and tuple(V.shape[1:]) == (6,) + shape):
        raise ValueError(f"V must be a contiguous {dt} device tensor of shape (k, 6) + {shape}")
    pr = _problem(phase, lame_tab, lame0)
    p = ctypes.c_int32()
    rc = _lib.rpm_fft_seed_basis(ctypes.byref(pr), ctypes.byref(opts), V.data_ptr() if V.shape[0] else None,
                                 V.shape[0], ctypes.byref(p), workspace.data_ptr(), workspace.numel(), _stream())
    if rc < 0:
        raise RpmError(rc, "rpm_fft_seed_basis")
    return p.value


def basis_dim(workspace):
    p = ctypes.c_int32()
    rc = _lib.rpm_workspace_basis_dim(workspace.data_ptr(), workspace.numel(), ctypes.byref(p), _stream())
    if rc != 0:
        raise RpmError(rc, "rpm_workspace_basis_dim")
    return p.value


def workspace_h(workspace):
    """H = Z^T F_u Z of the basis a workspace holds (p x p numpy array)."""
    H = np.zeros((64, 64))
    p = ctypes.c_int32()
    rc = _lib.rpm_workspace_h(ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), H.ctypes.data_as(_dp), 64,
                              ctypes.byref(p), _stream())
    if rc != 0:
        raise RpmError(rc, "rpm_workspace_h")
    return H[:p.value, :p.value].copy()


# --------------------------------------------------------------------------- learned warm start (rpmfno.h)

class FnoConfig(ctypes.Structure):
    _fields_ = [("c_in", ctypes.c_int32), ("c_out", ctypes.c_int32), ("width", ctypes.c_int32),
                ("layers", ctypes.c_int32), ("modes", ctypes.c_int32)]


_i64p = _P(ctypes.c_int64)
_fp = _vp
_lib.rpm_gemm_bf16.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _i64p, _vp, _i64p,
                               _vp, _i64p, ctypes.c_float, ctypes.c_float, _vp]
_lib.rpm_fno_param_count.argtypes = [_P(FnoConfig), _i64p]
_lib.rpm_fno_workspace_size.argtypes = [_P(FnoConfig), _P(ctypes.c_int32), ctypes.c_int32, _P(ctypes.c_size_t)]
_lib.rpm_fno_init.argtypes = [_P(FnoConfig), ctypes.c_uint64, _vp, _vp]
_lib.rpm_fno_forward.argtypes = [_P(FnoConfig), _vp, _P(ctypes.c_int32), ctypes.c_int32, _vp, _vp, _vp,
                                 ctypes.c_size_t, _vp]
_lib.rpm_fno_backward.argtypes = [_P(FnoConfig), _vp, _P(ctypes.c_int32), ctypes.c_int32, _vp, _vp, _vp, _vp, _vp,
                                  ctypes.c_size_t, _vp]
_lib.rpm_fno_train_step.argtypes = [_P(FnoConfig), _vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_float,
                                    _P(ctypes.c_int32), ctypes.c_int32, _vp, _vp, _dp, _vp, ctypes.c_size_t, _vp]
_lib.rpm_fno_features.argtypes = [_P(RpmProblem), _vp, _vp]
_lib.rpm_fno_warm_start.argtypes = [_P(FnoConfig), _vp, _P(RpmProblem), _dp, ctypes.c_int32, _vp, _vp,
                                    ctypes.c_size_t, _vp]
for _f in EXPORTED_FNO:
    getattr(_lib, _f).restype = ctypes.c_int


def fno_config(c_in=2, c_out=36, width=32, layers=4, modes=12):
    return FnoConfig(c_in, c_out, width, layers, modes)


def _grid(shape):
    nz, ny, nx = shape
    return (ctypes.c_int32 * 3)(nx, ny, nz)


def _f32(t, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 device tensor")
    return t.data_ptr()


def gemm_bf16(A, sA, B, sB, C, sC, M, N, K, batch=1, alpha=1.0, beta=0.0):
    """rpm_gemm_bf16 on float32 device tensors with element strides (sA, sB, sC: 3 each)."""
    rc = _lib.rpm_gemm_bf16(M, N, K, batch, _f32(A, "A"), (ctypes.c_int64 * 3)(*sA), _f32(B, "B"),
                            (ctypes.c_int64 * 3)(*sB), _f32(C, "C"), (ctypes.c_int64 * 3)(*sC), alpha, beta, _stream())
    if rc != 0:
        raise RpmError(rc, "rpm_gemm_bf16")
    return C


def fno_param_count(cfg):
    c = ctypes.c_int64()
    rc = _lib.rpm_fno_param_count(ctypes.byref(cfg), ctypes.byref(c))
    if rc != 0:
        raise RpmError(rc, "rpm_fno_param_count")
    return c.value


def fno_workspace(cfg, shape, batch, device="cuda"):
    b = ctypes.c_size_t()
    rc = _lib.rpm_fno_workspace_size(ctypes.byref(cfg), _grid(shape), batch, ctypes.byref(b))
    if rc != 0:
        raise RpmError(rc, "rpm_fno_workspace_size")
    return torch.empty(b.value, dtype=torch.uint8, device=device)


def fno_init(cfg, seed, device="cuda"):
    p = torch.empty(fno_param_count(cfg), dtype=torch.float32, device=device)
    rc = _lib.rpm_fno_init(ctypes.byref(cfg), seed, p.data_ptr(), _stream())
    if rc != 0:
        raise RpmError(rc, "rpm_fno_init")
    return p


def fno_forward(cfg, params, x, workspace=None):
    """x: (batch, c_in, nz, ny, nx) float32 device tensor; returns y (batch, c_out, nz, ny, nx)."""
    B, _, nz, ny, nx = x.shape
    ws = workspace if workspace is not None else fno_workspace(cfg, (nz, ny, nx), B, x.device)
    y = torch.empty((B, cfg.c_out, nz, ny, nx), dtype=torch.float32, device=x.device)
    rc = _lib.rpm_fno_forward(ctypes.byref(cfg), _f32(params, "params"), _grid((nz, ny, nx)), B, _f32(x, "x"),
                              y.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
    if rc != 0:
        raise RpmError(rc, "rpm_fno_forward")
    return y, ws


def fno_backward(cfg, params, x, dy, workspace, want_dx=False):
    """Parameter gradient (and input gradient) of sum(dy * y) after fno_forward on workspace."""
    B, _, nz, ny, nx = x.shape
    g = torch.empty_like(params)
    dx = torch.empty_like(x) if want_dx else None
    rc = _lib.rpm_fno_backward(ctypes.byref(cfg), _f32(params, "params"), _grid((nz, ny, nx)), B, _f32(x, "x"),
                               _f32(dy, "dy"), g.data_ptr(), dx.data_ptr() if dx is not None else None,
                               workspace.data_ptr(), workspace.numel(), _stream())
    if rc != 0:
        raise RpmError(rc, "rpm_fno_backward")
    return g, dx


def fno_train_step(cfg, params, grad, m, v, step, lr, x, target, workspace):
    B, _, nz, ny, nx = x.shape
    loss = ctypes.c_double()
    rc = _lib.rpm_fno_train_step(ctypes.byref(cfg), _f32(params, "params"), _f32(grad, "grad"), _f32(m, "m"),
                                 _f32(v, "v"), step, lr, _grid((nz, ny, nx)), B, _f32(x, "x"),
                                 _f32(target, "target"), ctypes.byref(loss), workspace.data_ptr(), workspace.numel(),
                                 _stream())
    if rc != 0:
        raise RpmError(rc, "rpm_fno_train_step")
    return loss.value


def fno_features(phase, lame_tab):
    pr = _problem(phase, lame_tab, (1.0, 1.0))
    nz, ny, nx = phase.shape
    x = torch.empty((2, nz, ny, nx), dtype=torch.float32, device=phase.device)
    rc = _lib.rpm_fno_features(ctypes.byref(pr), x.data_ptr(), _stream())
    if rc != 0:
        raise RpmError(rc, "rpm_fno_features")
    return x


def fno_warm_start(cfg, params, phase, lame_tab, lame0, E, precision="fp64", workspace=None):
    """Starting strain E + predicted fluctuation for rpm_fft_solve's eps0."""
    pr = _problem(phase, lame_tab, lame0)
    shape = tuple(phase.shape)
    ws = workspace if workspace is not None else fno_workspace(cfg, shape, 1, phase.device)
    dt = torch.float64 if precision == "fp64" else torch.float32
    eps0 = torch.empty((6,) + shape, dtype=dt, device=phase.device)
    Ea = (ctypes.c_double * 6)(*[float(e) for e in E])
    rc = _lib.rpm_fno_warm_start(ctypes.byref(cfg), _f32(params, "params"), ctypes.byref(pr), Ea, PRECISION[precision],
                                 eps0.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
    if rc != 0:
        raise RpmError(rc, "rpm_fno_warm_start")
    return eps0
