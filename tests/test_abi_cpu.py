"""C-ABI checks that need no GPU: the library loads, exports every declared entry
point, and rejects bad arguments before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("rpmfft.h", "rpmfno.h")]
LIB = os.path.join(ROOT, "paper_2003_07720_amd", "librpmfft.so")


@pytest.fixture(scope="module")
def B():
    if not os.path.exists(LIB):
        import __graft_entry__

        __graft_entry__.build()
    from paper_2003_07720_amd import binding

    return binding


def declared_functions():
    txt = "".join(open(h).read() for h in HEADERS)
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rpm_[a-z_0-9]+)\s*\(", txt)))


def test_header_symbols_exported(B):
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 8
    for n in names:
        assert hasattr(lib, n), f"{n} declared in rpmfft.h but not exported"
    assert sorted(B.EXPORTED + B.EXPORTED_FNO) == names


def test_default_options_and_status_strings(B):
    o = B.make_options()
    assert o.tol == 1e-6 and o.max_iter == 10000 and o.n_max == 10 and o.p_max == 32
    assert abs(o.kappa - 0.1) < 1e-15 and o.scheme == 1 and o.precision == 0 and o.check_every == 16
    assert o.map == 0 and o.alpha == 2.0 and o.beta == 2.0
    assert o.profile == 0 and o.profile_classes == 0 and o.profile_every == 1 and not o.tuning
    for code, name in B.STATUS.items():
        assert B.status_string(code) == name
    assert B.status_string(99) == "RPM_UNKNOWN"


def test_lame_from_young(B):
    lam, mu = B.lame_from_young(1.0, 0.3)
    assert abs(lam - 0.3 / (1.3 * 0.4)) < 1e-15 and abs(mu - 1.0 / 2.6) < 1e-15
    with pytest.raises(B.RpmError):
        B.lame_from_young(1.0, 0.5)
    with pytest.raises(B.RpmError):
        B.lame_from_young(float("nan"), 0.3)


def test_workspace_size_rules(B):
    o = B.make_options()
    for shape in [(1, 32, 32), (64, 64, 64), (128, 128, 128), (4, 6, 8), (96, 48, 12)]:
        assert B.workspace_size(shape, o) > 0
    for bad in [(1, 32, 5), (64, 7, 64), (1, 1, 32), (1024, 8, 8), (0, 8, 8)]:
        with pytest.raises(B.RpmError) as e:
            B.workspace_size(bad, o)
        assert e.value.code == -2
    # basis storage grows with p_max; fp32 fields are smaller than fp64
    s0 = B.workspace_size((32, 32, 32), B.make_options(p_max=0))
    s8 = B.workspace_size((32, 32, 32), B.make_options(p_max=8))
    assert s8 > s0 + 2 * 8 * 6 * 32 ** 3 * 8 - 1
    assert B.workspace_size((32, 32, 32), B.make_options(precision="fp32")) < B.workspace_size((32, 32, 32), o)
    with pytest.raises(B.RpmError):
        B.workspace_size((8, 8, 8), B.make_options(p_max=65))
    # only the error history (one double per main-loop F call) follows max_iter,
    # so calls that carry the basis may take different caps
    for prec in ("fp64", "fp32"):
        a = B.workspace_size((32, 32, 32), B.make_options(precision=prec, max_iter=1000))
        b = B.workspace_size((32, 32, 32), B.make_options(precision=prec, max_iter=1000 + 4096))
        assert b - a == 8 * 4096
    # the polarization iteration carries eps through the forward passes: twice the spectra
    sp = B.workspace_size((32, 32, 32), B.make_options(map="polarization"))
    assert sp >= B.workspace_size((32, 32, 32), o) + 2 * 6 * 17 * 32 * 32 * 16
    # its 12-component gamma tiles bound the FP64 pencil length (FP32 certifies in FP64)
    with pytest.raises(B.RpmError) as e:
        B.workspace_size((256, 8, 8), B.make_options(map="polarization"))
    assert e.value.code == -2


def _raw_problem(B, n=(8, 8, 8), lame=((1.0, 1.0),), lame0=(1.0, 1.0)):
    pr = B.RpmProblem()
    pr.n[0], pr.n[1], pr.n[2] = n
    pr.phase = 0x1000  # never dereferenced: every case below fails validation first
    lt = np.array(lame, dtype=np.float64)
    pr.n_phases = lt.shape[0]
    pr.lame = lt.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    pr.lame0[0], pr.lame0[1] = lame0
    pr._keep = lt
    return pr


@pytest.mark.parametrize("case", ["tol", "nan_E", "pmax", "mu0", "neg_mu", "scheme", "check", "size", "nphase",
                                  "workspace", "kappa", "replay", "map", "alpha", "classes", "every", "tune_neg",
                                  "tune_cols", "tune_wide", "tune_regs_neg", "tune_regs_2", "tune_regs_grid"])
def test_solve_rejects_bad_arguments_before_device_work(B, case):
    lib = B._lib
    o = B.make_options()
    pr = _raw_problem(B)
    E = (ctypes.c_double * 6)(0.01, 0, 0, 0, 0, 0)
    ws, wsb = 0x2000, 1 << 40
    expect = -1
    if case == "tol":
        o.tol = 0.0
    elif case == "nan_E":
        E[2] = float("nan")
    elif case == "pmax":
        o.p_max = 65
    elif case == "mu0":
        pr = _raw_problem(B, lame0=(1.0, 0.0))
    elif case == "neg_mu":
        pr = _raw_problem(B, lame=((1.0, -0.1),))
    elif case == "scheme":
        o.scheme = 7
    elif case == "check":
        o.check_every = 0
    elif case == "size":
        pr = _raw_problem(B, n=(8, 10, 8))
        expect = -2
    elif case == "nphase":
        pr.n_phases = 0
    elif case == "workspace":
        ws, wsb = None, 0
        expect = -3
    elif case == "kappa":
        o.kappa = 1.5
    elif case == "map":
        o.map = 3
    elif case == "alpha":
        o.map = 1
        o.alpha = -1.0
    elif case == "replay":
        o.replay_len = 3
    elif case == "classes":
        o.profile = 1
        o.profile_classes = 1 << B.RPM_NKERNEL
    elif case == "every":
        o.profile = 1
        o.profile_every = -2
    elif case == "tune_neg":
        tn = B.RpmTuning(0, -256, 0)
        o.tuning = ctypes.pointer(tn)
    elif case == "tune_cols":  # not a divisor of nz = 8
        tn = B.RpmTuning(3, 0, 0)
        o.tuning = ctypes.pointer(tn)
    elif case == "tune_wide":  # more z positions per y tile than the pass holds
        tn = B.RpmTuning(64, 0, 0)
        pr = _raw_problem(B, n=(64, 64, 64))
        o.tuning = ctypes.pointer(tn)
    elif case == "tune_regs_neg":
        tn = B.RpmTuning(0, 0, 0, -1)
        o.tuning = ctypes.pointer(tn)
    elif case == "tune_regs_2":
        tn = B.RpmTuning(0, 0, 0, 2)
        o.tuning = ctypes.pointer(tn)
    elif case == "tune_regs_grid":  # register y transforms need ny = 128 (here 8)
        tn = B.RpmTuning(0, 0, 0, 1)
        o.tuning = ctypes.pointer(tn)
    rc = lib.rpm_fft_solve(ctypes.byref(pr), E, ctypes.byref(o), None, None, None, None, None, ws, wsb, None)
    assert rc == expect, (case, rc)
    rc = lib.rpm_fft_effective_tensor(ctypes.byref(pr), ctypes.byref(o), (ctypes.c_double * 36)(), None, ws, wsb,
                                      None)
    if case != "nan_E":
        assert rc == expect, (case, rc)


def test_seed_basis_rejects_bad_arguments(B):
    lib = B._lib
    pr = _raw_problem(B)
    p = ctypes.c_int32(-7)
    o = B.make_options()
    assert lib.rpm_fft_seed_basis(ctypes.byref(pr), ctypes.byref(o), 0x3000, -1, ctypes.byref(p), 0x2000, 1 << 40,
                                  None) == -1
    assert lib.rpm_fft_seed_basis(ctypes.byref(pr), ctypes.byref(o), None, 2, ctypes.byref(p), 0x2000, 1 << 40,
                                  None) == -1
    ob = B.make_options(scheme="basic")
    assert lib.rpm_fft_seed_basis(ctypes.byref(pr), ctypes.byref(ob), 0x3000, 1, ctypes.byref(p), 0x2000, 1 << 40,
                                  None) == -1
    o.tol = 0.0
    assert lib.rpm_fft_seed_basis(ctypes.byref(pr), ctypes.byref(o), 0x3000, 1, ctypes.byref(p), 0x2000, 1 << 40,
                                  None) == -1
    assert p.value == -7  # untouched


def test_solve_stress_rejects_bad_arguments(B):
    lib = B._lib
    pr = _raw_problem(B)
    o = B.make_options()
    S = (ctypes.c_double * 6)(0.01, 0, 0, float("nan"), 0, 0)
    assert lib.rpm_fft_solve_stress(ctypes.byref(pr), S, ctypes.byref(o), None, None, None, None, None, 0x2000,
                                    1 << 40, None) == -1
    assert lib.rpm_fft_solve_stress(ctypes.byref(pr), None, ctypes.byref(o), None, None, None, None, None, 0x2000,
                                    1 << 40, None) == -1
    S[3] = 0.0
    o.tol = -1.0
    assert lib.rpm_fft_solve_stress(ctypes.byref(pr), S, ctypes.byref(o), None, None, None, None, None, 0x2000,
                                    1 << 40, None) == -1


def test_apply_rejects_aliasing_and_nulls(B):
    lib = B._lib
    o = B.make_options()
    pr = _raw_problem(B)
    E = (ctypes.c_double * 6)(0.01, 0, 0, 0, 0, 0)
    assert lib.rpm_fft_apply(ctypes.byref(pr), E, ctypes.byref(o), 0x3000, 0x3000, None, None, 0x2000, 1 << 40,
                             None) == -1
    assert lib.rpm_fft_apply(ctypes.byref(pr), E, ctypes.byref(o), None, 0x3000, None, None, 0x2000, 1 << 40,
                             None) == -1
    assert lib.rpm_fft_apply(None, E, ctypes.byref(o), 0x3000, 0x4000, None, None, 0x2000, 1 << 40, None) == -1


def test_table1_fixture():
    """The stored Table 1 of Sec. 5.5 (context for the contrast sweep): six contrasts,
    RPM around the Accelerated FFT needing fewer iterations and less time at each."""
    import bench

    t = bench.table1_paper()
    assert sorted(t) == [500, 1000, 5000, 10000, 50000, 100000]
    for K, (acc_it, rpm_it, acc_s, rpm_s) in t.items():
        assert rpm_it < acc_it and rpm_s < acc_s
    assert t[10000] == (1136, 82, 28.29, 4.44)


def test_apply_static_rejects_before_device_work(B):
    """The allocation-free map application refuses, with no device work, grids
    that need more than its static scratch, and the same bad arguments as
    rpm_fft_apply."""
    lib = B._lib
    pr = _raw_problem(B)
    E = (ctypes.c_double * 6)(0.01, 0, 0, 0, 0, 0)
    o = B.make_options(precision="fp64")
    assert lib.rpm_fft_apply_static(ctypes.byref(pr), E, ctypes.byref(o), 0x3000, 0x3000, None, None, None) == -1
    assert lib.rpm_fft_apply_static(ctypes.byref(pr), E, ctypes.byref(o), None, 0x3000, None, None, None) == -1
    big = _raw_problem(B)
    big.n[0], big.n[1], big.n[2] = 256, 256, 256
    for prec in ("fp64", "fp32"):
        o = B.make_options(precision=prec)
        assert lib.rpm_fft_apply_static(ctypes.byref(big), E, ctypes.byref(o), 0x3000, 0x4000, None, None,
                                        None) == -6
    big.n[0], big.n[1], big.n[2] = 128, 128, 128
    o = B.make_options(precision="fp64")  # 128^3 spectra in FP64 exceed the array
    assert lib.rpm_fft_apply_static(ctypes.byref(big), E, ctypes.byref(o), 0x3000, 0x4000, None, None, None) == -6
    assert B.status_string(-6) == "RPM_E_SCRATCH"


@pytest.mark.parametrize("case", ["reps0", "reps_big", "no_best", "bad_tuning_ignored"])
def test_autotune_rejects_bad_arguments(B, case):
    """rpm_fft_autotune validates before any device work; o->tuning is ignored."""
    lib = B._lib
    o = B.make_options()
    pr = _raw_problem(B)
    best = B.RpmTuning()
    reps, bp = 5, ctypes.byref(best)
    ws, wsb = 0x2000, 1 << 40
    expect = -1
    if case == "reps0":
        reps = 0
    elif case == "reps_big":
        reps = 1001
    elif case == "no_best":
        bp = None
    elif case == "bad_tuning_ignored":
        tn = B.RpmTuning(3, 0, 0)  # would be rejected by a solve
        o.tuning = ctypes.pointer(tn)
        ws, wsb = None, 0
        expect = -3  # the workspace check is reached: the tuning was not applied
    rc = lib.rpm_fft_autotune(ctypes.byref(pr), ctypes.byref(o), reps, bp, None, None, ws, wsb, None)
    assert rc == expect, (case, rc)
