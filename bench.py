"""Benchmark: voxel-iterations/s and time to a 1e-6 equilibrium error of RPM-FFT
on the 128^3 void cell (30 % spherical voids of stiffness 1e-8, matrix E = 1,
nu = 0.3, mean strain eps_zz = 0.01), FP32 fields and FFTs with FP64 RPM steps,
basis capped at 32, n_max = 10, reference medium at the arithmetic mean.

A step is one iteration of the solver at its steady state: one application of
the fixed-point map with the RPM recombination, projections and Newton step on
a basis of p_max columns.  An untimed solve builds the basis; the timed region
is one solve of exactly K steps that carries it (no growth inside the window);
value = voxels x (steps + JVP map applications) / s.  The growth events, the
time to tolerance, the small configurations (32^2 disk, 64^3 spheres) and the
CPU oracle legs are reported beside it.

Prints one JSON line (see the keys below).  --gpus above 1 is refused: this
build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0

# HBM traffic of the kernel classes, measured with hardware counters
# (rocprofv3 FETCH_SIZE / WRITE_SIZE) and written by --traffic-from; it is only
# reported while the kernel sources are the ones it was measured on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_128cube_voids_fp32.json")
KERNEL_SOURCES = ["include/rpmfft.h", "paper_2003_07720_amd/csrc/rpm_device.h",
                  "paper_2003_07720_amd/csrc/rpm_kernels.h", "paper_2003_07720_amd/csrc/rpm_solver.hip"]
# kernel symbols behind each timing class of rpm_stats ({T}: float or double)
CLASS_SYMBOLS = {
    "xfwd": r"rpm::k_xfwd<{T}, (true|false), false(, \d+)?(, (true|false)){0,3}>",
    "yfwd": r"rpm::k_ypipe<{T}, -1, \d+(, (true|false))?>|rpm::k_yfwd<{T}>|rpm::k_ywave<-1>",
    "gamma": r"rpm::k_(gamma|gpipe)<{T}, false(, (true|false))?>",
    "yinv": r"rpm::k_ypipe<{T}, 1, \d+(, (true|false))?>|rpm::k_yinv<{T}>|rpm::k_ywave<1>",
    "xinv": r"rpm::k_xinv<{T}, false(, \d+)?(, (true|false))?>",
    "project": r"rpm::k_gdots(_split)?<{T}, {T}, [12], 0(, \d+, \d+)?>",
    "recombine": r"rpm::k_recombine(_split)?<{T}(, \d+, \d+)?>",
}


def source_digest():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_from(fetch_csv, write_csv, copy_mib, steps, seed, out_path, precision, n, p):
    """Per-launch HBM bytes of each kernel class in the steady-state window (the
    last `steps` dispatches of the class: the timed solve, basis at p_max) from
    two rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE, KiB per
    dispatch), each scaled by what the same counter reads for the plain copy of
    copy_mib MiB that --calibrate-copy-mib appends to the run."""
    import csv
    import re

    def load(path, counter):
        rows = []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    rows.append((int(r.get("Dispatch_Id", len(rows))), r["Kernel_Name"],
                                 float(r["Counter_Value"]) * 1024.0))
        rows.sort()
        return [(k, v) for _, k, v in rows]

    T = "float" if precision == "fp32" else "double"
    copy_bytes = copy_mib * float(1 << 20)
    out = {"workload": f"{n}^3 voids {precision} (bench.py defaults), steady state at p_max", "steps": steps,
           "seed": seed, "precision": precision, "n": n, "p": p, "copy_mib": copy_mib,
           "source_sha256": source_digest(),
           "classes": {}}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = load(path, counter)
        # the calibration copies are the three largest copy dispatches
        copies = sorted(v for k, v in rows if "copyBuffer" in k)[-3:]
        scale = copy_bytes / (sum(copies) / len(copies))
        out[counter.lower() + "_scale"] = scale
        for cls, pat in CLASS_SYMBOLS.items():
            pat = pat.replace("{T}", T)
            vals = [v for k, v in rows if re.search(pat, k.split("(")[0])][-steps:]
            if not vals:
                continue
            c = out["classes"].setdefault(cls, {"dispatches": len(vals)})
            c[counter.lower() + "_bytes_per_launch"] = scale * sum(vals) / len(vals)
    for c in out["classes"].values():
        c["traffic_bytes_per_launch"] = c.get("fetch_size_bytes_per_launch", 0.0) + c.get(
            "write_size_bytes_per_launch", 0.0)
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def measured_traffic(cls, seed, precision, n, p):
    """Counter-measured bytes per launch of a class in the steady state (basis at
    p_max), or None when absent or measured on other sources, another cell or
    another precision.  Steady-state launches of a class all move the same bytes,
    so the figure does not depend on the number of steps."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if (t.get("source_sha256") != source_digest() or t.get("seed") != seed or t.get("precision") != precision
            or t.get("n") != n or t.get("p") != p):
        return None
    c = t.get("classes", {}).get(cls)
    return None if c is None else c.get("traffic_bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--seed", type=int, default=3000)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--ttt-iters", type=int, default=4000, help="iteration cap of the time-to-tolerance solves")
    ap.add_argument("--ttt-loose", default="1e-2,3e-3",
                    help="looser tolerances timed for RPM and the basic scheme (comma list, '' = none)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-tolerance solve")
    ap.add_argument("--no-small", action="store_true", help="skip the 32^2 disk and 64^3 sphere rows")
    ap.add_argument("--no-warm", action="store_true", help="skip training and timing the learned warm start")
    ap.add_argument("--warm-cells", type=int, default=64, help="solver-generated training cells (32^3)")
    ap.add_argument("--warm-steps", type=int, default=800, help="training steps of the warm-start network")
    ap.add_argument("--warm-eval-cells", type=int, default=0,
                    help="also evaluate the warm start on this many held-out 128^3 void cells (other seeds, void "
                         "stiffness 1e-3, to the tolerance)")
    ap.add_argument("--cpu-steps", type=int, default=14, help="oracle map applications in the CPU sample")
    ap.add_argument("--cpu-c2-maps", type=int, default=4,
                    help="single-threaded oracle map applications sampled on the 64^3 spheres")
    ap.add_argument("--p-max", type=int, default=32, help="basis cap")
    ap.add_argument("--basis-iters", type=int, default=400,
                    help="steps of the untimed solve that builds the basis before the timed window")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after the run, copy a float32 buffer of this many MiB three times (a plain copy kernel "
                         "of known size that scales hardware byte counters)")
    ap.add_argument("--table1", action="store_true",
                    help="instead of the benchmark: the contrast sweep of Sec. 5.5 (128^2 fibre, polarization "
                         "iteration alone and with RPM, FP64, tol 1e-4); prints its own JSON line")
    ap.add_argument("--stress", action="store_true",
                    help="instead of the benchmark: a prescribed-mean-stress solve of the 64^3 sphere workload "
                         "(FP64 and FP32 refined), timed; prints its own JSON line")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark: the 64^3 sphere C_eff over the five reference media between "
                         "the phase moduli, FP64 and FP32 refined (RPM p_max 64), and Algorithm 1 on the zz case; "
                         "prints its own JSON line")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU run: turn two rocprofv3 --pmc counter files (FETCH_SIZE, WRITE_SIZE) of "
                         "'bench.py --warmup 0 --no-cpu --no-ttt --no-small --no-warm --calibrate-copy-mib M' into "
                         "per-launch traffic (written to profiles/)")
    return ap.parse_args()


# Iterations and seconds printed in Table 1 (Sec. 5.5; Matlab, hardware not
# stated): K -> (Acc-FFT, RPM-Acc-FFT iterations, Acc-FFT s, RPM-Acc-FFT s).
TABLE1_FILE = os.path.join(ROOT, "tests", "golden", "table1_paper.json")


def table1_paper():
    """The paper's Table 1 (Sec. 5.5) as {K: (acc_iters, rpm_acc_iters, acc_s, rpm_acc_s)}."""
    with open(TABLE1_FILE) as fh:
        t = json.load(fh)
    return {int(r[0]): tuple(r[1:]) for r in t["rows"]}


def table1():
    """The contrast sweep of Table 1 on this implementation: the polarization
    iteration with alpha = beta = 2 (Accelerated FFT) alone and with RPM."""
    import torch

    from paper_2003_07720_amd import binding as B
    from paper_2003_07720_amd import microstructure as M

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    rows = []
    for K, paper in table1_paper().items():
        w = M.workload_fibre(K)
        phase = torch.from_numpy(w["phase"]).to("cuda")
        lt = np.array([B.lame_from_young(*p) for p in w["phases"]])
        l0 = B.lame_from_young(*w["ref"])
        row = dict(K=K, paper=dict(zip(("acc_iters", "rpm_acc_iters", "acc_s", "rpm_acc_s"), paper)))
        for scheme in ("basic", "rpm"):
            opts = B.make_options(scheme=scheme, map="polarization", tol=w["tol"], max_iter=20000, n_max=10,
                                  p_max=32)
            ws = B.make_workspace(tuple(phase.shape), opts)
            B.fft_solve(phase, lt, l0, w["E"], B.make_options(scheme=scheme, map="polarization", max_iter=3),
                        workspace=ws, want_eps=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = B.fft_solve(phase, lt, l0, w["E"], opts, workspace=ws, want_eps=False)
            torch.cuda.synchronize()
            row[scheme] = dict(status=r["status"], iterations=r["iterations"], jvps=r["jvps"], p=r["basis_dim"],
                               residual=r["residual"], seconds=round(time.perf_counter() - t0, 4))
        rows.append(row)
        print(f"table1: K={K} {row}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "iterations and seconds to 1e-4, 128^2 fibre, Accelerated FFT vs RPM-Accelerated FFT",
                      "n_gpus": 1, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": "128^2 centred fibre radius 32, nu 0.25, eps_12 0.5%, "
                                             "E0 = sqrt(K), alpha = beta = 2, n_max 10, p_max 32"},
                      "rows": rows}), flush=True)


def stress_bench():
    """Prescribed mean stress on the 64^3 sphere workload: uniaxial Sigma_zz with the
    other components zero, RPM, tol 1e-6 (FP64, and FP32 fields refined to an
    FP64-certified 1e-6), timed after one untimed solve of the same call."""
    import torch

    from paper_2003_07720_amd import binding as B
    from paper_2003_07720_amd import microstructure as M

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = M.workload_spheres64()  # E0 = 1000, the top of the sweep (the stiff phase)
    phase = torch.from_numpy(w["phase"]).to("cuda")
    lt = np.array([B.lame_from_young(*p) for p in w["phases"]])
    l0 = B.lame_from_young(*w["ref"])
    S = np.array([0.0, 0.0, 0.01, 0.0, 0.0, 0.0])
    rows = {}
    for prec in ("fp64", "fp32"):
        opts = B.make_options(scheme="rpm", precision=prec, tol=1e-6, n_max=10, p_max=32, check_every=32,
                              max_iter=20000)
        ws = B.make_workspace(tuple(phase.shape), opts)
        B.fft_solve_stress(phase, lt, l0, S, opts, workspace=ws, want_eps=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = B.fft_solve_stress(phase, lt, l0, S, opts, workspace=ws, want_eps=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        its = sum(c["iterations"] for c in r["cases"]) + r["final"]["iterations"]
        rows[prec] = dict(status=r["status"], seconds=round(el, 4), iterations=its,
                          final_iterations=r["final"]["iterations"], E=[round(x, 9) for x in r["E"]],
                          sig_avg=[round(x, 9) for x in r["sig_avg"]],
                          voxel_iters_per_s=round(phase.numel() * its / el, 1))
        print(f"stress: {prec} {rows[prec]}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "seconds per prescribed-mean-stress solve, 64^3 spheres", "n_gpus": 1,
                      "data": "synthetic",
                      "config": {"workload": "64^3 random spheres (radii 4-8, vf 0.2, seed 2000), E 1 / 1000, "
                                             "E0 1000, Sigma_zz = 0.01, RPM p_max 32, tol 1e-6"},
                      "rows": rows}), flush=True)


def sweep_bench():
    """The 64^3 sphere workload's effective tensor for each reference medium of
    the 5-point sweep between the phase moduli (E0 = 1 ... 1000): RPM (p_max 64,
    tol 1e-6) with FP64 fields and with FP32 fields refined to FP64-certified
    1e-6, each timed after an untimed call; and Algorithm 1 alone on the zz
    load case (FP64, 20 000 steps at most), whose map diverges for E0 below
    half the stiff modulus."""
    import torch

    from paper_2003_07720_amd import binding as B
    from paper_2003_07720_amd import microstructure as M

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    rows = []
    for ri in range(5):
        w = M.workload_spheres64(ref_index=ri)
        phase = torch.from_numpy(w["phase"]).to("cuda")
        lt = np.array([B.lame_from_young(*p) for p in w["phases"]])
        l0 = B.lame_from_young(*w["ref"])
        row = dict(E0=w["ref"][0])
        Cs = {}
        for prec in ("fp64", "fp32"):
            opts = B.make_options(scheme="rpm", precision=prec, tol=1e-6, n_max=10, p_max=64, check_every=32,
                                  max_iter=20000)
            ws = B.make_workspace(tuple(phase.shape), opts)
            B.effective_tensor(phase, lt, l0, opts, workspace=ws, history_cap=20001)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            C, stats, st = B.effective_tensor(phase, lt, l0, opts, workspace=ws, history_cap=20001)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            Cs[prec] = C
            row[prec] = dict(status=st, seconds=round(el, 3), iterations=[x["iterations"] for x in stats],
                             jvps=sum(x["jvps"] for x in stats),
                             residual_fp64=max(x["residual_fp64"] for x in stats),
                             C11=C[0][0], C12=C[0][1], C33=C[2][2], C44=C[3][3])
            print(f"sweep: E0 {w['ref'][0]} {prec} {row[prec]}", file=sys.stderr, flush=True)
        row["fp32_vs_fp64_max_rel"] = float(np.abs(Cs["fp32"] - Cs["fp64"]).max() / np.abs(Cs["fp64"]).max())
        ob = B.make_options(scheme="basic", precision="fp64", tol=1e-6, check_every=32, max_iter=20000)
        wb = B.make_workspace(tuple(phase.shape), ob)
        t0 = time.perf_counter()
        rb = B.fft_solve(phase, lt, l0, np.array([0, 0, 0.01, 0, 0, 0.0]), ob, workspace=wb, want_eps=False,
                         history_cap=20001)
        torch.cuda.synchronize()
        h = rb["history"]
        row["basic_zz_fp64"] = dict(status=rb["status"], iterations=rb["iterations"], residual=rb["residual"],
                                    seconds=round(time.perf_counter() - t0, 3),
                                    error_at={str(k): float(h[k]) for k in (10, 100, 1000, 10000) if k < len(h)})
        print(f"sweep: E0 {w['ref'][0]} basic {row['basic_zz_fp64']}", file=sys.stderr, flush=True)
        rows.append(row)
    print(json.dumps({"metric": "seconds per 6x6 effective tensor over the reference-medium sweep, 64^3 spheres",
                      "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": "64^3 random spheres (radii 4-8, vf 0.2, seed 2000), E 1 / 1000 "
                                             "(nu 0.3 / 0.25), E0 on the 5-point linear sweep 1 ... 1000, RPM "
                                             "p_max 64, n_max 10, tol 1e-6"},
                      "rows": rows}), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_legs(a, w_c3, phases_c3, E0_c3, N_c3, gpu_iters_c2):
    """The oracle on the host: the 128^3 headline cell on all threads (the
    cpu_baseline of the JSON line), and single-threaded legs on the 32^2 disk
    (basic and RPM to 1e-8, whole solves) and one load case of the 64^3
    spheres (seconds per map application, times the GPU's iteration count)."""
    import oracle as O
    from paper_2003_07720_amd import microstructure as M

    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    c0 = time.perf_counter()
    rc = O.solve(w_c3["phase"], O.lame_table(phases_c3), O.lame(E0_c3, 0.3), w_c3["E"], scheme="rpm", tol=a.tol,
                 max_iter=a.cpu_steps, n_max=10, p_max=32)
    c1 = time.perf_counter()
    base = dict(value=N_c3 * (rc["iterations"] + rc["jvps"]) / (c1 - c0), unit="voxel-iters/s", cores=cores,
                kind="oracle", cpu=cpu_model(),
                sample=f"{rc['iterations']} map applications and {rc['jvps']} JVPs of the FP64 oracle (literal "
                       f"18-transform map, RPM) on the same {a.n}^3 void cell, {c1 - c0:.1f} s, OpenMP threads")
    legs = {}
    # single-threaded legs: a child process with OMP_NUM_THREADS=1 (the OpenMP
    # runtime of this process is already sized)
    import subprocess

    code = r"""
import json, sys, time
import numpy as np
sys.path.insert(0, %r)
import oracle as O
from paper_2003_07720_amd import microstructure as M
out = {}
w = M.workload_disk32()
for scheme in ("basic", "rpm"):
    t0 = time.perf_counter()
    r = O.solve(w["phase"], O.lame_table(w["phases"]), O.lame(*w["ref"]), w["E"], scheme=scheme, tol=w["tol"],
                max_iter=20000, n_max=10, p_max=32)
    out["disk32_" + scheme] = dict(status=r["status"], iterations=r["iterations"], jvps=r["jvps"],
                                  seconds=round(time.perf_counter() - t0, 4))
s = M.workload_spheres64()
k = %d
t0 = time.perf_counter()
r = O.solve(s["phase"], O.lame_table(s["phases"]), O.lame(*s["ref"]), np.array([0, 0, 0.01, 0, 0, 0.]),
            scheme="rpm", tol=1e-6, max_iter=k, n_max=10, p_max=32)
el = time.perf_counter() - t0
out["spheres64_zz_sample"] = dict(map_applications=r["iterations"] + r["jvps"], seconds=round(el, 3),
                                  s_per_map=el / (r["iterations"] + r["jvps"]))
print(json.dumps(out))
""" % (ROOT, a.cpu_c2_maps)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    pr = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    if pr.returncode == 0:
        legs = json.loads(pr.stdout.strip().splitlines()[-1])
        sm = legs["spheres64_zz_sample"]
        if gpu_iters_c2:
            sm["gpu_map_applications"] = gpu_iters_c2
            sm["estimated_solve_s"] = round(sm["s_per_map"] * gpu_iters_c2, 1)
    else:
        legs = {"error": pr.stderr[-2000:]}
    legs["threads"] = 1
    legs["cpu"] = cpu_model()
    return base, legs


def main():
    a = parse()
    if a.traffic_from:
        traffic_from(a.traffic_from[0], a.traffic_from[1], a.calibrate_copy_mib or 1024, a.steps, a.seed,
                     TRAFFIC_FILE, a.precision, a.n, a.p_max)
        return
    if a.table1 and a.gpus == 1:
        table1()
        return
    if a.stress and a.gpus == 1:
        stress_bench()
        return
    if a.sweep and a.gpus == 1:
        sweep_bench()
        return
    if a.gpus != 1:
        print(f"bench.py: --gpus {a.gpus} refused: the benchmark runs on a single GPU (one process, one device); "
              f"run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2003_07720_amd import binding as B
    from paper_2003_07720_amd import microstructure as M

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = M.workload_voids128(seed=a.seed, n=a.n)
    phases = w["phases"]
    E = w["E"]
    lt = np.array([B.lame_from_young(*p) for p in phases])
    E0 = 0.5 * (phases[0][0] + phases[1][0])  # arithmetic mean of the phase moduli
    l0 = B.lame_from_young(E0, 0.3)
    phase = torch.from_numpy(w["phase"]).to("cuda")
    N = phase.numel()
    prec_txt = "FP32 fields + FP64 RPM steps" if a.precision == "fp32" else "FP64 fields and RPM steps"
    common = dict(scheme="rpm", precision=a.precision, n_max=10, p_max=a.p_max, kappa=0.1, tol=a.tol,
                  check_every=32)
    cap = max(a.steps, a.ttt_iters, a.warmup, a.basis_iters) + 1
    ws = B.make_workspace(tuple(phase.shape), B.make_options(max_iter=cap, **common))
    print(f"bench: workload {a.n}^3 voids vf={w['info']['vf']:.4f} ({w['info']['n_spheres']} spheres), "
          f"{a.precision}, warmup {a.warmup}, steps {a.steps}", file=sys.stderr, flush=True)

    # 1. untimed: build the basis up to p_max (a plain solve from the uniform
    # start; growth every n_max + 1 steps)
    rb = B.fft_solve(phase, lt, l0, E, B.make_options(max_iter=a.basis_iters, **dict(common, refine=0)),
                     workspace=ws, want_eps=False)
    p_steady = rb["basis_dim"]
    print(f"bench: basis solve {rb['iterations']} steps, {rb['jvps']} JVPs, p = {p_steady}", file=sys.stderr,
          flush=True)
    # steady-state windows: the basis carried (reuse_basis), no growth (p = p_max),
    # a tolerance no step reaches so every step does its full work
    steady = dict(common, reuse_basis=1, tol=1e-15, refine=0)
    if a.warmup > 0:
        B.fft_solve(phase, lt, l0, E, B.make_options(max_iter=a.warmup, **steady), workspace=ws, want_eps=False)
    # 2. untimed: the same K steps with HIP events around every kernel class
    rk = B.fft_solve(phase, lt, l0, E, B.make_options(max_iter=a.steps, profile=1, **steady), workspace=ws,
                     want_eps=False)
    kall = rk["kernel_ms"]
    per_kernel = {k: dict(ms_total=round(kall[k], 4), launches=rk["kernel_launches"][k],
                          avg_us=round(1e3 * kall[k] / max(rk["kernel_launches"][k], 1), 3),
                          gbs=round(rk["kernel_bytes"][k] / max(kall[k], 1e-12) / 1e6, 1))
                  for k in kall if rk["kernel_launches"][k] > 0}
    # the dominant class: the largest total event time among the classes with
    # algorithmic bytes (the small reduction / finalize kernels have none)
    dom = max((k for k in kall if rk["kernel_launches"][k] > 0 and rk["kernel_bytes"][k] > 0), key=lambda k: kall[k])
    # 3. timed region: K steps, events only around the dominant class
    mask = 1 << B.KERNEL_NAMES.index(dom)
    # events around about 30 of its launches, spread over the window (each event
    # pair costs a few microseconds of the step it brackets)
    every = max(1, a.steps // 30)
    opts = B.make_options(max_iter=a.steps, profile=1, profile_classes=mask, profile_every=every, **steady)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = B.fft_solve(phase, lt, l0, E, opts, workspace=ws, want_eps=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    steps = r["iterations"]
    fcalls = steps + r["jvps"]
    value = N * fcalls / el
    print(f"bench: timed {steps} steps at p = {r['basis_dim']}, {r['jvps']} JVPs, {el * 1e3:.1f} ms, "
          f"dominant class {dom}", file=sys.stderr, flush=True)
    launches = r["kernel_launches"][dom]
    avg_ms = r["kernel_ms"][dom] / launches
    bytes_per_launch = r["kernel_bytes"][dom] / launches
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom, a.seed, a.precision, a.n, r["basis_dim"])

    # time to tolerance: plain RPM from the uniform start and an empty basis
    ttt = None
    ttt_info = {}
    if not a.no_ttt:
        ttt, ttt_info = time_to_tol(a, B, M, torch, phase, lt, l0, E, common, ws)

    # the small configurations on the GPU: the 32^2 disk (basic and RPM to 1e-8, FP64)
    small = {} if a.no_small else disk32_row(B, M, torch)
    warm = None if a.no_warm else learned_warm_start(a, B, M, torch)

    cpu = None
    cpu_single = None
    if not a.no_cpu:
        c2 = small.get("spheres64_zz_fp64", {}).get("map_applications")
        cpu, cpu_single = cpu_legs(a, w, phases, E0, N, c2)

    out = {
        "metric": "voxel-iters/s + time to 1e-6 residual at 128³ voids; warm-start vs plain RPM",
        "value": value,
        "unit": "voxel-iters/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * el / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{a.n}^3 spherical voids (radii {6 * a.n / 128:g}-{12 * a.n / 128:g} voxels, "
                               f"vf {w['info']['vf']:.3f}, seed {a.seed}), void stiffness 1e-8, eps_zz 0.01, "
                               f"E0 = {E0:.6g} (arithmetic mean), plain RPM (no warm start), p_max {a.p_max}, "
                               f"n_max 10, {prec_txt}; timed: {steps} steady-state steps at p = "
                               f"{r['basis_dim']} (basis carried from an untimed solve)",
                   "voxels": N, "p_timed": r["basis_dim"], "jvps_timed": r["jvps"],
                   "time_to_tol_s": ttt, "time_to_tol_run": ttt_info, "learned_warm_start": warm,
                   "small_configs": small},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "avg_us": round(avg_ms * 1e3, 3), "bytes_per_launch": bytes_per_launch,
                     "launches_timed": launches, "events_every": every},
        "kernels": per_kernel,
        "cpu_baseline": cpu,
        "cpu_single_thread": cpu_single,
    }
    print(json.dumps(out), flush=True)
    if a.calibrate_copy_mib > 0:
        x = torch.ones(a.calibrate_copy_mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()


def time_to_tol(a, B, M, torch, phase, lt, l0, E, common, ws):
    """Plain RPM from the uniform start to tol (capped), then looser tolerances
    for RPM and the basic scheme, and the two warm starts."""
    o2 = B.make_options(max_iter=a.ttt_iters, **common)
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    r2 = B.fft_solve(phase, lt, l0, E, o2, workspace=ws, want_eps=False, history_cap=a.ttt_iters + 1)
    torch.cuda.synchronize()
    s1 = time.perf_counter()
    h = r2["history"]
    info = dict(status=r2["status"], iterations=r2["iterations"], jvps=r2["jvps"], p=r2["basis_dim"],
                residual=r2["residual"], residual_fp64=r2["residual_fp64"], refinements=r2["refinements"],
                seconds=round(s1 - s0, 4),
                error_at={str(k): float(h[k]) for k in (100, 300, 1000, 2000, 4000) if k < len(h)})
    ttt = (s1 - s0) if r2["status"] == "RPM_OK" else None
    print(f"bench: time-to-tol solve {info}", file=sys.stderr, flush=True)
    loose = {}
    for tl in [float(x) for x in a.ttt_loose.split(",") if x]:
        for scheme in ("rpm", "basic"):
            o3 = B.make_options(max_iter=a.ttt_iters, **dict(common, tol=tl, scheme=scheme, refine=0))
            torch.cuda.synchronize()
            u0 = time.perf_counter()
            r3 = B.fft_solve(phase, lt, l0, E, o3, workspace=ws, want_eps=False)
            torch.cuda.synchronize()
            u1 = time.perf_counter()
            loose[f"{scheme}@{tl:g}"] = dict(status=r3["status"], iterations=r3["iterations"],
                                             seconds=round(u1 - u0, 4), residual=r3["residual"])
    info["looser_tolerances"] = loose
    print(f"bench: looser tolerances {loose}", file=sys.stderr, flush=True)
    # basis warm start: the basis another load case (uniaxial xx) built on the
    # same cell, capped at half of p_max so the solve keeps room to grow
    bw = {}
    Exx = np.zeros(6)
    Exx[0] = E[2]
    for tl in [float(x) for x in a.ttt_loose.split(",") if x]:
        # about p_max / 2 columns: growth adds one or two every n_max + 1 steps
        ob = B.make_options(max_iter=min(a.ttt_iters, 11 * (a.p_max // 4) + 1),
                            **dict(common, tol=tl, refine=0, p_max=a.p_max))
        torch.cuda.synchronize()
        b0 = time.perf_counter()
        rb = B.fft_solve(phase, lt, l0, Exx, ob, workspace=ws, want_eps=False)
        torch.cuda.synchronize()
        b1 = time.perf_counter()
        ow = B.make_options(max_iter=a.ttt_iters, **dict(common, tol=tl, refine=0, reuse_basis=1))
        rw = B.fft_solve(phase, lt, l0, E, ow, workspace=ws, want_eps=False)
        torch.cuda.synchronize()
        b2 = time.perf_counter()
        bw[f"rpm@{tl:g}"] = dict(status=rw["status"], iterations=rw["iterations"], p_start=rb["basis_dim"],
                                 p_end=rw["basis_dim"], seconds=round(b2 - b1, 4), residual=rw["residual"],
                                 basis_solve=dict(status=rb["status"], iterations=rb["iterations"],
                                                  seconds=round(b1 - b0, 4)))
    info["basis_warm_start"] = bw
    print(f"bench: basis warm start {bw}", file=sys.stderr, flush=True)
    # the same geometry with a void stiffness where the tolerance is reachable
    # (1e-3 of the matrix; E0 at the matrix modulus): time to tol, plain RPM
    # from the uniform start, each after an untimed run of the same call
    lt3 = np.array([B.lame_from_young(*p) for p in [(1.0, 0.3), (1e-3, 0.3)]])
    l03 = B.lame_from_young(1.0, 0.3)
    reach = {}
    runs = [("rpm", prec, pm) for prec, pm in (("fp32", 32), ("fp32", 64), ("fp64", 32), ("fp64", 64))]
    runs += [("basic", "fp32", 32), ("basic", "fp64", 32)]  # Algorithm 1 to the same certified tolerance
    for scheme, prec, pm in runs:
        o3 = B.make_options(**dict(common, scheme=scheme, precision=prec, p_max=pm, max_iter=30000))
        w3 = B.make_workspace(tuple(phase.shape), o3)
        B.fft_solve(phase, lt3, l03, E, o3, workspace=w3, want_eps=False)
        torch.cuda.synchronize()
        r0 = time.perf_counter()
        r3 = B.fft_solve(phase, lt3, l03, E, o3, workspace=w3, want_eps=False)
        torch.cuda.synchronize()
        key = f"{prec}_p{pm}" if scheme == "rpm" else f"basic_{prec}"
        reach[key] = dict(status=r3["status"], iterations=r3["iterations"], jvps=r3["jvps"],
                                      refinements=r3["refinements"], residual_fp64=r3["residual_fp64"],
                                      seconds=round(time.perf_counter() - r0, 4))
        del w3
    info["voids_stiffness_1e-3_E0_1"] = reach
    print(f"bench: reachable-contrast voids {reach}", file=sys.stderr, flush=True)
    return ttt, info


def learned_warm_start(a, B, M, torch):
    """The learned warm start (NEXT-1): training data from the solver on seeded
    32^3 cells (spheres, contrast 1e-3 .. 1e3), training with the library's
    kernels, then the headline void cell solved from the uniform start and from
    the network's prediction, to looser tolerances (1e-6 is out of reach for
    both), and the same geometry with void stiffness 1e-3 to 1e-6."""
    from paper_2003_07720_amd import surrogate as S

    t0 = time.perf_counter()
    X, Y, _ = S.make_dataset(32, a.warm_cells, 0)
    Xv, Yv, _ = S.make_dataset(32, 8, 100000)
    t1 = time.perf_counter()
    cfg = B.fno_config(2, 36, 32, 4, 12)
    params, hist = S.train(cfg, X, Y, steps=a.warm_steps, batch=4, lr=3e-3, seed=1,
                           log_every=500 if a.warm_steps > 1000 else 0)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out = dict(network="FNO: 2 features -> width 32, 4 spectral layers, 12 signed modes per axis -> 36 channels; "
                       "BF16 matrix-core GEMMs, FP32 accumulation",
               params=B.fno_param_count(cfg), train_cells=a.warm_cells, train_grid="32^3", steps=a.warm_steps,
               data_seconds=round(t1 - t0, 1), train_seconds=round(t2 - t1, 1),
               loss_first_last=[hist[0], float(np.mean(hist[-50:]))],
               heldout_relative_error=round(S.relative_error(cfg, params, Xv, Yv), 4))
    w = M.workload_voids128(seed=a.seed, n=a.n)
    rows = {}
    for tol in [float(x) for x in a.ttt_loose.split(",") if x] + [a.tol]:
        rows[f"{tol:g}"] = S.compare_warm_start(cfg, params, w["phase"], w["phases"], w["E"], tol,
                                                precision=a.precision, ref=(0.5 * (1 + 1e-8), 0.3),
                                                max_iter=min(a.ttt_iters, 1000) if tol == a.tol else a.ttt_iters,
                                                seeded=tol != a.tol)
    out["voids128"] = rows
    # where 1e-6 is reachable: void stiffness 1e-3, E0 at the matrix modulus,
    # FP32 refined with p_max 64 (the fastest plain configuration there)
    out["voids128_stiffness_1e-3"] = S.compare_warm_start(cfg, params, w["phase"], [(1.0, 0.3), (1e-3, 0.3)], w["E"],
                                                          a.tol, precision="fp32", p_max=64, ref=(1.0, 0.3),
                                                          max_iter=30000, seeded=True)
    if a.warm_eval_cells > 0:
        # held-out void cells of the same recipe (other seeds), void stiffness 1e-3 so the tolerance is reachable
        ev = []
        for k in range(a.warm_eval_cells):
            wk = M.workload_voids128(seed=a.seed + 1 + k, n=a.n)
            r = S.compare_warm_start(cfg, params, wk["phase"], [(1.0, 0.3), (1e-3, 0.3)], wk["E"], a.tol,
                                     precision="fp32", p_max=64, ref=(1.0, 0.3), max_iter=30000)
            ev.append(dict(seed=a.seed + 1 + k, plain=r["plain"], warm=r["warm"]))
            print(f"bench: held-out cell {k}: {r}", file=sys.stderr, flush=True)
        ok = [e for e in ev if e["plain"]["status"] == "RPM_OK" and e["warm"]["status"] == "RPM_OK"]
        out["heldout_voids128_stiffness_1e-3"] = dict(
            cells=len(ev), both_converged=len(ok),
            mean_iterations_plain=float(np.mean([e["plain"]["iterations"] for e in ok])) if ok else None,
            mean_iterations_warm=float(np.mean([e["warm"]["iterations"] for e in ok])) if ok else None,
            mean_seconds_plain=float(np.mean([e["plain"]["seconds"] for e in ok])) if ok else None,
            mean_seconds_warm=float(np.mean([e["warm"]["seconds"] for e in ok])) if ok else None,
            per_cell=ev)
    print(f"bench: learned warm start {out}", file=sys.stderr, flush=True)
    return out


def disk32_row(B, M, torch):
    """The smaller configurations on the GPU, each timed after an untimed run of
    the same call, on a side stream so that iterations can be replayed from
    captured graphs: the 32^2 disk (basic and RPM to 1e-8, FP64; kernel by kernel
    and from graphs), one load case of the 64^3 spheres (E0 at the stiff
    modulus, RPM to 1e-6, FP64 and FP32 refined, basis cap 32 and 64) and their
    6 x 6 effective tensor (load cases one after the other, and batched on one
    shared basis), and the tile autotuner on 48^3 and 96^3 cells."""
    out = {}
    side = torch.cuda.Stream()

    def timed(fn):
        fn()
        side.synchronize()
        t0 = time.perf_counter()
        r = fn()
        side.synchronize()
        return r, time.perf_counter() - t0

    with torch.cuda.stream(side):
        w = M.workload_disk32()
        ph = torch.from_numpy(w["phase"]).to("cuda")
        lt = np.array([B.lame_from_young(*p) for p in w["phases"]])
        l0 = B.lame_from_young(*w["ref"])
        for scheme in ("basic", "rpm"):
            for graph in (0, 1):
                o = B.make_options(scheme=scheme, tol=w["tol"], max_iter=20000, precision="fp64", check_every=32,
                                   graph=graph)
                ws = B.make_workspace(tuple(ph.shape), o)
                r, el = timed(lambda: B.fft_solve(ph, lt, l0, w["E"], o, workspace=ws, want_eps=False))
                out[f"disk32_{scheme}" + ("_graph" if graph else "")] = dict(
                    status=r["status"], iterations=r["iterations"], jvps=r["jvps"], seconds=round(el, 5))
        s = M.workload_spheres64()
        ph = torch.from_numpy(s["phase"]).to("cuda")
        lt = np.array([B.lame_from_young(*p) for p in s["phases"]])
        l0 = B.lame_from_young(*s["ref"])
        Ezz = np.array([0, 0, 0.01, 0, 0, 0.0])
        for prec, p_max in (("fp64", 32), ("fp32", 32), ("fp64", 64)):
            o = B.make_options(scheme="rpm", tol=1e-6, max_iter=20000, precision=prec, check_every=32, p_max=p_max,
                               graph=1)
            ws = B.make_workspace(tuple(ph.shape), o)
            r, el = timed(lambda: B.fft_solve(ph, lt, l0, Ezz, o, workspace=ws, want_eps=False))
            out[f"spheres64_zz_{prec}" + ("" if p_max == 32 else f"_p{p_max}")] = dict(
                status=r["status"], iterations=r["iterations"], jvps=r["jvps"],
                map_applications=r["iterations"] + r["jvps"], refinements=r["refinements"],
                residual_fp64=r["residual_fp64"], seconds=round(el, 4))
        for batch, p_max in ((0, 32), (0, 64), (1, 64)):
            o = B.make_options(scheme="rpm", tol=1e-6, max_iter=20000, precision="fp64", check_every=32,
                               p_max=p_max, batch_cases=batch, graph=1)
            ws = B.make_workspace(tuple(ph.shape), o)
            (C, stats, st), el = timed(lambda: B.effective_tensor(ph, lt, l0, o, workspace=ws))
            out[f"spheres64_ceff_fp64_p{p_max}" + ("_batched" if batch else "")] = dict(
                status=st, seconds=round(el, 4), iterations=[x["iterations"] for x in stats],
                jvps=sum(x["jvps"] for x in stats), C11=C[0][0], C33=C[2][2])
        # the uneven grids of the batched benchmark family: the tile autotuner's
        # shape against the default, per map application (FP32); at 128^3 also
        # the y transforms held in registers (DPP exchanges), which the tuner
        # times as a candidate
        for n in (48, 96, 128):
            cell = M.random_phases((n, n, n), 2, seed=40 + n)
            ph = torch.from_numpy(cell).to("cuda")
            lt = np.array([B.lame_from_young(*p) for p in [(1.0, 0.3), (50.0, 0.3)]])
            l0 = B.lame_from_young(50.0, 0.3)
            o = B.make_options(scheme="rpm", precision="fp32", p_max=32)
            ws = B.make_workspace(tuple(ph.shape), o)
            t0 = time.perf_counter()
            t = B.autotune(ph, lt, l0, o, reps=20, workspace=ws)
            tune_s = time.perf_counter() - t0
            ms = {}
            shapes = [("default", None), ("tuned", t["tuning"])] + ([("y_regs", dict(y_regs=1))] if n == 128 else [])
            for name, tn in shapes:
                # 200 RPM steps each (a tolerance no step reaches), basis up to 32
                oo = B.make_options(scheme="rpm", precision="fp32", p_max=32, tol=1e-15, max_iter=200, refine=0,
                                    check_every=32, tuning=tn)
                r, el = timed(lambda: B.fft_solve(ph, lt, l0, Ezz, oo, workspace=ws, want_eps=False))
                ms[name] = round(el / (r["iterations"] + r["jvps"]) * 1e3, 4)
            out[f"autotune_{n}cube_fp32"] = dict(tuning=t["tuning"].as_dict(), tuner_ms_per_map=round(t["ms"], 4),
                                                 candidates=t["candidates"], tune_seconds=round(tune_s, 3),
                                                 **{f"ms_per_map_solve_{k}": v for k, v in ms.items()})
    # the batched family: seeded two-phase cells of uneven grids, the six unit
    # load cases each (FP32, FP64 refinement, tol 1e-6), one worker against four
    # and eight concurrent workers (a stream each), launch shapes tuned per grid
    from paper_2003_07720_amd import batch as bt

    cells = bt.random_cells(16, grids=(32, 48, 64), seed0=0, contrast=(1e-3, 1e2))
    kw = dict(scheme="rpm", precision="fp32", tol=1e-6, refine=4, p_max=32, max_iter=20000, check_every=32)
    t0 = time.perf_counter()
    tunings = bt.tune_grids(cells, kw, reps=10)
    tune_s = time.perf_counter() - t0
    row = dict(cells=len(cells), grids=sorted({c["n"] for c in cells}), tune_seconds=round(tune_s, 3),
               tunings={f"{k[0]}^3": v.as_dict() for k, v in tunings.items()})
    for workers in (1, 4, 8):
        res, wall = bt.effective_many(cells, kw, workers=workers, tunings=tunings)
        row[f"workers{workers}"] = dict(seconds=round(wall, 3), cells_per_s=round(len(cells) / wall, 3),
                                        statuses=sorted({r["status"] for r in res}),
                                        max_residual_fp64=max(r["residual_fp64"] for r in res),
                                        map_applications=sum(sum(r["iterations"]) + r["jvps"] for r in res))
    # the same batch with FP64 fields: on grids this small a pass costs its
    # launch, not its bytes, so FP32 saves nothing and its refinement adds work
    kw64 = dict(kw, precision="fp64")
    res, wall = bt.effective_many(cells, kw64, workers=4, tunings=bt.tune_grids(cells, kw64, reps=10))
    row["fp64_workers4"] = dict(seconds=round(wall, 3), cells_per_s=round(len(cells) / wall, 3),
                                statuses=sorted({r["status"] for r in res}),
                                max_residual_fp64=max(r["residual_fp64"] for r in res),
                                map_applications=sum(sum(r["iterations"]) + r["jvps"] for r in res))
    out["batched_cells_32_48_64"] = row
    print(f"bench: small configurations {out}", file=sys.stderr, flush=True)
    return out


if __name__ == "__main__":
    main()
