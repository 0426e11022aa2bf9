"""Many independent cells solved concurrently (the batched benchmark family:
seeded two-phase microstructures of uneven grids, the six unit load cases of
each, FP32 with FP64 refinement).

The cells share nothing a solve could reuse (each has its own operator, so its
own basis), and on small grids a map application is a handful of short pencil
passes whose launch and drain times dominate.  So the batch is spread over
worker threads, each owning a HIP stream (default priority) and, per grid, a
workspace: the library's entry points block only on their own stream, ctypes
releases the interpreter lock during the call, and the GPU overlaps the
passes of different cells.  Each distinct grid is first tuned once
(rpm_fft_autotune, on an idle GPU) and every solve on it uses that shape.
This module only schedules calls; every step of a solve runs in the library.
"""
from __future__ import annotations

import queue
import threading
import time

import numpy as np
import torch

from . import binding as B
from . import microstructure as M


def random_cells(count, grids=(32, 48, 64, 96), seed0=0, vf_range=(0.10, 0.40), contrast=(1e-6, 1e3)):
    """Seeded two-phase sphere cells: grid drawn from grids, volume fraction
    uniform in vf_range, inclusion/matrix modulus ratio log-uniform in
    contrast, radii 0.06-0.16 of the grid; matrix E = 1, both nu = 0.3.  The
    reference medium is taken at the stiffer phase."""
    out = []
    for k in range(count):
        r = np.random.Generator(np.random.PCG64(50_000 + seed0 + k))
        n = int(grids[r.integers(len(grids))])
        vf = float(r.uniform(*vf_range))
        K = float(np.exp(r.uniform(np.log(contrast[0]), np.log(contrast[1]))))
        ph, info = M.rsa_spheres(n, 0.06 * n, 0.16 * n, vf, seed0 + k)
        phases = [(1.0, 0.3), (K, 0.3)]
        out.append(dict(phase=ph, phases=phases, ref=(max(1.0, K), 0.3), vf=float(info["vf"]), n=n))
    return out


def tune_grids(cells, opts_kw, reps=10):
    """One launch shape per distinct grid (autotuned on the first cell of it)."""
    tunings = {}
    for c in cells:
        shape = tuple(c["phase"].shape)
        if shape in tunings:
            continue
        ph = torch.from_numpy(np.ascontiguousarray(c["phase"])).to("cuda")
        lt = np.array([B.lame_from_young(*p) for p in c["phases"]])
        l0 = B.lame_from_young(*c["ref"])
        o = B.make_options(**opts_kw)
        tunings[shape] = B.autotune(ph, lt, l0, o, reps=reps)["tuning"]
    torch.cuda.synchronize()
    return tunings


def effective_many(cells, opts_kw, workers=4, tunings=None):
    """C_eff of every cell, cells taken from a shared queue by `workers`
    threads with a stream each.  Returns (results in cell order, wall seconds)."""
    results = [None] * len(cells)
    work = queue.Queue()
    for i in sorted(range(len(cells)), key=lambda i: -cells[i]["phase"].size):  # large cells first
        work.put(i)
    errors = []

    def run(wid):
        stream = torch.cuda.Stream()
        spaces = {}
        try:
            with torch.cuda.stream(stream):
                while True:
                    try:
                        i = work.get_nowait()
                    except queue.Empty:
                        break
                    c = cells[i]
                    shape = tuple(c["phase"].shape)
                    tn = tunings.get(shape) if tunings else None
                    o = B.make_options(tuning=tn, **opts_kw)
                    if shape not in spaces:
                        spaces[shape] = B.make_workspace(shape, B.make_options(**opts_kw))
                    ph = torch.from_numpy(np.ascontiguousarray(c["phase"])).to("cuda")
                    lt = np.array([B.lame_from_young(*p) for p in c["phases"]])
                    l0 = B.lame_from_young(*c["ref"])
                    t0 = time.perf_counter()
                    C, stats, status = B.effective_tensor(ph, lt, l0, o, workspace=spaces[shape])
                    results[i] = dict(C=C, status=status, iterations=[s["iterations"] for s in stats],
                                      jvps=sum(s["jvps"] for s in stats),
                                      residual_fp64=max(s["residual_fp64"] for s in stats),
                                      seconds=time.perf_counter() - t0, worker=wid)
            stream.synchronize()
        except Exception as e:  # reported to the caller after the join
            errors.append(e)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    threads = [threading.Thread(target=run, args=(w,)) for w in range(workers)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if errors:
        raise errors[0]
    return results, wall
