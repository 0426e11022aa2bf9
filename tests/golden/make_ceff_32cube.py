"""Writes ceff_32cube.json: effective stiffness tensors of two 32^3 cells computed
by the FP64 CPU oracle (Algorithm 2, every unit load case, error tolerance
1e-7: the effective tensor is stationary at the solution, so its error is far
below 1e-7), the expected values of the FP32-refined effective-tensor parity tests.
Calls only the oracle and the seeded input generators.

  python tests/golden/make_ceff_32cube.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2003_07720_amd import microstructure as M  # noqa: E402

# cell name -> (generator arguments, phases (E, nu), reference medium (E0, nu0))
CELLS = {
    "spheres32_contrast1000": (dict(n=32, r_min=2.0, r_max=4.0, vf=0.20, seed=2000), [(1.0, 0.3), (1000.0, 0.25)],
                               (1000.0, 0.3)),
    "voids32_contrast1e-3": (dict(n=32, r_min=1.5, r_max=3.0, vf=0.30, seed=3000), [(1.0, 0.3), (1e-3, 0.3)],
                             (1.0, 0.3)),
}
TOL = 1e-7


def cell_phase(gen):
    ph, info = M.rsa_spheres(gen["n"], gen["r_min"], gen["r_max"], gen["vf"], gen["seed"])
    return ph, info


def main(names=None):
    out = {"tol": TOL, "scheme": "rpm", "n_max": 10, "p_max": 32, "cells": {}}
    path = os.path.join(HERE, "ceff_32cube.json")
    if os.path.exists(path):
        with open(path) as fh:
            out["cells"] = json.load(fh).get("cells", {})
    for name, (gen, phases, ref) in CELLS.items():
        if names and name not in names:
            continue
        ph, info = cell_phase(gen)
        t0 = time.time()
        C, runs = O.effective_tensor(ph, O.lame_table(phases), O.lame(*ref), scheme="rpm", tol=TOL,
                                     max_iter=40000, n_max=10, p_max=32)
        assert all(r["status"] == "converged" for r in runs), [r["status"] for r in runs]
        out["cells"][name] = dict(generator=gen, phases=phases, ref=ref, vf=float(info["vf"]), C_eff=C.tolist(),
                                  iterations=[r["iterations"] for r in runs], seconds=round(time.time() - t0, 1))
        print(name, out["cells"][name]["iterations"], out["cells"][name]["seconds"], flush=True)
        # merge with what another run wrote meanwhile
        if os.path.exists(path):
            with open(path) as fh:
                cells = json.load(fh).get("cells", {})
            cells[name] = out["cells"][name]
            out["cells"] = cells
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:])
