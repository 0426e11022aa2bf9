"""Build step of the HIP library (hipcc, gfx950).  Used by __graft_entry__.build()."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", "rpm_solver.hip"), os.path.join(HERE, "csrc", "rpm_fno.hip")]
OUT = os.path.join(HERE, "librpmfft.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off: plain scalar/float2 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-value",
]


def build(verbose=False):
    inc = ["-I", os.path.join(ROOT, "include")]
    objs = [os.path.join(HERE, "csrc", os.path.basename(s).replace(".hip", ".o")) for s in SRCS]
    procs = []
    for src, obj in zip(SRCS, objs):
        cmd = ["hipcc"] + HIPCC_FLAGS + inc + ["-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        _, err = p.communicate()
        if p.returncode != 0:
            raise RuntimeError("hipcc failed:\n" + err[-8000:])
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", OUT + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    for obj in objs:  # intermediate objects do not travel with the tree
        if os.path.exists(obj):
            os.remove(obj)
    if r.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + r.stderr[-8000:])
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
