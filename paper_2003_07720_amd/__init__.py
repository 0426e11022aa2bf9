"""MI355X (gfx950) implementation of the RPM-FFT solver (Peng, Nepal & Dayal 2020).

The solver lives in the HIP library ``librpmfft.so`` (C ABI: include/rpmfft.h);
:mod:`paper_2003_07720_amd.binding` marshals torch tensors into it and
:mod:`paper_2003_07720_amd.microstructure` generates seeded input cells.
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librpmfft.so")
CSRC = os.path.join(HERE, "csrc")
