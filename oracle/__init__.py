"""FP64 CPU oracle for the FFT-LB thermal liquid-vapour step.

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and by
bench.py's cpu_baseline leg.  The library and its Python binding never import,
call or link anything here, and nothing here imports the library.
"""
from . import fftlb_oracle, thermo  # noqa: F401
