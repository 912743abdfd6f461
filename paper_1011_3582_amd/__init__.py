"""MI355X-native FFT-LB solver for thermal liquid-vapour systems.

The compute path is the HIP library built from ``csrc/`` (``libfftlb.so``); the
Python side only marshals arguments.  Importing this package does not load the
library; ``paper_1011_3582_amd.fftlb`` does, and raises if it is not built.
"""
