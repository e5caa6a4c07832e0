"""MI355X-native FFT-accelerated, FIR-regularised MOT-JVIE (HIP library + thin binding).

The computation lives in libmotjvie.so (C interface: include/motjvie.h); this package
only builds it (build.py) and marshals arguments to it (motjvie.py).
"""
from .motjvie import MotJvieError, ProbeObjective, Solver, load_library, solver_for  # noqa: F401
