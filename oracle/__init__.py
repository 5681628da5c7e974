"""FP64 CPU oracle of the coupled two-phase EHD lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of the benchmark, never by the product library.  The C source is
`lbm_ehd_oracle.c`; `build()` compiles it with gcc and `Oracle` drives it
through ctypes.
"""
from .oracle import (Oracle, build, lib_path, lattice, geq, heq, leq, feq, rbar, source_g,  # noqa: F401
                     set_threads, max_threads, build_variant, source)
