"""CPU oracle for the dense Kohn-Sham path -- TEST INFRASTRUCTURE ONLY.

Plain FP64 C (``elsi_oracle.c``) behind ctypes.  Only the test-suite, the smoke
check and the benchmark's CPU-baseline leg may import this package; the GPU
library never does, and it shares no code with it.
"""
from .oracle import (  # noqa: F401
    FERMI,
    GAUSSIAN,
    MP0,
    MP1,
    backsub,
    band_energy,
    build,
    density,
    dm,
    dm_checked,
    dm_shared_mu,
    gevp,
    gevp_checked,
    occupations,
    occupation_value,
    potrf,
    reduce_standard,
    refine,
    residual_norms,
    tred,
    tridiag_eig,
    tridiag_eigvals,
    tridiag_shift_solve,
    zdensity,
    zdm,
    zgevp,
    zpotrf,
    zreduce_standard,
    ztred,
)
