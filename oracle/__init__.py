"""Plain FP64 CPU oracle of the coupled LBM + WENO step (arXiv 2106.07694).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product package never imports
it.  It shares no code with the HIP path; see ``lbw_oracle.c`` for what one
step computes and which passage of the paper each part follows.
"""
from .oracle import (  # noqa: F401
    OracleConfig,
    build,
    lattice,
    equilibrium,
    moments,
    rhs_c,
    faces_c,
    run,
    sums,
    library_path,
    adjoint_step,
    front_height,
    mass_below,
    front_psd,
)
