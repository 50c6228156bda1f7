"""FP64 CPU oracle of the Gaussian lattice Boltzmann hierarchy (arXiv:1905.04597).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``, never by the product package.
The arithmetic lives in ``glbm_oracle.c`` (plain C, FP64); this module only
builds it with gcc and marshals numpy arrays through ctypes.
"""
from .oracle import (  # noqa: F401
    AXIS_EVEN,
    AXIS_ODD,
    BC_EQ_ENDS,
    BC_PERIODIC,
    BC_WALL,
    OracleSolver,
    axis_equilibrium,
    axis_velocities,
    build_oracle,
    equilibrium_1d,
    rest_weights,
    step_probabilities,
    tau_from_kn,
)
