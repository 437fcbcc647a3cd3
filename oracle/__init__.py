"""Plain FP64 CPU oracle of the lattice update (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark import this package; the solver never does.
"""
from .pyoracle import (Oracle, OracleError, build, lattice, wetting_H, from_spec,  # noqa: F401
                       lattice_cos, wetting_H_lattice,
                       solubility_E, set_threads, SOLUTE_FORCE, EXPLICIT_COLLOID,
                       CAPILLARY_FORCE, STRESS_FORM)
