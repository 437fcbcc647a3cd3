"""Run the FP64 oracle's sanitizer build (liboracle_hostcheck.so, see
build.py) through a few steps of every option (TEST INFRASTRUCTURE).  Exit
status 0 and "oracle ok" mean no sanitizer report.

    python oracle_check.py LIB
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import pyoracle  # noqa: E402
from paper_2202_01631_amd import inputs as I  # noqa: E402


def main():
    pyoracle.LIB = sys.argv[1]
    pyoracle._lib = None
    w = I.workload_small()
    for over in ({}, dict(flags=pyoracle.SOLUTE_FORCE | pyoracle.CAPILLARY_FORCE),
                 dict(flags=pyoracle.EXPLICIT_COLLOID, ch_substeps=3, M_psi=0.25),
                 dict(soft_eps=1e-3, soft_sigma=1.0, soft_nu=2.0, soft_hc=2.5, lub_hc=1.5)):
        spec = dict(w, params=dict(w["params"], **over))
        o = pyoracle.from_spec(spec)
        pyoracle.set_threads(2)
        o.step(3)
        o.fields(), o.aux(), o.links(), o.owner(), o.observables(), o.step_diag()
        o.colloid_diag(0)
        o.close()
    pyoracle.set_threads(1)
    print("oracle ok", flush=True)


if __name__ == "__main__":
    main()
