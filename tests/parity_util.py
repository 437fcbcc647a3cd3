"""Helpers shared by the GPU parity tests: run a workload spec on the HIP
library and on the oracle, and the per-field error measure.

Error of field a against reference b over fluid nodes:
    e = max |a - b| / max(max |b|, floor)
with floors rho: 1, psi: 1, c: 1e-6, u: 1e-8 for the FP32 and FP16-storage
bars and u: 1e-3 for the FP64 bar.  Fields that start at zero would
otherwise make a relative measure meaningless.  The FP64 velocity floor is
the scale at which 1e-12 relative equals the FP64 round-off of the momentum
moment itself: 18 populations of size <= 1/18 summed each step carry
~1e-16 of rounding, which accumulates to ~1e-15 over O(100) steps.  The
largest reference |u| is printed beside every velocity error, so the reader
sees whether a floor was active."""
import sys

import numpy as np

import oracle
from paper_2202_01631_amd import lb

FLOORS = dict(rho=1.0, psi=1.0, c=1e-6, u=1e-3)
U_FLOOR_FP32 = 1e-8


def flush_print(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def field_errors(a, b, fluid, u_floor=None):
    """Per-field errors; u_floor overrides the FP64 velocity floor (pass
    U_FLOOR_FP32 for the FP32 and FP16-storage bars)."""
    out = {}
    for k in ("rho", "psi", "c"):
        ref = b[k][fluid]
        out[k] = float(np.abs(a[k][fluid] - ref).max() / max(np.abs(ref).max(), FLOORS[k]))
    ua, ub = a["u"][:, fluid], b["u"][:, fluid]
    umax = float(np.abs(ub).max())
    fl = FLOORS["u"] if u_floor is None else u_floor
    out["u"] = float(np.abs(ua - ub).max() / max(umax, fl))
    flush_print("[parity] max|u| of the reference %.3e (u floor %.0e%s)"
                % (umax, fl, ", active" if umax < fl else ""))
    return out


def run_pair(spec, steps, precision=None, **override):
    """Advance the same spec on the GPU and on the oracle; return both."""
    flush_print("[parity] %s shape=%s prec=%s steps=%d" % (spec.get("name"), spec["shape"],
                                                          precision or spec.get("precision"), steps))
    g = lb.from_spec(spec, precision=precision, **override)
    s2 = dict(spec)
    s2["params"] = dict(spec["params"], **override)
    o = oracle.from_spec(s2)
    if steps:
        g.step(steps)
        o.step(steps)
    return g, o
