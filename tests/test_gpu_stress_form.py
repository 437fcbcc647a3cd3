"""GPU checks of the divergence-form solvent force (LB_STRESS_FORM, with
LB_CAPILLARY_FORCE; the momentum exchange of Sec. II.B made exact for the
capillary coupling): FP32 and FP64 against the oracle on the paper's
regime box, and batched beside a box without the option bit for bit as
alone."""
import numpy as np
import pytest

import oracle
from paper_2202_01631_amd import inputs as I
from paper_2202_01631_amd import lb
from parity_util import U_FLOOR_FP32, field_errors, flush_print

pytestmark = pytest.mark.gpu


def _trap_spec(mu=0.05, E=-0.25, flags=lb.LB_CAPILLARY_FORCE | lb.LB_STRESS_FORM, R=4.5,
               M_psi=0.1, nsub=1, precision="fp32"):
    # a tilted axis: no link midpoint lies exactly on the cap's equator, where
    # the cap bit would hang on round-off in the turning axis
    col = I.janus((16.0, 48.0, 48.0), (0.3, 0.9, 0.2), R, alpha=0.0, mu=mu, theta=90.0)
    w = I.workload_paper([col], E=E)
    w["params"].update(flags=flags, M_psi=M_psi, ch_substeps=nsub)
    w["c"] = w["params"]["c_b0"] + E * np.tanh(w["psi"])
    w["precision"] = precision
    return w


@pytest.mark.parametrize("precision,steps,tol", [("fp64", 20, 1e-12), ("fp32", 20, 2e-5)])
def test_paper_box_matches_oracle(precision, steps, tol):
    # the paper's box with the option, a sphere on the interface pushed
    # phoretically, 20 steps: owner maps and links exact, fields within the
    # precision's bar, the particle's state within 1e-11 (FP64)
    w = _trap_spec(precision=precision)
    g = lb.from_spec(w)
    o = oracle.from_spec(dict(w, precision="fp64"))
    g.step(steps)
    o.step(steps)
    assert np.array_equal(g.owner(), o.owner())
    assert np.array_equal(g.links(), o.links())
    e = field_errors(g.fields(), o.fields(), o.owner() < 0,
                     u_floor=None if precision == "fp64" else U_FLOOR_FP32)
    flush_print("[stress form] %s errors %s" % (precision, e))
    assert max(e.values()) <= tol
    if precision == "fp64":
        _, cg = g.observables()
        _, co = o.observables()
        for a in ("vel", "omega", "pos"):
            assert np.abs(cg[0][a] - co[0][a]).max() <= 1e-11, a
    g.close()
    o.close()


def test_batched_beside_a_box_without_the_option():
    # one launch per kernel for both boxes: the box with the option takes
    # the one-node forms and the fix-ups, the other its own path; each gives
    # the bits it gives alone
    import torch
    s = torch.cuda.Stream()
    a_spec = _trap_spec()
    b_spec = _trap_spec(flags=lb.LB_CAPILLARY_FORCE, mu=0.1)
    a = lb.from_spec(a_spec, stream=s)
    b = lb.from_spec(b_spec, stream=s)
    lb.batch_step([a, b], 40)
    a1 = lb.from_spec(a_spec, stream=s)
    b1 = lb.from_spec(b_spec, stream=s)
    a1.step(40)
    b1.step(40)
    assert np.array_equal(a.populations(), a1.populations())
    assert np.array_equal(b.populations(), b1.populations())
    for x in (a, b, a1, b1):
        x.close()


def test_option_validated():
    with pytest.raises(lb.LBError):
        lb.Box((32, 32, 32), "fp32", **dict(I.FREE_ENERGY, flags=lb.LB_STRESS_FORM))
