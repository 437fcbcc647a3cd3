"""GPU tests of the production forms of the step: graph-replayed stepping,
batched multi-box launches and launch shapes.  Each box must come out
bitwise identical whatever way it is advanced, and stay within the FP64
oracle bars."""
import numpy as np
import pytest

import oracle
from paper_2202_01631_amd import inputs as I
from paper_2202_01631_amd import lb
from parity_util import field_errors, flush_print

pytestmark = pytest.mark.gpu


def _boxes(precision="fp32", seed=11, n=4):
    specs = I.batch_boxes(count=n, seed=seed, sides=(32, 48, 64), steps=20)
    return specs


def _state(b):
    return b.populations(), b.fields()["psi"], b.fields()["c"], b.owner(), b.links()


def _same(sa, sb):
    return all(np.array_equal(x, y) for x, y in zip(sa, sb))


def test_graph_replay_equals_eager():
    # a non-default stream enables the captured step-pair graph; replays are
    # interleaved with host reads (trap-safe: no memset nodes in the graph)
    import torch
    w = I.workload_small()
    stream = torch.cuda.Stream()
    g = lb.from_spec(w, precision="fp32", stream=stream)
    e = lb.from_spec(w, precision="fp32")  # default stream: eager launches
    for k in range(4):
        g.step(6)
        e.step(6)
        torch.cuda.synchronize()
        tg, _ = g.observables()
        te, _ = e.observables()
        flush_print("[graph] replay block", k, tg["mass"], te["mass"])
        assert _same(_state(g), _state(e))
    g.step(3)  # odd count: one pair from the graph, one eager step
    e.step(3)
    assert _same(_state(g), _state(e))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batched_equals_alone(precision):
    import torch
    specs = _boxes(n=5)
    stream = torch.cuda.Stream()
    batch = [lb.from_spec(s, precision=precision, stream=stream) for s in specs]
    alone = [lb.from_spec(s, precision=precision) for s in specs]
    # unequal histories first: box 1 is one step ahead (odd parity)
    batch[1].step(1)
    alone[1].step(1)
    lb.batch_step(batch, 9)
    for b in alone:
        b.step(9)
    for j, (b, a) in enumerate(zip(batch, alone)):
        flush_print("[batch] box", j, specs[j]["shape"])
        assert _same(_state(b), _state(a)), j
        tb, cb = b.observables()
        ta, ca = a.observables()
        assert tb["step"] == ta["step"]
        for k in range(len(cb)):
            for key in ("pos", "vel", "omega", "m"):
                assert np.array_equal(cb[k][key], ca[k][key])


def test_batched_fp64_matches_oracle():
    specs = _boxes(n=3, seed=5)
    batch = [lb.from_spec(s, precision="fp64") for s in specs]
    lb.batch_step(batch, 12)
    for j, s in enumerate(specs):
        o = oracle.from_spec(s)
        o.step(12)
        fl = o.owner() < 0
        assert np.array_equal(batch[j].owner(), o.owner())
        assert np.array_equal(batch[j].links(), o.links())
        e = field_errors(batch[j].fields(), o.fields(), fl)
        flush_print("[batch-oracle] box", j, s["shape"], e)
        assert max(e.values()) <= 1e-12


@pytest.mark.parametrize("shapes", [
    [(64, 4, 0), (64, 4, 0), (64, 4, 0)],
    [(32, 8, 2), (256, 1, 1), (16, 16, 2)],
    [(48, 5, 0), (24, 10, 0), (40, 6, 0)],
    [(64, 4, 0), (256, 1, 0), (64, 4, 8)],
    [(32, 8, 0), (32, 8, 0), (16, 16, 16)],
    [(32, 8, 0), (32, 8, 0), (32, 4, 40)],
])
def test_launch_shapes_do_not_change_results(shapes):
    w = I.workload_small()
    ref = lb.from_spec(w, precision="fp32")
    alt = lb.from_spec(w, precision="fp32")
    alt.set_launch_shapes(shapes)
    ref.step(15)
    alt.step(15)
    assert _same(_state(ref), _state(alt))


def test_batched_mixed_zmarch_equals_alone():
    # boxes of one batch disagreeing on the z-marching psi/c form fall back
    # to the one-node-per-thread form; results unchanged
    import torch
    specs = _boxes(n=3, seed=21)
    stream = torch.cuda.Stream()
    batch = [lb.from_spec(s, precision="fp32", stream=stream) for s in specs]
    batch[0].set_launch_shapes([(0, 0, 0), (0, 0, 0), (0, 0, 8)])
    alone = [lb.from_spec(s, precision="fp32") for s in specs]
    lb.batch_step(batch, 6)
    for b in alone:
        b.step(6)
    for b, a in zip(batch, alone):
        assert _same(_state(b), _state(a))


def test_batch_error_paths():
    specs = _boxes(n=2)
    a = lb.from_spec(specs[0], precision="fp32")
    b = lb.from_spec(specs[1], precision="fp64")
    with pytest.raises(lb.LBError):
        lb.batch_step([a, b], 2)  # mixed precision
    with pytest.raises(lb.LBError):
        lb.batch_step([a, a], 2)  # repeated context
