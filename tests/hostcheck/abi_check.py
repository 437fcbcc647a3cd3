"""Drive the sanitizer build of the library (liblb_hostcheck.so) through the
rest of the C ABI's call sequences (TEST INFRASTRUCTURE): every entry point,
the error paths, save/load, timing, launch shapes, a batch of uneven boxes on
a caller stream with an odd step count, contexts destroyed in any order,
particles with surface patterns.
Exit status 0 and "abi ok" mean no sanitizer or runtime-misuse report.

    python abi_check.py LIB
"""
import ctypes as C
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.modules["torch"] = None

import numpy as np  # noqa: E402

from paper_2202_01631_amd import inputs as I  # noqa: E402
from paper_2202_01631_amd import lb  # noqa: E402


def expect_error(fn, *a):
    try:
        fn(*a)
    except lb.LBError:
        return
    raise AssertionError("expected an LBError from %s" % fn)


def main():
    lb.LIB_PATH = sys.argv[1]
    lb._lib = None
    L = lb.load()
    L.hostcheck_live_allocations.restype = C.c_size_t
    st = C.c_void_p()
    assert L.hipStreamCreateWithFlags(C.byref(st), 1) == 0
    w = I.workload_small()
    for prec in ("fp64", "fp32", "fp16"):
        for stream in (None, st.value):
            b = lb.from_spec(w, precision=prec, stream=stream)
            b.step(3)
            b.observables(check=False)
            b.fields()
            b.populations()
            b.owner()
            b.links()
            b.colloid_forces()
            s = b.save_state()
            b.load_state(s)
            b.step(2)
            b.timing_enable(True)
            b.step(1)
            b.timing_read()
            b.timing_enable(False)
            b.set_launch_shapes([(64, 4, 0), (32, 8, 1), (0, 0, 2 + 8 * 4)])
            b.launch_shapes()
            b.step(4)
            # new shapes straight after a graph-replayed step: the captured
            # step pairs are dropped only once their replay has finished
            b.set_launch_shapes([(32, 8, 0), (64, 4, 0), (0, 0, 2 + 8 * 4)])
            b.step(2)
            expect_error(b.set_launch_shapes, [(-1, 0, 0)] * 3)
            b.close()
    # error paths before and after init
    b = lb.Box((16, 16, 16), "fp32", **lb.spec_params(w))
    expect_error(b.step, 1)
    expect_error(b.add_colloids, w["colloids"])
    b.close()
    expect_error(lambda: lb.Box((16, 16, 16), "fp32", tau=0.4))
    # a batch of uneven boxes (sizes, particle counts, options) on a caller
    # stream, odd step count, destroyed in a different order
    specs = I.batch_boxes(count=6, sides=(32, 40, 48), steps=5)
    boxes = [lb.from_spec(s, stream=st.value) for s in specs]
    boxes[2].add_colloids([])
    lb.batch_step(boxes, 5)
    lb.batch_step(boxes[::-1], 2)
    expect_error(lb.batch_step, [boxes[0], boxes[0]], 2)
    for b in boxes[::2] + boxes[1::2]:
        b.observables(check=False)
        b.links()
        b.close()
    # surface patterns: a patterned box alone (boundary fix-up launches), in
    # a batch beside a Janus box, saved and loaded; bad patterns refused
    pw = dict(w, colloids=[dict(w["colloids"][0], e=(0.0, 0.0, 0.0),
                                pattern=dict(bands=2, sectors=4, cos=[0.2], alpha=[1e-3] * 8,
                                             mu=[0.1] * 8, H=[0.0] * 8))])
    pb = lb.from_spec(pw, precision="fp32", stream=st.value)
    pb.step(3)
    pb.links()
    s = pb.save_state()
    pb.load_state(s)
    other = lb.from_spec(w, precision="fp32", stream=st.value)
    lb.batch_step([pb, other], 3)
    for bad in (dict(bands=9, sectors=1), dict(bands=2, sectors=3, cos=[0.0]),
                dict(bands=3, sectors=1, cos=[0.5, 0.1])):
        expect_error(pb.add_colloids, [dict(pw["colloids"][0], pattern=bad)])
    pb.close()
    other.close()
    # a spheroid (boundary fix-up launches), stepped and batched; refused
    # with soft-sphere forces
    sw = dict(w, colloids=[dict(w["colloids"][0], axial=6.0)])
    sb = lb.from_spec(sw, precision="fp32", stream=st.value)
    sb.step(3)
    other = lb.from_spec(w, precision="fp32", stream=st.value)
    lb.batch_step([other, sb], 2)
    sb.close()
    other.close()
    # the divergence-form solvent force (one-node forms, fix-ups, 7 more
    # arena fields), alone and batched beside a box without it
    dw = dict(w, params=dict(w["params"], flags=lb.LB_CAPILLARY_FORCE | lb.LB_STRESS_FORM))
    db = lb.from_spec(dw, precision="fp32", stream=st.value)
    db.step(3)
    other = lb.from_spec(w, precision="fp32", stream=st.value)
    lb.batch_step([other, db], 2)
    db.close()
    other.close()
    expect_error(lambda: lb.Box((32, 32, 32), "fp32",
                                **dict(lb.spec_params(w), flags=lb.LB_STRESS_FORM)))
    soft = lb.Box((32, 32, 32), "fp32", **dict(lb.spec_params(w), soft_eps=0.05, soft_sigma=1.0,
                                               soft_nu=1.0, soft_hc=1.0))
    soft.init_fields(np.zeros(32 ** 3), np.zeros(32 ** 3))
    expect_error(soft.add_colloids, sw["colloids"])
    soft.close()
    # host parameter maps: Eq. 10, the lattice's own wetting map (its
    # one-dimensional minimisers, with a wide interface too) and Eq. 1's E
    for th in (0.0, 60.0, 90.0, 135.0):
        assert np.isfinite(lb.wetting_H(th, 0.04, 0.0625))
        assert np.isfinite(lb.wetting_H_lattice(th, -0.0625, 0.0625, 0.04))
    assert np.isfinite(lb.wetting_H_lattice(60.0, -0.0625, 0.0625, 4.0))
    assert np.isnan(lb.wetting_H_lattice(60.0, 0.0625, 0.0625, 0.04))
    assert np.isnan(lb.wetting_H_lattice(float("nan"), -0.0625, 0.0625, 0.04))
    assert np.isfinite(lb.solubility_E(3.0, 0.5))
    lw = dict(w, wetting_map="lattice")
    lbox = lb.from_spec(lw, precision="fp32", stream=st.value)
    lbox.step(2)
    lbox.close()
    left = L.hostcheck_live_allocations()
    print("abi ok: %d device allocations left" % left, flush=True)
    if left:
        sys.exit(3)


if __name__ == "__main__":
    main()
