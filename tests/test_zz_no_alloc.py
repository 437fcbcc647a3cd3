"""GPU test of lb_batch_step_noalloc, the batched step that allocates
nothing (its tables in the library's fixed device array, launches one by
one): on two calls in a row, the second with a smaller batch, every box
equals the same box advanced by lb_batch_step, bit for bit; a batch whose
tables exceed the array is refused."""
import numpy as np
import pytest

from paper_2202_01631_amd import inputs as I
from paper_2202_01631_amd import lb

pytestmark = pytest.mark.gpu


def _state(b):
    f = b.fields()
    _, cols = b.observables(check=False)
    return [b.populations(), f["psi"], f["c"], f["u"], b.owner(), b.links()] + \
        [q[k] for q in cols for k in ("pos", "vel", "omega", "m")]


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("precision,nsub", [("fp32", 1), ("fp16", 2)])
def test_noalloc_batch_equals_batch_step(precision, nsub):
    import torch
    st = torch.cuda.Stream()
    for call, (count, sides, steps) in enumerate((((6, (32, 48, 64), 7)), ((2, (32,), 4)))):
        specs = I.batch_boxes(count=count, seed=23 + call, sides=sides, steps=steps)
        for s in specs:
            s["params"] = dict(s["params"], ch_substeps=nsub)
        ref = [lb.from_spec(s, precision=precision, stream=st) for s in specs]
        got = [lb.from_spec(s, precision=precision, stream=st) for s in specs]
        print("[noalloc] call %d: %d boxes, %s, %d steps" % (call, count, precision, steps),
              flush=True)
        lb.batch_step(ref, steps)
        lb.batch_step_noalloc(got, steps)
        for j, (a, b) in enumerate(zip(ref, got)):
            assert _same(_state(a), _state(b)), (call, j)
        for b in ref + got:
            b.close()


def test_noalloc_refuses_a_batch_beyond_its_array():
    # 4100 small boxes without particles: more descriptor tables than the
    # fixed array holds (about 4000 boxes): a clear error, nothing stepped
    specs = dict(I.batch_boxes(count=1, seed=3, sides=(32,), steps=1)[0])
    N = 8 ** 3
    boxes = []
    for k in range(4100):
        b = lb.Box((8, 8, 8), "fp32", **lb.spec_params(specs))
        b.init_fields(np.zeros(N), np.zeros(N))
        boxes.append(b)
    with pytest.raises(lb.LBError, match="too large"):
        lb.batch_step_noalloc(boxes, 2)
    t, _ = boxes[0].observables()
    assert t["step"] == 0
    lb.batch_step_noalloc(boxes[:100], 2)
    assert boxes[0].observables()[0]["step"] == 2
    for b in boxes:
        b.close()
