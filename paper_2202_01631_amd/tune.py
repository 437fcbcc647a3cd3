"""Launch-shape autotuner for the three lattice kernels.

For a box size and precision, time every candidate block shape (x segment
length, rows per block, block renumbering, row-vector form) on the GPU with the library's
per-kernel HIP-event timing, keep the fastest shape of each kernel, and cache
the result in ``tuning.json`` next to this file, keyed by device name, box
size and precision.  Shapes never change results (tested bit for bit); they
only change speed.

    python -m paper_2202_01631_amd.tune 256 256 256 fp32
    python -m paper_2202_01631_amd.tune batch 512 [CACHE_PATH]

A batch of boxes is tuned as a whole (``tune_batch``): rules that give each
box a shape for its size, timed on the batched step.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")


def candidates(nx, ny):
    """(bx, by, code) shapes, code = remap + 8 vec + 64 zc."""
    out = []
    for bx in (256, 128, 64, 32, 16):
        if bx > nx and bx != min(nx, 256):
            continue
        b = min(bx, nx)
        by = max(1, 256 // b)
        for remap in (0, 2):
            if remap == 2 and (ny % by != 0):
                continue
            out.append((b, by, remap))
    for vec in (2, 4):
        if nx % vec == 0:
            for remap in (0, 2):
                out.append((0, 0, remap + 8 * vec))
            for zc in (4, 8, 16):
                out.append((0, 0, 8 * vec + 64 * zc))
    # distinct, natural-order default first
    seen, uniq = set(), []
    for c in [(min(nx, 256), max(1, 256 // min(nx, 256)), 0)] + out:
        if c not in seen:
            seen.add(c)
            uniq.append(c)
    return uniq


def is_vec(cand):
    return cand[2] >= 16


def launch_for(cand):
    """(shapes of the three kernels, which kernels' times count) for a
    candidate: one-node and row-vector shapes go to all three kernels (the
    collide-stream keeps its one-node form where a row does not fit one lane
    group; its time then does not count); z-marching shapes to the psi/c
    update only (mu takes the same row-vector form, collide its default)."""
    if cand[2] >= 64:
        return [(0, 0, cand[2] & 63), (0, 0, 0), cand], (False, False, True)
    return [cand, cand, cand], (True, True, True)


def device_key():
    import torch
    if not torch.cuda.is_available():
        return "none"
    pr = torch.cuda.get_device_properties(0)
    return "%s-%dCU" % (getattr(pr, "gcnArchName", pr.name).split(":")[0], pr.multi_processor_count)


def _key(shape, precision):
    return "%s|%dx%dx%d|%s" % (device_key(), shape[0], shape[1], shape[2], precision)


def load_cache():
    if os.path.exists(CACHE):
        with open(CACHE) as fh:
            return json.load(fh)
    return {}


def tuned_shapes(shape, precision):
    """Cached shapes for this device, size and precision, or None."""
    v = load_cache().get(_key(shape, precision))
    return [tuple(s) for s in v["shapes"]] if v else None


def apply(box):
    """Give a box the cached tuned shapes, if any."""
    s = tuned_shapes(box.shape, box.precision)
    if s:
        box.set_launch_shapes(s)
    return s


def representative_spec(shape, precision):
    """Workload a shape is tuned on: particles change the cost of the stencil
    kernels (boundary nodes), so boxes are tuned with them.  Cubic boxes of
    side 256 take the benchmark workload (64 spheres of radius 6 on and near
    the interface); other boxes one sphere of radius 4.5 on the interface."""
    from . import inputs as I
    if tuple(shape) == (256, 256, 256):
        return I.workload_many(n=256, count=64, radius=6.0, precision=precision)
    psi = I.flat_interface(shape, shape[2] / 2.0, I.WIDTH, 0.01)
    h = [s / 2.0 for s in shape]
    cols = []
    if min(shape) >= 17:
        cols = [I.janus((h[0] + 0.3, h[1] - 0.2, h[2]), (0.6, 0.0, 0.8), 4.5, mu=0.1, theta=70.0)]
    return dict(shape=tuple(shape), precision=precision, params=dict(I.FREE_ENERGY),
                solubility_ratio=2.0, psi=psi, c=np.zeros(psi.size), colloids=cols)


def tune(shape, precision="fp32", steps=20, warmup=4, write=True, spec=None, log=print):
    """Time every candidate shape for the three lattice kernels; return the
    best (bx, by, code) of each and store it in the cache."""
    import torch

    from . import inputs as I
    from . import lb
    if spec is None:
        spec = representative_spec(shape, precision)
    box = lb.from_spec(spec, precision=precision)
    results = {}
    for cand in candidates(shape[0], shape[1]):
        shapes, scored = launch_for(cand)
        box.set_launch_shapes(shapes)
        if is_vec(cand) and not is_vec(box.launch_shapes()[1]):
            scored = (scored[0], False, scored[2])
        box.step(warmup)
        torch.cuda.synchronize()
        box.timing_enable(True)
        box.step(steps)
        ms, calls = box.timing_read()
        box.timing_enable(False)
        t = [float(ms[i] / max(calls[i], 1)) if scored[i] else float("inf") for i in range(3)]
        results[cand] = t
        log("[tune] %s %s %s us %s" % (shape, precision, cand,
                                        [round(1000 * v, 1) for v in results[cand]]))
    box.close()
    best = [min(results, key=lambda c: results[c][k]) for k in range(3)]
    if write:
        cache = load_cache()
        cache[_key(shape, precision)] = {
            "shapes": [list(b) for b in best],
            "us": [round(1000 * results[best[k]][k], 2) for k in range(3)],
            "kernels": ["k_mu", "k_collide", "k_scalar"]}
        with open(CACHE + ".tmp", "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(CACHE + ".tmp", CACHE)
    return best


# ------------------------------------------------------------------ batches
# A batch runs one launch per lattice kernel over all its boxes, and every
# box of a launch takes the same kernel form (one node per thread, or row
# vectors of 2 or 4 nodes per lane); block sizes, row counts and renumbering
# may differ per box.  The shapes tuned for a box stepped alone do not serve
# the batch: alone, a small box is latency-bound and its winners differ in
# form between sizes.  So the batch is tuned as a whole: each candidate is a
# rule that gives every box a shape for its size, and the batched step is
# timed with it.

def batch_rules():
    """Shape rules for one kernel of a batch: name -> f(nx, ny) giving
    (bx, by, code), or None for the library's default shape.  One-node rules: whole rows (or 64- / 32-node segments)
    with 256 threads per block, natural or plane-wise XCD order; row-vector
    rules: 2 or 4 nodes per lane, natural or plane-wise order."""
    def node(seg, remap):
        def f(nx, ny):
            b = min(nx, seg) if seg else min(nx, 256)
            by = max(1, 256 // b)
            return (b, by, remap if ny % by == 0 else 0)
        return f

    def vec(v, remap):
        return lambda nx, ny: (0, 0, remap + 8 * v)
    rules = {"default": lambda nx, ny: None}
    for seg in (0, 64, 32):
        for remap in (0, 2):
            rules["node%s_r%d" % (seg or "row", remap)] = node(seg, remap)
    for v in (2, 4):
        for remap in (0, 2):
            rules["vec%d_r%d" % (v, remap)] = vec(v, remap)
    return rules


def _batch_key(sides, count, precision):
    return "%s|batch%d:%s|%s" % (device_key(), count, ",".join(str(s) for s in sides), precision)


def tuned_batch_rules(sides, count, precision):
    """Cached rule names (mu, collide, psi/c) for this batch, or None."""
    v = load_cache().get(_batch_key(sides, count, precision))
    return list(v["rules"]) if v else None


def apply_batch(boxes, rule_names):
    """Give every box of a batch the shapes of the three rules for its size."""
    rules = batch_rules()
    for b in boxes:
        if not hasattr(b, "default_shapes"):
            b.default_shapes = b.launch_shapes()
        nx, ny, _ = b.shape
        sh = [rules[r](nx, ny) for r in rule_names]
        b.set_launch_shapes([b.default_shapes[k] if sh[k] is None else sh[k] for k in range(3)])


def tune_batch(specs, sides, precision="fp32", steps=60, write=True, cache=None, log=print):
    """Coordinate descent over the three kernels' rules (psi/c update, mu,
    collide-stream; two passes), timing the whole batched step on a
    non-default stream; caches the best rules under the batch's sides, box
    count and precision."""
    import time

    import torch

    from . import lb
    stream = torch.cuda.Stream()
    boxes = [lb.from_spec(s, precision=precision, stream=stream) for s in specs]
    rules = batch_rules()

    def timed(names):
        apply_batch(boxes, names)
        lb.batch_step(boxes, 4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lb.batch_step(boxes, steps)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    best = ["default", "default", "default"]
    tbest = timed(best)
    log("[tune-batch] start %s %.4f ms/step" % (best, 1e3 * tbest))
    for _ in range(2):
        for w in (2, 0, 1):
            for name in rules:
                if name == best[w] or (w == 1 and name.startswith("vec2")):
                    continue
                cand = list(best)
                cand[w] = name
                t = timed(cand)
                log("[tune-batch] %s %.4f ms/step" % (cand, 1e3 * t))
                if t < tbest:
                    best, tbest = cand, t
    for b in boxes:
        b.close()
    log("[tune-batch] best %s %.4f ms/step" % (best, 1e3 * tbest))
    if write:
        path = cache or CACHE
        data = {}
        if os.path.exists(path):
            with open(path) as fh:
                data = json.load(fh)
        data[_batch_key(sides, len(specs), precision)] = {
            "rules": best, "ms_per_step": round(1e3 * tbest, 4),
            "kernels": ["k_mu", "k_collide", "k_scalar"]}
        with open(path + ".tmp", "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    return best


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "batch":
        # python -m paper_2202_01631_amd.tune batch COUNT [CACHE_PATH]
        from . import inputs as I
        count = int(sys.argv[2])
        sides = (32, 48, 64)
        specs = I.batch_boxes(count=count, sides=sides, steps=2000)
        print(tune_batch(specs, sides, cache=sys.argv[3] if len(sys.argv) > 3 else None))
        sys.exit(0)
    if len(sys.argv) < 5:
        print(__doc__)
        sys.exit(2)
    nx, ny, nz = (int(v) for v in sys.argv[1:4])
    print(tune((nx, ny, nz), sys.argv[4]))
