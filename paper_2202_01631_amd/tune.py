"""Launch-shape autotuner for the three lattice kernels.

For a box size and precision, time every candidate block shape (x segment
length, rows per block, block renumbering, row-vector form) on the GPU with the library's
per-kernel HIP-event timing, keep the fastest shape of each kernel, and cache
the result in ``tuning.json`` next to this file, keyed by device name, box
size and precision.  Shapes never change results (tested bit for bit); they
only change speed.

    python -m paper_2202_01631_amd.tune 256 256 256 fp32
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


if __name__ == "__main__":
    if len(sys.argv) < 5:
        print(__doc__)
        sys.exit(2)
    nx, ny, nz = (int(v) for v in sys.argv[1:4])
    print(tune((nx, ny, nz), sys.argv[4]))
