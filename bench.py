"""Benchmark of the lattice update on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: a 256^3 periodic box, planar interface with noise, 64 Janus spheres
of radius 6 (32 on the interface, 32 near it), moving, FP32 shifted
population storage; every step is the whole update (chemical potential,
collide-stream, psi/c update, bounce-back links and particle update, cover/
uncover, geometry).  Inputs are resident in HBM before timing.  Prints one
JSON line; the same workload in FP64 (the plain double-precision form) and in
FP16 storage is timed beside it, and the FP64 CPU oracle is timed on one step
of it on the host (cpu_baseline).
"""
import argparse
import faulthandler
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = ("MLUPS & % HBM roofline (256³ FP32 vs FP64 plain); batched sweep p50/p99")
# algorithmic bytes per lattice update: 19 populations and psi, c read once
# and written once (storage bytes 8 / 4 / 2, psi and c in the compute type)
STEP_BYTES = {"fp64": 19 * 2 * 8 + 2 * 2 * 8, "fp32": 19 * 2 * 4 + 2 * 2 * 4,
              "fp16": 19 * 2 * 2 + 2 * 2 * 4,
              # single phase (Sec. III.A, psi absent): populations and c only
              "fp32_single_phase": 19 * 2 * 4 + 2 * 4}
# the collide-stream kernel alone moves the populations: 19 read + 19 written
COLLIDE_BYTES = {"fp64": 19 * 2 * 8, "fp32": 19 * 2 * 4, "fp16": 19 * 2 * 2}
KERNELS = ("k_mu", "k_collide", "k_scalar", "k_link_partial+k_colloid_update", "k_cover",
           "k_commit+k_link_count+k_link_write")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_collide_box256_fp32_traffic.json")


def kernel_source_hash():
    """Hash of the kernel sources with comments and whitespace removed: the
    stored HBM counters stay valid across comment edits, not code changes."""
    h = hashlib.sha256()
    for f in ("lb_kernels.hip", "lb_device.h", "lb_kernels.h"):
        with open(os.path.join(ROOT, "paper_2202_01631_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def settle(box, torch, seconds=1.0):
    """More untimed steps until `seconds` of stepping have passed: the first
    timed repetition after a short warm-up ran 3-6% slower than the ones after
    it (the GPU's clocks still settling), the later ones agreeing within 1%."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        box.step(20)
        torch.cuda.synchronize()


def time_gpu(spec, precision, steps, warmup, torch, lb):
    """Timed steps on the production path: a non-default stream, so the
    library replays captured step-pair graphs with the particle work on its
    side stream.  Then a separate run with per-kernel HIP-event timing (the
    kernels in order, no graphs) for the breakdown and the roofline."""
    stream = torch.cuda.Stream()
    arena = torch.empty(lb.footprint_bytes(spec["shape"], precision), dtype=torch.uint8,
                        device="cuda")
    box = lb.from_spec(spec, precision=precision, arena=arena, stream=stream)
    from paper_2202_01631_amd import tune
    tune.apply(box)  # cached autotuned launch shapes for this size, if any
    box.step(warmup)
    torch.cuda.synchronize()
    settle(box, torch)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    box.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    # four more repetitions of the same K steps, reported beside the timed one
    reps = [ms / steps]
    for _ in range(4):
        ev0.record(stream)
        box.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        reps.append(ev0.elapsed_time(ev1) / steps)
    ksteps = min(steps, 50)
    box.timing_enable(True)
    box.step(ksteps)
    torch.cuda.synchronize()
    kms, calls = box.timing_read()
    box.timing_enable(False)
    tot, _ = box.observables(check=False)
    box.close()
    del arena
    torch.cuda.synchronize()
    N = spec["shape"][0] * spec["shape"][1] * spec["shape"][2]
    per_kernel = {KERNELS[i]: (kms[i] / calls[i] if calls[i] else None) for i in range(6)}
    return dict(ms_per_step=ms / steps, mlups=N * steps / (ms * 1e-3) / 1e6,
                kernel_ms=per_kernel, kernel_steps=ksteps, error_bits=tot["error_bits"], N=N,
                reps_ms_per_step=[round(v, 5) for v in reps],
                median_ms_per_step=round(float(sorted(reps)[len(reps) // 2]), 5))


def single_phase_spec(spec):
    """The same box and particles in the single-phase form of Sec. III.A:
    A = kappa = E = c_b0 = 0 and psi = 0 (no interface, no wetting)."""
    import numpy as np
    p = dict(spec["params"], a=0.0, b=0.0, kappa=0.0, E=0.0, c_b0=0.0)
    cols = [dict(q, H=0.0) for q in spec["colloids"]]
    return dict(spec, name=spec.get("name", "") + "_single_phase", params=p,
                psi=np.zeros_like(spec["psi"]), colloids=cols)


def copy_ceiling(torch):
    """Device copy of 1 GiB (read 1 GiB + write 1 GiB), best of 5: the HBM
    rate a plain streaming kernel reaches on this part."""
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1)
        best = t if best is None else min(best, t)
    del src, dst
    return 2.0 * (1 << 30) / (best * 1e-3) / 1e9


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def batched_sweep(torch, lb, I, nbox, steps, eager_steps=100, baselines=True):
    """Boxes of the batched sweep (sides 32/48/64, one sphere each), FP32:
    aggregate MLUPS of the batched graph-replayed step against the same boxes
    advanced one after another on the single-box production path (a
    non-default stream, graph-replayed step pairs, tuned shapes where cached),
    and, for fewer steps, one after another with eager launches on the
    default stream."""
    from paper_2202_01631_amd import tune
    specs = I.batch_boxes(count=nbox, steps=steps)
    nodes = sum(s["shape"][0] * s["shape"][1] * s["shape"][2] for s in specs)
    lu = nodes * steps
    stream = torch.cuda.Stream()
    # the batch takes the shape rules tuned for this batch as a whole, where
    # cached (the shapes cached for small boxes stepped alone differ in form
    # between the sizes, and a mixed batch falls back to the one-node forms)
    boxes = [lb.from_spec(s, precision="fp32", stream=stream) for s in specs]
    rules = tune.tuned_batch_rules((32, 48, 64), nbox, "fp32")
    if rules:
        tune.apply_batch(boxes, rules)
    lb.batch_step(boxes, 4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lb.batch_step(boxes, steps)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    for b in boxes:
        b.close()

    def one_by_one(stream, k):
        # boxes one after another; the finish time of each (synchronised
        # after each box) is its time to result when all arrive together
        bs = [lb.from_spec(s, precision="fp32", stream=stream) for s in specs]
        for b in bs:
            tune.apply(b)
            b.step(4)
        torch.cuda.synchronize()
        done = []
        t0 = time.perf_counter()
        for b in bs:
            b.step(k)
            torch.cuda.synchronize()
            done.append(time.perf_counter() - t0)
        t = done[-1]
        for b in bs:
            b.close()
        return nodes * k / t / 1e6, done

    def pct(v, q):
        v = sorted(v)
        return v[min(len(v) - 1, max(0, int(math.ceil(q * len(v))) - 1))]

    bm = lu / tb / 1e6
    if not baselines:
        return dict(boxes=nbox, steps=steps, lattice_updates=lu, batched_mlups=round(bm, 1),
                    batch_shape_rules=rules or "library defaults")
    seq, done = one_by_one(torch.cuda.Stream(), steps)
    eager, _ = one_by_one(None, min(steps, eager_steps))
    # every member of the sweep submitted at once: batched, all results come
    # with the last batched step; one after another, member k waits for the
    # k - 1 before it
    ttr = {"batched": {"p50_s": round(tb, 3), "p99_s": round(tb, 3)},
           "sequential": {"p50_s": round(pct(done, 0.50), 3), "p99_s": round(pct(done, 0.99), 3)},
           "note": "all %d members submitted at t = 0; time from the first step to each "
                   "member's last step" % nbox}
    return dict(boxes=nbox, steps=steps, lattice_updates=lu, batched_mlups=round(bm, 1),
                batch_shape_rules=rules or "library defaults",
                sequential_mlups=round(seq, 1), speedup=round(bm / seq, 3),
                sequential_eager_mlups=round(eager, 1), sequential_eager_steps=min(steps, eager_steps),
                speedup_vs_eager=round(bm / eager, 3), time_to_result=ttr)


def serving_run(torch, I, nreq, rate, step_scale):
    """Continuous-batching server on a Poisson trace (rate/s, sides 32..96,
    1-8 spheres, FP32 or FP16 storage), request lengths scaled by step_scale
    to bound the run; p50/p99 time-to-result and sustained MLUPS."""
    from paper_2202_01631_amd import serve
    trace = I.serving_trace(n_requests=nreq, rate=rate)
    free, _ = torch.cuda.mem_get_info()
    streams = {"fp32": torch.cuda.Stream(), "fp16": torch.cuda.Stream()}
    _, summ, _ = serve.replay(trace, budget_bytes=int(0.5 * free), chunk=100,
                              step_scale=step_scale, streams=streams)
    summ = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()}
    summ.update(rate_per_s=rate, step_scale=step_scale)
    return summ


def _field_errors(a, b, fluid):
    """Per field max|a - b| over the fluid nodes relative to max|b| (floors:
    rho, psi 1; c 1e-6; u 1e-8), the measure the precision forms are stated in."""
    out = {}
    for key, floor in (("rho", 1.0), ("psi", 1.0), ("c", 1e-6), ("u", 1e-8)):
        x, y = a[key][..., fluid], b[key][..., fluid]
        out[key] = float(abs(x - y).max() / max(float(abs(y).max()), floor))
    # the velocity also absolutely: in a nearly quiescent box max|u| is small
    out["u_abs"] = float(abs(a["u"][..., fluid] - b["u"][..., fluid]).max())
    out["u_max"] = float(abs(b["u"][..., fluid]).max())
    return out


def _far_from_solid(solid, shape, reach):
    """Nodes more than `reach` face steps from every node of `solid` (periodic)."""
    import numpy as np
    nx, ny, nz = shape
    grown = solid.reshape(nz, ny, nx).copy()
    for _ in range(reach):
        g = grown.copy()
        for ax in range(3):
            g |= np.roll(grown, 1, axis=ax) | np.roll(grown, -1, axis=ax)
        grown = g
    return ~grown.reshape(-1)


def precision_runs(torch, lb, I, steps1=10000, steps2=5000, every=1000):
    """The precision forms against the FP64 GPU path (itself held to the oracle
    by the parity tests): 128^3 FP32 and one sphere of radius 8 on the
    interface for 10^4 steps, the particle's trajectory sampled every 1000
    steps; 256^3 with 64 spheres in FP16 storage for 5000 steps, with FP32
    beside it as the reference for how far round-off alone carries that
    many-particle run, per-field errors and the particles' velocities at the
    end.  Each run is timed."""
    import numpy as np
    out = {}
    many = I.workload_many(n=256, count=64, radius=6.0)
    cases = (("box128_fp32_vs_fp64", I.workload_single(n=128), ("fp32",), steps1),
             # FP32 beside FP16 storage: how far round-off alone carries the
             # many-particle run in the same number of steps
             ("box256_fp16_vs_fp64", many, ("fp16", "fp32"), steps2))
    for name, spec, precs, steps in cases:
        runs = {}
        for p in precs + ("fp64",):
            st = torch.cuda.Stream()
            b = lb.from_spec(spec, precision=p, stream=st)
            from paper_2202_01631_amd import tune
            tune.apply(b)
            traj, t = [], 0.0
            for k in range(steps // every):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                b.step(every)
                torch.cuda.synchronize()
                t += time.perf_counter() - t0
                _, cols = b.observables(check=False)
                traj.append([c["pos"].copy() for c in cols])
            tot, cols = b.observables(check=False)
            runs[p] = dict(traj=traj, cols=cols, fields=b.fields(), fluid=b.owner() < 0,
                           bits=tot["error_bits"], mlups=b.N * steps / t / 1e6)
            b.close()
        hi = runs["fp64"]
        L = np.array(spec["shape"], dtype=float)

        def dpos(p, q):
            d = (p - q + L / 2) % L - L / 2
            return float(np.abs(d).max())
        for prec in precs:
            lo = runs[prec]
            traj_dev = [max(dpos(p, q) for p, q in zip(a, b))
                        for a, b in zip(lo["traj"], hi["traj"])]
            vmax = max(float(np.abs(c["vel"]).max()) for c in hi["cols"])
            vdev = max(float(np.abs(a["vel"] - b["vel"]).max())
                       for a, b in zip(lo["cols"], hi["cols"]))
            key = name if prec == precs[0] else name.replace(precs[0], prec)
            out[key] = dict(
                steps=steps, precision=prec,
                mlups={prec: round(lo["mlups"], 1), "fp64": round(hi["mlups"], 1)},
                # nodes whose solid/fluid state differs (the particles' paths
                # differ slightly); the field errors are over the nodes fluid in both
                owner_differences=int((lo["fluid"] != hi["fluid"]).sum()),
                field_errors={k: float("%.3g" % v) for k, v in
                              _field_errors(lo["fields"], hi["fields"],
                                            lo["fluid"] & hi["fluid"]).items()},
                # the same away from the particles (more than 3 face steps from a
                # solid node of either run), where cover/uncover at slightly
                # different times leaves local transients
                field_errors_away_from_particles={
                    k: float("%.3g" % v) for k, v in
                    _field_errors(lo["fields"], hi["fields"],
                                  _far_from_solid(~(lo["fluid"] & hi["fluid"]), spec["shape"],
                                                  3)).items()},
                # largest particle position difference at every sample (every `every` steps)
                position_deviation=[float("%.3g" % v) for v in traj_dev], sample_every=every,
                velocity_deviation_of_max_v=float("%.3g" % (vdev / max(vmax, 1e-30))),
                velocity_deviation=float("%.3g" % vdev), max_v=float("%.3g" % vmax),
                error_bits=[lo["bits"], hi["bits"]])
    return out


def paper_regime_run(torch, lb, I, steps=2000, warmup=200):
    """The paper's own regime (Sec. II.C): 64 x 96 x 96, M_psi = 0.4 in two
    psi/c sub-steps, D_c = 0.05, R = 4.5, capillary stress on the particles;
    an active Janus sphere on the interface and an inactive one in the bulk,
    FP32, graph-replayed on a non-default stream.  Beside it the same box in
    the default form (M_psi = 0.1, one psi/c update per step, no capillary
    stress), to show what the sub-steps and the stress cost, and the paper's
    form with the divergence-form solvent force (LB_STRESS_FORM).  Tuned launch
    shapes where the cache has them."""
    from paper_2202_01631_amd import tune
    cols = [I.janus((16.3, 47.6, 48.2), (0.29, 0.94, 0.19), 4.5, alpha=1e-3, mu=0.3, theta=60.0),
            I.janus((33.0, 20.4, 70.7), (0.0, 0.0, 1.0), 4.5, alpha=0.0, mu=0.2, theta=90.0)]
    out = {}
    for name, over in (("paper", {}), ("default_form", dict(M_psi=0.1, ch_substeps=1, flags=0)),
                       ("paper_stress_form", dict(flags=lb.LB_CAPILLARY_FORCE | lb.LB_STRESS_FORM))):
        w = I.workload_paper(cols, E=-0.25)
        w["params"].update(over)
        st = torch.cuda.Stream()
        b = lb.from_spec(w, stream=st)
        tune.apply(b)
        b.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        t, _ = b.observables()
        b.close()
        N = w["shape"][0] * w["shape"][1] * w["shape"][2]
        out[name] = dict(ms_per_step=round(ms, 5), mlups=round(N / ms / 1e3, 1),
                         error_bits=t["error_bits"])
    # the single-phase runs of Fig. 3 (A = kappa = E = 0, psi = 0): no mu
    # pass, chi read from c
    col = dict(cols[0], H=0.0)
    w = I.workload_paper([col], single_phase=True)
    b = lb.from_spec(w, stream=torch.cuda.Stream())
    tune.apply(b)
    b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    t, _ = b.observables()
    b.close()
    out["single_phase"] = dict(ms_per_step=round(ms, 5), mlups=round(64 * 96 * 96 / ms / 1e3, 1),
                               error_bits=t["error_bits"], particles=1, ch_substeps=2)
    out.update(shape=[64, 96, 96], precision="fp32", particles=2, steps=steps,
               paper=dict(out["paper"], M_psi=0.4, ch_substeps=2, capillary_force=True))
    # a parameter scan of the kind behind Figs. 3-4: 8 boxes of the regime
    # (mu in {0.05, 0.1}, E in {-0.25, -0.125, 0, 0.125}: |mu E| small enough
    # that the slip stays at low Mach number), one batched launch per kernel,
    # graph-replayed
    st = torch.cuda.Stream()
    boxes = []
    for mu in (0.05, 0.1):
        for E in (-0.25, -0.125, 0.0, 0.125):
            c = [dict(cols[0], mu_minus=mu, mu_plus=mu), cols[1]]
            boxes.append(lb.from_spec(I.workload_paper(c, E=E), stream=st))
    lb.batch_step(boxes, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lb.batch_step(boxes, steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    errs = 0
    for b in boxes:
        errs |= b.observables()[0]["error_bits"]
        b.close()
    n8 = len(boxes) * 64 * 96 * 96
    out["scan_8_boxes_batched"] = dict(ms_per_step=round(ms, 5), mlups=round(n8 / ms / 1e3, 1),
                                       error_bits=errs)
    return out


def cpu_baseline(spec):
    """The FP64 oracle on one step of the workload, on one host thread and on
    all of them (OpenMP over the per-node loops; bitwise the same result)."""
    import oracle
    model, ncpu = cpu_info()
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = ncpu
    nthreads = int(os.environ.get("OMP_NUM_THREADS", avail) or avail)
    N = spec["shape"][0] * spec["shape"][1] * spec["shape"][2]
    out = {}
    for label, nt in (("one", 1), ("all", nthreads)):
        used = oracle.set_threads(nt)
        log("[bench] cpu baseline: FP64 oracle, 1 step of the workload, %d thread(s)" % used)
        t0 = time.time()
        o = oracle.from_spec(spec)
        t1 = time.time()
        o.step(1)
        t2 = time.time()
        o.close()
        out[label] = dict(mlups=round(N / (t2 - t1) / 1e6, 4), threads=used,
                          step_s=round(t2 - t1, 2), setup_s=round(t1 - t0, 1))
    oracle.set_threads(1)
    return dict(value=out["one"]["mlups"], unit="MLUPS", cores=1, kind="oracle",
                all_cores=out["all"],
                sample="1 time step of the full 256^3 64-sphere workload, FP64 oracle, one "
                       "thread (step %.1f s, setup %.1f s excluded); the same step on %d "
                       "threads: %.3f MLUPS; %s, %s logical CPUs visible, %d usable"
                       % (out["one"]["step_s"], out["one"]["setup_s"], out["all"]["threads"],
                          out["all"]["mlups"], model, ncpu, avail))


def main():
    faulthandler.enable()  # a native crash prints the Python stack
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", default=None, help="time one precision only (profiling runs)")
    ap.add_argument("--paper-only", action="store_true",
                    help="run only the paper-regime leg (profiling runs)")
    ap.add_argument("--batch", type=int, default=512, help="boxes in the batched sweep (0: skip)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched sweep (profiling runs)")
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--serve", type=int, default=0,
                    help="requests in the serving run (0: skip, the default: the serving replay "
                         "ended twice in a host segmentation fault whose cause is not found, so "
                         "it stays off until it is)")
    ap.add_argument("--serve-scale", type=float, default=0.25,
                    help="request length scale of the serving run (at 0.25 the offered load "
                         "at 50 requests/s is ~45k MLUPS, above one GPU's capacity)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (torch) five times, for "
                         "scaling the HBM byte counters against a kernel of known traffic")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: one GPU only (--gpus 1); no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_calibration:
        torch.cuda.set_device(0)
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": 1 << 30, "bytes_written": 1 << 30,
                                               "launches": 5}}), flush=True)
        return

    from paper_2202_01631_amd import inputs as I
    from paper_2202_01631_amd import lb
    lb.load()
    torch.cuda.set_device(0)
    if args.batch_only:
        print(json.dumps({"batched_sweep": batched_sweep(torch, lb, I, args.batch, args.batch_steps,
                                                          baselines=False)}), flush=True)
        return
    if args.paper_only:
        # the paper-regime leg alone (profiling runs)
        print(json.dumps({"paper_regime": paper_regime_run(torch, lb, I, steps=args.steps,
                                                           warmup=args.warmup)}), flush=True)
        return
    n = args.size
    spec = I.workload_many(n=n, count=64, radius=6.0, precision="fp32")
    res = {}
    precs = [args.only] if args.only else ["fp32", "fp64", "fp16"]
    for prec in precs:
        log("[bench] %d^3 %s: warmup %d, timed %d" % (n, prec, args.warmup, args.steps))
        res[prec] = time_gpu(spec, prec, args.steps, args.warmup, torch, lb)
        log("[bench] %s: %.3f ms/step, %.0f MLUPS, kernels %s" % (
            prec, res[prec]["ms_per_step"], res[prec]["mlups"], res[prec]["kernel_ms"]))
    if not args.only:
        log("[bench] %d^3 fp32 single phase: warmup %d, timed %d" % (n, args.warmup, args.steps))
        res["fp32_single_phase"] = time_gpu(single_phase_spec(spec), "fp32", args.steps,
                                            args.warmup, torch, lb)
        log("[bench] single phase: %.3f ms/step, %.0f MLUPS" % (
            res["fp32_single_phase"]["ms_per_step"], res["fp32_single_phase"]["mlups"]))
    main_prec = precs[0]
    r = res[main_prec]
    N = r["N"]
    kc = r["kernel_ms"]["k_collide"]
    achieved = COLLIDE_BYTES[main_prec] * N / (kc * 1e-3) / 1e9
    traffic = None
    if main_prec == "fp32" and os.path.exists(TRAFFIC_FILE):
        t = json.load(open(TRAFFIC_FILE))
        if t.get("kernel_source_hash") == kernel_source_hash() and t.get("size") == n:
            traffic = t.get("bytes_per_launch")
    copy_gbs = copy_ceiling(torch)
    log("[bench] copy ceiling %.0f GB/s" % copy_gbs)
    out = {
        "metric": METRIC,
        "value": round(r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "fp16": "f16-storage/f32"}[main_prec],
        "data": "synthetic",
        "config": {"workload": "box%d_64spheres_%s" % (n, main_prec), "shape": [n, n, n],
                   "spheres": 64, "radius": 6.0, "precision": main_prec,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_collide",
                     "bytes_per_lu": COLLIDE_BYTES[main_prec],
                     # the kernel's counted HBM bytes over its time, and both
                     # rates against a plain device copy measured in this run
                     "traffic_GBs": (round(traffic / (kc * 1e-3) / 1e9, 1) if traffic else None),
                     "copy_ceiling_GBs": round(copy_gbs, 1),
                     "frac_of_copy": round(achieved / copy_gbs, 4),
                     "traffic_frac_of_copy": (round(traffic / (kc * 1e-3) / 1e9 / copy_gbs, 4)
                                              if traffic else None),
                     # the whole step beside the kernel: its algorithmic bytes
                     # (state read and written once) at the measured rate
                     "step_bytes_per_lu": STEP_BYTES[main_prec],
                     "step_achieved": round(r["mlups"] * 1e6 * STEP_BYTES[main_prec] / 1e9, 1),
                     "step_frac": round(r["mlups"] * 1e6 * STEP_BYTES[main_prec] / 1e9
                                        / HBM_PEAK_GBS, 4)},
        "reps_ms_per_step": r["reps_ms_per_step"],
        "median_ms_per_step": r["median_ms_per_step"],
        "step_roofline": {p: {"mlups": round(v["mlups"], 1),
                              "algorithmic_GBs": round(v["mlups"] * 1e6 * STEP_BYTES[p] / 1e9, 1),
                              "frac": round(v["mlups"] * 1e6 * STEP_BYTES[p] / 1e9 / HBM_PEAK_GBS, 4),
                              "bytes_per_lu": STEP_BYTES[p],
                              "kernel_ms": {k: (round(x, 5) if x else None)
                                            for k, x in v["kernel_ms"].items()},
                              "error_bits": v["error_bits"]} for p, v in res.items()},
    }
    # secondary legs: a library error there is recorded in the line rather
    # than losing it
    if args.batch and not args.only:
        log("[bench] batched sweep: %d boxes x %d steps" % (args.batch, args.batch_steps))
        try:
            out["batched_sweep"] = batched_sweep(torch, lb, I, args.batch, args.batch_steps)
        except lb.LBError as e:
            out["batched_sweep"] = {"error": str(e)}
        log("[bench] batched sweep %s" % out["batched_sweep"])
    if not args.only:
        log("[bench] precision forms against the FP64 GPU path (128^3 x 10^4, 256^3 x 5000)")
        try:
            out["precision_forms"] = precision_runs(torch, lb, I)
        except lb.LBError as e:
            out["precision_forms"] = {"error": str(e)}
        log("[bench] precision forms %s" % out["precision_forms"])
        log("[bench] paper regime 64x96x96")
        try:
            out["paper_regime"] = paper_regime_run(torch, lb, I)
        except lb.LBError as e:
            out["paper_regime"] = {"error": str(e)}
        log("[bench] paper regime %s" % out["paper_regime"])
    if args.serve and not args.only:
        log("[bench] serving: %d requests" % args.serve)
        out["serving"] = serving_run(torch, I, args.serve, 50.0, args.serve_scale)
        log("[bench] serving %s" % out["serving"])
        # below capacity: 5 requests/s
        out["serving_low_rate"] = serving_run(torch, I, max(1, min(12, args.serve)), 5.0,
                                              args.serve_scale)
        log("[bench] serving at 5/s %s" % out["serving_low_rate"])
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(spec)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
