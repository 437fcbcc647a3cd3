"""Drive the sanitizer build of the library (liblb_hostcheck.so, see build.py)
with the serving loop's own call sequence (TEST INFRASTRUCTURE).

Runs ``paper_2202_01631_amd.serve.Server`` unchanged on a Poisson trace of
sweep requests: contexts created on admission, grouped by storage precision
on one caller stream per precision, advanced with ``lb_batch_step`` in
chunks (graph capture of step pairs on those streams), read back and
destroyed on retirement while the others keep going.  The kernels do not
run, so a simulated clock (lattice updates at a fixed rate) stands in for the
GPU's time; it keeps as many requests live at once as the GPU run had.

Must run in a process that preloads the shared AddressSanitizer runtime
(tests/test_host_sanitizers.py starts it so).  Exit status 0 and "replay ok"
mean no sanitizer or runtime-misuse report.

    python replay_check.py LIB N_REQUESTS RATE MLUPS BUDGET_BYTES COLLECT_EVERY
"""
import ctypes as C
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.modules["torch"] = None  # the sanitizer build has no use for torch's HIP runtime

from paper_2202_01631_amd import inputs as I  # noqa: E402
from paper_2202_01631_amd import lb, serve  # noqa: E402


def main():
    lib, nreq, rate, mlups, budget, every = sys.argv[1:7]
    nreq, rate, mlups, budget, every = int(nreq), float(rate), float(mlups), int(budget), int(every)
    lb.LIB_PATH = lib
    lb._lib = None
    L = lb.load()
    L.hostcheck_live_allocations.restype = C.c_size_t
    h = [C.c_void_p(), C.c_void_p()]
    for x in h:
        assert L.hipStreamCreateWithFlags(C.byref(x), 1) == 0
    streams = {"fp32": x_value(h[0]), "fp16": x_value(h[1])}

    seen = [0]

    def collect(box):
        # every few retirements, the full readback the serving tests use
        seen[0] += 1
        if seen[0] % every:
            return {}
        f = box.fields()
        return dict(pop=box.populations().shape, psi=f["psi"].shape, links=box.links().shape,
                    forces=box.colloid_forces()["F"].shape)

    trace = I.serving_trace(n_requests=nreq, rate=rate)
    srv = serve.Server(budget, max_slots=256, chunk=100, collect=collect, streams=streams)

    class VirtualTime:
        """Time of the replay: idle waits advance it directly, GPU work by
        its lattice updates at the given rate."""
        idle = 0.0

        def sleep(self, dt):
            VirtualTime.idle += dt

        def perf_counter(self):
            return VirtualTime.idle + srv.lattice_updates / (mlups * 1e6)

    serve.time = VirtualTime()
    for i, r in enumerate(trace):
        spec = I.serving_request(r)
        spec["steps"] = max(2, int(round(r["steps"] * 0.25)))
        srv.submit(i, spec, r["t"])
    res = srv.run()
    done = sum(1 for v in res.values() if "time_to_result" in v)
    left = L.hostcheck_live_allocations()
    print("replay ok: %d requests, %d completed, peak %d live, %d device allocations left"
          % (nreq, done, srv.peak_live, left), flush=True)
    if done != nreq or left != 0:
        sys.exit(3)


def x_value(p):
    return p.value


if __name__ == "__main__":
    main()
