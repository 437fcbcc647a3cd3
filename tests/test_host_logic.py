"""Host-side logic that needs no GPU: autotuner candidates and cache
format, serving admission sizes, the binding's structure layouts."""
import json
import os

import pytest

from paper_2202_01631_amd import inputs as I
from paper_2202_01631_amd import lb, serve, tune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _decode(code):
    return code & 7, (code >> 3) & 7, code >> 6


@pytest.mark.parametrize("nx,ny", [(256, 256), (32, 32), (48, 48), (30, 17), (1, 40), (70, 9)])
def test_tuner_candidates_are_valid_codes(nx, ny):
    cands = tune.candidates(nx, ny)
    assert cands[0] == (min(nx, 256), max(1, 256 // min(nx, 256)), 0)  # natural default first
    assert len(set(cands)) == len(cands)
    for bx, by, code in cands:
        rm, vec, zc = _decode(code)
        assert rm in (0, 1, 2) and vec in (0, 2, 4)
        if vec:
            assert nx % vec == 0  # row-vector forms only where they apply
        else:
            assert 1 <= bx <= 256 and bx * by <= 256 and zc == 0
        shapes, scored = tune.launch_for((bx, by, code))
        assert len(shapes) == 3
        # only the psi/c update marches in z
        assert _decode(shapes[0][2])[2] == 0 and _decode(shapes[1][2])[2] == 0
        if zc:
            assert scored == (False, False, True)
            assert shapes[1] == (0, 0, 0)
        else:
            assert shapes == [(bx, by, code)] * 3 and scored == (True, True, True)


@pytest.mark.parametrize("side", [32, 48, 64, 96, 30])
def test_batch_rules_give_valid_shapes(side):
    # every rule gives a box of any side a shape the library accepts: one
    # node per thread within the 256-thread launch bound, or a row-vector
    # code; plane-wise renumbering only where the rows per block divide ny
    for name, rule in tune.batch_rules().items():
        sh = rule(side, side)
        if name == "default":
            assert sh is None
            continue
        bx, by, code = sh
        rm, vec, zc = _decode(code)
        assert zc == 0 and rm in (0, 2)
        if vec:
            assert (bx, by) == (0, 0) and vec in (2, 4)
        else:
            assert 1 <= bx <= min(side, 256) and bx * by <= 256
            assert rm == 0 or side % by == 0


def test_tuning_cache_entries_decode():
    path = tune.CACHE
    if not os.path.exists(path):
        pytest.skip("no tuning cache")
    cache = json.load(open(path))
    rules = tune.batch_rules()
    for key, v in cache.items():
        dev, size, prec = key.split("|")
        assert prec in ("fp32", "fp64", "fp16")
        if size.startswith("batch"):
            # a batch tuned as a whole: one rule per kernel
            assert len(v["rules"]) == 3 and all(r in rules for r in v["rules"])
            continue
        assert len(size.split("x")) == 3
        assert len(v["shapes"]) == 3
        for k, (bx, by, code) in enumerate(v["shapes"]):
            rm, vec, zc = _decode(code)
            assert rm <= 2 and vec in (0, 1, 2, 4)
            assert k == 2 or zc == 0


def test_serving_request_bytes_cover_the_arena():
    tr = I.serving_trace(n_requests=6, rate=50.0, sides=(32, 60))
    for r in tr:
        spec = I.serving_request(r)
        need = serve.request_bytes(spec)
        arena = lb.footprint_bytes(spec["shape"], spec["precision"])
        assert need > arena  # plus the particle tables
        assert need < 2 * arena + (64 << 20)


def test_bench_refuses_more_than_one_gpu():
    # the benchmark is single-GPU: asking for more exits with a message
    # before touching a device
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_bench_kernel_hash_ignores_comments(tmp_path):
    # the stored HBM counters stay valid across comment and whitespace edits
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    h0 = bench.kernel_source_hash()
    csrc = os.path.join(root, "paper_2202_01631_amd", "csrc")
    copy = tmp_path / "paper_2202_01631_amd" / "csrc"
    copy.mkdir(parents=True)
    for f in ("lb_kernels.hip", "lb_device.h", "lb_kernels.h"):
        src = open(os.path.join(csrc, f)).read()
        if f == "lb_kernels.hip":
            src = "// a new comment\n/* and a block\n comment */\n" + src.replace("\n", "\n\n", 3)
        (copy / f).write_text(src)
    bench.ROOT = str(tmp_path)
    assert bench.kernel_source_hash() == h0
    (copy / "lb_device.h").write_text(open(os.path.join(csrc, "lb_device.h")).read() + "\nint x;\n")
    assert bench.kernel_source_hash() != h0


def test_params_struct_layout_matches_header(tmp_path):
    # the bindings' parameter and particle structures (library and oracle)
    # must lay out every field where the C headers do (sizeof and offsetof
    # from a gcc-compiled probe)
    import ctypes
    import subprocess
    from oracle import pyoracle
    from paper_2202_01631_amd import lb
    inc = os.path.join(ROOT, "include")
    structs = (("lb_params", lb.Params), ("lb_colloid", lb.Colloid),
               ("or_params", pyoracle.Params), ("or_colloid", pyoracle.Colloid))
    checks = []
    for cname, py in structs:
        checks.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            checks.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    src = tmp_path / "probe.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "lb.h"\n#include "oracle.h"\n'
                   'int main(void) {\n'
                   + "\n".join(checks) + "\nreturn 0;\n}\n")
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c99", "-I", inc, "-I", os.path.join(ROOT, "oracle"),
                           "-o", str(exe), str(src)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().split("\n"):
        if line:
            a, b, v = line.split()
            got[(a, b)] = int(v)
    for cname, py in structs:
        assert got[(cname, "size")] == ctypes.sizeof(py)
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_oversized_request_is_refused():
    # admission by footprint alone: host-side sizes, no GPU call
    srv = serve.Server(budget_bytes=1 << 20)
    spec = I.serving_request(dict(I.serving_trace(1)[0], side=40, spheres=1))
    spec["steps"] = 4
    srv.submit(0, spec, 0.0)
    res = srv.run()
    assert "error" in res[0]


def test_bench_error_helpers():
    # the precision leg's measures: the relative error per field with its
    # floor, and the mask of nodes beyond a reach from solid nodes
    import sys
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    shape = (8, 7, 6)
    N = 336
    solid = np.zeros(N, bool)
    solid[0] = True
    far1 = bench._far_from_solid(solid, shape, 1)
    assert far1.sum() == N - 7                   # the node and its 6 face neighbours
    far2 = bench._far_from_solid(solid, shape, 2)
    assert far2.sum() == N - 25                  # Manhattan distance <= 2: 1 + 6 + 18
    a = dict(rho=np.ones(N), psi=np.zeros(N), c=np.full(N, 1e-7), u=np.zeros((3, N)))
    b = dict(rho=np.ones(N) + 1e-3, psi=np.full(N, 0.5), c=np.zeros(N), u=np.zeros((3, N)))
    b["u"][0, 3] = 2e-3
    e = bench._field_errors(a, b, np.ones(N, bool))
    assert abs(e["rho"] - 1e-3 / (1 + 1e-3)) < 1e-12
    assert e["psi"] == 0.5 and abs(e["c"] - 1e-7 / 1e-6) < 1e-12  # floors 1 and 1e-6
    assert e["u"] == 1.0 and e["u_abs"] == 2e-3 and e["u_max"] == 2e-3
