"""Host-side logic that needs no GPU: autotuner candidates and cache
format, serving admission sizes."""
import json
import os

import pytest

from paper_2202_01631_amd import inputs as I
from paper_2202_01631_amd import lb, serve, tune


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


def test_tuning_cache_entries_decode():
    path = tune.CACHE
    if not os.path.exists(path):
        pytest.skip("no tuning cache")
    cache = json.load(open(path))
    for key, v in cache.items():
        dev, size, prec = key.split("|")
        assert prec in ("fp32", "fp64", "fp16")
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
