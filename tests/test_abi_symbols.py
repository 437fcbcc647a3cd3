"""The C-ABI library loads on a machine without a GPU and exports every
function include/lb.h declares; host-only helpers agree with the oracle's."""
import ctypes as C
import math
import os
import re

import pytest

import oracle
from paper_2202_01631_amd import lb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lb.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_0-9A-Z]+)\s*\(", text)))


def test_library_built():
    assert os.path.exists(lb.LIB_PATH), "run python -m paper_2202_01631_amd.build"


def test_every_declared_symbol_is_exported():
    names = declared()
    assert "lb_create" in names and "lb_step" in names and "lb_observables" in names
    L = C.CDLL(lb.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(lb.EXPORTS)


def test_host_parameter_maps_match_oracle():
    for th in (0.0, 30.0, 45.0, 60.0, 90.0, 120.0, 135.0, 180.0):
        assert lb.wetting_H(th, 0.04, 0.0625) == pytest.approx(oracle.wetting_H(th, 0.04, 0.0625), abs=1e-15)
    assert math.isnan(lb.wetting_H(60.0, 0.0, 0.0625))
    for th in (45.0, 60.0, 90.0, 120.0, 135.0):
        for kap in (0.04, 0.5):
            assert lb.wetting_H_lattice(th, -0.0625, 0.0625, kap) == pytest.approx(
                oracle.wetting_H_lattice(th, -0.0625, 0.0625, kap), abs=1e-14)
    assert math.isnan(lb.wetting_H_lattice(60.0, 0.0625, 0.0625, 0.04))
    assert math.isnan(lb.wetting_H_lattice(60.0, -0.0625, 0.0625, 0.0))
    for r in (1.0, 2.0, 3.5, 5.0):
        assert lb.solubility_E(r, 0.5) == pytest.approx(oracle.solubility_E(r, 0.5), rel=1e-15)


def test_footprint_is_host_only():
    n32 = lb.footprint_bytes((256, 256, 256), "fp32")
    n64 = lb.footprint_bytes((256, 256, 256), "fp64")
    n16 = lb.footprint_bytes((256, 256, 256), "fp16")
    N = 256 ** 3
    # two population lattices + psi, c twice + mu + u + owner byte
    assert n32 >= N * (2 * 19 * 4 + 4 * 4 + 4 + 12 + 1)
    assert n64 >= N * (2 * 19 * 8 + 4 * 8 + 8 + 24 + 1)
    assert n16 >= N * (2 * 19 * 2 + 4 * 4 + 4 + 12 + 1)
    assert n16 < n32 < n64
    with pytest.raises(lb.LBError):
        lb.footprint_bytes((0, 4, 4), "fp32")
    # scalar fields are addressed with 32-bit byte offsets: one field must
    # stay below 4 GiB (2^29 nodes in FP64, 2^30 otherwise)
    with pytest.raises(lb.LBError):
        lb.footprint_bytes((1024, 1024, 512), "fp64")
    with pytest.raises(lb.LBError):
        lb.footprint_bytes((1024, 1024, 1024), "fp32")
    assert lb.footprint_bytes((1024, 1024, 511), "fp64") > 0
    assert lb.footprint_bytes((1024, 1024, 1023), "fp32") > 0


def test_binding_shares_torch_hip_runtime():
    # loading the library through the binding, with nothing imported before,
    # must leave one HIP runtime in the process (torch's), not two
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2202_01631_amd import lb\n"
            "lb.load()\n"
            "maps = open('/proc/self/maps').read().split('\\n')\n"
            "print(sorted(set(l.split()[-1] for l in maps if 'libamdhip64' in l)))\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    libs = eval(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1, libs
