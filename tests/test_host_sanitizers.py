"""AddressSanitizer and UndefinedBehaviorSanitizer on the host side of the
library and on the oracle (CPU, no GPU).

The library's host code is built host-only against a CPU stand-in of the HIP
runtime (tests/hostcheck) that also checks stream, event, graph and memory
lifetimes, and is driven through
  * the serving loop's own call sequence: serve.Server on a 100-request
    Poisson trace at 50/s, two storage precisions on two caller streams,
    contexts created and destroyed between batched steps (with graph capture
    of step pairs), up to ~90 live at once, and a full readback every tenth
    retirement;
  * every other ABI entry point, the error paths and an uneven batch.
The oracle is built with the same sanitizers and stepped through every
option.  Kernels do not run in these builds: they check the host code only.
"""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HC = os.path.join(HERE, "hostcheck")
sys.path.insert(0, HC)


@pytest.fixture(scope="module")
def san():
    import build as hcbuild
    if not os.path.exists(hcbuild.CLANG) or shutil.which("nm") is None:
        pytest.skip("clang or nm not available")
    try:
        rt = hcbuild.asan_runtime()
    except (RuntimeError, subprocess.CalledProcessError):
        pytest.skip("shared AddressSanitizer runtime not available")
    hcbuild.build()
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", ORACLE_THREADS="1")
    return hcbuild, env


def _run(env, *args):
    r = subprocess.run([sys.executable] + list(args), env=env, capture_output=True, text=True,
                       timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert "hostcheck:" not in out, out[-6000:]
    return out


def test_serving_call_sequence_is_clean(san):
    hcbuild, env = san
    out = _run(env, os.path.join(HC, "replay_check.py"), hcbuild.LIB, "100", "50", "13700",
               str(140 * 10 ** 9), "10")
    assert "replay ok: 100 requests, 100 completed" in out
    peak = int(out.split("peak ")[1].split()[0])
    assert peak >= 50   # as many live requests as the GPU run had (93)


def test_abi_call_sequences_are_clean(san):
    hcbuild, env = san
    assert "abi ok: 0 device allocations left" in _run(env, os.path.join(HC, "abi_check.py"),
                                                        hcbuild.LIB)


def test_oracle_is_clean(san):
    hcbuild, env = san
    assert "oracle ok" in _run(env, os.path.join(HC, "oracle_check.py"), hcbuild.ORACLE_LIB)
