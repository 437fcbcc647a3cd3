"""Build the sanitizer builds of the library's host code and of the oracle
(TEST INFRASTRUCTURE).

The library sources (lb_api.hip and lb_kernels.hip) are compiled host-only in
clang's HIP mode against the CPU stand-in of the HIP runtime in this folder
(include/hip/*.h, hip_cpu.cpp), with AddressSanitizer and
UndefinedBehaviorSanitizer, into liblb_hostcheck.so.  Kernels are not built
or run; the product library is built by paper_2202_01631_amd/build.py.  The
FP64 oracle is built the same way (liboracle_hostcheck.so).

    python tests/hostcheck/build.py
"""
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2202_01631_amd", "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(OUT, "liblb_hostcheck.so")
ORACLE_LIB = os.path.join(OUT, "liboracle_hostcheck.so")
CLANG = os.environ.get("HOSTCHECK_CLANG", "/opt/rocm/llvm/bin/clang++")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer", "-shared-libasan"]
COMMON = ["-std=c++17", "-O1", "-g", "-fPIC", "-fdeclspec", "-I" + os.path.join(HERE, "include"),
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def asan_runtime():
    """Path of the shared AddressSanitizer runtime the library links against
    (to be preloaded into the host process)."""
    r = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True, check=True)
    p = r.stdout.strip()
    if not os.path.isabs(p) or not os.path.exists(p):
        raise RuntimeError("shared AddressSanitizer runtime not found")
    return p


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("%s\n%s" % (" ".join(cmd), r.stderr[-4000:]))
    return r


def build():
    os.makedirs(OUT, exist_ok=True)
    objs = []
    for src in ("lb_kernels.hip", "lb_api.hip"):
        o = os.path.join(OUT, src.replace(".hip", ".o"))
        _run([CLANG] + COMMON + SAN + ["-x", "hip", "--offload-host-only", "-nogpuinc", "-nogpulib",
                                       "--offload-arch=gfx950", "-c", os.path.join(CSRC, src),
                                       "-o", o])
        objs.append(o)
    o = os.path.join(OUT, "hip_cpu.o")
    _run([CLANG] + COMMON + SAN + ["-c", os.path.join(HERE, "hip_cpu.cpp"), "-o", o])
    objs.append(o)
    # host-only HIP objects refer to the device code image of their unit,
    # which a host-only build does not produce: define empty images
    names = set()
    for ob in objs:
        r = _run(["nm", "-u", ob])
        names.update(re.findall(r"\b(__hip_fatbin\w*)", r.stdout))
    stub = os.path.join(OUT, "fatbin_stub.c")
    with open(stub, "w") as f:
        for n in sorted(names):
            f.write("char %s[16] __attribute__((aligned(16)));\n" % n)
    o = os.path.join(OUT, "fatbin_stub.o")
    _run(["gcc", "-c", "-fPIC", stub, "-o", o])
    objs.append(o)
    _run([CLANG, "-shared", "-fPIC"] + SAN + ["-Wl,-Bsymbolic", "-o", LIB] + objs)
    # the oracle, with the flags of its own build (no contraction)
    cc = os.path.join(os.path.dirname(CLANG), "clang")
    _run([cc, "-std=c99", "-O1", "-g", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
          "-shared", "-D_DEFAULT_SOURCE"] + SAN + ["-o", ORACLE_LIB,
                                                   os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    return LIB


if __name__ == "__main__":
    print(build())
    sys.exit(0)
