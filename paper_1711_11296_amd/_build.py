"""Build the HIP shared library libsht.so in-tree for gfx950.

Every HIP source is compiled by hipcc for --offload-arch=gfx950; the host
planner is plain C++.  The result lands next to this file, where the Python
binding loads it.
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsht.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_SOURCES = ["sht_fft.hip", "sht_legendre.hip", "sht_legendre_bf16.hip", "sht_transfer.hip", "sht_api.hip"]
CXX_SOURCES = ["sht_host.cpp", "sht_plan.cpp"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-I" + CSRC, "-I" + os.path.join(os.path.dirname(HERE), "include")]
HIP_FLAGS = COMMON + ["--offload-arch=" + ARCH, "-mcode-object-version=5",
                      "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                      # keep MFMA accumulators in ordinary VGPRs: with the
                      # accumulation-register form the compiler copies every
                      # accumulator out and back once per K-block
                      "-mllvm", "-amdgpu-mfma-vgpr-form=1",
                      "-Wno-unused-result"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), out))
    if verbose and out.strip():
        print(out)


def build(verbose=False, jobs=4):
    os.makedirs(BUILD, exist_ok=True)
    cmds = []
    objs = []
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        cmds.append([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in CXX_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        cmds.append(["g++"] + COMMON + ["-pthread", "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = OUT + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-pthread"], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
