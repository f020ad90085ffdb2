"""Build libmcmi.so for gfx950 in-tree with hipcc.

Flags: IEEE arithmetic with no contraction (every compared floating-point step
is one correctly rounded operation), hardware float atomics, and packed FP32
instructions disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmcmi.so")
# benchmark tooling, not part of the library's ABI: the dependent-gather probe
PROBE_SRC = os.path.join(HERE, "bench_probe", "gather_probe.hip")
PROBE_LIB = os.path.join(HERE, "bench_probe", "libmcmi_probe.so")
SOURCES = ["cdf.hip", "walk.hip", "walk_block.hip", "learn.hip", "mlp.hip", "plan.hip", "krylov.hip", "alloc.hip", "order.hip", "scan.hip", "api.hip"]
ARCH = os.environ.get("MCMI_ARCH", "gfx950")


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found (ROCm is required to build libmcmi.so)")
    return exe


FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function",
         "-Wno-unused-variable", "-Wno-unused-result", "-Wno-unused-value"]


def build(verbose: bool = False, jobs: int = 4) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [hipcc()] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    probe_tmp = PROBE_LIB + ".tmp"
    procs.append((os.path.basename(PROBE_SRC),
                  subprocess.Popen([hipcc()] + FLAGS + ["-shared", PROBE_SRC, "-o", probe_tmp],
                                   stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out = p.communicate()[0].decode(errors="replace")
        out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)
        if p.returncode != 0:
            failed.append(src)
            print(out, file=sys.stderr)
        elif verbose and out.strip():
            print(out)
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    tmp = LIB + ".tmp"
    subprocess.check_call([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    os.replace(probe_tmp, PROBE_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
