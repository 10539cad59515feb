"""Builds the HIP library libmera_hip.so in place (hipcc, gfx950).

Usage: python -m paper_2007_03638_amd.build  (or build() from Python). Always recompiles.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmera_hip.so")
ROOT = os.path.dirname(HERE)

SOURCES = ["gett.hip", "vec.hip", "noalloc.hip", "network.cpp", "linalg.cpp", "model.cpp", "mera.cpp", "optim.cpp",
           "server.cpp", "capi.cpp"]

HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include")]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False, jobs=8):
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    procs = []
    objs = []
    for s in srcs:
        obj = os.path.join(objdir, s + ".o")
        objs.append(obj)
        cmd = [hipcc, *HIPFLAGS, "-x", "hip", "-c", os.path.join(CSRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len([p for p in procs if p[1].poll() is None]) >= jobs:
            procs[0][1].wait()
    failed = []
    for s, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass warns about the GPU-only target feature; that line is expected
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip() != "")
        if p.returncode != 0:
            failed.append(s)
            sys.stderr.write(f"--- {s} ---\n{text}\n")
        elif verbose and text:
            print(text)
    if failed:
        raise RuntimeError("HIP build failed: " + ", ".join(failed))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
