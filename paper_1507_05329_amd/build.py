"""Builds libcola.so (HIP for gfx950) in place next to this file.

Usage: python -m paper_1507_05329_amd.build   (or build_library() from Python)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcola.so")
SOURCES = ["cola_api.cpp", "cosmo.cpp", "k_sort.hip", "k_deposit.hip", "k_fft.hip",
           "k_particles.hip", "k_ic.hip", "k_pk.hip", "k_adjoint.hip",
           "k_velocity.hip", "k_fof.hip", "cola_noalloc.hip"]
# translation units whose float results must follow the written order bit for bit
STRICT = {"k_sort.hip", "k_deposit.hip"}
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-ffp-contract=fast", "-Wno-unused-result", "-Wno-unused-command-line-argument"]


def build_library(verbose=False, jobs=8):
    """Compiles every source to an object (in parallel) and links libcola.so."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        strict = ["-ffp-contract=off"] if src in STRICT else []
        cmd = [HIPCC, *FLAGS, *strict, *lang, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    if p.returncode != 0:
        sys.stderr.write(out.decode(errors="replace"))
        raise RuntimeError(f"hipcc failed on {src}")
    text = out.decode(errors="replace").strip()
    if text and "warning" in text and "packed-fp32-ops" not in text:
        sys.stderr.write(text + "\n")


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
