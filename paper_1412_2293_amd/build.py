"""Build libqsim.so (gfx950) in place from csrc/ with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqsim.so")

SOURCES = ["kernels.hip", "fused.hip", "fr.hip", "api.cpp", "planner.cpp", "serve.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def common_flags():
    return ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
            "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
            # packed FP32 instructions stay off: hand-written code never uses them and the
            # compiler must not form them either
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # keep the per-qubit register-update branches apart: sinking their common code
            # merges them behind pointer phis, which forces the register tile into scratch
            "-mllvm", "-simplifycfg-sink-common=false"]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        cmd = [hipcc(), *common_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".hip"):
            cmd[1:1] = ["-x", "hip"]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        for src, text in failed:
            sys.stderr.write(f"---- {src} ----\n{text}\n")
        raise RuntimeError("libqsim build failed: " + ", ".join(s for s, _ in failed))
    tmp = LIB + ".tmp"
    subprocess.check_call([hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
