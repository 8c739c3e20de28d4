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

SOURCES = ["kernels.hip", "fused.hip", "fr.hip", "noalloc.hip", "api.cpp", "planner.cpp", "serve.cpp"]
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


# Host-side sanitizers for the C++ host code (api.cpp, planner.cpp, serve.cpp): each -fsanitize
# applies to the host compilation only (-Xarch_host); the device code is built as usual.
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
ASAN_LIB = os.path.join(BUILD, "asan", "libqsim.so")


def asan_runtime() -> str:
    """The clang ASan runtime that a host process preloads to load ASAN_LIB."""
    root = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(hipcc()))), "llvm", "lib", "clang")
    if not os.path.isdir(root):
        root = "/opt/rocm/llvm/lib/clang"
    for ver in sorted(os.listdir(root), reverse=True):
        p = os.path.join(root, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    raise FileNotFoundError("clang ASan runtime not found under " + root)


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile csrc/ into libqsim.so; sanitize=True builds ASAN_LIB instead: the host C++ with
    AddressSanitizer and UndefinedBehaviorSanitizer, the kernels as usual."""
    out_dir = os.path.join(BUILD, "asan") if sanitize else BUILD
    os.makedirs(out_dir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(out_dir, src + ".o")
        objs.append(obj)
        flags = common_flags()
        if sanitize and not src.endswith(".hip"):
            flags = [f for f in flags if f != "-O3"] + ["-O1", "-g", *SANITIZE_HOST, "-shared-libasan"]
        cmd = [hipcc(), *flags, "-c", os.path.join(CSRC, src), "-o", obj]
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
    lib_path = ASAN_LIB if sanitize else LIB
    tmp = lib_path + ".tmp"
    link = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if sanitize:
        link[1:1] = ["-shared-libasan", "-fsanitize=address,undefined"]
    subprocess.check_call(link)
    os.replace(tmp, lib_path)
    return lib_path


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
