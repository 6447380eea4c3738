"""Build the native library libdh2.so in-tree with hipcc for gfx950.

    python -m paper_1510_07087_amd.build        (or build() from Python)

Host-only C++ sources are compiled with -ffp-contract=off so that the plan's
floating-point predicates are evaluated exactly as written.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdh2.so")
ARCH = os.environ.get("DH2_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

SOURCES = [
    ("plan.cpp", ["-x", "c++", "-ffp-contract=off"]),
    ("engine.cpp", ["-x", "c++", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"]),
    ("api.cpp", ["-x", "c++", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"]),
    ("kernels.hip", DEVICE),
]


def _compile(src, extra):
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC] + COMMON + extra + ["-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (p.stdout + p.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{out}")
    return obj, out


def build(verbose: bool = False) -> str:
    """Compile every source and link libdh2.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        res = list(ex.map(lambda a: _compile(*a), SOURCES))
    objs = [o for o, _ in res]
    if verbose:
        for _, out in res:
            if out.strip():
                print(out)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{p.stdout}{p.stderr}")
    os.replace(tmp, LIB)
    return LIB


SAN_DIR = os.path.join(BUILD, "sanitize")
SAN_LIB = os.path.join(SAN_DIR, "libdh2_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer"]


def build_sanitized() -> str:
    """Host code (plan, engine, C ABI) built with g++ under AddressSanitizer
    and UndefinedBehaviorSanitizer, linked with the regular gfx950 kernel
    object; returns the library's path.  Load it with DH2_LIBRARY set to that
    path and the sanitizer runtimes preloaded (see sanitizer_env)."""
    kobj = os.path.join(BUILD, "kernels.hip.o")
    if not os.path.exists(kobj):
        build()
    os.makedirs(SAN_DIR, exist_ok=True)
    objs = []
    for src in ("plan.cpp", "engine.cpp", "api.cpp"):
        obj = os.path.join(SAN_DIR, src + ".o")
        cmd = ["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
               "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I", CSRC] + SAN_FLAGS + \
              ["-c", os.path.join(CSRC, src), "-o", obj]
        p = subprocess.run(cmd, capture_output=True, text=True)
        if p.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{p.stdout}{p.stderr}")
        objs.append(obj)
    cmd = ["g++", "-shared", "-o", SAN_LIB] + objs + [kobj, "-L/opt/rocm/lib", "-lamdhip64",
                                                     "-Wl,-rpath,/opt/rocm/lib"] + SAN_FLAGS
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{p.stdout}{p.stderr}")
    return SAN_LIB


def sanitizer_env() -> dict:
    """Environment for a Python process that loads the sanitizer build: the
    runtimes preloaded (libstdc++ too, so that the exception interceptor finds
    its target), leak checks off (the interpreter's own allocations)."""
    def lib(name):
        return subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True,
                              text=True).stdout.strip()
    env = dict(os.environ)
    env["LD_PRELOAD"] = " ".join([lib("libasan.so"), lib("libubsan.so"), lib("libstdc++.so")])
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["DH2_LIBRARY"] = SAN_LIB
    return env


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized())
    else:
        print(build(verbose="-v" in sys.argv))
