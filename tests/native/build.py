"""Build the native ABI check (tests/native/abi_check): the library's sources
compiled again with the device-side invariant checks on (-DPV_CHECKED) and
with AddressSanitizer and UndefinedBehaviorSanitizer on their host code,
linked with abi_check.cpp (also sanitized).  Device code is never built with
a sanitizer here: only host compilation actions get the flags.

    python tests/native/build.py

Objects go to _build/checked/ at the repository root.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2001_06784_amd import build as libbuild  # noqa: E402

OUT = os.path.join(HERE, "abi_check")
ORACLE_OUT = os.path.join(HERE, "oracle_check")
ORACLE_SRC = os.path.join(ROOT, "oracle", "oracle.c")
OBJ = os.path.join(ROOT, "_build", "checked")
CLANG = "/opt/rocm/llvm/bin/clang++"
ROCM_INC = "/opt/rocm/include"
ROCM_LIB = "/opt/rocm/lib"


def _host_san() -> list[str]:
    # every sanitizer flag applies to the host compilation only
    return ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [libbuild.HIPCC, *libbuild.FLAGS, "-DPV_CHECKED", "-g", *_host_san(),
           "-c", os.path.join(libbuild.CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"checked build failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build_oracle_check(out: str = ORACLE_OUT) -> str:
    """oracle.c and oracle_check.c, both sanitized, into one host program."""
    cmd = ["gcc", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g", "-O1", "-std=gnu11", "-Wall", "-o", out, os.path.join(HERE, "oracle_check.c"), ORACLE_SRC, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"oracle_check failed to build:\n{r.stdout}\n{r.stderr}")
    return out


def build(verbose: bool = False) -> str:
    build_oracle_check()
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(libbuild.SOURCES)) as ex:
        objs = list(ex.map(_compile, libbuild.SOURCES))
    drv = os.path.join(OBJ, "abi_check.o")
    # host-only translation unit and link: no device code, so no GPU sanitizer
    cmd = [CLANG, "-fno-gpu-sanitize", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-g", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", libbuild.INCLUDE, "-I", ROCM_INC, "-c", os.path.join(HERE, "abi_check.cpp"), "-o", drv]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"abi_check.cpp failed:\n{r.stdout}\n{r.stderr}")
    tmp = OUT + ".tmp"
    cmd = [CLANG, "-fno-gpu-sanitize", "-fsanitize=address,undefined", "-o", tmp, drv, *objs, "-L", ROCM_LIB, "-lamdhip64", "-Wl,-rpath," + ROCM_LIB]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
