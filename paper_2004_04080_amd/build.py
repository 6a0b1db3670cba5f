"""Build liblbhip.so (HIP, gfx950) in-tree: paper_2004_04080_amd/_lib/liblbhip.so.

Each csrc/*.hip file is compiled to an object with hipcc for gfx950 only and
the objects are linked into one shared library exporting the C interface of
include/lbhip.h.

Packed FP32 instructions (v_pk_add_f32, v_pk_mul_f32, v_pk_fma_f32) are kept
out of all device code: the target feature -packed-fp32-ops is passed to the
gfx950 device pass (the x86 host pass does not know the feature and says it
ignores it, which is harmless). The build then compiles every source once
more to gfx950 assembly and fails if any packed FP32 instruction is there.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "liblbhip.so")
OBJ_DIR = os.path.join(ROOT, "_build", "lbhip")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"),
]
SOURCES = ["lb_fluid.hip", "lb_particles.hip", "lb_adjoint.hip", "lb_domain.hip", "lb_api.hip",
           "lb_noalloc.hip", "lb_probe.hip"]
LIBS = ["-L/opt/rocm/lib", "-lrocfft", "-Wl,-rpath,/opt/rocm/lib"]


PACKED_FP32 = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")


def device_asm(src_path: str, out: str, flags=None) -> str:
    """gfx950 assembly of one source (device pass only), as text."""
    cmd = [HIPCC, *(FLAGS if flags is None else flags), "--cuda-device-only", "-S", src_path,
           "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc -S failed for {src_path}:\n{r.stdout}\n{r.stderr}")
    with open(out) as fh:
        return fh.read()


def _check_no_packed_fp32(src: str) -> None:
    asm = device_asm(os.path.join(CSRC, src), os.path.join(OBJ_DIR, os.path.splitext(src)[0] + ".s"))
    found = sorted(set(m.group(0) for m in PACKED_FP32.finditer(asm)))
    if found:
        raise RuntimeError(f"{src}: packed FP32 instructions in the device code: {found}")


# host code only (the device passes are never sanitised): AddressSanitizer and
# UndefinedBehaviorSanitizer with every UB report fatal, for the CPU tests of
# the host runtime; the process that loads such a build preloads the runtime
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def _compile(src: str, verbose: bool, obj_dir: str = OBJ_DIR, extra=()) -> str:
    obj = os.path.join(obj_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, flush=True)
    return obj


def build(verbose: bool = False, out: str = LIB, sanitize: bool = False) -> str:
    """Build the library to `out`; with sanitize the host code carries ASan and
    UBSan (objects in a directory of their own, no device-assembly check)."""
    obj_dir = OBJ_DIR + ("-san" if sanitize else "")
    extra = SANITIZE_HOST if sanitize else ()
    os.makedirs(os.path.dirname(out), exist_ok=True)
    os.makedirs(obj_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, obj_dir, extra), SOURCES))
        if not sanitize:
            list(ex.map(_check_no_packed_fp32, SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, *LIBS, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
