"""Builds the HIP library ``liblbm.so`` in-tree for gfx950 with hipcc.

The kernel file is compiled once per storage type (FP64, FP32, FP16 and BF16
deviation storage) so the objects build in parallel; the host files and the
dispatch are separate objects; hipcc links them into one shared library.

Usage: ``python -m paper_1611_00907_amd.build`` (or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbm.so")
OBJ = os.path.join(PKG, "_build")

KERNEL_SOURCE = "lbm_kernels.hip"
STORAGE = [("double", "f64"), ("float", "f32"), ("__half", "f16dev"), ("__hip_bfloat16", "bf16dev")]
HOST_SOURCES = ["lbm_dispatch.cpp", "lbm_host.cpp", "lbm_batch.cpp", "thermo_host.cpp", "sur_kernels.hip",
                "sur_host.cpp", "lbm3d_kernels.hip", "lbm3d_host.cpp", "warm_host.cpp"]
HEADERS = ["lbm_internal.h", "lbm_common.h", "thermo_host.h", "sur_internal.h", "lbm3d_internal.h",
           "lbm_eos_device.h"]
SOURCES = [KERNEL_SOURCE] + HOST_SOURCES

ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep the compiler from forming packed FP32 instructions (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_commands():
    cmds = []
    for st, sfx in STORAGE:
        out = os.path.join(OBJ, "lbm_kernels_%s.o" % sfx)
        cmds.append((out, [hipcc()] + FLAGS + ["-DCPLBM_ST=%s" % st, "-DCPLBM_SUFFIX=%s" % sfx, "-c",
                                               os.path.join(CSRC, KERNEL_SOURCE), "-o", out]))
    for src in HOST_SOURCES:
        out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        cmds.append((out, [hipcc()] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", out]))
    return cmds


def build(verbose: bool = True) -> str:
    os.makedirs(OBJ, exist_ok=True)
    cmds = compile_commands()

    def run(cmd):
        r = subprocess.run(cmd, capture_output=True, text=True)
        return cmd, r

    jobs = max(1, min(len(cmds), os.cpu_count() or 4, 16))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda c: run(c[1]), cmds))
    for cmd, r in results:
        if verbose:
            print(" ".join(cmd), flush=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed: %s" % cmd[-3])
    tmp = LIB + ".tmp%d" % os.getpid()
    link = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}"] + [c[0] for c in cmds] + ["-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking liblbm.so")
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS] + [os.path.join(ROOT, "include", "lbm.h")]
    return any(os.path.getmtime(d) > t for d in deps)


if __name__ == "__main__":
    build()
