"""Build libevx.so (gfx950) in-tree with hipcc.

Every supported transform length is compiled as its own object from evx_kernels.hip (in
parallel), then linked with the C ABI object into paper_2507_21748_amd/libevx.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libevx.so")

ARCH = "gfx950"
HIPFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no FP contraction: every kernel that transforms the same data rounds identically, which
    # makes resume from a stored state and checkpoint recomputation bit-exact
    "-ffp-contract=off",
    # packed FP32 instructions stay off: the compiler must not emit v_pk_{add,mul,fma}_f32
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", CSRC,
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def transform_lengths() -> list[int]:
    text = open(os.path.join(CSRC, "evx_schedule.hpp")).read()
    m = re.search(r"#define EVX_FOR_EACH_N\(X\)(.*?)\n\n", text, re.S)
    return [int(v) for v in re.findall(r"X\((\d+)\)", m.group(1))]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
        raise RuntimeError(f"command failed: {' '.join(cmd)}\n{err}")
    return cmd[-1]


def build(jobs: int | None = None, verbose: bool = False, lib: str = LIB,
          defines: tuple = (), build_dir: str = BUILD) -> str:
    """Compile every object and link `lib`; `defines` are extra -D options for all objects."""
    os.makedirs(build_dir, exist_ok=True)
    cc = hipcc()
    flags = HIPFLAGS + [f"-D{d}" for d in defines]
    jobs = jobs or min(16, os.cpu_count() or 4)
    cmds = []
    for n in transform_lengths():
        obj = os.path.join(build_dir, f"evx_k{n}.o")
        cmds.append([cc, *flags, f"-DEVX_INST_N={n}", "-c",
                     os.path.join(CSRC, "evx_kernels.hip"), "-o", obj])
    for src in ("evx_api.hip", "evx_aux.hip", "evx_net.hip"):
        obj = os.path.join(build_dir, src.replace(".hip", ".o"))
        cmds.append([cc, *flags, "-c", os.path.join(CSRC, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_run, cmds))
    tmp = lib + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
