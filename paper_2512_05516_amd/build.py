"""Build libsphmi.so (HIP kernels for gfx950 plus the C-ABI host code).

    python -m paper_2512_05516_amd.build

Objects go to paper_2512_05516_amd/_build/, the library next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsphmi.so")
SOURCES = ["abi.cpp", "host_convert.cpp", "tune.cpp", "serve.cpp", "bin.hip", "convert.hip", "pair.hip", "kick.hip",
           "worklist.hip", "pair_dens_f32.hip", "pair_dens_r.hip", "pair_dens_gen.hip",
           "pair_dens_aos.hip", "pair_dens_h.hip", "pair_dens_b.hip", "pair_force_f32.hip",
           "pair_force_r.hip", "pair_force_gen.hip", "pair_force_h.hip", "pair_force_b.hip",
           "pair_force_aos.hip", "pair_task_f32.hip", "pair_task_r.hip", "pair_task_gen.hip", "hiter.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("SPH_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          "-I", os.path.join(ROOT, "include")]
# packed FP32 instructions stay off: hipcc -O3 would otherwise form them from
# ordinary float code
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src + ".o")
    path = os.path.join(CSRC, src)
    cmd = [HIPCC, *COMMON, "-c", path, "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = DEVICE
    p = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (p.stderr or "").splitlines()
                     if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{errs}")
    if errs.strip():
        sys.stderr.write(errs + "\n")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(os.cpu_count() or 8, 16)) as ex:
        # longest first: the kernel instantiation units
        order = sorted(SOURCES, key=lambda f: (not f.startswith("pair_"), f))
        done = dict(zip(order, ex.map(_compile, order)))
        objs = [done[f] for f in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{p.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
