"""Build libmgfwa.so (HIP, gfx950) in-tree with hipcc.

Every .hip file under csrc/ is compiled to an object in csrc/_build/ (in
parallel, slowest first) and linked into paper_2501_03944_amd/libmgfwa.so.
build() recompiles everything; build(incremental=True) skips objects newer
than their source and every header.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(CSRC, "_build")
LIB = os.path.join(HERE, "libmgfwa.so")
ARCH = os.environ.get("MGFWA_OFFLOAD_ARCH", "gfx950")

# the wide fitness instances take the longest: start them first
SOURCES = ["fit_l4_wide_f32.hip", "fit_l4_wide_bf16.hip", "fit_lds_bf16.hip", "fit_lds_f32.hip",
           "fit_l2_wide.hip", "fit_l3_wide_f32.hip", "fit_l3_wide_bf16.hip", "fit_l4_f32.hip",
           "fit_l4_bf16.hip", "fit_l3.hip", "fit_std.hip", "fit_l2.hip", "fit_l1.hip",
           "fit_wide.hip", "fitness.hip", "capi.hip", "spark.hip", "guide.hip", "select.hip",
           "server.hip", "net_input.hip"]
HEADERS = ["device_common.h", "internal.h", "fit_kernel.h", "fit_wide.h"]

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
    # state-path arithmetic is specified operation by operation: no contraction
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    # packed FP32 instructions stay off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


# Instance files whose kernels read the weights from global memory: their layer
# loops (every (K block, row block) pair of a layer, fully unrolled so that the
# activation tiles stay in registers) exceed the compiler's default size limit
# for a requested full unroll; left partly rolled, the activation arrays are
# indexed at run time and live in scratch memory.
UNROLL_FLAGS = ["-mllvm", "-pragma-unroll-threshold=1000000"]
GLOBAL_WEIGHT_SOURCES = {"fit_l1.hip", "fit_l2.hip", "fit_l2_wide.hip", "fit_l3.hip",
                         "fit_l3_wide_bf16.hip", "fit_l3_wide_f32.hip", "fit_l4_bf16.hip",
                         "fit_l4_f32.hip", "fit_l4_wide_bf16.hip", "fit_l4_wide_f32.hip"}


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found: the HIP toolchain is required to build libmgfwa.so")
    return p


def _obj(src: str) -> str:
    return os.path.join(BUILD, os.path.splitext(src)[0] + ".o")


def _fresh(src: str) -> bool:
    obj = _obj(src)
    if not os.path.exists(obj):
        return False
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in HEADERS]
    deps.append(os.path.join(ROOT, "include", "mgfwa.h"))
    return all(os.path.getmtime(d) <= t for d in deps)


def _compile(src: str, verbose: bool) -> str:
    obj = _obj(src)
    extra = UNROLL_FLAGS if src in GLOBAL_WEIGHT_SOURCES else []
    cmd = [hipcc(), *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


def build(verbose: bool = False, jobs: int | None = None, incremental: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    listed = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    missing = set(listed) ^ set(SOURCES)
    if missing:
        raise RuntimeError(f"csrc/*.hip and build.SOURCES differ: {sorted(missing)}")
    todo = [s for s in SOURCES if not (incremental and _fresh(s))]
    jobs = jobs or min(len(SOURCES), max(1, min(16, os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda s: _compile(s, verbose), todo))
    objs = [_obj(s) for s in SOURCES]
    if incremental and not todo and os.path.exists(LIB) and \
            all(os.path.getmtime(o) <= os.path.getmtime(LIB) for o in objs):
        return LIB
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
