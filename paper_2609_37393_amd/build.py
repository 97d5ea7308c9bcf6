"""Build librift_ile.so (HIP, gfx950) in the package directory, and the LDS
read-bandwidth microbenchmark `lds_peak` beside it.

The evaluation kernels are instantiated per detector class and kernel kind in
separate objects (csrc/inst.hip compiled with -DRIFT_KT, -DRIFT_KIND) so they
compile in parallel; the host code and setup kernels are csrc/rift_ile.hip.

    python -m paper_2609_37393_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librift_ile.so")
LDS_PEAK = os.path.join(HERE, "lds_peak")  # LDS read-bandwidth microbenchmark (a program)
OBJDIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("RIFT_ILE_ARCH", "gfx950")
KT_CLASSES = (2, 3, 5, 8)
KINDS = (0, 1, 2, 3, 4, 5, 6, 7, 8)  # FP64 tiles, FP32 tiles, FP64 refine, gradient, distance / time / psi
#                                      marginals, data passes of the band-limited time rule and of ERAI

FLAGS = [
    "-O3",
    "-std=c++17",
    f"--offload-arch={ARCH}",
    "-fPIC",
    # packed FP32 VALU ops are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds fused only inside one source expression: the same
    # expression gives the same bits in every kernel that inlines it
    "-ffp-contract=on",
    "-Wall",
    "-Wno-unused-function",
]


def _objects():
    objs = [(os.path.join(CSRC, "rift_ile.hip"), os.path.join(OBJDIR, "rift_ile.o"), []),
            (os.path.join(CSRC, "wide.hip"), os.path.join(OBJDIR, "wide.o"), []),
            (os.path.join(CSRC, "sampler.hip"), os.path.join(OBJDIR, "sampler.o"), []),
            (os.path.join(CSRC, "pregrid.hip"), os.path.join(OBJDIR, "pregrid.o"), []),
            (os.path.join(CSRC, "importance.hip"), os.path.join(OBJDIR, "importance.o"), [])]
    for kt in KT_CLASSES:
        for kind in KINDS:
            objs.append((os.path.join(CSRC, "inst.hip"), os.path.join(OBJDIR, f"inst_kt{kt}_k{kind}.o"),
                         [f"-DRIFT_KT={kt}", f"-DRIFT_KIND={kind}"]))
    return objs


def _compile(job, extra, verbose):
    src, obj, defs = job
    cmd = [HIPCC, *FLAGS, *defs, *extra, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = ("is not a recognized feature", "unknown target feature")
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if l and not any(n in l for n in noise))
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {obj}:\n{msg}")
    return obj, msg


def build(verbose: bool = False, extra=None, jobs: int | None = None) -> str:
    """Compile every HIP object for the target arch and link librift_ile.so."""
    extra = list(extra or [])
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    objs = _objects()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for obj, msg in ex.map(lambda j: _compile(j, extra, verbose), objs):
            if msg and verbose:
                print(f"[{os.path.basename(obj)}]\n{msg}", flush=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *[o for _, o, _ in objs], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # the LDS microbenchmark behind the LDS ceiling in the measurements
    cmd = [HIPCC, *[f for f in FLAGS if f != "-fPIC"], os.path.join(CSRC, "lds_peak.hip"), "-o", LDS_PEAK + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL if not verbose else None)
    os.replace(LDS_PEAK + ".tmp", LDS_PEAK)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
