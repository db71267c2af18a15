"""Build libsttsv.so (HIP, gfx950) in-tree.

    python -m paper_2311_08595_amd.build [-j JOBS]

Every HIP translation unit is compiled with hipcc for gfx950 in parallel,
then linked into ``paper_2311_08595_amd/libsttsv.so`` next to this file.
Packed FP32 instructions are switched off for all device code
(``-target-feature -packed-fp32-ops``).
"""
import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libsttsv.so")
ARCH = os.environ.get("STTSV_ARCH", "gfx950")

HIP_SOURCES = (["edge_part%d.hip" % i for i in range(8)] + ["edge_gen%d.hip" % i for i in range(8)]
               + ["edge_coop%d.hip" % i for i in range(4)]
               + ["edge_cpart%d.hip" % i for i in range(8)] + ["edge_cgen%d.hip" % i for i in range(2)]
               + ["edge_ccoop%d.hip" % i for i in range(2)]
               + ["apply.hip", "reduce.hip", "nqz.hip", "mpnn.hip", "naive.hip", "sshopm.hip", "ccss.hip", "cp.hip"])
CXX_SOURCES = ["plan.cpp", "api.cpp", "tune.cpp"]
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=off"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "is not a recognized feature" not in l)
    if p.returncode != 0:
        raise RuntimeError("command failed: %s\n%s" % (" ".join(cmd), out))
    return out


def _stale(src, obj):
    """True if obj is missing or older than src or any header it may include."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".inc"))]
    deps.append(os.path.join(ROOT, "include", "sttsv.h"))
    return any(os.path.getmtime(d) > t for d in deps)


def build(jobs=None, verbose=False, incremental=False):
    """Compile every translation unit (all of them unless ``incremental``)
    and link libsttsv.so."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    inc = ["-I", CSRC, "-I", os.path.join(ROOT, "include")]
    cmds = []
    for s in HIP_SOURCES:
        src, obj = os.path.join(CSRC, s), os.path.join(BUILD, s + ".o")
        if incremental and not _stale(src, obj):
            continue
        cmds.append([hipcc, "-x", "hip", "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
                     *DEVICE_FLAGS, *inc, "-c", src, "-o", obj])
    for s in CXX_SOURCES:
        src, obj = os.path.join(CSRC, s), os.path.join(BUILD, s + ".o")
        if incremental and not _stale(src, obj):
            continue
        cmds.append([hipcc, "-O2", "-std=c++17", "-fPIC", *inc, "-c", src, "-o", obj])
    jobs = jobs or min(16, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out.strip():
                print(out)
    objs = [os.path.join(BUILD, s + ".o") for s in HIP_SOURCES + CXX_SOURCES]
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    ap.add_argument("-i", "--incremental", action="store_true",
                    help="recompile only translation units older than their sources")
    a = ap.parse_args()
    print(build(a.j, a.v, a.incremental))


if __name__ == "__main__":
    sys.exit(main())
