"""Build libfscc.so (gfx950) in-tree with hipcc.

Each source is compiled to an object in parallel (no relocatable device code:
every kernel is launched from its own translation unit), then linked into
the shared library.  All HIP code is compiled with packed-FP32 instruction
selection disabled.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfscc.so")
SOURCES = ["fscc_api.hip", "batch_api.hip", "noalloc_api.hip", "kernels.hip", "kernels_real.hip", "kernels_split.hip",
           "kernels_dl.hip", "mlp.hip", "probe.hip", "plan_ccsd.cpp", "host_linalg.cpp"]
# per-source extra flags: the throughput probe's accumulators stay in VGPRs
# (no accumulator copies around its loop)
EXTRA = {"probe.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    return r.returncode, r.stdout


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    tag = "%d" % os.getpid()
    cmds = []
    objs = []
    for s in SOURCES:
        obj = os.path.join(OBJ, os.path.splitext(s)[0] + "." + tag + ".o")
        objs.append(obj)
        cmds.append([HIPCC] + FLAGS + EXTRA.get(s, []) + ["-c", "-o", obj, os.path.join(CSRC, s)])
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_run, cmds))
    bad = [(c, out) for c, (rc, out) in zip(cmds, results) if rc != 0]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    if bad:
        for c, out in bad:
            sys.stderr.write(" ".join(c) + "\n" + out)
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
        raise RuntimeError("hipcc failed building libfscc.so")
    tmp = LIB + ".tmp" + tag
    link = [HIPCC, "--offload-arch=gfx950", "-fPIC", "-shared", "-o", tmp] + objs
    if verbose:
        print(" ".join(link), flush=True)
    rc, out = _run(link)
    for o in objs:
        if os.path.exists(o):
            os.remove(o)
    if rc != 0:
        sys.stderr.write(out)
        raise RuntimeError("hipcc failed linking libfscc.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
