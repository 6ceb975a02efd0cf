"""Build libempc.so (HIP, gfx950) in-tree.

    python -m paper_2001_04931_amd.build [--changed]

Each .hip file under csrc/ is compiled to an object with hipcc, then the
objects are linked into paper_2001_04931_amd/libempc.so.  Packed FP32 VALU
instructions are disabled for every device compilation.
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libempc.so")
ARCH = "gfx950"

DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Per-file device options.  The rollout kernels keep MFMA accumulators in
# ordinary VGPRs: the state the matrix cores produce is read back by the
# next step's MFMAs and by VALU cost code, and the AGPR form would force
# copies between the two register files on every step.
FILE_FLAGS = {"rollout_linear_f32.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
              "batched.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
          "-Wno-unused-function", "-Wno-unused-result"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: cannot build libempc.so")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), "-c", *COMMON, *DEVICE_FLAGS, *FILE_FLAGS.get(os.path.basename(src), []),
           "-I", os.path.join(HERE, "..", "include"), src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, r.stderr[-8000:]))
    if r.stderr.strip():
        warn = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if warn:
            sys.stderr.write("\n".join(warn[-40:]) + "\n")
    return obj


def _stale(src: str, headers) -> bool:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in [src, *headers])


def build(verbose: bool = True, changed_only: bool = False) -> str:
    """Compile every source (changed_only: only those whose object is older
    than the source or any header) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    headers = glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(
        os.path.join(HERE, "..", "include", "*.h"))
    todo = [s for s in srcs if not changed_only or _stale(s, headers)]
    if todo:
        with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(todo))) as ex:
            list(ex.map(_compile, todo))
    objs = [os.path.join(BUILD, os.path.basename(s) + ".o") for s in srcs]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-8000:])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(changed_only="--changed" in sys.argv[1:])
