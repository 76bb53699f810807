"""Builds the HIP library ``libcmtcs.so`` for gfx950 in-tree (next to this file).

Usage: ``python -m paper_2310_00420_amd.build`` or ``build()`` from Python.  Each ``csrc/*.hip``
file is compiled to an object in ``_build/`` in parallel, then linked into one shared library.
"""

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libcmtcs.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
# All device code is built without packed-FP32 instructions.
CFLAGS = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include")]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # the host pass does not know the packed-fp32 feature and says so; that line is noise
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    return p.returncode, out


def build(verbose=False):
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    bdir = os.path.join(ROOT, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = [os.path.join(bdir, os.path.basename(s)[:-4] + ".o") for s in srcs]
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with concurrent.futures.ThreadPoolExecutor(max_workers=max(jobs, 1)) as ex:
        res = list(ex.map(lambda so: _run([HIPCC] + CFLAGS + ["-c", so[0], "-o", so[1]]),
                          zip(srcs, objs)))
    for (rc, out), s in zip(res, srcs):
        if verbose and out.strip():
            print(out)
        if rc != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (s, out))
    tmp = LIB + ".tmp"
    rc, out = _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    if rc != 0:
        raise RuntimeError("link failed:\n" + out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
