"""Build libtsqr.so (HIP, gfx950) in-tree with hipcc.

Every .hip file under csrc/ is compiled to an object in parallel, then linked
into paper_0808_2664_amd/libtsqr.so.  tsqr_factor_inst.hip is compiled once per
instantiation of the factor launcher (type x panels x implicit Q kept), so the
unrolled factor kernels build in parallel.  Run:
``python -m paper_0808_2664_amd.build``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtsqr.so")
ARCH = os.environ.get("TSQR_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

# -packed-fp32-ops: keep the compiler from forming packed FP32 VALU ops.
CFLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


INST = "tsqr_factor_inst.hip"
FACTOR_INST = [(t, np_, wq) for t in ("double", "float") for np_ in (4, 2, 1) for wq in (1, 0)]


def sources():
    """(source, object name, extra flags) of every compilation unit."""
    units = []
    for f in sorted(os.listdir(CSRC)):
        if not f.endswith(".hip"):
            continue
        src = os.path.join(CSRC, f)
        if f == INST:
            for t, np_, wq in FACTOR_INST:
                units.append((src, "factor_%s_np%d_%s" % (t[0], np_, "q" if wq else "r"),
                              ["-DTSQR_INST_T=" + t, "-DTSQR_INST_NP=%d" % np_, "-DTSQR_INST_WQ=%d" % wq]))
        else:
            units.append((src, f[:-4], []))
    # longest compilations first
    return sorted(units, key=lambda u: 0 if u[1].startswith("factor_d") else 1)


def _compile(unit) -> str:
    src, name, extra = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC] + CFLAGS + extra + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, p.stderr))
    return obj


def build(jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n%s" % p.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else None))
