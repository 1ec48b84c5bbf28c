"""Builds the gfx950 HIP library ``libfvsrn.so`` in-tree with hipcc.

The network kernels are compiled once per precision (FP32, FP16, BF16) as
separate translation units, in parallel, then linked with the C ABI and the
utility kernels into one shared library.
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
LIB = os.path.join(HERE, "libfvsrn.so")

# (source, extra defines, object name)
UNITS = [
    ("fvsrn_api.cpp", [], "api.o"),
    ("fvsrn_misc.hip", [], "misc.o"),
    ("fvsrn_march.hip", ["-DFVSRN_PREC=0"], "march_f32.o"),
    ("fvsrn_march.hip", ["-DFVSRN_PREC=1"], "march_f16.o"),
    ("fvsrn_march.hip", ["-DFVSRN_PREC=2"], "march_bf16.o"),
    ("fvsrn_train.hip", [], "train.o"),
]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 VALU instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _sources():
    out = [os.path.join(ROOT, "include", "fvsrn.h")]
    for f in os.listdir(CSRC):
        out.append(os.path.join(CSRC, f))
    return out


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    text = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l)
    return res.returncode, text


def build(force: bool = True, verbose: bool = False, jobs: int = 0) -> str:
    """Compile the library (always when force is set)."""
    if not force and os.path.exists(LIB):
        if os.path.getmtime(LIB) >= max(os.path.getmtime(p) for p in _sources()):
            return LIB
    os.makedirs(BUILD, exist_ok=True)
    units = [u for u in UNITS if os.path.exists(os.path.join(CSRC, u[0]))]
    cmds = []
    for src, defs, obj in units:
        cmds.append([hipcc()] + HIPCC_FLAGS + defs + ["-I", os.path.join(ROOT, "include"), "-c",
                                                      os.path.join(CSRC, src), "-o", os.path.join(BUILD, obj)])
    jobs = jobs or min(len(cmds), os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_run, cmds))
    for (src, _, obj), (rc, text) in zip(units, results):
        if rc != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (src, text))
        if verbose and text.strip():
            print(text, file=sys.stderr)
    tmp = LIB + ".tmp%d" % os.getpid()
    rc, text = _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] +
                    [os.path.join(BUILD, u[2]) for u in units])
    if rc != 0:
        raise RuntimeError("link failed:\n" + text)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
