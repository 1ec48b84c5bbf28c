"""Builds the gfx950 HIP library ``libfvsrn.so`` in-tree with hipcc.

The network kernels are compiled once per precision (FP32, FP16, BF16) as
separate translation units (the adjoint-gradient, time-encoded and
Fourier-matrix kernels in units of their own), in parallel, then linked with
the C ABI and the utility kernels into one shared library.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import json
import os
import re
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
    ("fvsrn_adjoint.hip", ["-DFVSRN_PREC=0"], "adj_f32.o"),
    ("fvsrn_adjoint.hip", ["-DFVSRN_PREC=1"], "adj_f16.o"),
    ("fvsrn_adjoint.hip", ["-DFVSRN_PREC=2"], "adj_bf16.o"),
    ("fvsrn_time.hip", ["-DFVSRN_PREC=0"], "time_f32.o"),
    ("fvsrn_time.hip", ["-DFVSRN_PREC=1"], "time_f16.o"),
    ("fvsrn_time.hip", ["-DFVSRN_PREC=2"], "time_bf16.o"),
    ("fvsrn_rff.hip", ["-DFVSRN_PREC=0"], "rff_f32.o"),
    ("fvsrn_rff.hip", ["-DFVSRN_PREC=1"], "rff_f16.o"),
    ("fvsrn_rff.hip", ["-DFVSRN_PREC=2"], "rff_bf16.o"),
    # the training kernels schedule for instruction-level parallelism (measured
    # 5% faster per step; the render kernels are faster with the default)
    ("fvsrn_train.hip", ["-mllvm", "-amdgpu-sched-strategy=max-ilp"], "train.o"),
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
    for f in sorted(os.listdir(CSRC)):
        out.append(os.path.join(CSRC, f))
    return out


def source_hash() -> str:
    """SHA-256 over the header and every file of csrc/ (names and contents):
    the library records it at build time (fvsrn_build_id), and the binding
    refuses a library whose record differs from the sources beside it."""
    import hashlib
    h = hashlib.sha256()
    for path in _sources():
        h.update(os.path.relpath(path, ROOT).encode() + b"\0")
        with open(path, "rb") as fh:
            h.update(fh.read())
        h.update(b"\0")
    return h.hexdigest()


def _run(cmd, cwd=None):
    res = subprocess.run(cmd, capture_output=True, text=True, cwd=cwd)
    text = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l)
    return res.returncode, text


_VMEM = ("global_", "buffer_", "flat_", "scratch_")
_REGS = re.compile(r"\b([va])\[(\d+):(\d+)\]|\b([va])(\d+)\b")


def _reg_set(text):
    out = set()
    for m in _REGS.finditer(text):
        if m.group(1):
            out |= {(m.group(1), i) for i in range(int(m.group(2)), int(m.group(3)) + 1)}
        else:
            out.add((m.group(4), int(m.group(5))))
    return out


def mfma_early_vmem_reads(asm: str):
    """Memory instructions that read an MFMA result fewer wait states after
    the MFMA than the result needs (passes + 3: 11 for the 16x16 shapes, 19
    for 32x32), on any path through the listing's branches (one function or
    several). The compiler pads VALU and LDS readers of MFMA results, but a
    global store of a result reached through a taken branch was issued right
    after the MFMA. Returns (function, mfma, reader) triples."""
    funcs, cur = [], None
    for line in asm.splitlines():
        if line.startswith("_Z") and ":" in line:
            cur = (line.split(":", 1)[0], [])
            funcs.append(cur)
        elif cur is not None:
            cur[1].append(line)
    bad = []
    for fn, lines in funcs:
        ins, labels = [], {}
        for raw in lines:
            l = raw.split(";")[0].rstrip()
            if not l.strip():
                continue
            m = re.match(r"^(\.LBB\w+):", l)
            if m:
                labels[m.group(1)] = len(ins)
            elif l[0].isspace() and not l.strip().startswith("."):
                t = l.strip()
                op = t.split()[0]
                ins.append((op, t[len(op):]))
        for i, (op, rest) in enumerate(ins):
            if not op.startswith("v_mfma"):
                continue
            dst = _reg_set(rest.split(",")[0])
            need = 19 if "32x32" in op else 11
            stack, seen = [(i + 1, 0)], set()
            while stack:
                j, w = stack.pop()
                while j < len(ins) and w < need and (j, w) not in seen:
                    seen.add((j, w))
                    o, r = ins[j]
                    # registers the memory instruction reads: a load's first
                    # operand is its destination
                    src = r.split(",", 1)[1] if ("_load" in o and "," in r) else r
                    if o.startswith(_VMEM) and _reg_set(src) & dst:
                        bad.append((fn, "%s%s" % ins[i], "%s%s" % ins[j]))
                        break
                    if o.startswith("v_mfma") and _reg_set(r.split(",")[0]) >= dst:
                        break
                    w += int(r.strip(), 0) + 1 if o == "s_nop" else 1
                    if o == "s_branch":
                        j = labels[r.strip()]
                        continue
                    if o.startswith("s_cbranch"):
                        stack.append((labels[r.strip()], w))
                    if o in ("s_endpgm", "s_setpc_b64"):
                        break
                    j += 1
    return bad


def device_asm_files():
    return sorted(glob.glob(os.path.join(BUILD, "*", "*-hip-amdgcn-amd-amdhsa-gfx950.s")))


KERNEL_HASHES = os.path.join(HERE, "libfvsrn_kernels.json")


def kernel_isa_hashes(asm: str):
    """sha256 of each kernel's instruction listing (label to end of function,
    comments and directives dropped): it changes only when the kernel's code
    does, unlike a hash of the source files."""
    import hashlib
    out, name, body = {}, None, []
    for line in asm.splitlines():
        head = line.split(";")[0].rstrip()
        if head.startswith("_Z") and head.endswith(":"):
            name, body = head[:-1], []
        elif name is not None:
            if line.startswith(".Lfunc_end"):
                out[name] = hashlib.sha256("\n".join(body).encode()).hexdigest()
                name = None
                continue
            t = line.split(";")[0].strip()
            if t and not t.startswith("."):
                body.append(t)
    return out


def build(force: bool = True, verbose: bool = False, jobs: int = 0) -> str:
    """Compile the library (always when force is set)."""
    if not force and os.path.exists(LIB):
        if os.path.getmtime(LIB) >= max(os.path.getmtime(p) for p in _sources()):
            return LIB
    os.makedirs(BUILD, exist_ok=True)
    units = [u for u in UNITS if os.path.exists(os.path.join(CSRC, u[0]))]
    cmds = []
    src_hash = source_hash()
    for src, defs, obj in units:
        if src == "fvsrn_api.cpp":
            defs = defs + ['-DFVSRN_SOURCE_HASH="%s"' % src_hash]
        # each unit keeps its intermediate files (device assembly included) in
        # a folder of its own
        tmp = os.path.join(BUILD, obj[:-2])
        os.makedirs(tmp, exist_ok=True)
        extra = ["-save-temps=cwd"] if src.endswith(".hip") else []
        cmds.append(([hipcc()] + HIPCC_FLAGS + defs + extra + ["-I", os.path.join(ROOT, "include"), "-c",
                                                               os.path.join(CSRC, src), "-o",
                                                               os.path.join(BUILD, obj)], tmp))
    jobs = jobs or min(len(cmds), os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda c: _run(c[0], cwd=c[1]), cmds))
    for (src, _, obj), (rc, text) in zip(units, results):
        if rc != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (src, text))
        if verbose and text.strip():
            print(text, file=sys.stderr)
    # refuse a library in which a memory instruction reads an MFMA result
    # before it is complete (such a store wrote partly stale tiles on gfx950)
    for path in device_asm_files():
        with open(path) as fh:
            text = fh.read()
        bad = mfma_early_vmem_reads(text)
        if bad:
            raise RuntimeError("%s: memory instruction reads an MFMA result too early:\n%s" %
                               (path, "\n".join("%s: %s -> %s" % b for b in bad[:10])))
    hashes = {}
    for path in device_asm_files():
        with open(path) as fh:
            hashes.update(kernel_isa_hashes(fh.read()))
    with open(KERNEL_HASHES, "w") as fh:
        json.dump(hashes, fh, indent=0, sort_keys=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    rc, text = _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] +
                    [os.path.join(BUILD, u[2]) for u in units])
    if rc != 0:
        raise RuntimeError("link failed:\n" + text)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
