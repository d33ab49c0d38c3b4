"""Build libscrooge_hip.so in-tree with hipcc for gfx950.

    python -m paper_2208_09985_amd.build

Every source is compiled on each call (this is also the project's "does it
build" check); the shared library lands next to this file.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libscrooge_hip.so")
SOURCES = ["pack.hip", "align.hip", "align_cols.hip", "align_wide.hip", "align_lane.hip", "mlp.hip", "io.hip", "noalloc.hip", "capi.cpp"]
# the resource microbenchmarks (VALU, LDS, load latency) are a library of their own
PEAK_LIB = os.path.join(HERE, "libscrooge_peak.so")
PEAK_SOURCES = ["peak.hip"]
ARCH = os.environ.get("SCG_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall",
    # keep the device compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def register_boundary_problems(asm: str) -> list:
    """Kernels in gfx950 assembly text where a 64-bit VALU instruction takes a
    32-bit VGPR operand in the last register of the wavefront's allocation
    (allocation = next_free_vgpr rounded up to 8).  A build of this kind gave
    wrong results in wavefronts that did not start at VGPR 0 of their SIMD,
    while the same code with a larger allocation was correct, so the build
    refuses such code rather than ship it."""
    problems = []
    for m in re.finditer(r"^(_Z\w+):[^\n]*\n(.*?)s_endpgm", asm, re.S | re.M):
        name, body = m.group(1), m.group(2)
        d = re.search(r"\.amdhsa_kernel " + re.escape(name) + r"\n(.*?)\.end_amdhsa_kernel", asm, re.S)
        if not d:
            continue
        nfv = re.search(r"\.amdhsa_next_free_vgpr (\d+)", d.group(1))
        if not nfv:
            continue
        alloc = (int(nfv.group(1)) + 7) // 8 * 8
        for line in body.splitlines():
            code = line.split(";")[0].strip()
            if not re.match(r"v_\w*(b64|i64|u64)\b", code) or " " not in code:
                continue
            for r in re.finditer(r"(?<![\[:])\bv(\d+)\b", code.split(None, 1)[1]):
                if int(r.group(1)) + 1 >= alloc:
                    problems.append(f"{name}: '{code}' uses v{r.group(1)}, the last of {alloc} allocated VGPRs")
    return problems


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compile both libraries; returns the alignment library's path."""
    _build_one(SOURCES, LIB, verbose, jobs)
    _build_one(PEAK_SOURCES, PEAK_LIB, verbose, jobs)
    return LIB


def _build_one(sources, lib, verbose: bool, jobs: int) -> str:
    cc = hipcc()
    tmp = tempfile.mkdtemp(prefix="scg_build_")
    try:
        objs, procs, asms = [], [], []
        for src in sources:
            obj = os.path.join(tmp, src + ".o")
            lang = ["-x", "hip"] if src.endswith(".cpp") else []
            cmds = [[cc, *HIPCC_FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj]]
            if src.endswith(".hip"):
                # device assembly for the register-boundary check
                asm = os.path.join(tmp, src + ".s")
                cmds.append([cc, *HIPCC_FLAGS, "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", asm])
                asms.append(asm)
            for cmd in cmds:
                if verbose:
                    print(" ".join(cmd), flush=True)
                procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
                while len([p for _, p in procs if p.poll() is None]) >= jobs:
                    next(p for _, p in procs if p.poll() is None).wait()
            objs.append(obj)
        for src, p in procs:
            out, _ = p.communicate()
            text = out.decode(errors="replace")
            text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
            if p.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{text}")
            if verbose and text.strip():
                print(text)
        problems = [q for a in asms for q in register_boundary_problems(open(a).read())]
        if problems:
            raise RuntimeError("register-boundary check failed:\n" + "\n".join(problems))
        tmp_lib = lib + ".tmp"
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp_lib]
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
        os.replace(tmp_lib, lib)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
