"""Compile the HIP library libtnn.so for gfx950 (in-tree)."""
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtnn.so")
SOURCES = ["build.hip", "query.hip", "mixed.hip", "radius.hip", "gka.hip", "noalloc.hip",
           "host.cpp", "api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Wall",
         "-Wno-unused-result", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(HERE, "..", "include")]


# Per-source flags.  The BF16 linear search reads every tile value with
# vector ALU instructions: MFMA results in VGPRs save one register read each.
SOURCE_FLAGS = {"mixed.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}

LITERAL64 = re.compile(r"\b(s_mov_b64|v_mov_b64|s_[a-z0-9_]+_b64)\b[^;]*\b0x[0-9a-fA-F]{9,}")

# Kernels that must not use scratch memory: in the BF16 linear search a
# scratch reload waits on the vector-memory counter, which also drains the
# stage loads in flight (they complete in issue order).
NO_SCRATCH = {"mixed.hip": ("mixed_brute_kernel",)}
KERNEL_DESC = re.compile(r"\.amdhsa_kernel\s+(\S+)")
PRIVATE_SIZE = re.compile(r"\.amdhsa_private_segment_fixed_size\s+(\d+)")


def _scratch_users(asm_path, names):
    """Kernels among `names` (substrings of the symbol) whose descriptor
    reserves private (scratch) memory."""
    bad, current = [], None
    for ln in open(asm_path):
        m = KERNEL_DESC.search(ln)
        if m:
            current = m.group(1)
            continue
        m = PRIVATE_SIZE.search(ln)
        if m and current and int(m.group(1)) > 0 and any(n in current for n in names):
            bad.append(current)
    return bad


def _compile(src):
    obj = os.path.join(BUILD, src + ".o")
    flags = FLAGS + SOURCE_FLAGS.get(src, [])
    cmd = [HIPCC] + flags + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode == 0 and src.endswith(".hip"):
        # The gfx950 assembler of this toolchain encodes a 64-bit scalar
        # literal move by its low 32 bits only (+inf becomes 0): refuse any.
        asm = os.path.join(BUILD, src + ".s")
        a = subprocess.run([HIPCC] + flags + ["-x", "hip", "--cuda-device-only", "-S",
                                              os.path.join(CSRC, src), "-o", asm],
                           capture_output=True, text=True)
        if a.returncode == 0:
            bad = [ln.strip() for ln in open(asm) if LITERAL64.search(ln)]
            if bad:
                r = subprocess.CompletedProcess(cmd, 1, "", "64-bit scalar literal in device code "
                                                "(miscompiled on gfx950): " + "; ".join(bad[:5]))
            scratch = _scratch_users(asm, NO_SCRATCH.get(src, ()))
            if scratch:
                r = subprocess.CompletedProcess(cmd, 1, "", "kernel uses scratch memory: "
                                                + "; ".join(scratch))
    return src, obj, r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    objs = []
    for src, obj, r in results:
        errs = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln]
        if r.returncode != 0:
            sys.stderr.write("\n".join(errs) + "\n")
            raise RuntimeError(f"hipcc failed on {src}")
        if verbose and errs:
            sys.stderr.write("\n".join(errs) + "\n")
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
