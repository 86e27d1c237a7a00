"""Builds libtnhip.so (the HIP library behind include/tensorneat_hip.h) in place.

Every source under csrc/ is compiled for gfx950 with hipcc, in parallel, then
linked into paper_2504_08339_amd/libtnhip.so. Packed FP32 instructions are
disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtnhip.so")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


# Per-file flags. Branches on wavefront-uniform values (a node's aggregation
# or activation code, an in-edge count) are left unstructured in the kernels of
# these files: plain scalar branches instead of structurized flow variables,
# 8-14 % fewer cycles on the evaluation kernels. Not applied to the NEAT
# generation and reproduction kernels (the generation's speciation gave wrong
# species with it). The program-interpreting kernels (forward engines,
# HyperNEAT, adjoints, recurrent) also start every block that is only reached
# by a branch on a 32-byte boundary: their per-node code is a chain of taken
# branches, and aligned targets made them 1-3 % faster (distance: 1 % slower,
# transform: no change, so not there).
_UNIFORM = ["-mllvm", "-structurizecfg-skip-uniform-regions=true"]
_ALIGN = ["-mllvm", "-align-all-nofallthru-blocks=5"]
FILE_FLAGS = {f: _UNIFORM for f in ("transform.hip", "distance.hip")}
FILE_FLAGS.update({f: _UNIFORM + _ALIGN for f in ("forward.hip", "forward_reg.hip", "hyperneat.hip",
                                                  "backward.hip", "recurrent.hip")})


def _compile(src: str, extra) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), *COMMON, *FILE_FLAGS.get(os.path.basename(src), []), *extra, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def _define(header: str, name: str) -> int:
    with open(os.path.join(CSRC, header)) as f:
        m = re.search(r"#define %s (\d+)" % name, f.read())
    if not m:
        raise RuntimeError(f"{name} not found in {header}")
    return int(m.group(1))


def _rf_base(kernel: str) -> int:
    """First VGPR of the register file of a register-file kernel."""
    if "backward_rf_kernel" in kernel:
        return _define("backward.hip", "TN_BW_RF_BASE")
    return _define("fwd_reg.hpp", "TN_RF_BASE")


# kernels that keep an explicit register file (names as they appear mangled)
RF_KERNELS = ("forward_rf", "cppn_query_kernel", "cppn_backward_kernel", "backward_rf_kernel")
RF_SOURCES = ("forward_reg.hip", "hyperneat.hip", "backward.hip")


def check_register_file(src: str, extra=()) -> None:
    """The register engine keeps node values in VGPRs from TN_RF_BASE up, which
    only its inline assembly addresses (through the index window); the
    compiler must never place a value there. Compiles `src` to AMDGPU assembly
    and fails if any instruction outside the inline-assembly blocks of a
    register-file kernel names such a VGPR (an SGPR spill lane, a temporary)."""
    asm = os.path.join(BUILD, os.path.basename(src) + ".s")
    cmd = [hipcc(), *COMMON, *FILE_FLAGS.get(os.path.basename(src), []), *extra,
           "--cuda-device-only", "-S", src, "-o", asm]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc -S failed on {src}:\n{res.stdout}\n{res.stderr}")
    with open(asm) as f:
        text = f.read()
    heads = [(m.start(), m.group(1)) for m in re.finditer(r"^(_Z\S+):\s", text, re.M)]
    checked = 0
    for i, (pos, name) in enumerate(heads):
        if not any(k in name for k in RF_KERNELS):
            continue
        checked += 1
        base = _rf_base(name)
        end = heads[i + 1][0] if i + 1 < len(heads) else len(text)
        body = re.sub(r";;#ASMSTART.*?;;#ASMEND", "", text[pos:end], flags=re.S)
        for line in body.split("\n"):
            code = line.split(";")[0].strip()
            if not code or code.startswith("."):
                continue
            for m in re.finditer(r"\bv\[?(\d+)(?::(\d+))?\]?", code):
                hi = int(m.group(2) or m.group(1))
                if hi >= base:
                    raise RuntimeError(
                        f"{os.path.basename(src)}: compiler-generated code of {name} uses "
                        f"v{hi} (register file starts at v{base}): {code}")
    if checked == 0:
        raise RuntimeError(f"{os.path.basename(src)}: no register-file kernel found to check")


def build(verbose: bool = False, extra=()) -> str:
    """Compile every csrc/*.hip, check the register engine's register file,
    and link libtnhip.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = min(len(srcs) + 2, max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        rf_checks = [ex.submit(check_register_file, os.path.join(CSRC, f), list(extra))
                     for f in RF_SOURCES]
        objs = list(ex.map(lambda s: _compile(s, list(extra)), srcs))
        for c in rf_checks:
            c.result()
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources", file=sys.stderr)
    return LIB


SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
            "-fno-omit-frame-pointer"]


def build_host_sanitized(verbose: bool = False) -> str:
    """Every csrc/*.hip with AddressSanitizer and UndefinedBehaviorSanitizer on
    the host code only (argument checks, plan bookkeeping, workspace carving;
    the device code is the product's), linked into
    _build/sanitize/libtnhip_host_san.so, for host-only tests on the CPU."""
    out_dir = os.path.join(BUILD, "sanitize")
    os.makedirs(out_dir, exist_ok=True)
    flags = [*COMMON, "-Xarch_host", "-g", *SANITIZE]

    def one(src):
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        cmd = [hipcc(), *flags, *FILE_FLAGS.get(os.path.basename(src), []), "-c", src, "-o", obj]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{' '.join(cmd)}\n{res.stderr}")
        return obj

    srcs = sources()
    with cf.ThreadPoolExecutor(min(8, len(srcs))) as ex:
        objs = list(ex.map(one, srcs))
    lib = os.path.join(out_dir, "libtnhip_host_san.so")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *SANITIZE, "-o", lib, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{res.stderr}")
    if verbose:
        print(f"built {lib}", file=sys.stderr)
    return lib


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--host-sanitized":
        build_host_sanitized(verbose=True)
    else:
        build(verbose=True)
