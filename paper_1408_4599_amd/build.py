"""Build libmdcell.so in-tree with hipcc for gfx950 (kernels) and the host C++ (ABI layer).

Flags: -O3, no floating-point contraction (explicit fma() where fused arithmetic is intended, so
the cutoff test and the periodic wrap are bit-reproducible), packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmdcell.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
KERNEL_SOURCES = ["md_cells.hip", "md_pair.hip", "md_step.hip", "md_adjoint.hip"]
HOST_SOURCES = ["md_api.cpp"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", f"-I{os.path.join(HERE, '..', 'include')}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link the shared library; returns its path."""
    with tempfile.TemporaryDirectory(prefix="mdcell_build_") as tmp:
        procs = []
        objs = []
        for src in KERNEL_SOURCES + HOST_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            flags = COMMON + (DEVICE if src.endswith(".hip") else ["-D__HIP_PLATFORM_AMD__"])
            cmd = [HIPCC] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
        failed = []
        for src, p in procs:
            out, _ = p.communicate()
            text = "\n".join(l for l in out.decode(errors="replace").splitlines() if "packed-fp32-ops" not in l)
            if p.returncode != 0:
                failed.append((src, text))
            elif verbose and text.strip():
                print(text)
        if failed:
            for src, text in failed:
                sys.stderr.write(f"--- {src}\n{text}\n")
            raise RuntimeError("libmdcell build failed: " + ", ".join(s for s, _ in failed))
        tmp_lib = LIB + ".tmp"
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp_lib] + objs
        subprocess.run(cmd, check=True)
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
