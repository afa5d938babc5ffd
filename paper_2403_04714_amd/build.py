"""Build libfibersim.so for gfx950 in-tree with hipcc (no JIT cache).

    python -m paper_2403_04714_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfibersim.so")
SOURCES = ["compiler.cpp", "runtime.cpp", "serve.cpp", "kernels_plain.hip", "kernels_batched.hip", "scratch.hip"]
HEADERS = ["compiler.h", "isa.h", "kernels.h", "device_common.h"]
ARCH = os.environ.get("FSIM_OFFLOAD_ARCH", "gfx950")


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose: bool = False) -> str:
    """Compile every source (always; this is the build check)."""
    objs = []
    common = ["-O3", "-std=c++17", "-fPIC", f"-I{CSRC}", f"-I{os.path.join(HERE, '..', 'include')}"]
    for src in sources():
        obj = os.path.join(CSRC, os.path.basename(src) + ".o")
        # every translation unit targets gfx950 only (host-only files carry no
        # device code, but must not default to another architecture)
        cmd = ["hipcc", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
               "-packed-fp32-ops", *common, "-c", src, "-o", obj]
        if src.endswith(".hip"):
            # Uniform branches (the interpreters' opcode and class dispatch)
            # are left unstructured: structurizing them adds a scalar flag
            # block per branch on every interpreted instruction.
            cmd[1:1] = ["-x", "hip"]
            cmd += ["-mllvm", "-structurizecfg-skip-uniform-regions=true"]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"hipcc failed on {src}")
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
