"""Build libperm_mi355x.so in-tree with hipcc for gfx950.

Sources: paper_2501_15126_amd/csrc/*.cpp (host code: validation, ordering,
partitioning, code generation, hipRTC driver, runtime) and *.hip (the
precompiled final-reduction kernel).  The result is
paper_2501_15126_amd/libperm_mi355x.so, loaded by perm.py.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libperm_mi355x.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# No packed-FP32 instructions in any HIP code of this project.
NO_PACKED_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.cpp")) + glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-Wall",
               "-I", os.path.join(ROOT, "include"), "-I", CSRC, *NO_PACKED_FP32, "-c", src, "-o", obj]
        if src.endswith(".cpp"):
            # host-only translation units
            cmd.insert(1, "-x")
            cmd.insert(2, "c++")
            cmd = [c for c in cmd if c not in ("--offload-arch=gfx950",) and c not in NO_PACKED_FP32]
            cmd += ["-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = False
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed = True
            sys.stderr.write("build failed: %s\n%s\n" % (src, text))
        elif verbose and text.strip():
            sys.stderr.write(text + "\n")
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs,
                    "-L/opt/rocm/lib", "-lhiprtc", "-lamd_comgr", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
