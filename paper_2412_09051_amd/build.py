"""Build libsllbm.so (HIP for gfx950) in-tree.

Usage: python paper_2412_09051_amd/build.py [-v]   (by path: importing the package
loads the library this script builds)
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsllbm.so")

SOURCES = ["sllbm_host.cpp", "sllbm_csr.cpp", "sllbm_device.hip", "sllbm_kernels.hip", "sllbm_tile.hip", "sllbm_csr_kernel.hip", "sllbm_mlp.hip"]

# -packed-fp32-ops: keep the compiler from emitting packed FP32 VALU ops.
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return h


def build(verbose=False, jobs=4, defines=()):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        s = os.path.join(CSRC, src)
        o = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc()] + HIPFLAGS + ["-D" + d for d in defines] + lang + ["-c", s, "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), src))
        objs.append(o)
    failed = False
    for p, src in procs:
        out, _ = p.communicate()
        if out:
            sys.stdout.write(out.decode())
        if p.returncode != 0:
            failed = True
            print("compile failed:", src, file=sys.stderr)
    if failed:
        raise RuntimeError("libsllbm build failed")
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, defines=[a[2:] for a in sys.argv[1:] if a.startswith("-D")]))
