"""Compile the HIP library libkpm.so for gfx950 (in-tree, next to this file).

    python paper_2212_05685_amd/build.py     (by file path: importing the package loads the library)

Every HIP source is compiled with packed FP32 instructions disabled
(-target-feature -packed-fp32-ops).
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = ["kpm_build.hip", "kpm_cheb.hip", "kpm_api.hip", "kpm_rmft.hip", "kpm_ldos.hip",
       "kpm_supercell.hip"]
ROCM_LIB = "/opt/rocm/lib"
LIB = os.path.join(HERE, "libkpm.so")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def command(out: str = LIB, extra=()) -> list:
    srcs = [os.path.join(HERE, "csrc", s) for s in SRC]
    return [hipcc(), "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", *extra, *srcs,
            f"-L{ROCM_LIB}", f"-Wl,-rpath,{ROCM_LIB}", "-lrocsolver", "-lrocblas", "-o", out]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libkpm.so")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
