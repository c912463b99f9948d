"""Builds the HIP library libvca.so in-tree for gfx950 with hipcc (the three
translation units compile in parallel, then link into one shared library)."""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "csrc", n) for n in ("vca.hip", "vca_batch.hip", "vca_grad.hip")]
LIB = os.path.join(HERE, "libvca.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # packed FP32 instructions stay off in every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA results straight into VGPRs (no accumulator-register copies)
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
]


def build(verbose: bool = False, extra=()) -> str:
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory(prefix="vca_build_") as work:
        objs = [os.path.join(work, os.path.basename(s) + ".o") for s in SRCS]
        cmds = [[HIPCC, *FLAGS, *extra, "-c", src, "-o", obj] for src, obj in zip(SRCS, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with ThreadPoolExecutor(len(cmds)) as pool:
            procs = list(pool.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
        for c, p in zip(cmds, procs):
            sys.stderr.write(p.stderr)
            if p.returncode != 0:
                raise subprocess.CalledProcessError(p.returncode, c)
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
