"""Build libcorr.so (all HIP kernels and the host runtime) for gfx950 with hipcc.

Each translation unit is compiled to an object in parallel, then linked into
paper_1102_0148_amd/libcorr.so.  Run `python -m paper_1102_0148_amd.build`.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libcorr.so")
SOURCES = ["host.hip", "fstage.hip", "xstage.hip", "dump.hip", "batch.hip", "ingest.hip", "fused.hip"]
ARCH = "gfx950"
# Packed fp32 VALU forms are kept out of every kernel on this target, and
# floating-point contraction is off: fused multiply-adds are written out.
FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-Wno-unused-result"]
# Units holding the F-stage, whose transform feeds matrix-product results
# straight back into vector arithmetic: the products write vector registers
# (the accumulation-register form costs a copy of every result).
UNIT_FLAGS = {src: ["-mllvm", "-amdgpu-mfma-vgpr-form"] for src in ("fstage.hip", "fused.hip", "batch.hip")}


def _compile(src, verbose):
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *FLAGS, *UNIT_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
