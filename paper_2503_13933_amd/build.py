"""Build the TAPS HIP library (libtaps.so, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtaps.so")
SOURCES = [
    "taps_handle.hip",
    "taps_basis.hip",
    "taps_contract.hip",
    "taps_solve.hip",
    "taps_sweep.hip",
    "taps_batch.hip",
    "taps_reconstruct.hip",
    "taps_reconstruct_mfma.hip",
    "taps_mlp.hip",
    "taps_tune.hip",
]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
# per source: the reconstruction's matrix-core accumulators in ordinary
# vector registers (each AGPR result would otherwise be copied out by one
# vector instruction per value before the epilogue uses it)
EXTRA = {"taps_reconstruct_mfma.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    from concurrent.futures import ThreadPoolExecutor
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmds.append([hipcc, *[f for f in FLAGS if f != "-shared"], *EXTRA.get(src, []), "-c", os.path.join(CSRC, src),
                     "-o", obj])
        objs.append(obj)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", "4"))))
    with ThreadPoolExecutor(jobs) as pool:
        list(pool.map(run, cmds))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
