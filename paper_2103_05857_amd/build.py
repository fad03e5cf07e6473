"""Builds libsrot.so (HIP, gfx950) in-tree next to this file, and the
copy_calibrate program used to scale HBM traffic counters."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsrot.so")
CALIB = os.path.join(HERE, "copy_calibrate")
SOURCES = ["srot_kernels.hip", "srot_adjoint.hip", "srot_batched.hip", "srot_fw.hip", "srot_variants.hip",
           "srot_ga.hip", "srot_screen.hip", "srot_team.hip", "srot_plan.hip", "srot_api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    """Compiles the translation units in parallel, then links the library."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [HIPCC] + FLAGS + ["-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for p, cmd in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, cmd)
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    exe = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-o", CALIB + ".tmp", os.path.join(CSRC, "copy_calibrate.hip")]
    if verbose:
        print(" ".join(exe), flush=True)
    subprocess.run(exe, check=True)
    os.replace(CALIB + ".tmp", CALIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
