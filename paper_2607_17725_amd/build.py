"""Build the HIP library (libfvem.so) in-tree for gfx950."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfvem.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

SOURCES = ["api.hip", "kernels.hip", "sell.hip", "transport.hip", "elem.hip", "setup_host.cpp", "geom.cpp", "vem.cpp", "grid.cpp"]

# -packed-fp32-ops keeps the compiler from emitting packed FP32 arithmetic
HIP_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-fopenmp", "-Wno-unused-result"]


def build(verbose=False):
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc] + HIP_FLAGS + lang + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fopenmp", "--offload-arch=gfx950", "-o", tmp] + objs + [
        f"-Wl,-rpath,{ROCM}/llvm/lib", f"-Wl,-rpath,{ROCM}/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
