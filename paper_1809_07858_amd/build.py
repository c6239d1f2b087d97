"""Build the HIP library libshouji.so in-tree for gfx950 (hipcc cross-compiles without a GPU)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libshouji.so")
SOURCES = ["csrc/shouji_plain.hip", "csrc/shouji_batched.hip", "csrc/shouji_abi.hip",
           "csrc/shouji_server.hip", "csrc/shouji_verify.hip", "csrc/shouji_window.hip",
           "csrc/shouji_magnet.hip", "csrc/shouji_relayout.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # no packed-FP32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


def build(verbose=False):
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + [os.path.join(HERE, s) for s in SOURCES] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL if not verbose else None)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
