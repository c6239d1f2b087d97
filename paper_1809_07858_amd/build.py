"""Build the HIP library libshouji.so in-tree for gfx950 (hipcc cross-compiles without a GPU)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libshouji.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["csrc/shouji_plain.hip", "csrc/shouji_batched.hip", "csrc/shouji_abi.hip",
           "csrc/shouji_server.hip", "csrc/shouji_verify.hip", "csrc/shouji_window.hip",
           "csrc/shouji_magnet.hip", "csrc/shouji_relayout.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # no packed-FP32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]
# Per-source flags.  The plain, tile and two-length kernels' window loop is
# long straight-line gate code run at two wavefronts per SIMD: the machine
# scheduler's ILP strategy (within the 256 VGPRs that occupancy allows, no
# scratch) gave 2-5% shorter launches than the default one on the shapes
# measured, with identical outputs.
EXTRA = {
    "csrc/shouji_plain.hip": ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"],
}


def build(verbose=False, jobs=8):
    os.makedirs(OBJDIR, exist_ok=True)
    cmds, objs = [], []
    for s in SOURCES:
        obj = os.path.join(OBJDIR, os.path.basename(s) + ".o")
        cmds.append([HIPCC] + FLAGS + EXTRA.get(s, []) + ["-c", os.path.join(HERE, s), "-o", obj])
        objs.append(obj)
    # compile the sources in parallel, then link
    running = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        running.append((cmd, subprocess.Popen(cmd, stderr=subprocess.DEVNULL if not verbose else None)))
        if len(running) >= jobs:
            c, p = running.pop(0)
            if p.wait() != 0:
                raise subprocess.CalledProcessError(p.returncode, c)
    for c, p in running:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, c)
    tmp = SO + ".tmp%d" % os.getpid()
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link, stderr=subprocess.DEVNULL if not verbose else None)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
