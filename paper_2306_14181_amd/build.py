"""Build the gfx950 shared library of the phonon-BTE hot path in-tree.

    python -m paper_2306_14181_amd.build

Produces paper_2306_14181_amd/_lib/libbte.so from csrc/*.hip and csrc/*.cpp
with hipcc (--offload-arch=gfx950).  Compiles every time it is called.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_lib", "libbte.so")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-warning-option",
]


def build(verbose=False):
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))
    objs = []
    procs = []
    for f in srcs:
        obj = os.path.join(build_dir, f + ".o")
        cmd = ["hipcc", "-c", os.path.join(CSRC, f), "-o", obj] + HIP_FLAGS
        if f.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        procs.append((f, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = False
    for f, pr in procs:
        out, _ = pr.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 feature: harmless
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if pr.returncode != 0:
            failed = True
            sys.stderr.write("---- %s\n%s\n" % (f, "\n".join(lines)))
        elif verbose and lines:
            sys.stderr.write("---- %s\n%s\n" % (f, "\n".join(lines)))
    if failed:
        raise RuntimeError("HIP compilation failed")
    tmp = OUT + ".tmp%d" % os.getpid()
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
