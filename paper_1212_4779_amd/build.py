"""Compile the HIP library (libim.so) for gfx950 with hipcc."""
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libim.so")
SOURCES = [os.path.join(PKG, "csrc", f) for f in ("im.hip", "mlp.hip", "undirected.hip")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from emitting packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose=False):
    """Always recompiles libim.so in place: one object per source, compiled
    in parallel, then linked."""
    tmp = LIB + ".tmp"
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(PKG, "csrc")]
    objs, procs = [], []
    for src in SOURCES:
        obj = src[:-4] + ".o"
        cmd = ["hipcc", *HIPCC_FLAGS, *inc, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                            text=True)))
        objs.append(obj)
    errors = []
    for cmd, p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            errors.append(" ".join(cmd) + "\n" + out + err)
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    cmd = ["hipcc", *HIPCC_FLAGS, "-shared", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    for obj in objs:
        os.remove(obj)
    if proc.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + proc.stdout + proc.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
