"""Builds the HIP library libmpmc.so for gfx950, in-tree.

All sources are compiled by hipcc with floating-point contraction off (every
fp32 operation of the sampler must round exactly once) and without packed
fp32 instructions.
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmpmc.so")
ARCH = os.environ.get("MPMC_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
         "--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include")]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(force=True, jobs=8):
    srcs = sources()
    deps = srcs + glob.glob(os.path.join(HERE, "csrc", "*.hpp")) + [os.path.join(ROOT, "include", "mpmc.h")]
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(os.path.getmtime(d) for d in deps):
        return LIB
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for s in srcs:
        o = os.path.join(objdir, os.path.basename(s) + ".o")
        objs.append(o)
        procs.append((s, subprocess.Popen(["hipcc", "-c", s, "-o", o] + FLAGS,
                                          stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        while sum(p.poll() is None for _, p in procs) >= jobs:
            procs[[p.poll() is None for _, p in procs].index(True)][1].wait()
    failed = False
    for s, p in procs:
        out = p.communicate()[0].decode()
        if p.returncode != 0:
            failed = True
            sys.stderr.write("hipcc failed for %s:\n%s\n" % (s, out))
        elif out.strip():
            lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l and "is not a recognized feature" not in l]
            if lines:
                sys.stderr.write("\n".join(lines) + "\n")
    if failed:
        raise RuntimeError("HIP build failed")
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["hipcc", "-shared", "-o", tmp] + objs + ["--offload-arch=" + ARCH, "-fPIC"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
