"""Builds the CPU oracle (test infrastructure) into oracle/liborc.so.

Plain C, single-threaded, compiled without floating-point contraction so that
every fp32 operation rounds exactly once, as the definitions require.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
# ORC_SANITIZE=1 builds and loads a copy instrumented with AddressSanitizer
# and UndefinedBehaviorSanitizer (run Python with libasan preloaded)
SANITIZE = os.environ.get("ORC_SANITIZE") == "1"
LIB = os.path.join(HERE, "liborc_san.so" if SANITIZE else "liborc.so")


def build(force: bool = False) -> str:
    src = os.path.join(HERE, "orc.c")
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(
            os.path.getmtime(src), os.path.getmtime(os.path.join(HERE, "orc.h"))):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter", "-D_GNU_SOURCE",
           src, "-o", tmp, "-lm"]
    if SANITIZE:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-g"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
