"""Builds the host-side rocRAND Philox reference used to pin the oracle's RNG."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build():
    src = os.path.join(HERE, "rocrand_philox_ref.cpp")
    out = os.path.join(HERE, "librocrand_philox_ref.so")
    if os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["hipcc", "-O1", "-fPIC", "-shared", src, "-o", tmp])
    os.replace(tmp, out)
    return out
