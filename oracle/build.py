"""Builds the oracle library ``oracle/liboracle.so`` with gcc.

Test infrastructure: the compiled oracle is used only by the tests, the smoke
check and the CPU-baseline leg of the benchmark.  Plain IEEE double
arithmetic: no -ffast-math, no FMA contraction beyond the default target.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose=False, force=True):
    """Compiles the oracle; with force=False only if the library is missing
    or older than its source."""
    src = os.path.join(HERE, "oracle.c")
    out = os.path.join(HERE, "liboracle.so")
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC", "-Wall",
           src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
