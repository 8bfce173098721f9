"""Build the FP64 CPU oracle (``liblbo.so``) with gcc.

Test infrastructure: the oracle checks the GPU library and is never part of
it.  ``-ffp-contract=off`` keeps every FP64 expression rounded as written
(the head geometry is decided in FP64 and must not depend on FMA fusion).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "lbo.c")
    out = os.path.join(HERE, "liblbo.so")
    cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
