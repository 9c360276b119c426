"""Compile the CPU oracle (test infrastructure only) into two shared libraries:
``liblbmref_f64.so`` (double precision) and ``liblbmref_f32.so`` (single precision
diagnostic build).  Plain gcc, no GPU code."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbmref.c")
FLAGS = ["-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
         "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> None:
    for tag, extra in (("f64", []), ("f32", ["-DLBMREF_REAL=float"])):
        out = os.path.join(HERE, f"liblbmref_{tag}.so")
        cmd = ["gcc", *FLAGS, *extra, SRC, "-o", out + ".tmp", "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
