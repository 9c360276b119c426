"""Compile the CPU oracle (test infrastructure only) into two shared libraries:
``liblbmref_f64.so`` (double precision) and ``liblbmref_f32.so`` (single precision
diagnostic build), and the sanitizer driver ``lbmref_sanitize`` (the double-precision
oracle with AddressSanitizer and UndefinedBehaviorSanitizer, host code only).  Plain gcc,
no GPU code."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbmref.c")
DRIVER = os.path.join(HERE, "sanitize_main.c")
SANITIZE_EXE = os.path.join(HERE, "lbmref_sanitize")
FLAGS = ["-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
         "-Wall", "-Wno-unused-function"]
SAN_FLAGS = ["-O1", "-g", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-Wall", "-Wno-unused-function"]


def build_sanitized(verbose: bool = False) -> str:
    cmd = ["gcc", *SAN_FLAGS, SRC, DRIVER, "-o", SANITIZE_EXE + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(SANITIZE_EXE + ".tmp", SANITIZE_EXE)
    return SANITIZE_EXE


def build(verbose: bool = False) -> None:
    for tag, extra in (("f64", []), ("f32", ["-DLBMREF_REAL=float"])):
        out = os.path.join(HERE, f"liblbmref_{tag}.so")
        cmd = ["gcc", *FLAGS, *extra, SRC, "-o", out + ".tmp", "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    build_sanitized(verbose)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
