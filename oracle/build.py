"""Builds the CPU oracle (test infrastructure) into oracle/liboracle.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter"]


# AddressSanitizer and UndefinedBehaviorSanitizer build of the oracle (host
# code only), for running the CPU tests under the sanitizers: load it with
# HT_ORACLE_LIB=<path> and the sanitizer runtime preloaded (see DESIGN).
SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=undefined"]


def build(verbose=False, sanitize=False, out=None):
    src = os.path.join(HERE, "oracle.c")
    lib = out or (os.path.join(HERE, "liboracle_san.so") if sanitize else LIB)
    tmp = lib + ".tmp"
    flags = [f for f in CFLAGS if f != "-O2"] + SANITIZE if sanitize else CFLAGS
    cmd = ["gcc", *flags, "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    import sys
    print(build(verbose=True, sanitize="--sanitize" in sys.argv))
