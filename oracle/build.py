"""Build the CPU oracle (test infrastructure): liboracle.so (double) and
liboracle_ld.so (long double, the arbiter) and liboracle_q.so (__float128)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "shg_oracle.c")


def build(verbose: bool = False) -> None:
    for out, extra in (("liboracle.so", []), ("liboracle_ld.so", ["-DORACLE_LONG_DOUBLE"]),
                       ("liboracle_q.so", ["-DORACLE_QUAD"])):
        libs = ["-lquadmath"] if "-DORACLE_QUAD" in extra else []
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", *extra,
               "-o", os.path.join(HERE, out), SRC, *libs, "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
