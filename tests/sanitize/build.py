"""Build the sanitizer drivers (test infrastructure): the CPU oracle and the
host mirror, each linked into a small executable with AddressSanitizer and
UndefinedBehaviorSanitizer (every finding fatal), into tests/_build/sanitize/.
CPU-only builds; no GPU code is involved.

The host mirror instantiates only the classes l_a, l_b <= 2 with derivatives
here (HM_KEEP): the full table takes minutes to compile with instrumentation.
A build is reused while the stamp (sha256 of the flags and of every source and
header involved) matches."""
import concurrent.futures as cf
import glob
import hashlib
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(ROOT, "tests", "_build", "sanitize")
ORACLE_SRC = os.path.join(ROOT, "oracle", "shg_oracle.c")
MIRROR_DIR = os.path.join(ROOT, "tests", "hostmirror")
CSRC = os.path.join(ROOT, "paper_1701_06588_amd", "csrc")
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
KEEP = "-DHM_KEEP(la,lb,d)=((la)<=2&&(lb)<=2&&(d))"
# the same C++ compiler as the host mirror's own build
CXX = "/opt/rocm/llvm/bin/clang++" if os.path.exists("/opt/rocm/llvm/bin/clang++") else "g++"
MIRROR_SRCS = ["shg_hostmirror.cpp"] + [f"shg_hostmirror_op{k}.cpp" for k in range(5)]


def _stamp() -> str:
    h = hashlib.sha256("\0".join(SAN + [KEEP, CXX]).encode())
    files = sorted(glob.glob(os.path.join(HERE, "*")) + glob.glob(os.path.join(MIRROR_DIR, "*")) +
                   [ORACLE_SRC] + [os.path.join(CSRC, f) for f in ("shg_math.h", "shg_r2n_math.h", "boys_table.h")])
    for f in files:
        if os.path.isfile(f):
            h.update(os.path.relpath(f, ROOT).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\n{r.stderr[-3000:]}")


def build() -> dict:
    """Compile both drivers (unless the stamp matches); returns {"oracle": path, "mirror": path}."""
    os.makedirs(OUT, exist_ok=True)
    exes = {"oracle": os.path.join(OUT, "oracle_driver"), "mirror": os.path.join(OUT, "mirror_driver")}
    stamp = _stamp()
    stamp_path = os.path.join(OUT, "stamp")
    if all(os.path.exists(e) for e in exes.values()) and os.path.exists(stamp_path):
        with open(stamp_path) as fh:
            if fh.read().strip() == stamp:
                return exes
    srcs = [os.path.join(MIRROR_DIR, f) for f in MIRROR_SRCS] + [os.path.join(HERE, "mirror_driver.cpp")]

    def cc(src):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        _run([CXX, *SAN, KEEP, "-std=c++17", "-I", HERE, "-c", src, "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(min(len(srcs) + 1, 8)) as ex:
        fut_oracle = ex.submit(_run, ["gcc", *SAN, "-fopenmp", "-Wall", "-I", HERE, ORACLE_SRC,
                                      os.path.join(HERE, "oracle_driver.c"), "-o", exes["oracle"], "-lm"])
        objs = list(ex.map(cc, srcs))
        fut_oracle.result()
    _run([CXX, *SAN, "-o", exes["mirror"], *objs])
    with open(stamp_path, "w") as fh:
        fh.write(stamp + "\n")
    return exes


if __name__ == "__main__":
    print(build())
