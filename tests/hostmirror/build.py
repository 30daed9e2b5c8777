"""Build the test-only host mirror (tests/_build/libshg_hostmirror.so)."""
import concurrent.futures as cf
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT_DIR = os.path.join(ROOT, "tests", "_build")
LIB = os.path.join(OUT_DIR, "libshg_hostmirror.so")
# clang compiles these template-heavy sources several times faster than g++
CXX = "/opt/rocm/llvm/bin/clang++" if os.path.exists("/opt/rocm/llvm/bin/clang++") else "g++"
DEPS = [os.path.join(ROOT, "paper_1701_06588_amd", "csrc", f) for f in ("shg_math.h", "shg_r2n_math.h", "boys_table.h")]


def _stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    srcs = glob.glob(os.path.join(HERE, "*")) + DEPS
    return any(os.path.getmtime(s) > t for s in srcs)


def build(force: bool = False) -> str:
    if not force and not _stale():
        return LIB
    os.makedirs(OUT_DIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(HERE, "*.cpp")))

    def cc(src):
        obj = os.path.join(OUT_DIR, os.path.basename(src) + ".o")
        subprocess.run([CXX, "-O2", "-std=c++17", "-fPIC", "-c", src, "-o", obj], check=True)
        return obj
    with cf.ThreadPoolExecutor(min(len(srcs), 8)) as ex:
        objs = list(ex.map(cc, srcs))
    subprocess.run([CXX, "-shared", "-o", LIB + ".tmp", *objs], check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(force=True)
