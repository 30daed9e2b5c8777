"""Build libshg.so (HIP for gfx950) in-tree.

Every ``csrc/*.hip`` file is compiled to an object in ``_build/`` (in parallel)
and linked into ``paper_1701_06588_amd/libshg.so``.

Two builds of one tree must never interleave (a library linked from objects of
two source states is the result), so a build holds an exclusive lock on
``_build/.lock`` from the first compile to the final rename. Each object has a
stamp: the sha256 of the compiler flags and the text of its source and of every
local header it includes. An incremental build recompiles an object whose stamp
differs; objects and the library are written under unique temporary names and
renamed into place, so a reader never sees a half-written file."""
import concurrent.futures as cf
import contextlib
import fcntl
import glob
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libshg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# packed FP32 instructions are kept out of every kernel: some of their forms have been
# seen to give wrong results silently
FLAGS = ["-O3", f"--offload-arch={ARCH}", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # GVN's memory-dependence analysis dominates the compile time of the large
         # straight-line tile kernels and changes nothing in their code (same VGPRs)
         "-mllvm", "-enable-gvn-memdep=false"]


def _deps(path: str, seen=None) -> set:
    """The file and every local header it includes, recursively."""
    seen = set() if seen is None else seen
    if path in seen or not os.path.exists(path):
        return seen
    seen.add(path)
    for line in open(path, errors="ignore"):
        line = line.strip()
        if line.startswith("#include") and '"' in line:
            inc = line.split('"')[1]
            _deps(os.path.normpath(os.path.join(os.path.dirname(path), inc)), seen)
    return seen


def source_stamp(src: str, flags=None) -> str:
    """sha256 over the flags and the bytes of `src` and its local headers."""
    h = hashlib.sha256()
    h.update("\0".join(FLAGS if flags is None else flags).encode())
    for f in sorted(_deps(src)):
        h.update(os.path.relpath(f, HERE).encode())
        h.update(b"\0")
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


@contextlib.contextmanager
def build_lock(build_dir: str = BUILD):
    """Exclusive lock on build_dir/.lock for the duration of the block."""
    os.makedirs(build_dir, exist_ok=True)
    with open(os.path.join(build_dir, ".lock"), "w") as fh:
        fcntl.flock(fh, fcntl.LOCK_EX)
        try:
            yield
        finally:
            fcntl.flock(fh, fcntl.LOCK_UN)


def _compile(src: str, verbose: bool, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
    stamp_path = obj + ".stamp"
    stamp = source_stamp(src)
    if incremental and os.path.exists(obj) and os.path.exists(stamp_path):
        with open(stamp_path) as fh:
            if fh.read().strip() == stamp:
                return obj
    tmp = f"{obj}.tmp{os.getpid():x}"
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        if os.path.exists(tmp):
            os.remove(tmp)
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
    warn = "\n".join(x for x in r.stderr.splitlines() if "packed-fp32-ops" not in x and x.strip())
    if warn and verbose:
        print(warn)
    os.replace(tmp, obj)
    with open(stamp_path + ".tmp", "w") as fh:
        fh.write(stamp + "\n")
    os.replace(stamp_path + ".tmp", stamp_path)
    return obj


def _weight(path: str) -> int:
    b = os.path.basename(path)
    if b.startswith("shg_tile_la") and "_lb" in b:
        la = int(b.split("_la")[1].split("_")[0])
        lb = int(b.split("_lb")[1].split(".")[0])
        return 1000 * (2 * la + 1) * (2 * lb + 1)
    return 50000 if b in ("shg_aab.hip", "shg_persist_d1.hip") else 0


def build(verbose: bool = False, jobs: int | None = None, incremental: bool = False) -> str:
    """Compile every source (always, unless `incremental`, which keeps objects
    whose stamp matches) and link libshg.so, under the build lock."""
    with build_lock():
        # longest compiles first so the pool stays busy
        srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")), key=lambda f: -os.path.getsize(f) - _weight(f))
        jobs = jobs or min(len(srcs), os.cpu_count() or 4, 16)
        with cf.ThreadPoolExecutor(jobs) as ex:
            objs = list(ex.map(lambda s: _compile(s, verbose, incremental), srcs))
        tmp = f"{LIB}.tmp{os.getpid():x}"
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv)
