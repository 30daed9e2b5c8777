"""The engine build cannot mix objects of two source states: a build holds an
exclusive lock on the build folder, and an object is reused only when its
stamp (flags + source + every local header it includes) matches."""
import fcntl
import os
import subprocess
import sys
import textwrap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_stamp_follows_included_headers(tmp_path):
    from paper_1701_06588_amd import build
    (tmp_path / "inner.h").write_text("#define X 1\n")
    (tmp_path / "outer.h").write_text('#include "inner.h"\n')
    src = tmp_path / "k.hip"
    src.write_text('#include "outer.h"\nint f() { return X; }\n')
    s0 = build.source_stamp(str(src))
    assert build.source_stamp(str(src)) == s0
    (tmp_path / "inner.h").write_text("#define X 2\n")        # a header two levels down
    s1 = build.source_stamp(str(src))
    assert s1 != s0
    assert build.source_stamp(str(src), flags=["-O2"]) != s1    # and the flags


def test_build_lock_is_exclusive(tmp_path):
    from paper_1701_06588_amd import build
    lock = tmp_path / ".lock"
    probe = textwrap.dedent(f"""
        import fcntl, sys
        fh = open({str(lock)!r}, "w")
        try:
            fcntl.flock(fh, fcntl.LOCK_EX | fcntl.LOCK_NB)
        except BlockingIOError:
            sys.exit(3)
        sys.exit(0)
    """)
    with build.build_lock(str(tmp_path)):
        assert subprocess.run([sys.executable, "-c", probe]).returncode == 3
    assert subprocess.run([sys.executable, "-c", probe]).returncode == 0


def test_every_object_has_a_current_stamp():
    """After a build, every object's stamp matches its sources (skipped when nothing is built)."""
    from paper_1701_06588_amd import build
    import glob
    import pytest
    srcs = glob.glob(os.path.join(build.CSRC, "*.hip"))
    objs = [os.path.join(build.BUILD, os.path.basename(s).replace(".hip", ".o")) for s in srcs]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("library not built in this tree")
    for s, o in zip(srcs, objs):
        with open(o + ".stamp") as fh:
            assert fh.read().strip() == build.source_stamp(s), s
