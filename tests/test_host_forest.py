"""Host forest code built two ways from the library's own sources: the
default leaf lookup (a dense cell map for shallow forests, a hash for deep
ones) and the hash alone.  Both must give the same balance, regrid,
transfer plans, neighbour records and lookups, and every updated plan must
equal a fresh build."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1308_1472_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "host", "forest_check.cpp")


def _build(tmp, name, defines):
    exe = os.path.join(tmp, name)
    subprocess.run(["g++", "-O2", "-std=c++17", *defines, "-I", CSRC,
                    "-I", os.path.join(ROOT, "include"), SRC,
                    os.path.join(CSRC, "forest.cpp"), "-o", exe, "-lpthread"],
                   check=True)
    return exe


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_dense_and_hashed_lookups_agree(tmp_path):
    tmp = str(tmp_path)
    dense = _build(tmp, "dense", [])
    hashed = _build(tmp, "hash", ["-DFCX_DENSE_FACTOR=0"])
    runs = [subprocess.run(cmd, capture_output=True, text=True)
            for cmd in ([dense], [hashed])]
    for r in runs:
        assert r.returncode == 0, r.stdout + r.stderr
    outs = [r.stdout for r in runs]
    assert len(outs[0].splitlines()) == 60
    assert outs[0] == outs[1]
