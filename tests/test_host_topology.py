"""Host logic without a GPU: the block-sparse pattern, the element -> slot maps
and the sliced-ELL positions built by csrc/topology.cpp, checked against brute
force on 300 random meshes (including out-of-range and repeated vertex
indices and vertices outside every tetrahedron, which must be refused) by
tests/host/topology_check.cpp, compiled with g++ and run under
AddressSanitizer and UndefinedBehaviorSanitizer when the toolchain has them;
the same program checks that the PCG product's panel order of workgroups
(csrc/wg_order.h) is a bijection of every chunk size and panel length."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2505_21013_amd", "csrc")


def _build(tmp_path, flags):
    exe = str(tmp_path / "topology_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", *flags, "-I", CSRC,
           os.path.join(HERE, "host", "topology_check.cpp"), os.path.join(CSRC, "topology.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return exe if r.returncode == 0 else None


def test_topology_against_brute_force(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    exe = _build(tmp_path, ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"])
    if exe is None:  # no sanitizer runtime: plain build
        exe = _build(tmp_path, [])
    assert exe is not None, "topology_check did not compile"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "ok (0 failures)" in r.stdout
