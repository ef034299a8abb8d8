"""Host-side pieces of bench.py, without a GPU: the algorithmic bytes of one
matrix product, and the counter traffic taken from the committed profile
summaries, which is reported only while the kernel source is the one the
counters were taken on (null once it changes)."""
import os
import shutil

import bench


def test_product_bytes_per_launch():
    # 64^3 compressed cube: N = 274,625 vertices, E = 1,872,064 edges,
    # NB = N + 2E = 4,018,753 blocks, 4,292 groups of 64 rows
    N, E = 274625, 1872064
    NB = N + 2 * E
    assert NB == 4018753
    assert bench.spmv_bytes(N, NB, False) == 8 * NB + 72 * (N + E) + 4 * 4292 + 96 * N
    assert bench.spmv_bytes(N, NB, True) == 8 * NB + 36 * (N + E) + 4 * 4292 + 96 * N
    assert round(bench.spmv_bytes(N, NB, False) / 1e6, 1) == 213.1


def test_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    """The counter traffic is read from a profile summary only while its
    recorded source hash equals the current kernel source's (a summary of the
    tree's form, written here, and the same with one byte of source changed)."""
    import hashlib
    root = tmp_path / "repo"
    (root / "profiles").mkdir(parents=True)
    (root / "paper_2505_21013_amd" / "csrc").mkdir(parents=True)
    src = open(os.path.join(bench.ROOT, "paper_2505_21013_amd", "csrc", "k_pcg.hip"), "rb").read()
    (root / "paper_2505_21013_amd" / "csrc" / "k_pcg.hip").write_bytes(src)
    sha = hashlib.sha256(src).hexdigest()[:16]
    for f, v in (("fp64", 345500000), ("mixed", 206000000)):
        (root / "profiles" / f"k_pcg_spmv_cube64_compress_ppn_{f}.md").write_text(
            f"kernel_source: paper_2505_21013_amd/csrc/k_pcg.hip sha256[:16] = {sha}\n"
            f"traffic_bytes_per_launch: {v}\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.measured_traffic(False) == 345500000 and bench.measured_traffic(True) == 206000000
    (root / "paper_2505_21013_amd" / "csrc" / "k_pcg.hip").write_bytes(src + b"\n")
    assert bench.measured_traffic(False) is None and bench.measured_traffic(True) is None


def test_committed_traffic_is_close_to_the_algorithmic_bytes():
    """When the committed summary was taken on the current kernel source, its
    traffic is within 20% above the algorithmic bytes (no wasted re-reads)."""
    fp64 = bench.measured_traffic(False)
    if fp64 is None:
        import pytest
        pytest.skip("the committed counter summary predates the current kernel source")
    assert 1.0 <= fp64 / bench.spmv_bytes(274625, 4018753, False) < 1.2
