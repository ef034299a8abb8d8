"""Host-side pieces of bench.py, without a GPU: the algorithmic bytes of one
matrix product, and the counter traffic taken from the committed profile
summaries, which is reported only while the kernel source is the one the
counters were taken on (null once it changes)."""
import os
import shutil

import bench


def test_product_bytes_per_launch():
    # 64^3 compressed cube: N = 274,625 vertices, NB = 4,018,753 blocks
    assert bench.spmv_bytes(274625, 4018753, False) == 76 * 4018753 + 4 * 274626 + 96 * 274625
    assert bench.spmv_bytes(274625, 4018753, True) == 40 * 4018753 + 4 * 274626 + 96 * 274625
    assert round(bench.spmv_bytes(274625, 4018753, False) / 1e6, 1) == 332.9


def test_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    fp64, fp32 = bench.measured_traffic(False), bench.measured_traffic(True)
    assert fp64 is not None and fp32 is not None
    assert 1.0 <= fp64 / bench.spmv_bytes(274625, 4018753, False) < 1.2
    # a copy of the tree whose kernel source differs by one byte: no traffic
    root = tmp_path / "repo"
    (root / "profiles").mkdir(parents=True)
    (root / "paper_2505_21013_amd" / "csrc").mkdir(parents=True)
    for f in ("k_pcg_spmv_cube64_compress_ppn_fp64.md", "k_pcg_spmv_cube64_compress_ppn_mixed.md"):
        shutil.copy(os.path.join(bench.ROOT, "profiles", f), root / "profiles" / f)
    src = open(os.path.join(bench.ROOT, "paper_2505_21013_amd", "csrc", "k_pcg.hip"), "rb").read()
    (root / "paper_2505_21013_amd" / "csrc" / "k_pcg.hip").write_bytes(src)
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.measured_traffic(False) == fp64
    (root / "paper_2505_21013_amd" / "csrc" / "k_pcg.hip").write_bytes(src + b"\n")
    assert bench.measured_traffic(False) is None and bench.measured_traffic(True) is None
