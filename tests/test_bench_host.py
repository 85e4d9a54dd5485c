"""Host logic of bench.py (no GPU): the HBM traffic it reports comes from the
committed counter summary only while that summary matches the kernel source
and the block size it was taken at."""
import os
import shutil
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

SUMMARY = os.path.join("profiles", "gemm1_f16_grid64_v128c512_traffic.txt")
SOURCE = os.path.join("paper_2310_20103_amd", "csrc", "gemm_mfma.hip")


def _copy_tree(dst):
    for rel in (SUMMARY, SOURCE):
        os.makedirs(os.path.join(dst, os.path.dirname(rel)), exist_ok=True)
        shutil.copy(os.path.join(ROOT, rel), os.path.join(dst, rel))


def test_traffic_matches_committed_summary():
    import hashlib
    with open(os.path.join(ROOT, SUMMARY)) as f:
        kv = dict(ln.split(":", 1) for ln in f if ":" in ln and not ln.startswith(" "))
    with open(os.path.join(ROOT, SOURCE), "rb") as f:
        current = hashlib.sha256(f.read()).hexdigest() == kv["source_sha256"].strip()
    got = bench.measured_traffic("gemm1_f16", "grid64_v128c512", 128)
    if current:
        assert got == float(kv["hbm_bytes_per_launch"])
    else:
        assert got is None


def test_traffic_null_for_other_block_or_changed_source(tmp_path, monkeypatch):
    _copy_tree(str(tmp_path))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # make the copied summary match the copied source, whatever the tree holds
    import hashlib
    with open(os.path.join(str(tmp_path), SOURCE), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    path = os.path.join(str(tmp_path), SUMMARY)
    with open(path) as f:
        lines = [("source_sha256: " + sha + "\n") if ln.startswith("source_sha256:") else ln
                 for ln in f]
    with open(path, "w") as f:
        f.writelines(lines)
    assert bench.measured_traffic("gemm1_f16", "grid64_v128c512", 128) is not None
    assert bench.measured_traffic("gemm1_f16", "grid64_v128c512", 64) is None
    assert bench.measured_traffic("gemm1_f16", "grid32_v32c128", 128) is None
    with open(os.path.join(str(tmp_path), SOURCE), "a") as f:
        f.write("\n")
    assert bench.measured_traffic("gemm1_f16", "grid64_v128c512", 128) is None


def test_more_than_one_gpu_is_refused(monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err
