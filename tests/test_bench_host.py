"""Host logic of bench.py's traffic bookkeeping: the kernel-source hash that
decides whether committed counter summaries still describe the timed kernel
ignores comments, follows code and the tuning-table entries of the
workload's dimensionality, and gates the reported traffic."""
import json
import os
import shutil

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _copy_tree(tmp):
    for sub in ("paper_1807_06507_amd/csrc", "include"):
        shutil.copytree(os.path.join(ROOT, sub), os.path.join(tmp, sub))
    shutil.copy(os.path.join(ROOT, "paper_1807_06507_amd", "tune_table.txt"),
                os.path.join(tmp, "paper_1807_06507_amd", "tune_table.txt"))
    os.makedirs(os.path.join(tmp, "profiles"))


def test_hash_follows_code_not_comments(tmp_path, monkeypatch):
    tmp = str(tmp_path)
    _copy_tree(tmp)
    monkeypatch.setattr(bench, "ROOT", tmp)
    h1, h4b = bench._kernel_source_hash("c1"), bench._kernel_source_hash("c4b")
    src = os.path.join(tmp, "paper_1807_06507_amd", "csrc", "swc_corr2d_fast.hpp")
    with open(src, "a") as f:
        f.write("\n// a remark\n/* a block\n   remark */\n")
    assert bench._kernel_source_hash("c1") == h1
    with open(src, "a") as f:
        f.write("static int swc_unused_probe_value = 1;\n")
    h1b = bench._kernel_source_hash("c1")
    assert h1b != h1
    # the 1-D kernel does not include the 2-D header
    assert bench._kernel_source_hash("c4b") == h4b
    # a tuning line of another dimensionality leaves the 2-D hash alone
    tt = os.path.join(tmp, "paper_1807_06507_amd", "tune_table.txt")
    with open(tt, "a") as f:
        f.write("2 1 0 63 8 32 1 0\n")
    assert bench._kernel_source_hash("c1") == h1b
    assert bench._kernel_source_hash("c4b") != h4b
    with open(tt, "a") as f:
        f.write("2 2 0 63 4 0 2 0\n")
    assert bench._kernel_source_hash("c1") != h1b


def test_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    tmp = str(tmp_path)
    _copy_tree(tmp)
    monkeypatch.setattr(bench, "ROOT", tmp)
    h = bench._kernel_source_hash("c1")
    assert bench._traffic_from_profiles(h, "c1") is None          # no summary
    with open(os.path.join(tmp, "profiles", "c1_pmc.json"), "w") as f:
        json.dump({"kernel_source_hash": h, "hbm_bytes_per_launch": 1234.0}, f)
    assert bench._traffic_from_profiles(h, "c1") == 1234.0
    assert bench._traffic_from_profiles("0" * 16, "c1") is None   # stale summary
