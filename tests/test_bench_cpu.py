"""Host logic of bench.py: which launch a class's quartets run in, and the lookup of the
committed HBM-traffic lines (no GPU needed)."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import bench  # noqa: E402


def _stats(n, n32, not_split):
    cv = [0] * 21
    cv[1] = (3 if not_split else 0) | (4 << 3) | (64 if not_split else 0)
    q = [0] * 21
    q32 = [0] * 21
    q[1], q32[1] = n, n32
    return {"class_quartets": q, "class_fp32_quartets": q32, "class_variant": cv}


def test_launch_quartets_split_and_merged():
    # split class: the FP64 launch holds the FP64-routed quartets, the FP32 launch the rest
    st = _stats(1000, 300, not_split=False)
    assert bench.launch_quartets(st, 1, "fp64") == 700
    assert bench.launch_quartets(st, 1, "fp32") == 300
    # kept in FP64: one launch of all quartets (the statistics then report no FP32 quartets)
    st = _stats(1000, 0, not_split=True)
    assert bench.launch_quartets(st, 1, "fp64") == 1000
    assert bench.launch_quartets(st, 1, "fp32") == 0


def test_traffic_lookup_needs_matching_sources_and_launch(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    sha = bench._sources_sha()
    (prof / "k_test_hbm_traffic.txt").write_text(
        "# header\n"
        f"traffic 1000 3 fp64 {sha} 1000 24 1583444    # kernel\n"
        f"traffic 1000 0 fp64 0000000000000000 5 5 1583444    # other sources\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "_sources_sha", lambda: sha)
    assert bench._traffic((1, 0, 0, 0), 3, "fp64", 1583444) == 1024
    assert bench._traffic((1, 0, 0, 0), 3, "fp64", 1583443) is None   # another launch size
    assert bench._traffic((1, 0, 0, 0), 0, "fp64", 1583444) is None   # other kernel sources
    assert bench._traffic((1, 0, 0, 0), 3, "fp32", 1583444) is None


def test_committed_traffic_lines_are_well_formed():
    import glob
    lines = []
    for path in glob.glob(os.path.join(os.path.dirname(HERE), "profiles", "*_hbm_traffic.txt")):
        lines += [l.split() for l in open(path) if l.startswith("traffic ")]
    assert lines
    for f in lines:
        assert len(f) >= 8 and len(f[1]) == 4 and f[2] in "01234" and f[3] in ("fp64", "fp32")
        assert len(f[4]) == 16 and all(int(x) >= 0 for x in f[5:8])
