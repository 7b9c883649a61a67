"""Host-side checks of bench.py (no GPU): the one-GPU contract and the byte model."""
from __future__ import annotations

import numpy as np

import bench
from gen.netlist import CFG0, make_design
from oracle import sta_oracle as O


def test_more_than_one_gpu_exits_with_message(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_every_workload_has_a_runner():
    for name in ("run_single", "run_batch", "run_serve", "run_fusion", "run_rc", "run_place", "checkpoint_comparison"):
        assert callable(getattr(bench, name))


def test_algorithmic_bytes_add_over_designs():
    # A union of two copies has exactly twice the per-level bytes of one copy.
    d = make_design(CFG0)
    lv = O.levelize(d).level
    one = bench.algorithmic_bytes(d, lv)
    L = int(lv.max()) + 1
    assert len(one["fwd_level"]) == L - 1 and len(one["bwd_level"]) == L
    assert all(np.all(v > 0) for k, v in one.items() if k != "fwd_level") and np.all(one["fwd_level"] >= 0)
    wider = bench.algorithmic_bytes(d, lv, n_levels=L + 3)
    assert len(wider["bwd_level"]) == L + 3 and np.all(wider["bwd_level"][:3] == 0)
    assert np.array_equal(wider["bwd_level"][3:], one["bwd_level"])


def test_traffic_is_reported_only_for_matching_kernel_sources(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    assert len(h) == 16
    prof = tmp_path / "profiles"
    prof.mkdir()
    f = prof / "sta_sweep_2p5Mpins_hbm_counters.md"
    f.write_text(f"x\ntraffic_bytes_per_launch k_bwd_level 1234 kernel_source {h}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    assert bench.counted_traffic("k_bwd_level") == 1234.0
    f.write_text("traffic_bytes_per_launch k_bwd_level 1234 kernel_source 0000000000000000\n")
    assert bench.counted_traffic("k_bwd_level") is None


def test_schedule_flags_reject_unsupported_values():
    import pytest
    for argv in (["--fwd-cell-lanes", "12"], ["--sweep-group-log2", "1"]):
        with pytest.raises(SystemExit):
            bench.main(argv)
    assert callable(bench.snapshot_graph_only)
