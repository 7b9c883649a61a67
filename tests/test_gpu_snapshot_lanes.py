"""Placement snapshots with the snapshot innermost (STA_SNAP_INNER: the lanes of a wave take
snapshots) against the FP64 oracle, and against the snapshots-outermost sweep."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from gen.netlist import CFG0, jitter, make_design, scaled_spec
from oracle import sta_oracle as O
from paper_2603_28381_amd import Graph
from paper_2603_28381_amd.sta import StaError
from tests._parity import assert_times
from tests.test_gpu_parity import GAMMA, check_grad, check_values

pytestmark = pytest.mark.gpu


def _snapshots(d, S, sigma=5.0):
    snaps = [(d.x, d.y)] + [jitter(d, sigma, stream=s) for s in range(1, S)]
    return [(np.asarray(a, np.float32), np.asarray(b, np.float32)) for a, b in snaps]


def _run(d, snaps, inner, canonical=False, wns=False, capture=False, lane_block=512):
    """Forward + backward of all snapshots in one call; returns per-snapshot numpy outputs
    (original pin order)."""
    S = len(snaps)
    g = Graph.from_design(d)
    g.levelize()
    g.set_schedule(2, 2, 64, lane_block=lane_block)
    g.set_snapshots(S)
    g.set_snapshot_layout(inner)
    perm = g.levelization()["pin_perm"]
    xs = np.stack([sx[perm] if canonical else sx for sx, _ in snaps])
    ys = np.stack([sy[perm] if canonical else sy for _, sy in snaps])
    if inner:
        xs, ys = xs.T.copy(), ys.T.copy()
    x = torch.tensor(xs, device="cuda")
    y = torch.tensor(ys, device="cuda")
    outs = []
    for _ in range(2 if capture else 1):     # a captured call replays its graph the second time
        f = g.forward(x, y, gamma=GAMMA, pins=True, canonical=canonical, capture=capture)
        o = g.backward(x, y, f, rat=True, grad=True, wns=wns, pins=True, capture=capture)
        torch.cuda.synchronize()
        outs.append((f, o))
    f, o = outs[-1]
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    res = []
    for s in range(S):
        r = {}
        for k, v in list(o.items()) + [("fwd_at", f.at), ("fwd_slew", f.slew), ("atg", f.atg)]:
            a = v.cpu().numpy()
            a = a[:, s] if inner else a[s]
            r[k] = a[inv] if canonical else a
        r["scalars"] = f.scalars[s].cpu().numpy()
        res.append(r)
    if capture:
        for k in ("dx", "rat", "slack"):
            assert torch.equal(outs[0][1][k], outs[1][1][k]), k
    return res


def _check_snapshots(d, snaps, got, picks, wns=False):
    for s in picks:
        ref = O.run(d, x=snaps[s][0], y=snaps[s][1], gamma=GAMMA, grad="wns" if wns else "tns")
        check_values(d, got[s], ref)
        check_grad(got[s], ref, 1e-3, 1e-6)


@pytest.mark.parametrize("S,canonical,lane_block", [(64, True, 512), (80, False, 1024), (3, True, 256)])
def test_snapshot_lanes_match_oracle_and_outer_layout(S, canonical, lane_block):
    # Heavy-tailed nets (every lane-group class and nets over 12 sinks in the workgroup path),
    # 64 snapshots (one wave per item), 80 (two blocks of snapshots), 3 (16 items per wave),
    # backward workgroups of 512, 1024 and 256 threads.
    d = make_design(scaled_spec(30_000, cfg_id=42, box_um=500.0))
    assert np.diff(d.net_offsets).max() - 1 > 128
    snaps = _snapshots(d, S)
    got = _run(d, snaps, inner=True, canonical=canonical, lane_block=lane_block)
    _check_snapshots(d, snaps, got, sorted({0, S // 2, S - 1}))
    outer = _run(d, snaps, inner=False, canonical=canonical)
    for s in range(S):
        for k in ("at", "slew", "rat", "slack", "atg"):
            assert_times(got[s][k], outer[s][k], f"snapshot {s} {k}")
        for k in ("dx", "dy"):
            r = outer[s][k].astype(np.float64)
            assert np.all(np.abs(got[s][k] - r) <= 1e-4 * np.abs(r) + 1e-6 * np.abs(r).max()), (s, k)
        assert np.allclose(got[s]["scalars"], outer[s]["scalars"], rtol=1e-5, atol=1e-3), s


def test_snapshot_lanes_wide_cells_wns_and_capture():
    # Cells of 5-8 inputs (the second chunk of arcs) with the WNS_g gradient, 8 snapshots
    # (8 items of 8 lanes per wave), replayed from a captured hipGraph.
    from tests._designs import wide_dag
    d = wide_dag(n_levels=9, gates_per_level=60, n_pi=16, seed=3)
    snaps = _snapshots(d, 8, sigma=3.0)
    got = _run(d, snaps, inner=True, wns=True, capture=True)
    _check_snapshots(d, snaps, got, [0, 7], wns=True)


def test_snapshot_lanes_star_net_over_512_sinks():
    # A 1300-sink net driven by a cell: the workgroup path with 5 snapshots (8 lanes each),
    # the threads of a backward workgroup (64 per snapshot) splitting the sinks.
    from tests._designs import fanout_design
    d = fanout_design(via_cell=True)
    snaps = _snapshots(d, 5, sigma=20.0)
    got = _run(d, snaps, inner=True)
    _check_snapshots(d, snaps, got, [0, 4])


def test_snapshot_layout_errors():
    d = make_design(CFG0)
    g = Graph.from_design(d)
    with pytest.raises(StaError):
        g.set_snapshot_layout(True)            # not levelized
    g.levelize()
    g.set_checkpointing(-1)
    with pytest.raises(StaError):
        g.set_snapshot_layout(True)            # checkpointing on
    g.set_checkpointing(0)
    g.set_snapshot_layout(True)
    with pytest.raises(StaError):
        g.set_checkpointing(-1)                # and the other way round
    from gen.netlist import heap_trees
    t = Graph.from_design(heap_trees(d))
    t.levelize()
    with pytest.raises(StaError):
        t.set_snapshot_layout(True)            # RC trees
