"""GPU parity of the RC-tree path (pin_parent given): the tree passes and their adjoint against
the FP64 oracle, and the tree form of a star against the star kernels."""
from __future__ import annotations

from dataclasses import replace

import numpy as np
import pytest
import torch

from gen.netlist import heap_trees, make_design, scaled_spec
from oracle import sta_oracle as O
from paper_2603_28381_amd import Graph
from tests._designs import fanout_design
from tests.test_gpu_parity import GAMMA, check_grad, check_values, gpu_run

pytestmark = pytest.mark.gpu


def test_tree_design_matches_oracle():
    d = heap_trees(make_design(scaled_spec(40_000, cfg_id=71, box_um=600.0)))
    ref = O.run(d, gamma=GAMMA, grad="tns")
    got = gpu_run(d)
    check_values(d, got, ref)
    check_grad(got, ref, 1e-3, 1e-6)
    # the canonical pin order gives the same bits, permuted
    can = gpu_run(d, canonical=True)
    perm = got["graph"].levelization()["pin_perm"]
    for k in ("at", "slew", "rat", "slack", "dx", "dy", "atg"):
        assert np.array_equal(got[k][perm], can[k], equal_nan=True), k


def test_tree_wns_gradient_and_deep_chains():
    # Chains (each sink hangs off the previous one in net order) give trees as deep as the net.
    d = make_design(scaled_spec(20_000, cfg_id=72, box_um=400.0))
    pp = np.full(d.n_pins, -1, np.int32)
    for n in range(d.n_nets):
        pins = d.net_pins[d.net_offsets[n]:d.net_offsets[n + 1]]
        pp[pins[1:]] = pins[:-1]
    d = replace(d, pin_parent=pp)
    assert np.diff(d.net_offsets).max() > 100
    ref = O.run(d, gamma=GAMMA, grad="wns")
    got = gpu_run(d, wns=True)
    check_values(d, got, ref)
    check_grad(got, ref, 1e-3, 1e-6)


def test_star_given_as_tree_matches_star_kernels():
    d = make_design(scaled_spec(30_000, cfg_id=73, box_um=500.0))
    lv = O.levelize(d)
    drv = lv.driver[lv.net_of_pin]
    t = replace(d, pin_parent=np.where(drv == np.arange(d.n_pins), -1, drv).astype(np.int32))
    a = gpu_run(d)
    b = gpu_run(t)
    for k in ("at", "slew", "rat", "slack", "scalars"):
        x, y = a[k], b[k]
        fin = np.isfinite(x)
        assert np.array_equal(fin, np.isfinite(y)), k
        assert np.allclose(x[fin], y[fin], rtol=1e-5, atol=1e-3), k
    # gradients: rounding order differs (fused star adjoint vs the tree passes)
    check_grad(b, {"dx": a["dx"].astype(np.float64), "dy": a["dy"].astype(np.float64)}, 1e-3, 1e-6)


def test_tree_batch_checkpointing_and_snapshots_bitwise():
    # A tree design batched with a star design, swept plain, checkpointed and as two snapshots:
    # every form gives the same bits.
    a = heap_trees(make_design(scaled_spec(15_000, cfg_id=74, box_um=300.0)))
    b = make_design(scaled_spec(6_000, cfg_id=75, box_um=200.0))
    g = Graph.batch([Graph.from_design(a), Graph.from_design(b)])
    g.levelize()
    x = torch.tensor(np.concatenate([a.x, b.x]), device="cuda")
    y = torch.tensor(np.concatenate([a.y, b.y]), device="cuda")

    def run():
        f = g.forward(x, y, gamma=GAMMA)
        o = g.backward(x, y, f, rat=True, grad=True, pins=True)
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in o.items()}
        res["scalars"] = f.scalars.cpu().numpy()
        return res
    plain = run()
    g.set_checkpointing(-1)
    ck = run()
    g.set_checkpointing(0)
    for k in plain:
        assert np.array_equal(plain[k], ck[k], equal_nan=True), k
    g.set_snapshots(2)
    x2, y2 = torch.stack([x, x + 1.0]), torch.stack([y, y])
    f = g.forward(x2, y2, gamma=GAMMA)
    o = g.backward(x2, y2, f, rat=True, grad=True, pins=True)
    torch.cuda.synchronize()
    for k in ("at", "rat", "dx", "dy"):
        assert np.array_equal(o[k][0].cpu().numpy(), plain[k], equal_nan=True), k
    g.set_snapshots(1)
    shifted = {k: v for k, v in zip(("x", "y"), (x + 1.0, y))}
    f1 = g.forward(shifted["x"], shifted["y"], gamma=GAMMA)
    o1 = g.backward(shifted["x"], shifted["y"], f1, rat=True, grad=True, pins=True)
    torch.cuda.synchronize()
    for k in ("at", "rat", "dx", "dy"):
        assert np.array_equal(o[k][1].cpu().numpy(), o1[k].cpu().numpy(), equal_nan=True), k
    # the tree member of the batch (the union's first pins, in its own order) against the oracle
    ref = O.run(a, gamma=GAMMA, grad="tns")
    P_a = a.n_pins
    fin = np.isfinite(ref["at"])
    assert np.allclose(plain["at"][:P_a][fin], ref["at"][fin], rtol=1e-4, atol=1e-3)
    check_grad({"dx": plain["dx"][:P_a], "dy": plain["dy"][:P_a]}, ref, 1e-3, 1e-6)


def test_tree_net_over_one_chunk_uses_the_fallback_kernels():
    d = heap_trees(fanout_design())
    assert np.diff(d.net_offsets).max() > 1024
    ref = O.run(d, gamma=GAMMA, grad="tns")
    got = gpu_run(d)
    check_values(d, got, ref)
    check_grad(got, ref, 1e-3, 1e-6)
