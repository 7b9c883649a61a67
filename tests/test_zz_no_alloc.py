"""sta_backward_noalloc (the backward sweep on the library's fixed device workspace) against
sta_backward on a workspace the caller allocates: two calls in a row, the second on a
smaller design, every output identical; plus the size limit and the argument checks."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from gen.netlist import CFG0, make_design, scaled_spec
from oracle import sta_oracle as O
from paper_2603_28381_amd import Graph
from paper_2603_28381_amd.sta import STA_E_NOMEM, STA_E_STATE, Forward, StaError
from tests._parity import assert_times

pytestmark = pytest.mark.gpu

GAMMA = 10.0
NOALLOC_BYTES = 96 << 20


def _both(d, wns):
    g = Graph.from_design(d)
    g.levelize()
    g.upload()
    x = torch.tensor(d.x, device="cuda")
    y = torch.tensor(d.y, device="cuda")
    fwd = g.forward(x, y, gamma=GAMMA)
    ref = g.backward(x, y, fwd, rat=True, grad=True, wns=wns, pins=True)
    torch.cuda.synchronize()
    ref = {k: v.cpu().numpy() for k, v in ref.items()}
    got = g.backward(x, y, fwd, rat=True, grad=True, wns=wns, pins=True, noalloc=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in got.items()}
    return g, ref, got


@pytest.mark.parametrize("wns", [False, True])
def test_noalloc_backward_equals_allocating_backward(wns):
    big = make_design(scaled_spec(60_000, cfg_id=71, box_um=400.0))
    small = make_design(CFG0)
    assert small.n_pins < big.n_pins
    for d in (big, small):          # the second call runs on a smaller input than the first
        print(f"noalloc backward: {d.spec.name} {d.n_pins} pins wns={wns}", flush=True)
        g, ref, got = _both(d, wns)
        assert g.info()["bwd_workspace_bytes"] <= NOALLOC_BYTES
        assert set(got) == set(ref)
        for k in ref:
            assert np.array_equal(got[k], ref[k], equal_nan=True), (d.n_pins, k)
    # the smaller design's results also meet the oracle
    o = O.run(small, gamma=GAMMA, grad="wns" if wns else "tns")
    assert_times(got["rat"], o["rat"], "RAT")
    for k in ("dx", "dy"):
        tol = 1e-3 * np.abs(o[k]) + 1e-6 * np.abs(o[k]).max()
        assert np.all(np.abs(got[k] - o[k]) <= tol), k


def test_noalloc_backward_limits_and_arguments():
    d = make_design(CFG0)
    g = Graph.from_design(d)
    g.levelize()
    x = torch.tensor(d.x, device="cuda")
    y = torch.tensor(d.y, device="cuda")
    fake = Forward(torch.empty(16, dtype=torch.uint8, device="cuda"), torch.empty(4, dtype=torch.float64,
                                                                                  device="cuda"))
    with pytest.raises(StaError) as e:        # not uploaded yet: uploading would allocate
        g.backward(x, y, fake, rat=True, grad=False, pins=False, noalloc=True)
    assert e.value.code == STA_E_STATE
    per_snap = g.info()["bwd_workspace_bytes"]
    n = NOALLOC_BYTES // per_snap + 1        # just past the array
    g.set_snapshots(n)
    g.upload()
    assert g.info()["bwd_workspace_bytes"] > NOALLOC_BYTES
    with pytest.raises(StaError) as e:
        g.backward(x, y, fake, rat=True, grad=False, pins=False, noalloc=True, out={})
    assert e.value.code == STA_E_NOMEM and "exceeds" in str(e.value)
    g.set_snapshots(1)
    g.upload()
    f = g.forward(x, y, gamma=GAMMA)
    with pytest.raises(ValueError):
        g.backward(x, y, f, noalloc=True, capture=True)
    # a gradient against a forward computed without smoothing is refused as by sta_backward
    f0 = g.forward(x, y, gamma=GAMMA, smooth=False)
    with pytest.raises(StaError) as e:
        g.backward(x, y, f0, rat=False, grad=True, pins=False, noalloc=True)
    assert e.value.code == STA_E_STATE
    torch.cuda.synchronize()
