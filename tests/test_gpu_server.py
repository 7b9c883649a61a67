"""GPU tests of the serving loop (C server through the C ABI): results in a mix of
concurrent requests, and in sweeps that merge waiting requests as snapshots, equal the same
requests run alone; admission under a tight budget."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from gen.netlist import CFG0, heap_trees, jitter, make_design, scaled_spec
from oracle import sta_oracle as O
from paper_2603_28381_amd import Graph, Server, StaError
from paper_2603_28381_amd import sta as S

pytestmark = pytest.mark.gpu

GAMMA = 10.0


def _designs():
    # the last design carries an RC tree per net (served like the star designs)
    ds = [make_design(CFG0), make_design(scaled_spec(20_000, cfg_id=46, box_um=700.0)),
          make_design(scaled_spec(5_000, cfg_id=47, box_um=300.0)),
          heap_trees(make_design(scaled_spec(8_000, cfg_id=58, box_um=400.0)))]
    gs = []
    for d in ds:
        g = Graph.from_design(d)
        g.levelize()
        gs.append(g)
    return ds, gs


def _requests(ds, n=36):
    rng = np.random.default_rng(7)
    reqs = []
    for i in range(n):
        k = int(rng.integers(len(ds)))
        grad = bool(rng.random() < 0.4)
        xy = jitter(ds[k], 2.0, stream=100 + i) if rng.random() < 0.5 else None
        reqs.append((k, grad, xy))
    return reqs


def _alone(g, d, grad, xy):
    x = torch.tensor(d.x if xy is None else xy[0], device="cuda")
    y = torch.tensor(d.y if xy is None else xy[1], device="cuda")
    f = g.forward(x, y, gamma=GAMMA)
    res = {}
    if grad:
        o = g.backward(x, y, f, rat=False, grad=True, pins=False)
        res["dx"], res["dy"] = o["dx"].cpu().numpy(), o["dy"].cpu().numpy()
    torch.cuda.synchronize()
    res["scalars"] = f.scalars.cpu().numpy()
    return res


def _serve(ds, gs, reqs, budget, slots=4, merge=8):
    srv = Server(budget, max_slots=slots, max_merge=merge)
    ids = [srv.add_design(g, d.x, d.y) for g, d in zip(gs, ds)]
    tickets = []
    for k, grad, xy in reqs:
        tickets.append(srv.submit(ids[k], grad=grad, x=None if xy is None else xy[0],
                                  y=None if xy is None else xy[1], gamma=GAMMA))
    out = [srv.wait(t) for t in tickets]
    srv.close()
    return out


def _same(a, b):
    assert np.array_equal(a["scalars"], b["scalars"])
    assert ("dx" in a) == ("dx" in b)
    if "dx" in a:
        assert np.array_equal(a["dx"], b["dx"]) and np.array_equal(a["dy"], b["dy"])


@pytest.mark.parametrize("merge", [1, 8])
def test_served_mix_equals_requests_run_alone(merge):
    ds, gs = _designs()
    reqs = _requests(ds)
    served = _serve(ds, gs, reqs, budget=8 << 30, slots=4, merge=merge)
    lat = np.array([r["latency_ms"] for r in served])
    print(f"latency p50 {np.percentile(lat, 50):.3f} ms, p99 {np.percentile(lat, 99):.3f} ms")
    for (k, grad, xy), r in zip(reqs, served):
        _same(r, _alone(gs[k], ds[k], grad, xy))
    # One served gradient against the FP64 oracle.
    i = next(i for i, (k, grad, xy) in enumerate(reqs) if k == 0 and grad and xy is None)
    ref = O.run(ds[0], gamma=GAMMA, grad="tns")
    assert served[i]["scalars"][3] == pytest.approx(ref["tns_g"], rel=1e-4, abs=1e-3)
    g, r = served[i]["dx"].astype(np.float64), ref["dx"]
    assert np.all(np.abs(g - r) <= 1e-3 * np.abs(r) + 1e-6 * np.abs(r).max())


def _need(g, grad, new_xy):
    a = lambda v: (v + 255) // 256 * 256
    info = g.info()
    P = info["n_pins"]
    b = a(info["fwd_state_bytes"]) + a(32)
    if grad:
        b += a(info["bwd_workspace_bytes"]) + 2 * a(4 * P)
    if new_xy:
        b += 2 * a(4 * P)
    return b


def test_tight_budget_queues_and_keeps_results():
    ds, gs = _designs()
    reqs = _requests(ds, n=16)
    wide = _serve(ds, gs, reqs, budget=8 << 30, slots=4)
    for g in gs:
        g.upload()
    resident = sum(g.info()["device_bytes"] + 8 * g.info()["n_pins"] for g in gs)
    one = max(_need(gs[k], grad, xy is not None) for k, grad, xy in reqs)
    narrow = _serve(ds, gs, reqs, budget=resident + one, slots=4)   # one request at a time
    for a, b in zip(wide, narrow):
        _same(a, b)
    assert max(r["queue_ms"] for r in narrow) > 0.0
    # A request that can never fit, and a design that does not fit.
    srv = Server(resident + 1024, max_slots=2)
    ids = [srv.add_design(g, d.x, d.y) for g, d in zip(gs, ds)]
    with pytest.raises(StaError) as e:
        srv.submit(ids[0], grad=True)
    assert e.value.code == S.STA_E_NOMEM
    with pytest.raises(StaError) as e:
        srv.add_design(gs[0], ds[0].x, ds[0].y)
    assert e.value.code == S.STA_E_NOMEM
    srv.close()


def test_ticket_errors_and_full_queue():
    d = make_design(scaled_spec(200_000, cfg_id=48, box_um=1500.0))
    g = Graph.from_design(d)
    g.levelize()
    srv = Server(8 << 30, max_slots=1, queue_capacity=1)
    i = srv.add_design(g, d.x, d.y)
    with pytest.raises(StaError) as e:
        srv.poll(12345)
    assert e.value.code == S.STA_E_UNKNOWN_TICKET
    tickets, busy = [], 0
    for _ in range(5):
        try:
            tickets.append(srv.submit(i, grad=True))
        except StaError as err:
            assert err.code == S.STA_E_BUSY
            busy += 1
    assert busy >= 1
    res = [srv.wait(t) for t in tickets]
    for r in res[1:]:
        _same(r, res[0])
    with pytest.raises(StaError) as e:
        srv.release(tickets[0])
    assert e.value.code == S.STA_E_UNKNOWN_TICKET
    with pytest.raises(StaError):
        srv.submit(i, grad=False, gamma=-1.0)
    srv.close()


def test_waiting_requests_merge_into_snapshot_sweeps():
    # One slot: while the first request captures and runs, the others wait, and the scheduler
    # sweeps waiting requests of one kind and gamma together as snapshots (2, 4 or 8), new and
    # resident coordinates mixed.  A design under the thread-per-net schedule always runs alone.
    d = make_design(scaled_spec(30_000, cfg_id=49, box_um=800.0))
    g = Graph.from_design(d)
    g.levelize()
    t = Graph.from_design(d)
    t.levelize()
    t.set_schedule(2, 2, 64, level_scheme="thread")
    rng = np.random.default_rng(11)
    reqs = []
    for i in range(23):
        xy = jitter(d, 2.0, stream=300 + i) if rng.random() < 0.5 else None
        reqs.append((i % 7 == 3, bool(rng.random() < 0.5), xy, 10.0 if i % 5 else 20.0))
    srv = Server(8 << 30, max_slots=1, max_merge=8)
    ids = [srv.add_design(g, d.x, d.y), srv.add_design(t, d.x, d.y)]
    tickets = [srv.submit(ids[int(th)], grad=grad, x=None if xy is None else xy[0],
                          y=None if xy is None else xy[1], gamma=gm) for th, grad, xy, gm in reqs]
    out = [srv.wait(q) for q in tickets]
    st = srv.stats()
    srv.set_max_merge(1)                     # from now on each request alone
    more = [srv.submit(ids[0], grad=False) for _ in range(8)]
    again = [srv.wait(q) for q in more]
    st2 = srv.stats()
    srv.close()
    print(st, st2)
    assert st["completed"] == len(reqs) and st["merged"] >= 4 and st["sweeps"] < len(reqs)
    assert st2["merged"] == st["merged"] and st2["sweeps"] == st["sweeps"] + 8
    for r in again[1:]:
        _same(r, again[0])
    for (th, grad, xy, gm), r in zip(reqs, out):
        h = t if th else g
        x = torch.tensor(d.x if xy is None else xy[0], device="cuda")
        y = torch.tensor(d.y if xy is None else xy[1], device="cuda")
        f = h.forward(x, y, gamma=gm)
        ref = {"scalars": None}
        if grad:
            o = h.backward(x, y, f, rat=False, grad=True, pins=False)
            ref["dx"], ref["dy"] = o["dx"].cpu().numpy(), o["dy"].cpu().numpy()
        torch.cuda.synchronize()
        ref["scalars"] = f.scalars.cpu().numpy()
        _same(r, ref)


def test_concurrent_clients_get_their_own_results():
    # Four client threads submit and wait at once (mixed kinds, new and resident coordinates,
    # merging on); every result equals the same request run alone.
    import threading
    ds, gs = _designs()
    reqs = _requests(ds, n=48)
    srv = Server(8 << 30, max_slots=4, max_merge=8)
    ids = [srv.add_design(g, d.x, d.y) for g, d in zip(gs, ds)]
    out = [None] * len(reqs)
    errors = []

    def client(part):
        try:
            mine = []
            for i in part:
                k, grad, xy = reqs[i]
                mine.append((i, srv.submit(ids[k], grad=grad, x=None if xy is None else xy[0],
                                           y=None if xy is None else xy[1], gamma=GAMMA)))
            for i, t in mine:
                out[i] = srv.wait(t)
        except Exception as e:                  # reported below, on the test's thread
            errors.append(e)

    threads = [threading.Thread(target=client, args=(range(c, len(reqs), 4),)) for c in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    st = srv.stats()
    srv.close()
    assert not errors, errors
    assert st["completed"] == len(reqs)
    for (k, grad, xy), r in zip(reqs, out):
        _same(r, _alone(gs[k], ds[k], grad, xy))
