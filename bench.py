"""Benchmark of the levelized STA sweep on one MI355X.

One step = sta_forward (RC net delay, all forward levels with the LSE-smoothed late arrival,
endpoint WNS/TNS and their smoothed forms) + sta_backward (seeds, all backward levels with
required times, slack and the fused adjoint of the smoothed TNS), writing every per-pin
output: AT, slew, RAT, slack (4 conditions each) and d TNS_g / dx, dy.  Levelization and
the graph upload happen once, before timing (the netlist does not change between calls).

Default workload: a 2.5M-pin synthetic design (650k gates, 91 net levels, 6000 um box,
heavy-tailed nets up to 500 pins), inputs resident in HBM in the canonical pin order.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, 8 TB/s


def algorithmic_bytes(d, level: np.ndarray, n_levels: int | None = None, snapshots: int = 1) -> dict:
    """Bytes each kernel family must move per step (float32 values, int32 indices).

    `level` is the net level of every net of d; the per-level lists are indexed by level
    (fwd_level: levels 1..L-1; bwd_level: levels L-1..0, the launch order), so the lists of
    designs swept together in one batch add up element by element.  With `snapshots` S
    placements of d swept together, topology is counted once and every per-placement value
    S times.

    Counts only what the method reads and writes once; re-reads served by caches are not
    counted.  Per unit, as topology + per placement:
      rc         per net 12 (sched, offset, driver cap) + 12 (driver x, y, load write), +40
                 record write for level-0 nets; per sink 4 (cap) + 16 (x, y, wire write)
      fwd_level  per cell 12 (type, offset, arc base) + 44 (load, record write); per cell
                 input 9 (source net, pin, unateness) + 48 (wire, source record)
      ep_partial per endpoint 8 (pin, net) + 36 (late AT 8, smoothed AT 8, wire delay 4, its
                 smoothed slack and weights kept for the seeds 16)
      ep_seed    per endpoint 4 (pin) + 48 (kept values, required-time and adjoint seeds)
      bwd_level  per net 8 (sched, offset) + 40 (record, driver x, y); per cell 12 + 4 (load);
                 per cell input 9 + 64 (wire, source slew and smoothed AT, seed writes); per
                 sink 4 (cap) + 48 (RAT, adjoint, wire, x, y); per pin 72 output writes (AT,
                 slew, RAT, slack, dx, dy)
    """
    S = int(snapshots)
    N, P = d.n_nets, d.n_pins
    sinks = np.diff(d.net_offsets).astype(np.int64) - 1
    level = level.astype(np.int64)
    L = int(level.max()) + 1 if n_levels is None else n_levels
    drv = d.net_pins[d.net_offsets[:-1]]
    cell_of_out = np.full(P, -1, np.int64)
    cell_of_out[d.cell_out_pin] = np.arange(d.n_cells)
    cell = cell_of_out[drv]
    fanin = np.where(cell >= 0, np.diff(d.cell_in_offsets)[np.maximum(cell, 0)], 0).astype(np.int64)
    is_cell = (cell >= 0).astype(np.int64)
    nets_l = np.bincount(level, minlength=L)
    sinks_l = np.bincount(level, weights=sinks, minlength=L)
    cells_l = np.bincount(level, weights=is_cell, minlength=L)
    ins_l = np.bincount(level, weights=fanin, minlength=L)
    pins_l = nets_l + sinks_l
    E = int(np.count_nonzero((d.pin_kind == 3) | (d.pin_kind == 4)))
    n0 = int(nets_l[0])
    out = {}
    out["rc"] = np.array([float(N * (12 + 12 * S) + n0 * 40 * S + sinks.sum() * (4 + 16 * S))])
    out["fwd_level"] = np.array([float(cells_l[l] * (12 + 44 * S) + ins_l[l] * (9 + 48 * S)) for l in range(1, L)])
    out["ep_partial"] = np.array([float(E * (8 + 36 * S))])
    out["ep_seed"] = np.array([float(E * (4 + 48 * S))])
    out["bwd_level"] = np.array([float(nets_l[l] * (8 + 40 * S) + cells_l[l] * (12 + 4 * S) + ins_l[l] * (9 + 64 * S)
                                       + sinks_l[l] * (4 + 48 * S) + pins_l[l] * 72 * S)
                                 for l in range(L - 1, -1, -1)])
    return out


def whole_sweep_bytes(d) -> dict:
    """The per-step byte model of the sweep as a whole, written per pin (P pins, N nets,
    S = P - N sinks, C cells, A cell inputs; float32 values, int32 indices):
      forward   8P x,y + 4S cap + 4N offsets + 8C type and input offset + 4A input pin ids
                + 40A gathers (4 AT, 4 slew, 2 smoothed AT per cell input) + 40P writes of
                the same per pin + the library tables once
      backward  topology 4N + 8C + 4A, RC inputs again 8P + 4S, 40P state read, 16P RAT and
                16P slack writes, 32P adjoint scratch written and read, 8P dx, dy
    Unlike algorithmic_bytes it does not follow where the kernels actually move each value
    (here the per-pin AT and slew are written by the backward sweep)."""
    P, N, C = d.n_pins, d.n_nets, d.n_cells
    S, A = P - N, int(d.cell_in_offsets[-1])
    tables = int(d.lib.tables.size) * 4
    fwd = 8 * P + 4 * S + 4 * N + 8 * C + 4 * A + 40 * A + 40 * P + tables
    bwd = (4 * N + 8 * C + 4 * A) + (8 * P + 4 * S) + 40 * P + 16 * P + 16 * P + 32 * P + 8 * P
    return {"forward": float(fwd), "backward": float(bwd)}


def whole_sweep_roofline(d, kernels: dict, ms_step: float) -> dict:
    """Fractions of HBM peak under whole_sweep_bytes: the backward level kernel (the whole backward
    sweep's bytes over its summed launch time), the forward sweep (RC, levels, endpoint
    scalars) and the whole step."""
    b = whole_sweep_bytes(d)
    fwd_ms = sum(kernels[k]["ms_per_step"] for k in ("rc", "fwd_level", "ep_partial", "ep_final") if k in kernels)
    bl = kernels["bwd_level"]
    out = {"model": "whole_sweep_bytes (whole-sweep byte model per pin)",
           "bwd_level": {"bytes_per_launch": round(b["backward"] / bl["launches_per_step"], 1),
                         "avg_launch_us": round(bl["avg_us"], 3)},
           "forward_sweep": {"bytes": b["forward"], "ms": round(fwd_ms, 4)},
           "step": {"bytes": b["forward"] + b["backward"], "ms": round(ms_step, 4)}}
    gbs = b["backward"] / (bl["ms_per_step"] * 1e-3) / 1e9
    out["bwd_level"].update(achieved_gbs=round(gbs, 2), frac=round(gbs / HBM_PEAK_GBS, 5))
    for k in ("forward_sweep", "step"):
        gb = out[k]["bytes"] / (out[k]["ms"] * 1e-3) / 1e9
        out[k].update(achieved_gbs=round(gb, 2), frac=round(gb / HBM_PEAK_GBS, 5))
    return out


def cpu_host() -> dict:
    """The host CPU the oracle ran on: model name, logical CPUs, and those this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def time_oracle(d, gamma: float, threads: int, x=None, y=None) -> float:
    """Seconds of one FP64 oracle forward+backward+gradient of d (levelization excluded) on
    `threads` host threads (torch and BLAS pools limited to that)."""
    import torch
    from threadpoolctl import threadpool_limits
    from oracle import sta_oracle as O
    lv = O.levelize(d)
    plan = O._Plan(d, lv)
    prev = torch.get_num_threads()
    torch.set_num_threads(threads)
    try:
        with threadpool_limits(threads):
            c0 = time.perf_counter()
            O.run(d, x=x, y=y, gamma=gamma, grad="tns", lv=lv, plan=plan)
            return time.perf_counter() - c0
    finally:
        torch.set_num_threads(prev)


def kernel_source_hash() -> str:
    """First 16 hex digits of the SHA-256 of the kernel sources (kernels and their shared header)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("sta_kernels.hip", "sta_internal.h"):
        with open(os.path.join(ROOT, "paper_2603_28381_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counted_traffic(kernel: str, summary: str = "sta_sweep_2p5Mpins_hbm_counters.md") -> float | None:
    """HBM bytes per launch of `kernel` from a committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary (by default the 2.5M-pin sweep's), or None when the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    want = kernel_source_hash()
    with open(path) as fh:
        for line in fh:
            f = line.split()
            if len(f) == 5 and f[0] == "traffic_bytes_per_launch" and f[1] == kernel and f[3] == "kernel_source":
                return float(f[2]) if f[4] == want else None
    return None


def kernel_table(prof: dict, alg: dict, steps: int) -> tuple[dict, dict]:
    """Per-kernel launch statistics and the roofline entry of the dominant kernel."""
    kernels = {}
    for k, (n, tot) in prof.items():
        if n == 0:
            continue
        per_step = float(np.sum(alg.get(k, [0.0])))
        kernels[k] = dict(launches_per_step=n // steps, avg_us=1e3 * tot / n, ms_per_step=tot / steps,
                          alg_bytes_per_step=per_step,
                          gbs=(per_step * steps / (tot * 1e-3) / 1e9) if per_step else None)
    # the dominant kernel among those the byte model covers
    dom = max((k for k in kernels if kernels[k]["gbs"] is not None), key=lambda k: kernels[k]["ms_per_step"])
    kd = kernels[dom]
    achieved = kd["gbs"]
    roofline = dict(bound="hbm", kernel=dom, achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 5), traffic=None,
                    alg_bytes_per_launch=kd["alg_bytes_per_step"] / kd["launches_per_step"],
                    avg_launch_us=round(kd["avg_us"], 3))
    return kernels, roofline


def step_buffers(g, P, dev, n_designs=1, snaps=1):
    import torch
    lead = (snaps,) if snaps > 1 else ()
    state = g.new_state(dev)
    ws = g.new_workspace(dev)
    scal = torch.empty(lead + ((n_designs, 4) if n_designs > 1 else (4,)), dtype=torch.float64, device=dev)
    outs = {k: torch.empty(lead + (P, 4), dtype=torch.float32, device=dev) for k in ("at", "slew", "rat", "slack")}
    outs["dx"] = torch.empty(lead + (P,), dtype=torch.float32, device=dev)
    outs["dy"] = torch.empty(lead + (P,), dtype=torch.float32, device=dev)
    return state, ws, scal, outs


def launch_floor_us(dev, n: int, reps: int = 200) -> float:
    """Average time of back-to-back dependent launches of a trivial kernel (one float add per
    thread), replayed from a captured graph so that host-side dispatch does not pace them."""
    import torch
    t = torch.zeros(n, device=dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(3):
            t.add_(1.0)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(reps):
            t.add_(1.0)
    graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    return 1e3 * e0.elapsed_time(e1) / (3 * reps)


def timed(step, steps: int, warmup: int) -> tuple[float, float]:
    """(ms per step from events on the current stream, wall seconds)."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps, time.perf_counter() - w0


def run_batch(args) -> dict:
    """Batched sweep: 64 jittered placement snapshots of the 800k-pin design plus 16
    designs of 10k-400k pins (log-uniform), fwd+bwd with every output, three ways:
      shared     the 64 snapshots as one graph with 64 snapshots (one topology) on one
                 stream, the 16 designs as one batch graph on a second stream, both replayed
                 from captured hipGraphs (the reported value);
      union      one batch graph of all 80 members (64 copies of the topology), captured;
      plain      80 sequential plain call pairs, one member at a time."""
    import torch
    from gen.netlist import CFG1, batch_designs, jitter, make_design
    from paper_2603_28381_amd import Graph

    t0 = time.time()
    d1 = make_design(CFG1)
    others = batch_designs(16, 10_000, 400_000, cfg_id=3)
    snaps = [jitter(d1, 5.0, stream=s) for s in range(1, 65)]
    members = [(d1, sx, sy) for sx, sy in snaps] + [(d, d.x, d.y) for d in others]
    dev = torch.device("cuda")
    P = sum(m[0].n_pins for m in members)

    # shared: snapshots graph + batch of the 16 others
    g1 = Graph.from_design(d1)
    L1 = g1.levelize()
    perm1 = g1.levelization()["pin_perm"]
    g1.set_snapshots(64)
    inner = args.snapshot_layout == "inner"
    g1.set_snapshot_layout(inner)
    g1.upload()
    x1 = np.stack([sx[perm1] for sx, _ in snaps])
    y1 = np.stack([sy[perm1] for _, sy in snaps])
    if inner:                                   # snapshot innermost: [pin][snapshot]
        x1, y1 = np.ascontiguousarray(x1.T), np.ascontiguousarray(y1.T)
    x1 = torch.from_numpy(x1).to(dev)
    y1 = torch.from_numpy(y1).to(dev)
    u16 = Graph.batch([Graph.from_design(d) for d in others])
    L16 = u16.levelize()
    u16.upload()
    perm16 = u16.levelization()["pin_perm"]
    x16 = torch.from_numpy(np.concatenate([d.x for d in others])[perm16]).to(dev)
    y16 = torch.from_numpy(np.concatenate([d.y for d in others])[perm16]).to(dev)
    t_setup = time.time() - t0
    best1 = g1.tune(x1, y1, gamma=args.gamma, reps=2)
    if args.snapshots_only:
        return snapshot_graph_only(args, g1, d1, x1, y1, dev, best1, t_setup)
    best16 = u16.tune(x16, y16, gamma=args.gamma, reps=2)
    b1 = step_buffers(g1, d1.n_pins, dev, 1, 64)
    b16 = step_buffers(u16, u16.n_pins, dev, 16)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()

    def sweep(g, x, y, bufs, stream):
        state, ws, scal, outs = bufs
        cap = not args.no_batch_capture
        f = g.forward(x, y, gamma=args.gamma, canonical=True, state=state, scalars=scal, capture=cap, stream=stream)
        g.backward(x, y, f, rat=True, grad=True, workspace=ws, out=outs, capture=cap, stream=stream)

    def step_shared():
        cur = torch.cuda.current_stream()
        sa.wait_stream(cur)
        sb.wait_stream(cur)
        sweep(g1, x1, y1, b1, sa)
        sweep(u16, x16, y16, b16, sb)
        cur.wait_stream(sa)
        cur.wait_stream(sb)

    ms, wall = timed(step_shared, args.steps, args.warmup)
    value = P / (ms * 1e-3)

    ms_u = None
    if not getattr(args, "lean", False):
        # union: one batch graph of all 80 members
        gu = Graph.batch([Graph.from_design(d1)] * 64 + [Graph.from_design(d) for d in others])
        gu.levelize()
        gu.upload()
        dsg, pin = gu.batch_pin_map()
        base = np.cumsum([0] + [m[0].n_pins for m in members])
        src = base[dsg] + pin
        xu = torch.from_numpy(np.concatenate([m[1] for m in members])[src]).to(dev)
        yu = torch.from_numpy(np.concatenate([m[2] for m in members])[src]).to(dev)
        bu = step_buffers(gu, P, dev, 80)
        ms_u, _ = timed(lambda: sweep(gu, xu, yu, bu, None), max(1, args.steps // 2), 1)
        del bu, xu, yu
        gu.close()

    # plain: the same 80 sweeps as plain call pairs, each member in its own canonical order
    gp1 = Graph.from_design(d1)
    gp1.levelize()
    gp1.upload()
    plain = []
    bp1 = step_buffers(gp1, d1.n_pins, dev)
    for sx, sy in snaps:
        plain.append((gp1, torch.from_numpy(sx[perm1]).to(dev), torch.from_numpy(sy[perm1]).to(dev), bp1))
    for d in others:
        g = Graph.from_design(d)
        g.levelize()
        g.upload()
        pm = g.levelization()["pin_perm"]
        plain.append((g, torch.from_numpy(d.x[pm]).to(dev), torch.from_numpy(d.y[pm]).to(dev),
                      step_buffers(g, d.n_pins, dev)))

    def seq_step():
        for g, xx, yy, (st, w, sc, o) in plain:
            f = g.forward(xx, yy, gamma=args.gamma, canonical=True, state=st, scalars=sc)
            g.backward(xx, yy, f, rat=True, grad=True, workspace=w, out=o)

    ms_seq, _ = timed(seq_step, max(1, args.steps // 4), 1)

    roofline = kernels = None
    if not args.no_profile:
        # The snapshot graph alone (its launches would overlap the other stream's otherwise).
        g1.profile(True)
        for _ in range(args.steps):
            sweep(g1, x1, y1, b1, None)
        torch.cuda.synchronize()
        prof = g1.profile_read()
        g1.profile(False)
        alg = algorithmic_bytes(d1, g1.levelization()["level"], snapshots=64)
        kernels, roofline = kernel_table(prof, alg, args.steps)
        roofline["scope"] = "the 64-snapshot graph's launches"
        roofline["traffic"] = (counted_traffic("k_bwd_level_si", "sta_snapshot_lanes_64snap_kernel_stats.md")
                               if inner and roofline["kernel"] == "bwd_level" else None)

    cpu = None
    if not args.no_cpu_baseline and not getattr(args, "lean", False):
        from oracle import sta_oracle as O
        c0 = time.perf_counter()
        done = 0
        for d, mx, my in members[:1] + members[64:]:
            O.run(d, x=mx, y=my, gamma=args.gamma, grad="tns")
            done += d.n_pins
        ct = time.perf_counter() - c0
        cpu = dict(value=round(done / ct, 1), unit="pins/s", cores=int(torch.get_num_threads()), kind="oracle",
                   sample=f"FP64 forward+backward+gradient of snapshot 1 and the 16 designs "
                          f"({done} of {P} pins, levelization included), {ct:.1f} s")
    return {
        "metric": "STA fwd+bwd pins/sec, batched sweep vs plain calls",
        "value": round(value, 1),
        "unit": "pins/s",
        "ms_per_step": round(ms, 4),
        "dtype": "f32",
        "config": {"workload": f"cfg3: 64 snapshots (sigma 5 um) of the {d1.n_pins}-pin design + 16 designs "
                               f"of 10k-400k pins; {P} pins, fwd+bwd with d TNS_g/dx,dy, gamma {args.gamma} ps; "
                               f"snapshots share one graph ({L1} levels, snapshot-{args.snapshot_layout} layout) on "
                               f"one stream, the 16 designs one batch "
                               f"graph ({L16} levels) on another, "
                               + ("launched directly" if args.no_batch_capture else "both hipGraph-captured"),
                   "pins": P, "members": 80, "schedule_snapshots": best1, "schedule_designs": best16,
                   "io": "canonical order, HBM resident"},
        "union": None if ms_u is None else {
            "value": round(P / (ms_u * 1e-3), 1), "unit": "pins/s", "ms_per_step": round(ms_u, 4),
            "note": "one batch graph of all 80 members" + ("" if args.no_batch_capture else ", captured")},
        "plain_sequential": {"value": round(P / (ms_seq * 1e-3), 1), "unit": "pins/s",
                             "ms_per_step": round(ms_seq, 4), "calls": 2 * len(plain),
                             "speedup_batched": round(ms_seq / ms, 3)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "wall_s_timed": round(wall, 3),
        "setup_s": round(t_setup, 2),
    }


def snapshot_graph_only(args, g1, d1, x1, y1, dev, best1, t_setup) -> dict:
    """The 64-snapshot graph of the batched workload alone, launched directly on the default
    stream (the form the counter runs use)."""
    import torch
    b1 = step_buffers(g1, d1.n_pins, dev, 1, 64)
    state, ws, scal, outs = b1

    def step():
        f = g1.forward(x1, y1, gamma=args.gamma, canonical=True, state=state, scalars=scal)
        g1.backward(x1, y1, f, rat=True, grad=True, workspace=ws, out=outs)

    ms, wall = timed(step, args.steps, args.warmup)
    roofline = kernels = None
    if not args.no_profile:
        g1.profile(True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        prof = g1.profile_read()
        g1.profile(False)
        alg = algorithmic_bytes(d1, g1.levelization()["level"], snapshots=64)
        kernels, roofline = kernel_table(prof, alg, args.steps)
        roofline["scope"] = "the 64-snapshot graph's launches"
        roofline["traffic"] = (counted_traffic("k_bwd_level_si", "sta_snapshot_lanes_64snap_kernel_stats.md")
                               if args.snapshot_layout == "inner" and roofline["kernel"] == "bwd_level"
                               else None)
    P = 64 * d1.n_pins
    return {
        "metric": "STA fwd+bwd pins/sec, 64 placement snapshots in one sweep",
        "value": round(P / (ms * 1e-3), 1),
        "unit": "pins/s",
        "ms_per_step": round(ms, 4),
        "dtype": "f32",
        "config": {"workload": f"64 snapshots (sigma 5 um) of the {d1.n_pins}-pin design as one graph, "
                               f"fwd+bwd with d TNS_g/dx,dy, gamma {args.gamma} ps, default stream, "
                               f"launched directly", "pins": P, "schedule_snapshots": best1,
                   "io": "canonical order, HBM resident"},
        "roofline": roofline,
        "kernels": kernels,
        "wall_s_timed": round(wall, 3),
        "setup_s": round(t_setup, 2),
    }


def run_single(args) -> dict:
    import torch
    from gen.netlist import CFG0, CFG1, CFG2, make_design
    from paper_2603_28381_amd import Graph

    spec = {"cfg0": CFG0, "cfg1": CFG1, "cfg2": CFG2}[args.workload]
    t0 = time.time()
    d = make_design(spec)
    if args.trees:
        from gen.netlist import heap_trees
        d = heap_trees(d)
    g = Graph.from_design(d)
    n_levels = g.levelize()
    if args.fwd_cell_lanes != 16 or args.sweep_group_log2 != 2:
        g.set_schedule(args.sweep_group_log2, 2, 64, "groups", args.fwd_cell_lanes)
    g.upload()
    lev = g.levelization()
    t_setup = time.time() - t0
    P = d.n_pins
    dev = torch.device("cuda")
    perm = torch.from_numpy(lev["pin_perm"].astype(np.int64))
    x = torch.from_numpy(d.x)[perm].contiguous().to(dev)        # canonical order, resident in HBM
    y = torch.from_numpy(d.y)[perm].contiguous().to(dev)
    state, ws, scal, outs = step_buffers(g, P, dev)

    def step():
        f = g.forward(x, y, gamma=args.gamma, smooth=True, canonical=True, state=state, scalars=scal,
                      capture=args.capture)
        g.backward(x, y, f, rat=True, grad=True, workspace=ws, out=outs, capture=args.capture)

    ms, wall = timed(step, args.steps, args.warmup)
    value = P / (ms * 1e-3)

    roofline = kernels = None
    if not args.no_profile:
        # Same steps again with an event pair around every launch, on the library's stream.
        g.profile(True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        prof = g.profile_read()
        g.profile(False)
        kernels, roofline = kernel_table(prof, algorithmic_bytes(d, lev["level"]), args.steps)
        if args.workload == "cfg2" and not args.trees and args.fwd_cell_lanes == 16 and args.sweep_group_log2 == 2:
            roofline["traffic"] = counted_traffic("k_" + roofline["kernel"])
        # The per-launch floor of this machine for comparison: back-to-back dependent launches of
        # a trivial elementwise kernel over as many threads as a level launch has.
        roofline["launch_floor_us"] = round(launch_floor_us(dev, 256 * 450), 2)
        if not args.trees:
            roofline["whole_sweep_model"] = whole_sweep_roofline(d, kernels, ms)

    ckpt = None
    if args.ckpt_compare:
        ckpt = checkpoint_comparison(g, x, y, P, dev, args)

    cpu = None
    if not args.no_cpu_baseline:
        host = cpu_host()
        ct = time_oracle(d, args.gamma, 1)
        cpu = dict(value=round(P / ct, 1), unit="pins/s", cores=1, kind="oracle",
                   sample=f"one full FP64 forward+backward+gradient of the same {P}-pin design "
                          f"(levelization excluded) on one host thread, {ct:.1f} s", **host)
        nt = min(16, host["usable_cpus"] or 1)
        ctm = time_oracle(d, args.gamma, nt)
        cpu["multithread"] = dict(value=round(P / ctm, 1), unit="pins/s", cores=nt, seconds=round(ctm, 2))
    return {
        "metric": "STA fwd+bwd pins/sec @2.5M pins",
        "value": round(value, 1),
        "unit": "pins/s",
        "ms_per_step": round(ms, 4),
        "dtype": "f32",
        "config": {"workload": f"{args.workload}: {P} pins, {d.n_nets} nets, {d.n_cells} cells, "
                               f"{n_levels} net levels, fwd+bwd with d TNS_g/dx,dy, gamma {args.gamma} ps"
                               + (", hipGraph-captured" if args.capture else "")
                               + (", an RC tree per net (binary heaps by distance)" if args.trees else "")
                               + (f", {args.fwd_cell_lanes} lanes per forward cell" if args.fwd_cell_lanes != 16 else "")
                               + (f", backward groups from {1 << args.sweep_group_log2} lanes"
                                  if args.sweep_group_log2 != 2 else ""),
                   "pins": P, "levels": n_levels, "io": "canonical order, HBM resident"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "checkpointing": ckpt,
        "wall_s_timed": round(wall, 3),
        "setup_s": round(t_setup, 2),
    }


def checkpoint_comparison(g, x, y, P, dev, args) -> dict:
    """Gradient steps (forward + backward with d TNS_g/dx,dy, no per-pin outputs) with and
    without per-level checkpointing: time, arrival-state bytes and peak device memory."""
    import torch
    res = {}
    # The stride with the least sweep memory (state + workspace) among 2..2*sqrt(L), from the
    # host-side layout alone (ceil(sqrt(L - 1)) is the textbook choice; the frontier of this
    # DAG decides).
    L = g.info()["n_levels"]
    best = None
    for k in range(2, int(2 * np.sqrt(L)) + 1):
        g.set_checkpointing(k)
        info = g.info()
        b = info["fwd_state_bytes"] + info["bwd_workspace_bytes"]
        if best is None or b < best[0]:
            best = (b, k)
    g.set_checkpointing(0)
    for name, stride in (("plain", 0), ("checkpointed", best[1])):
        g.set_checkpointing(stride)
        g.upload()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        state, ws = g.new_state(dev), g.new_workspace(dev)
        scal = torch.empty(4, dtype=torch.float64, device=dev)
        out = {"dx": torch.empty(P, device=dev), "dy": torch.empty(P, device=dev)}

        def step():
            f = g.forward(x, y, gamma=args.gamma, canonical=True, state=state, scalars=scal)
            g.backward(x, y, f, rat=False, grad=True, workspace=ws, out=out)

        ms, _ = timed(step, args.steps, args.warmup)
        info, ck = g.info(), g.checkpointing()
        res[name] = dict(ms_per_step=round(ms, 4), stride_levels=ck["stride_levels"],
                         record_slots=ck["record_slots"], kept_nets=ck["kept_nets"],
                         fwd_state_bytes=info["fwd_state_bytes"], workspace_bytes=info["bwd_workspace_bytes"],
                         graph_device_bytes=info["device_bytes"],
                         peak_bytes=torch.cuda.max_memory_allocated() - base + info["device_bytes"])
        del state, ws, scal, out
    g.set_checkpointing(0)
    for k in ("plain", "checkpointed"):
        res[k]["sweep_bytes"] = res[k]["fwd_state_bytes"] + res[k]["workspace_bytes"]
    res["state_ratio"] = round(res["checkpointed"]["fwd_state_bytes"] / res["plain"]["fwd_state_bytes"], 4)
    res["sweep_ratio"] = round(res["checkpointed"]["sweep_bytes"] / res["plain"]["sweep_bytes"], 4)
    res["peak_ratio"] = round(res["checkpointed"]["peak_bytes"] / res["plain"]["peak_bytes"], 4)
    res["time_ratio"] = round(res["checkpointed"]["ms_per_step"] / res["plain"]["ms_per_step"], 4)
    return res


def run_fusion(args) -> dict:
    """Operation-fusion ablation (Sec. 3.2, Table 4 of the paper): the time of plain STA, and of STA
    plus the smoothed-TNS gradient computed (a) by a separate smoothed forward and gradient
    backward after STA, (b) by a gradient sweep on a second stream beside the required-time sweep
    (the two-stream overlap of Sec. 3.2), (c) fused into the required-time sweep.  Mid-size and
    2.5M-pin designs, every per-pin output, canonical order, inputs resident in HBM."""
    import torch
    from gen.netlist import CFG1, CFG2, make_design
    from paper_2603_28381_amd import Graph

    res = {}
    for name, spec in (("cfg1", CFG1), ("cfg2", CFG2)):
        d = make_design(spec)
        g = Graph.from_design(d)
        g.levelize()
        g.upload()
        lev = g.levelization()
        P = d.n_pins
        dev = torch.device("cuda")
        perm = torch.from_numpy(lev["pin_perm"].astype(np.int64))
        x = torch.from_numpy(d.x)[perm].contiguous().to(dev)
        y = torch.from_numpy(d.y)[perm].contiguous().to(dev)
        state, ws, scal, outs = step_buffers(g, P, dev)
        state2, ws2 = g.new_state(dev), g.new_workspace(dev)
        scal2 = torch.empty(4, dtype=torch.float64, device=dev)
        rat_out = {k: outs[k] for k in ("at", "slew", "rat", "slack")}
        grad_out = {k: outs[k] for k in ("dx", "dy")}
        s1, s2 = torch.cuda.current_stream(), torch.cuda.Stream()
        ev_f, ev_j = torch.cuda.Event(), torch.cuda.Event()
        gm = args.gamma

        def sta():
            f = g.forward(x, y, gamma=gm, smooth=False, canonical=True, state=state, scalars=scal)
            g.backward(x, y, f, rat=True, grad=False, workspace=ws, out=rat_out)

        def separate():
            sta()
            f = g.forward(x, y, gamma=gm, smooth=True, canonical=True, state=state2, scalars=scal2)
            g.backward(x, y, f, rat=False, grad=True, workspace=ws2, out=grad_out)

        def two_stream():
            f = g.forward(x, y, gamma=gm, smooth=True, canonical=True, state=state, scalars=scal)
            ev_f.record(s1)
            s2.wait_event(ev_f)
            g.backward(x, y, f, rat=True, grad=False, workspace=ws, out=rat_out, stream=s1)
            g.backward(x, y, f, rat=False, grad=True, workspace=ws2, out=grad_out, stream=s2)
            ev_j.record(s2)
            s1.wait_event(ev_j)

        def fused():
            f = g.forward(x, y, gamma=gm, smooth=True, canonical=True, state=state, scalars=scal)
            g.backward(x, y, f, rat=True, grad=True, workspace=ws, out=outs)

        r = {"pins": P, "levels": int(lev["level"].max()) + 1}
        for vname, fn in (("sta", sta), ("separate", separate), ("two_stream", two_stream), ("fused", fused)):
            r[vname + "_ms"] = round(timed(fn, args.steps, args.warmup)[0], 4)
        for vname in ("separate", "two_stream", "fused"):
            r[vname + "_pct_of_sta"] = round(100.0 * r[vname + "_ms"] / r["sta_ms"], 1)
        res[name] = r
        del state, ws, state2, ws2, outs, g
        torch.cuda.empty_cache()
    c2 = res["cfg2"]
    return {"metric": "STA + smoothed-TNS gradient time as % of plain STA (fused sweep)", "value": c2["fused_pct_of_sta"],
            "unit": "% of plain STA", "ms_per_step": c2["fused_ms"], "higher_is_better": False, "dtype": "f32",
            "config": {"workload": "fusion ablation: plain STA vs gradient as a separate pass, on a second stream, "
                                   "fused; 800k-pin and 2.5M-pin designs, every per-pin output, gamma "
                                   f"{args.gamma} ps", "io": "canonical order, HBM resident"},
            "variants": res,
            "paper": "Table 4 (RTX 4090): differentiable STA as a separate pass costs about 133% of STA time, "
                     "fused about 116%"}


def run_rc(args) -> dict:
    """RC-stage mapping ablation (Sec. 3.1.1, Alg. 1-2, Table 2 of the paper): the RC net delay
    kernel and the whole forward+backward step with the RC stage mapped as lane groups per net
    (the pin-based scheme), as Alg. 2's workgroup task pool (CTE), and one thread per net (the
    mapping of earlier GPU timers); mid-size and 2.5M-pin designs, canonical order."""
    import torch
    from gen.netlist import CFG1, CFG2, make_design
    from paper_2603_28381_amd import Graph

    res = {}
    for name, spec in (("cfg1", CFG1), ("cfg2", CFG2)):
        d = make_design(spec)
        g = Graph.from_design(d)
        g.levelize()
        g.upload()
        lev = g.levelization()
        alg = algorithmic_bytes(d, lev["level"])
        P = d.n_pins
        dev = torch.device("cuda")
        perm = torch.from_numpy(lev["pin_perm"].astype(np.int64))
        x = torch.from_numpy(d.x)[perm].contiguous().to(dev)
        y = torch.from_numpy(d.y)[perm].contiguous().to(dev)
        state, ws, scal, outs = step_buffers(g, P, dev)

        def step():
            f = g.forward(x, y, gamma=args.gamma, smooth=True, canonical=True, state=state, scalars=scal)
            g.backward(x, y, f, rat=True, grad=True, workspace=ws, out=outs)

        r = {"pins": P, "rc_alg_bytes": float(np.sum(alg["rc"]))}
        # RC stage as lane groups, task pool or one thread per net (level kernels in lane
        # groups), the task pool in the RC stage and the level kernels ("cte_all", the paper's
        # whole-STA CTE column), and one thread per net and cell in every stage ("thread_all")
        for scheme, level in (("groups", "groups"), ("cte", "groups"), ("thread", "groups"),
                              ("cte_all", "cte"), ("thread_all", "thread")):
            rc = {"thread_all": "thread", "cte_all": "cte"}.get(scheme, scheme)
            g.set_schedule(2, 2, 64, rc, 16, level)
            ms = timed(step, args.steps, args.warmup)[0]
            g.profile(True)
            for _ in range(args.steps):
                step()
            torch.cuda.synchronize()
            prof = g.profile_read()
            n_rc, t_rc = prof["rc"]
            g.profile(False)
            us = 1e3 * t_rc / n_rc
            r[scheme] = {"rc_us": round(us, 2), "rc_gbs": round(r["rc_alg_bytes"] / (us * 1e-6) / 1e9, 1),
                         "fwd_level_us": round(1e3 * prof["fwd_level"][1] / max(1, prof["fwd_level"][0]), 2),
                         "bwd_level_us": round(1e3 * prof["bwd_level"][1] / max(1, prof["bwd_level"][0]), 2),
                         "step_ms": round(ms, 4)}
        g.set_schedule(2, 2, 64, "groups", 16, "groups")
        r["groups_speedup_vs_thread"] = round(r["thread"]["rc_us"] / r["groups"]["rc_us"], 2)
        r["cte_speedup_vs_thread"] = round(r["thread"]["rc_us"] / r["cte"]["rc_us"], 2)
        r["step_speedup_vs_thread_all"] = {k: round(r["thread_all"]["step_ms"] / r[k]["step_ms"], 3)
                                           for k in ("groups", "cte", "thread", "cte_all")}
        r["cte_all_step_vs_groups"] = round(r["cte_all"]["step_ms"] / r["groups"]["step_ms"], 3)
        res[name] = r
        del state, ws, outs, g
        torch.cuda.empty_cache()
    c2 = res["cfg2"]
    return {"metric": "RC net delay kernel speedup of lane groups over one thread per net", "value":
            c2["groups_speedup_vs_thread"], "unit": "x", "ms_per_step": c2["groups"]["step_ms"], "dtype": "f32",
            "config": {"workload": "mapping ablation: RC stage as lane groups (pin-based), CTE task pool or one "
                                   "thread per net, and one thread per net and cell in every stage; 800k-pin and "
                                   "2.5M-pin designs", "io": "canonical order, HBM resident"},
            "variants": res,
            "paper": "Table 2 (RTX 4090, whole STA): pin-based 236% and CTE 124% of GPU-Timer's speed"}


def run_place(args) -> dict:
    """Synthetic timing-driven placement loop (Sec. 3.3): every iteration runs the smoothed
    forward sweep and the fused gradient sweep of the mid-size design, gathers the pin gradients
    to cells and takes one Adam step of the cells.  Reports iterations per second and the
    timing before and after."""
    import torch
    from gen.netlist import CFG1, make_design
    from paper_2603_28381_amd import Graph, TimingDescent

    d = make_design(CFG1)
    g = Graph.from_design(d)
    g.levelize()
    g.upload()
    td = TimingDescent(g, d.x, d.y, d.cell_in_offsets, d.cell_in_pins, d.cell_out_pin, gamma=args.gamma, lr=1.0,
                       anchor=1e-4)
    iters = max(args.steps, 1) * 5
    first = td.evaluate().cpu().numpy()
    ms, _ = timed(td.step, iters, args.warmup)
    last = td.evaluate().cpu().numpy()
    x, y = td.coordinates()
    disp = torch.sqrt((x - td.x0) ** 2 + (y - td.y0) ** 2)
    names = ("wns", "tns", "wns_g", "tns_g")
    return {"metric": "timing-driven placement iterations/sec (STA + TNS_g gradient + cell step)",
            "value": round(1e3 / ms, 1), "unit": "iterations/s", "ms_per_step": round(ms, 4), "dtype": "f32",
            "config": {"workload": f"placement loop: {d.n_pins}-pin design, {d.n_cells} movable cells, "
                                   f"{iters + args.warmup} Adam steps of 1 um on cell x, y against TNS_g "
                                   f"(gamma {args.gamma} ps) with a quadratic anchor", "pins": d.n_pins},
            "timing_before": {k: float(v) for k, v in zip(names, first)},
            "timing_after": {k: float(v) for k, v in zip(names, last)},
            "mean_displacement_um": round(float(disp.mean()), 3), "max_displacement_um": round(float(disp.max()), 3)}


def run_serve(args) -> dict:
    """Served workload: 12 resident designs of 5k-2.5M pins (log-uniform), an open-loop
    Poisson stream of requests (70% forward slack queries on resident coordinates, 30%
    forward+backward gradient queries on coordinates jittered by N(0, 2 um)), admitted
    against a 200 GB budget.  Latency runs from the scheduled arrival to the results being
    on the host."""
    import threading
    import torch
    from gen.netlist import batch_designs, jitter
    from paper_2603_28381_amd import Graph, Server

    t0 = time.time()
    designs = batch_designs(12, 5_000, 2_500_000, cfg_id=4)
    graphs = []
    for d in designs:
        g = Graph.from_design(d)
        g.levelize()
        graphs.append(g)
    srv = Server(200 << 30, max_slots=args.serve_slots, queue_capacity=1 << 16, max_merge=args.serve_merge)
    ids = [srv.add_design(g, d.x, d.y) for g, d in zip(graphs, designs)]
    n_jit = 4
    jit = [[jitter(d, 2.0, stream=500 + j) for j in range(n_jit)] for d in designs]
    rng = np.random.default_rng([260328381, 4, 77])
    n_req = int(args.serve_rate * args.serve_seconds)
    arrivals = np.cumsum(rng.exponential(1.0 / args.serve_rate, n_req))
    which = rng.integers(len(designs), size=n_req)
    grad = rng.random(n_req) < 0.3
    t_setup = time.time() - t0
    # Warm every slot on every (design, kind, new or resident coordinates) it may serve alone,
    # so that few captures fall in the timed window: with merging off, a burst of `slots`
    # requests of one key at a time occupies every slot.  Merged sweeps capture when they
    # first occur on a slot; the line counts the captures in the window.
    srv.set_max_merge(1)
    for i in ids:
        for g_ in (False, True):
            tk = [srv.submit(i, grad=g_, x=jit[i][0][0] if g_ else None, y=jit[i][0][1] if g_ else None)
                  for _ in range(args.serve_slots)]
            for q in tk:
                srv.wait(q)
    srv.set_max_merge(args.serve_merge)
    # Then bursts that merge (the first request of a burst runs alone, the others wait and
    # are swept together), so that merged sweeps have run before the window.
    for i in ids:
        for g_ in (False, True):
            tk = [srv.submit(i, grad=g_, x=jit[i][0][0] if g_ else None, y=jit[i][0][1] if g_ else None)
                  for _ in range(4 * args.serve_slots)]
            for q in tk:
                srv.wait(q)
    warm = srv.stats()
    tickets = [None] * n_req
    lag = np.zeros(n_req)
    results = [None] * n_req
    sample_every = 100

    def collect():
        for r in range(n_req):
            while tickets[r] is None:
                time.sleep(0.0002)
            res = srv.wait(tickets[r], grad=r % sample_every == 0)
            results[r] = (res["latency_ms"], res["queue_ms"], res["scalars"],
                          (res.get("dx"), res.get("dy")) if r % sample_every == 0 else None)

    # The client's own pauses count as submission lag: no garbage collection in the window.
    import gc
    gc.collect()
    gc.disable()
    th = threading.Thread(target=collect)
    th.start()
    start = time.perf_counter()
    for r in range(n_req):
        due = start + arrivals[r]
        while True:
            now = time.perf_counter()
            if now >= due:
                break
            time.sleep(min(due - now, 0.001))
        k = int(which[r])
        # lag: scheduled arrival to the submit call (the server's latency starts inside it)
        lag[r] = (time.perf_counter() - due) * 1e3
        if grad[r]:
            x, y = jit[k][r % n_jit]
            tickets[r] = srv.submit(ids[k], grad=True, x=x, y=y)
        else:
            tickets[r] = srv.submit(ids[k], grad=False)
    th.join()
    elapsed = time.perf_counter() - start
    gc.enable()
    after = srv.stats()
    captures_in_window = after["captures"] - warm["captures"]
    srv.close()

    def burst(slots: int, merge: int, n: int = 400) -> dict:
        """Capacity: n requests of the same mix submitted at once, served with `slots` slots,
        waiting requests of one design and kind merged up to `merge` per sweep."""
        b = Server(200 << 30, max_slots=slots, queue_capacity=1 << 16, max_merge=merge)
        bid = [b.add_design(g, d.x, d.y) for g, d in zip(graphs, designs)]
        def run_all():
            tk = []
            for r in range(n):
                k = int(which[r])
                if grad[r]:
                    x, y = jit[k][r % n_jit]
                    tk.append(b.submit(bid[k], grad=True, x=x, y=y))
                else:
                    tk.append(b.submit(bid[k], grad=False))
            for q in tk:
                b.wait(q, grad=False)      # results are on the host; no client copy

        for _ in range(6):             # until a pass captures no new launch sequence
            c0 = b.stats()["captures"]
            run_all()
            if b.stats()["captures"] == c0:
                break
        s0 = b.stats()
        t = time.perf_counter()
        run_all()
        dt = time.perf_counter() - t
        s1 = b.stats()
        b.close()
        pp = float(sum(designs[int(which[r])].n_pins for r in range(n)))
        return {"slots": slots, "max_merge": merge, "requests": n, "s": round(dt, 4), "pins_per_s": round(pp / dt, 1),
                "sweeps": s1["sweeps"] - s0["sweeps"], "merged": s1["merged"] - s0["merged"],
                "captures": s1["captures"] - s0["captures"],
                "capture_ms": round(s1["capture_ms"] - s0["capture_ms"], 3)}

    if getattr(args, "served_samples", ""):
        # Every 100th result with what regenerates its inputs, for check_served on the host:
        # the scalars, and of a gradient result the entries of up to SAMPLE_PINS seeded pins.
        rs = list(range(0, n_req, sample_every))
        picks = [served_sample_pins(designs[int(which[r])].n_pins, r) if grad[r] else np.zeros(0, np.int64)
                 for r in rs]
        dx = [results[r][3][0][pk] if grad[r] else np.zeros(0, np.float32) for r, pk in zip(rs, picks)]
        dy = [results[r][3][1][pk] if grad[r] else np.zeros(0, np.float32) for r, pk in zip(rs, picks)]
        os.makedirs(os.path.dirname(os.path.abspath(args.served_samples)), exist_ok=True)
        np.savez_compressed(args.served_samples, request=np.array(rs), design=which[rs], grad=grad[rs],
                            jitter=np.array(rs) % n_jit, scalars=np.stack([results[r][2] for r in rs]),
                            grad_offsets=np.cumsum([0] + [len(a) for a in dx]), pins=np.concatenate(picks),
                            dx=np.concatenate(dx), dy=np.concatenate(dy),
                            latency_ms=np.array([results[r][0] for r in rs]) + lag[rs], gamma=10.0)
    cap_many = burst(args.serve_slots, args.serve_merge)
    cap_alone = burst(args.serve_slots, 1)
    cap_one = burst(1, 1)
    lat = np.array([results[r][0] for r in range(n_req)]) + lag
    qms = np.array([results[r][1] for r in range(n_req)])
    pins = np.array([designs[int(k)].n_pins for k in which], np.float64)
    checked = []
    if not args.no_cpu_baseline and args.serve_check > 0:
        from oracle import sta_oracle as O
        c0 = time.perf_counter()
        done = 0
        # every 100th result; one per design, smallest designs first (the oracle's time)
        first = {}
        for r in range(0, n_req, sample_every):
            first.setdefault(int(which[r]), r)
        cands = sorted(first.values(), key=lambda r: designs[int(which[r])].n_pins)
        for r in cands[:args.serve_check]:
            k = int(which[r])
            d = designs[k]
            x, y = (jit[k][r % n_jit] if grad[r] else (d.x, d.y))
            ref = O.run(d, x=x, y=y, gamma=10.0, grad="tns" if grad[r] else None)
            sc = results[r][2]
            ok = abs(sc[1] - ref["tns"]) <= 1e-4 * abs(ref["tns"]) + 1e-3 and \
                abs(sc[3] - ref["tns_g"]) <= 1e-4 * abs(ref["tns_g"]) + 1e-3
            if grad[r]:
                gx = results[r][3][0].astype(np.float64)
                ok = ok and bool(np.all(np.abs(gx - ref["dx"]) <= 1e-3 * np.abs(ref["dx"])
                                        + 1e-6 * np.abs(ref["dx"]).max()))
            checked.append(dict(request=r, pins=d.n_pins, grad=bool(grad[r]), ok=bool(ok)))
            done += d.n_pins
        cpu_s = time.perf_counter() - c0
    value = pins.sum() / elapsed
    return {
        "metric": "served STA pins/sec with p50/p99 latency",
        "value": round(value, 1),
        "unit": "pins/s",
        "ms_per_step": round(float(np.percentile(lat, 50)), 4),
        "dtype": "f32",
        "config": {"workload": f"cfg4: {len(designs)} resident designs of {min(d.n_pins for d in designs)}-"
                               f"{max(d.n_pins for d in designs)} pins, Poisson {args.serve_rate} req/s for "
                               f"{args.serve_seconds} s, 30% fwd+bwd (jitter 2 um), budget 200 GB, "
                               f"{args.serve_slots} slots, merging up to {args.serve_merge}",
                   "designs_pins": [d.n_pins for d in designs], "requests": n_req},
        "serving": {"p50_ms": round(float(np.percentile(lat, 50)), 4),
                    "p99_ms": round(float(np.percentile(lat, 99)), 4),
                    "max_ms": round(float(lat.max()), 4),
                    "p99_queue_ms": round(float(np.percentile(qms, 99)), 4),
                    "slowest": [{"ms": round(float(lat[r]), 3), "queue_ms": round(float(qms[r]), 3),
                                 "submit_lag_ms": round(float(lag[r]), 3),
                                 "pins": int(pins[r]), "grad": bool(grad[r]), "arrival_s": round(float(arrivals[r]), 3)}
                                for r in np.argsort(lat)[::-1][:6]],
                    "capture_ms_in_window": round(after["capture_ms"] - warm["capture_ms"], 3),
                    "slot_grows_in_window": after["slot_grows"] - warm["slot_grows"],
                    "grow_ms_in_window": round(after["grow_ms"] - warm["grow_ms"], 3),
                    "pinned_allocs_in_window": after["pinned_allocs"] - warm["pinned_allocs"],
                    "pinned_ms_in_window": round(after["pinned_ms"] - warm["pinned_ms"], 3),
                    "p99_submit_lag_ms": round(float(np.percentile(lag, 99)), 4),
                    "fwd_p50_ms": round(float(np.percentile(lat[~grad], 50)), 4),
                    "fwd_bwd_p50_ms": round(float(np.percentile(lat[grad], 50)), 4) if grad.any() else None,
                    "achieved_req_per_s": round(n_req / elapsed, 2), "elapsed_s": round(elapsed, 3),
                    "captures_warmup": warm["captures"], "captures_in_window": captures_in_window,
                    "sweeps_in_window": after["sweeps"] - warm["sweeps"],
                    "merged_in_window": after["merged"] - warm["merged"],
                    "capacity": cap_many, "capacity_unmerged": cap_alone, "capacity_one_at_a_time": cap_one,
                    "capacity_speedup": round(cap_many["pins_per_s"] / cap_one["pins_per_s"], 3),
                    "merge_speedup": round(cap_many["pins_per_s"] / cap_alone["pins_per_s"], 3),
                    "oracle_checked": checked},
        "roofline": None,
        "cpu_baseline": None,
        "setup_s": round(t_setup, 2),
    }


SAMPLE_PINS = 20_000


def served_sample_pins(n_pins: int, request: int) -> np.ndarray:
    """The pins (original ids) whose gradient entries a served sample keeps: all of a small
    design, else SAMPLE_PINS seeded by the request number."""
    if n_pins <= SAMPLE_PINS:
        return np.arange(n_pins)
    return np.sort(np.random.default_rng([260328381, 4, 100, request]).choice(n_pins, SAMPLE_PINS, replace=False))


def check_served(path: str, gamma: float = 10.0) -> dict:
    """Checks served results saved by --served-samples against the FP64 oracle on the host:
    the designs and jittered coordinates are regenerated from their seeds.  Scalars must meet
    1e-4 relative (1e-3 ps absolute); the sampled gradient entries are counted against
    1e-3 |g| + 1e-6 max|g| and at most 2e-4 of them may exceed it (the full-size parity
    test's cap: values float32 cannot pin down in these extrapolated designs)."""
    from gen.netlist import batch_designs, jitter
    from oracle import sta_oracle as O
    z = np.load(path)
    designs = batch_designs(12, 5_000, 2_500_000, cfg_id=4)
    out = []
    t0 = time.perf_counter()
    for i, r in enumerate(z["request"]):
        k, gr = int(z["design"][i]), bool(z["grad"][i])
        d = designs[k]
        x, y = jitter(d, 2.0, stream=500 + int(z["jitter"][i])) if gr else (d.x, d.y)
        c0 = time.perf_counter()
        ref = O.run(d, x=x, y=y, gamma=gamma, grad="tns" if gr else None)
        sc = z["scalars"][i]
        errs = [abs(sc[j] - ref[n]) / (1e-4 * abs(ref[n]) + 1e-3) for j, n in enumerate(("wns", "tns", "wns_g", "tns_g"))]
        rec = dict(request=int(r), design=k, pins=d.n_pins, grad=gr, scalar_worst_x_tol=round(max(errs), 4),
                   oracle_s=round(time.perf_counter() - c0, 2))
        ok = max(errs) <= 1.0
        if gr:
            o0, o1 = z["grad_offsets"][i], z["grad_offsets"][i + 1]
            pk = z["pins"][o0:o1]
            for name in ("dx", "dy"):
                g = z[name][o0:o1].astype(np.float64)
                ref_g = ref[name][pk]
                tol = 1e-3 * np.abs(ref_g) + 1e-6 * np.abs(ref[name]).max()
                n_out = int(np.count_nonzero(np.abs(g - ref_g) > tol))
                norm = float(np.linalg.norm(g - ref_g) / max(np.linalg.norm(ref_g), 1e-300))
                rec[name] = dict(outside=n_out, norm_rel=norm)
                ok = ok and n_out <= 2e-4 * len(g)
        rec["ok"] = bool(ok)
        out.append(rec)
        print(json.dumps(rec), file=sys.stderr, flush=True)
    return {"checked": len(out), "ok": sum(r["ok"] for r in out), "designs": sorted({r["design"] for r in out}),
            "largest_pins": max(r["pins"] for r in out), "grad_results": sum(r["grad"] for r in out),
            "host_s": round(time.perf_counter() - t0, 1), "results": out}


def part_of_line(res: dict) -> dict:
    """A workload's result as a sub-object of the headline line."""
    keep = ("metric", "value", "unit", "ms_per_step", "config", "plain_sequential", "serving", "roofline",
            "cpu_baseline", "setup_s")
    return {k: res[k] for k in keep if k in res and res[k] is not None}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg2", choices=["cfg0", "cfg1", "cfg2", "cfg3", "cfg4", "fusion", "rc", "place"])
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-merge", type=int, default=8,
                    help="waiting requests of one design and kind swept together as snapshots, at most")
    ap.add_argument("--serve-check", type=int, default=6, help="served results checked against the oracle")
    ap.add_argument("--gamma", type=float, default=10.0)
    ap.add_argument("--capture", action="store_true", help="replay each call from a captured hipGraph")
    ap.add_argument("--no-batch-capture", action="store_true",
                    help="cfg3: launch the batched sweeps directly instead of replaying captured hipGraphs")
    ap.add_argument("--snapshot-layout", default="inner", choices=["inner", "outer"],
                    help="cfg3: the 64-snapshot graph with the snapshot innermost (lanes over snapshots) "
                         "or outermost (each snapshot its own workgroups)")
    ap.add_argument("--snapshots-only", action="store_true",
                    help="cfg3: only the 64-snapshot graph, launched directly on the default stream")
    ap.add_argument("--no-ckpt-compare", dest="ckpt_compare", action="store_false",
                    help="skip the gradient-step comparison with per-level checkpointing")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="first run one plain device copy of this size (a reference for HBM counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the event-timed roofline pass")
    ap.add_argument("--fwd-cell-lanes", type=int, default=16, choices=[16, 8, 4],
                    help="cfg0-2: lanes per cell of the forward level kernel (the schedule's fwd_cell_lanes)")
    ap.add_argument("--sweep-group-log2", type=int, default=2, choices=[2, 3, 4, 5, 6],
                    help="cfg0-2: log2 of the smallest backward lane group (the schedule's sweep_group_log2)")
    ap.add_argument("--trees", action="store_true",
                    help="cfg0-2 with an RC tree per net (binary heaps by distance) instead of stars")
    ap.add_argument("--headline-only", action="store_true",
                    help="cfg2: skip the batched and served parts of the metric")
    ap.add_argument("--served-samples", default="",
                    help="cfg4: save every 100th served result (request, inputs' seeds, outputs) to this .npz")
    ap.add_argument("--check-served", default="",
                    help="check a --served-samples file against the FP64 oracle on the host (no GPU)")
    args = ap.parse_args(argv)
    if args.check_served:
        print(json.dumps(check_served(args.check_served, args.gamma)), flush=True)
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the STA sweep of one design runs on a single device "
              "(independent designs would be routed one per GPU); run with --gpus 1.", file=sys.stderr)
        return 2
    if args.copy_probe_mb > 0:
        import torch
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    run = {"cfg3": run_batch, "cfg4": run_serve, "fusion": run_fusion, "rc": run_rc,
           "place": run_place}.get(args.workload, run_single)
    res = run(args)
    if args.workload == "cfg2" and not args.headline_only and not args.trees:
        # The rest of the metric: the batched form against plain calls, and the served form.
        import gc
        import torch
        gc.collect()
        torch.cuda.empty_cache()
        res["batched"] = part_of_line(run_batch(argparse.Namespace(**{**vars(args), "lean": True,
                                                                        "steps": max(5, args.steps // 2)})))
        gc.collect()
        torch.cuda.empty_cache()
        res["served"] = part_of_line(run_serve(argparse.Namespace(**{**vars(args), "serve_seconds": min(
            args.serve_seconds, 15.0)})))
    line = {"metric": res.pop("metric"), "value": res.pop("value"), "unit": res.pop("unit"), "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": res.pop("ms_per_step"),
            "higher_is_better": res.pop("higher_is_better", True), "scaling": "weak", "vs_baseline": None, "dtype": res.pop("dtype"),
            "data": "synthetic"}
    line.update(res)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
