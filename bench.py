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


def algorithmic_bytes(d, lev) -> dict:
    """Bytes each kernel family must move per step (float32 values, int32 indices).

    Counts only what the method reads and writes once; re-reads served by caches are not
    counted.  Per unit:
      rc         per net 4 sched + 4 offset + 8 driver x,y + 4 driver cap + 4 load write
                 (+40 record write for level-0 nets); per sink 8 x,y + 4 cap + 8 wire write
      fwd_level  per cell 16 (type, offset, arc base, load) + 40 record write; per cell
                 input 9 (source net, pin, unateness) + 8 wire + 40 source record
      ep_partial per endpoint 28 (pin, net, late AT 8, smoothed AT 8, wire delay 4)
      ep_seed    per endpoint 28 + 32 (required-time and adjoint seeds)
      bwd_level  per net 4 sched + 4 offset + 32 record + 8 driver x,y; per cell 16; per
                 cell input 9 + 8 wire + 24 source slew/smoothed AT + 32 seed writes;
                 per sink 16 RAT + 16 adjoint + 8 wire + 8 x,y + 4 cap; per pin 72 output
                 writes (AT, slew, RAT, slack, dx, dy)
    """
    N, P = d.n_nets, d.n_pins
    sinks = np.diff(d.net_offsets).astype(np.int64) - 1
    level = lev["level"].astype(np.int64)
    L = int(level.max()) + 1
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
    out["rc"] = [float(N * 24 + n0 * 40 + sinks.sum() * 20)]
    out["fwd_level"] = [float(cells_l[l] * 56 + ins_l[l] * 57) for l in range(1, L)]
    out["ep_partial"] = [float(E * 28)]
    out["ep_seed"] = [float(E * 60)]
    out["bwd_level"] = [float(nets_l[l] * 48 + cells_l[l] * 16 + ins_l[l] * 73 + sinks_l[l] * 52 + pins_l[l] * 72)
                        for l in range(L - 1, -1, -1)]
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg2", choices=["cfg0", "cfg1", "cfg2"])
    ap.add_argument("--gamma", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the event-timed roofline pass")
    args = ap.parse_args(argv)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the STA sweep of one design runs on a single device "
              "(independent designs would be routed one per GPU); run with --gpus 1.", file=sys.stderr)
        return 2

    import torch
    from gen.netlist import CFG0, CFG1, CFG2, make_design
    from paper_2603_28381_amd import Graph

    spec = {"cfg0": CFG0, "cfg1": CFG1, "cfg2": CFG2}[args.workload]
    t0 = time.time()
    d = make_design(spec)
    g = Graph.from_design(d)
    n_levels = g.levelize()
    g.upload()
    lev = g.levelization()
    t_setup = time.time() - t0
    P = d.n_pins
    dev = torch.device("cuda")
    perm = torch.from_numpy(lev["pin_perm"].astype(np.int64))
    x = torch.from_numpy(d.x)[perm].contiguous().to(dev)        # canonical order, resident in HBM
    y = torch.from_numpy(d.y)[perm].contiguous().to(dev)
    state = g.new_state(dev)
    ws = g.new_workspace(dev)
    scal = torch.empty(4, dtype=torch.float64, device=dev)
    outs = {k: torch.empty((P, 4), dtype=torch.float32, device=dev) for k in ("at", "slew", "rat", "slack")}
    outs["dx"] = torch.empty(P, dtype=torch.float32, device=dev)
    outs["dy"] = torch.empty(P, dtype=torch.float32, device=dev)

    def step():
        f = g.forward(x, y, gamma=args.gamma, smooth=True, canonical=True, state=state, scalars=scal)
        g.backward(x, y, f, rat=True, grad=True, workspace=ws, out=outs)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = ev0.elapsed_time(ev1) / args.steps
    value = P / (ms * 1e-3)

    roofline = None
    kernels = None
    if not args.no_profile:
        # Same steps again with an event pair around every launch, on the library's stream.
        g.profile(True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        prof = g.profile_read()
        g.profile(False)
        alg = algorithmic_bytes(d, lev)
        kernels = {}
        for k, (n, tot) in prof.items():
            if n == 0:
                continue
            per_step = sum(alg.get(k, [0.0]))
            kernels[k] = dict(launches_per_step=n // args.steps, avg_us=1e3 * tot / n,
                              ms_per_step=tot / args.steps,
                              alg_bytes_per_step=per_step,
                              gbs=(per_step * args.steps / (tot * 1e-3) / 1e9) if per_step else None)
        dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
        kd = kernels[dom]
        achieved = kd["gbs"]
        roofline = dict(bound="hbm", kernel=dom, achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(achieved / HBM_PEAK_GBS, 5), traffic=None,
                        alg_bytes_per_launch=kd["alg_bytes_per_step"] / kd["launches_per_step"],
                        avg_launch_us=round(kd["avg_us"], 3))

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import sta_oracle as O
        lv = O.levelize(d)
        plan = O._Plan(d, lv)
        c0 = time.perf_counter()
        O.run(d, gamma=args.gamma, grad="tns", lv=lv, plan=plan)
        ct = time.perf_counter() - c0
        cpu = dict(value=round(P / ct, 1), unit="pins/s", cores=int(torch.get_num_threads()), kind="oracle",
                   sample=f"one full FP64 forward+backward+gradient of the same {P}-pin design "
                          f"(levelization excluded), {ct:.1f} s")

    line = {
        "metric": "STA fwd+bwd pins/sec @2.5M pins",
        "value": round(value, 1),
        "unit": "pins/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {P} pins, {d.n_nets} nets, {d.n_cells} cells, "
                               f"{n_levels} net levels, fwd+bwd with d TNS_g/dx,dy, gamma {args.gamma} ps",
                   "pins": P, "levels": n_levels, "io": "canonical order, HBM resident"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "wall_s_timed": round(wall, 3),
        "setup_s": round(t_setup, 2),
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
