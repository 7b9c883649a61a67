"""FP64 CPU oracle for levelized static timing analysis (STA) and its LSE-smoothed adjoint.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check of the entry module and
the CPU-baseline leg of the benchmark import this file.  The GPU library never
calls, links or reads it, and it shares no code, table or helper with the library.

It evaluates the plain definitions, in float64, in the order the paper states them:

* levelization: nets grouped into dependency levels (Sec. 2.1 stage 2, Sec. 3.1.2);
* RC net delay with the Elmore model of Eq. 1 (Load), Eq. 2 (Delay), Eq. 3 (Impulse)
  (Sec. 3.1.1);
* forward propagation: cell-arc delay by NLDM table interpolation, late arrival =
  max over inputs of (input arrival + arc delay), early = min (Sec. 3.1.2);
* backward propagation of required times from the endpoints, slack (Sec. 2.1, 3.1.2);
* the LSE smoothing of Eq. 4 applied to the late max, and the gradient of a smoothed
  total negative slack with respect to pin coordinates (Sec. 3.2), taken by torch
  autograd of the smoothed forward (the derivative by definition).

Readings of what the paper leaves open (each used below):
  R1  nets are stars: each sink hangs off the driver through one wire segment, so
      Eq. 2 needs no parent-delay term; wire length is the Manhattan distance;
  R2  half of a segment's wire capacitance sits at each end (pi split);
  R3  in Eq. 3, Res(u) is the resistance of the segment into u and Cap(u) the node
      capacitance of u; the argument of the root is clamped at 0;
  R4  a sink's slew is sqrt(driver slew^2 + Impulse^2);
  R5  table rows are indexed by input slew, columns by the driven net's root load;
      bilinear interpolation, linear extrapolation from the edge cell, cell index
      upper_bound - 1 clamped to [0, 5];
  R6  output slew is the worst arc slew (max late, min early), independent of which
      arc sets the arrival; its gradient follows the arg max, ties to the lowest arc;
  R7  conditions are k = 2*mode + transition (mode 0 early, 1 late; 0 rise, 1 fall);
      a positive-unate arc keeps the transition, a negative-unate arc flips it;
  R8  primary inputs: AT = pi_at, slew = pi_slew; endpoints (flop D pins, primary
      outputs): late RAT = t_clk - setup, early RAT = hold; unconstrained pins get
      RAT = +inf (late) / -inf (early);
  R9  late slack = RAT - AT, early slack = AT - RAT; WNS/TNS over endpoints on the
      worst late transition, WNS = min(0, min slack), TNS = sum of min(0, slack);
  R10 only the late max merge is smoothed, using the hard-path arc delays and slews;
      smoothed slack s_e = -LSE(-slack_rise, -slack_fall), TNS_g = -sum_e LSE(0, -s_e),
      WNS_g = -LSE({0} u {-s_e}).
  R13 a design may instead give every net an RC tree over its own pins (each sink's
      parent pin, the driver at the root; one segment per sink, Manhattan length).
      Eq. 1 then sums Loads over children recursively, Eq. 2 gains the parent's delay,
      Delay(u) = Delay(fa(u)) + Res(fa(u) -> u) * Load(u) (the paper's Eq. 2 omits it,
      which is exact for the depth-1 trees of R1), and the impulse of Eq. 3 takes the
      second moment of the TAU 2015 model the paper cites for Eq. 1-3:
      LDelay(u) = Cap(u) * Delay(u) + sum over children of LDelay(v),
      Beta(u) = Beta(fa(u)) + Res(fa(u) -> u) * LDelay(u),
      Impulse(u) = sqrt(2 * Beta(u) - Delay(u)^2), clamped at 0.  On a star, Beta(u) =
      Res(u) * Cap(u) * Delay(u) and this is Eq. 3.
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np
import torch

PIN_PI, PIN_CELL_IN, PIN_CELL_OUT, PIN_FF_D, PIN_PO = 0, 1, 2, 3, 4
F64 = torch.float64


class CycleError(ValueError):
    pass


# --------------------------------------------------------------------------------------
# Levelization (Sec. 2.1 stage 2; Sec. 3.1.2): independent nets share a level, a net's
# level is one more than the deepest net feeding its driver cell, PI-driven nets are 0.
# --------------------------------------------------------------------------------------
@dataclass
class Levelization:
    n_levels: int
    level: np.ndarray          # int32 [N], level of each original net
    level_offsets: np.ndarray  # int32 [L+1], over the canonical net order
    net_perm: np.ndarray       # int32 [N], original id of the net at canonical position i;
                               # canonical order is (level, pins of the net, original id)
    pin_perm: np.ndarray       # int32 [P], original id of the pin at canonical position i
    net_of_pin: np.ndarray     # int64 [P]
    driver: np.ndarray         # int64 [N], driver pin of each net
    cell_of_net: np.ndarray    # int64 [N], driving cell or -1
    cell_of_out_pin: np.ndarray  # int64 [P], cell driven by the pin or -1


def levelize(d) -> Levelization:
    P, N, C = d.n_pins, d.n_nets, d.n_cells
    off = d.net_offsets.astype(np.int64)
    if len(off) != N + 1 or off[0] != 0 or off[-1] != P or np.any(np.diff(off) < 1):
        raise ValueError("bad net offsets")
    net_of_pin = np.full(P, -1, np.int64)
    for n in range(N):
        for p in d.net_pins[off[n]:off[n + 1]]:
            if net_of_pin[p] != -1:
                raise ValueError("pin in two nets")
            net_of_pin[p] = n
    if np.any(net_of_pin < 0):
        raise ValueError("pin in no net")
    driver = d.net_pins[off[:-1]].astype(np.int64)
    kind = d.pin_kind
    cell_of_out_pin = np.full(P, -1, np.int64)
    cell_of_out_pin[d.cell_out_pin] = np.arange(C)
    cell_of_net = np.full(N, -1, np.int64)
    for n in range(N):
        p = driver[n]
        if kind[p] == PIN_PI:
            continue
        if kind[p] != PIN_CELL_OUT or cell_of_out_pin[p] < 0:
            raise ValueError("net driver is neither a PI nor a cell output")
        cell_of_net[n] = cell_of_out_pin[p]

    # Net DAG: edge m -> n when a sink of m is an input of the cell driving n.
    preds = [[] for _ in range(N)]
    succs = [[] for _ in range(N)]
    cin = d.cell_in_offsets.astype(np.int64)
    for n in range(N):
        c = cell_of_net[n]
        if c < 0:
            continue
        if cin[c + 1] <= cin[c]:
            raise ValueError("cell without inputs")
        for p in d.cell_in_pins[cin[c]:cin[c + 1]]:
            m = int(net_of_pin[p])
            preds[n].append(m)
            succs[m].append(n)

    # Kahn's algorithm, frontier by frontier.
    indeg = np.array([len(pr) for pr in preds], np.int64)
    level = np.full(N, -1, np.int64)
    frontier = [n for n in range(N) if indeg[n] == 0]
    for n in frontier:
        if cell_of_net[n] >= 0:
            raise ValueError("cell-driven net without predecessors")
        level[n] = 0
    seen = 0
    while frontier:
        nxt = []
        for m in frontier:
            seen += 1
            for n in succs[m]:
                level[n] = max(level[n], level[m] + 1)
                indeg[n] -= 1
                if indeg[n] == 0:
                    nxt.append(n)
        frontier = nxt
    if seen != N:
        raise CycleError("combinational cycle")
    L = int(level.max()) + 1
    # Canonical order: (level, pins of the net, original id).
    pins = np.diff(off)
    net_perm = np.lexsort((np.arange(N), pins, level)).astype(np.int32)
    level_offsets = np.searchsorted(level[net_perm], np.arange(L + 1), side="left").astype(np.int32)
    pin_perm = np.concatenate([d.net_pins[off[n]:off[n + 1]] for n in net_perm]).astype(np.int32)
    return Levelization(L, level.astype(np.int32), level_offsets, net_perm, pin_perm,
                        net_of_pin, driver, cell_of_net, cell_of_out_pin)


# --------------------------------------------------------------------------------------
# RC net delay, Sec. 3.1.1, Eq. 1-3 (readings R1-R3).
# --------------------------------------------------------------------------------------
def rc(d, lv: Levelization, x: torch.Tensor, y: torch.Tensor):
    """Per-pin wire length, node capacitance, Load (Eq. 1), Delay (Eq. 2), Impulse (Eq. 3).

    Returns dict of float64 tensors indexed by original pin id; Load is also given per net
    (the root load of the net, which is the load a driving cell sees).  Designs with RC
    trees (d.pin_parent) go through rc_tree (reading R13).
    """
    if getattr(d, "pin_parent", None) is not None:
        return rc_tree(d, lv, x, y)
    P, N = d.n_pins, d.n_nets
    r, c = float(d.cons.r_per_um), float(d.cons.c_per_um)
    net = torch.from_numpy(lv.net_of_pin)
    drv = torch.from_numpy(lv.driver)[net]                      # driver pin of each pin's net
    is_sink = torch.from_numpy(lv.driver[lv.net_of_pin] != np.arange(P))
    cpin = torch.from_numpy(d.pin_cap.astype(np.float64))
    length = torch.where(is_sink, (x - x[drv]).abs() + (y - y[drv]).abs(), torch.zeros((), dtype=F64))
    res = r * length                                            # Res(fa(u) -> u), ohm
    cwire = c * length                                          # wire capacitance, fF
    # Node capacitances: half of each segment at the sink, half at the driver (R2).
    cap_node = torch.where(is_sink, cpin + 0.5 * cwire, torch.zeros((), dtype=F64))
    cap_root = cpin[torch.from_numpy(lv.driver)] + torch.zeros(N, dtype=F64).index_add(0, net, 0.5 * cwire)
    # Eq. 1: a leaf's Load is its own Cap; the root adds all of its fanout Loads.
    load_leaf = cap_node
    load_root = cap_root + torch.zeros(N, dtype=F64).index_add(0, net, torch.where(is_sink, load_leaf, torch.zeros((), dtype=F64)))
    # Eq. 2: Delay(u) = Res(fa(u) -> u) * Load(u); ohm * fF = 1e-3 ps.
    delay = torch.where(is_sink, 1e-3 * res * load_leaf, torch.zeros((), dtype=F64))
    # Eq. 3: Impulse(u) = sqrt(2 * Res(u) * Cap(u) * Delay(u) - Delay(u)^2), argument clamped at 0.
    arg = 2.0 * (1e-3 * res * cap_node) * delay - delay * delay
    pos = arg > 0
    imp = torch.where(pos, torch.sqrt(torch.where(pos, arg, torch.ones((), dtype=F64))), torch.zeros((), dtype=F64))
    return dict(length=length, cap_node=cap_node, load_root=load_root, delay=delay, imp=imp)


def tree_depth(parent: np.ndarray) -> np.ndarray:
    """Depth of every pin in its net's RC tree (0 at the driver), by following parents."""
    P = len(parent)
    depth = np.full(P, -1, np.int64)
    depth[parent < 0] = 0
    for _ in range(P + 1):
        todo = depth < 0
        if not todo.any():
            return depth
        ready = todo & (depth[np.where(parent >= 0, parent, 0)] >= 0) & (parent >= 0)
        if not ready.any():
            raise ValueError("pin_parent has a cycle")
        depth[ready] = depth[parent[ready]] + 1
    raise ValueError("pin_parent has a cycle")


def rc_tree(d, lv: Levelization, x: torch.Tensor, y: torch.Tensor):
    """Eq. 1-3 on RC trees (reading R13): segment u runs from pin fa(u) to pin u.

    Children are summed depth by depth, deepest first (Load, LDelay); delays and second
    moments accumulate from the root down (Delay, Beta).
    """
    N = d.n_nets
    r, c = float(d.cons.r_per_um), float(d.cons.c_per_um)
    parent = np.asarray(d.pin_parent, np.int64)
    depth = tree_depth(parent)
    zero = torch.zeros((), dtype=F64)
    nonroot = torch.from_numpy(parent >= 0)
    fa = torch.from_numpy(np.where(parent >= 0, parent, np.arange(len(parent))))
    cpin = torch.from_numpy(d.pin_cap.astype(np.float64))
    length = torch.where(nonroot, (x - x[fa]).abs() + (y - y[fa]).abs(), zero)
    res = r * length                                            # Res(fa(u) -> u), ohm
    cwire = c * length
    # Node capacitance: the pin, half of the segment into it, half of each segment out of it (R2).
    half = torch.where(nonroot, 0.5 * cwire, zero)
    cap = cpin + half + torch.zeros_like(cpin).index_add(0, fa[nonroot], half[nonroot])
    levels = [torch.from_numpy(np.nonzero(depth == k)[0]) for k in range(int(depth.max()) + 1)]
    # Eq. 1: Load(u) = Cap(u) + sum of the children's Loads, deepest level first.
    load = cap
    for nodes in reversed(levels[1:]):
        load = load.index_add(0, fa[nodes], load[nodes])
    # Eq. 2 with the parent's delay: Delay(u) = Delay(fa(u)) + Res(fa(u) -> u) * Load(u).
    delay = torch.zeros_like(cap)
    for nodes in levels[1:]:
        delay = delay.index_put((nodes,), delay[fa[nodes]] + 1e-3 * res[nodes] * load[nodes])
    # Second moment: LDelay bottom-up, Beta top-down.
    ldelay = cap * delay
    for nodes in reversed(levels[1:]):
        ldelay = ldelay.index_add(0, fa[nodes], ldelay[nodes])
    beta = torch.zeros_like(cap)
    for nodes in levels[1:]:
        beta = beta.index_put((nodes,), beta[fa[nodes]] + 1e-3 * res[nodes] * ldelay[nodes])
    arg = 2.0 * beta - delay * delay
    pos = arg > 0
    imp = torch.where(pos, torch.sqrt(torch.where(pos, arg, torch.ones((), dtype=F64))), zero)
    drv = torch.from_numpy(lv.driver.astype(np.int64))
    load_root = load[drv]
    return dict(length=length, cap_node=torch.where(nonroot, cap, zero), load_root=load_root,
                delay=torch.where(nonroot, delay, zero), imp=imp, beta=beta)


# --------------------------------------------------------------------------------------
# NLDM table lookup, Sec. 3.1.2 (reading R5).
# --------------------------------------------------------------------------------------
def lut_index(axis: torch.Tensor, v: torch.Tensor) -> torch.Tensor:
    """Cell index: upper_bound(axis, v) - 1, clamped to [0, len(axis) - 2]."""
    i = torch.searchsorted(axis, v.detach().contiguous(), right=True) - 1
    return i.clamp(0, axis.numel() - 2)


def lut(tab: torch.Tensor, xa: torch.Tensor, ya: torch.Tensor, xv: torch.Tensor, yv: torch.Tensor):
    """Bilinear interpolation (linear extrapolation outside the axes) of tab[..., i, j].

    tab: [..., 7, 7] tables, one per query; xv (input slew) and yv (load) broadcast to tab[..., 0, 0].
    Returns (value, i, j).
    """
    i = lut_index(xa, xv)
    j = lut_index(ya, yv)
    tx = (xv - xa[i]) / (xa[i + 1] - xa[i])
    ty = (yv - ya[j]) / (ya[j + 1] - ya[j])
    flat = tab.reshape(*tab.shape[:-2], -1)
    n = xa.numel()

    def at(ii, jj):
        return torch.gather(flat, -1, (ii * n + jj).unsqueeze(-1)).squeeze(-1)

    v = ((1 - tx) * (1 - ty) * at(i, j) + tx * (1 - ty) * at(i + 1, j)
         + (1 - tx) * ty * at(i, j + 1) + tx * ty * at(i + 1, j + 1))
    return v, i, j


def lut_partials(tab: torch.Tensor, xa: torch.Tensor, ya: torch.Tensor, xv: torch.Tensor, yv: torch.Tensor):
    """Partial derivatives of the bilinear lookup with respect to its two inputs (same cell
    choice as lut()): d/dx = ((1-ty)(T[i+1][j]-T[i][j]) + ty(T[i+1][j+1]-T[i][j+1])) / (X[i+1]-X[i])."""
    i = lut_index(xa, xv)
    j = lut_index(ya, yv)
    tx = (xv - xa[i]) / (xa[i + 1] - xa[i])
    ty = (yv - ya[j]) / (ya[j + 1] - ya[j])
    flat = tab.reshape(*tab.shape[:-2], -1)
    n = xa.numel()

    def at(ii, jj):
        return torch.gather(flat, -1, (ii * n + jj).unsqueeze(-1)).squeeze(-1)

    dx = ((1 - ty) * (at(i + 1, j) - at(i, j)) + ty * (at(i + 1, j + 1) - at(i, j + 1))) / (xa[i + 1] - xa[i])
    dy = ((1 - tx) * (at(i, j + 1) - at(i, j)) + tx * (at(i + 1, j + 1) - at(i + 1, j))) / (ya[j + 1] - ya[j])
    return dx, dy


def lse(xs: torch.Tensor, gamma: float, dim: int = -1) -> torch.Tensor:
    """Eq. 4: y = c + gamma * log sum_i exp((x_i - c) / gamma), c = max_i x_i."""
    c = xs.max(dim=dim, keepdim=True).values
    c = torch.where(torch.isfinite(c), c, torch.zeros_like(c))
    return (c + gamma * torch.log(torch.exp((xs - c) / gamma).sum(dim=dim, keepdim=True))).squeeze(dim)


# --------------------------------------------------------------------------------------
# Forward propagation (Sec. 2.1 stage 3; Sec. 3.1.2; smoothed late AT from Sec. 3.2).
# --------------------------------------------------------------------------------------
class _Plan:
    """Per-level index lists built from the oracle's own levelization."""

    def __init__(self, d, lv: Levelization):
        P = d.n_pins
        self.L = lv.n_levels
        level = lv.level.astype(np.int64)
        kind = d.pin_kind
        off = d.net_offsets.astype(np.int64)
        cin = d.cell_in_offsets.astype(np.int64)
        self.max_fanin = int(np.max(np.diff(cin))) if d.n_cells else 1
        self.drv = []        # driver pins of the level's nets
        self.sinks = []      # sink pins of the level's nets
        self.sink_drv = []   # local driver index of each sink
        self.cells = []      # cell driving each net (-1 for PI nets)
        self.row = np.full(P, -1, np.int64)  # row of each pin in the level-ordered state
        start = 0
        for l in range(self.L):
            nets = np.nonzero(level == l)[0]
            drv = lv.driver[nets]
            sinks, sd = [], []
            for i, n in enumerate(nets):
                s = d.net_pins[off[n] + 1:off[n + 1]]
                sinks.append(s)
                sd.append(np.full(len(s), i, np.int64))
            sinks = np.concatenate(sinks).astype(np.int64) if sinks else np.zeros(0, np.int64)
            sd = np.concatenate(sd) if sd else np.zeros(0, np.int64)
            self.drv.append(drv)
            self.sinks.append(sinks)
            self.sink_drv.append(sd)
            self.cells.append(lv.cell_of_net[nets])
            self.row[drv] = start + np.arange(len(drv))
            self.row[sinks] = start + len(drv) + np.arange(len(sinks))
            start += len(drv) + len(sinks)
        # Padded input lists of each level's cells.
        self.in_pins, self.in_arc, self.in_unate, self.in_mask = [], [], [], []
        F = self.max_fanin
        for l in range(self.L):
            cells = self.cells[l]
            nc = len(cells)
            pins = np.zeros((nc, F), np.int64)
            arc = np.zeros((nc, F), np.int64)
            mask = np.zeros((nc, F), bool)
            if l > 0:
                for r_, c in enumerate(cells):
                    ins = d.cell_in_pins[cin[c]:cin[c + 1]]
                    a0 = d.lib.arc_offsets[d.cell_type[c]]
                    if len(ins) != d.lib.arc_offsets[d.cell_type[c] + 1] - a0:
                        raise ValueError("cell fanin does not match its type's arc count")
                    pins[r_, :len(ins)] = ins
                    arc[r_, :len(ins)] = a0 + np.arange(len(ins))
                    mask[r_, :len(ins)] = True
            self.in_pins.append(pins)
            self.in_arc.append(arc)
            self.in_unate.append(d.lib.arc_unate.astype(np.int64)[arc])
            self.in_mask.append(mask)
        self.endpoints = np.nonzero((kind == PIN_FF_D) | (kind == PIN_PO))[0]


def forward(d, lv: Levelization, x: torch.Tensor, y: torch.Tensor, gamma: float = 10.0,
            plan: _Plan | None = None, want_decisions: bool = False, perturb=None, base=None,
            start_level: int = 0):
    """Arrival time, slew and smoothed late arrival time for every pin.

    x, y: float64 tensors [P] by original pin id (may require grad).
    perturb: None (the default, exact float64), or a function applied to each wire delay,
    impulse and root load and to the result of each table lookup and of each propagated
    arrival, slew and smoothed arrival; the rounding experiments of oracle/sta_rounding.py
    use it.
    base, start_level: levels below start_level are taken from `base`, an earlier result of
    this function on the same design and plan, instead of being recomputed.  That is exact
    when x, y changed only in nets of level start_level or above (a net's coordinates reach
    its own level first), and is how finite differences avoid redoing the whole sweep.
    Returns dict with at[P,4], slew[P,4], atg[P,2] (torch, by original pin id),
    arc_delay[P,4] (numpy; delay of the arc entered at each cell-input pin, for each
    output condition k), the RC results, and the level-ordered state blocks.
    """
    plan = plan or _Plan(d, lv)
    pt = perturb or (lambda v: v)
    lib, cons = d.lib, d.cons
    xa = torch.from_numpy(lib.slew_axis.astype(np.float64))
    ya = torch.from_numpy(lib.load_axis.astype(np.float64))
    tables = torch.from_numpy(lib.tables.astype(np.float64))       # [arcs, 4, 7, 7]
    rcr = dict(rc(d, lv, x, y))
    for k in ("delay", "imp", "load_root"):
        rcr[k] = pt(rcr[k])
    delay, imp, load_root = rcr["delay"], rcr["imp"], rcr["load_root"]
    net_of_pin = torch.from_numpy(lv.net_of_pin)
    P = d.n_pins
    arc_delay = np.full((P, 4), np.nan) if base is None else base["arc_delay"].copy()
    decisions = []
    blocks = []           # level-ordered pin states [rows, 10]: at(4) slew(4) atg(2)
    for l in range(plan.L):
        if l < start_level:
            blocks.append(base["blocks"][l])
            continue
        drv = plan.drv[l]
        n_d = len(drv)
        if l == 0:
            st = torch.empty((n_d, 10), dtype=F64)
            st[:, 0:4] = cons.pi_at
            st[:, 4:8] = cons.pi_slew
            st[:, 8:10] = cons.pi_at
            drv_state = st
        else:
            prev = torch.cat(blocks)
            pins = plan.in_pins[l]
            mask = torch.from_numpy(plan.in_mask[l])
            rows = torch.from_numpy(np.where(plan.in_mask[l], plan.row[pins], 0))
            arc = torch.from_numpy(plan.in_arc[l])
            unate = plan.in_unate[l]
            src = prev[rows]                                       # [nc, F, 10]
            load_o = load_root[net_of_pin[torch.from_numpy(drv)]]  # [nc]
            cols = []
            late_delay = {}
            for k in range(4):
                m, t = k // 2, k % 2
                tp = np.where(unate > 0, t, 1 - t)                  # input transition t'
                kp = torch.from_numpy(2 * m + tp)
                at_in = torch.gather(src[:, :, 0:4], 2, kp.unsqueeze(-1)).squeeze(-1)
                slew_in = torch.gather(src[:, :, 4:8], 2, kp.unsqueeze(-1)).squeeze(-1)
                lo = load_o.unsqueeze(1).expand_as(slew_in)
                dval, di, dj = lut(tables[arc, t], xa, ya, slew_in, lo)
                sval, si, sj = lut(tables[arc, 2 + t], xa, ya, slew_in, lo)
                dval, sval = pt(dval), pt(sval)
                cand = pt(at_in + dval)
                big = torch.tensor(math.inf, dtype=F64)
                if m == 1:
                    at_o = torch.where(mask, cand, -big).max(dim=1).values
                    sm = torch.where(mask, sval, -big)
                    am = torch.argmax(sm, dim=1)                   # first max: ties to lowest arc
                    slew_o = torch.gather(sm, 1, am.unsqueeze(1)).squeeze(1)
                    atg_in = torch.gather(src[:, :, 8:10], 2, torch.from_numpy(tp).unsqueeze(-1)).squeeze(-1)
                    late_delay[t] = (pt(atg_in + dval), mask)
                    if want_decisions:
                        decisions.append(am.numpy().copy())
                else:
                    at_o = torch.where(mask, cand, big).min(dim=1).values
                    slew_o = torch.where(mask, sval, big).min(dim=1).values
                if want_decisions:
                    decisions += [di.numpy().copy(), dj.numpy().copy(), si.numpy().copy()]
                cols.append((at_o, slew_o))
                ad = dval.detach().numpy()
                pm = plan.in_mask[l]
                arc_delay[pins[pm], k] = ad[pm]
            atg_cols = []
            for t in range(2):
                vals, mask_t = late_delay[t]
                atg_cols.append(pt(lse(torch.where(mask_t, vals, torch.tensor(-math.inf, dtype=F64)), gamma, dim=1)))
            drv_state = torch.stack([c[0] for c in cols] + [c[1] for c in cols] + atg_cols, dim=1)
        # Net step: sinks take the driver's arrival plus the wire (R4 for the slew).
        sinks = torch.from_numpy(plan.sinks[l])
        sd = torch.from_numpy(plan.sink_drv[l])
        dsv = drv_state[sd]
        w = delay[sinks].unsqueeze(1)
        im = imp[sinks].unsqueeze(1)
        sink_state = torch.cat([pt(dsv[:, 0:4] + w), pt(torch.sqrt(dsv[:, 4:8] ** 2 + im ** 2)), pt(dsv[:, 8:10] + w)],
                               dim=1)
        blocks.append(torch.cat([drv_state, sink_state]))
    allst = torch.cat(blocks)
    rows = torch.from_numpy(plan.row)
    st = allst[rows]
    if want_decisions:
        # the sign of each wire segment's extent (to the driver, or to the parent pin of R13)
        pp = getattr(d, "pin_parent", None)
        ref = (torch.from_numpy(np.where(pp >= 0, pp, np.arange(P)).astype(np.int64)) if pp is not None
               else torch.from_numpy(lv.driver)[net_of_pin])
        decisions.append(np.sign((x - x[ref]).detach().numpy()))
        decisions.append(np.sign((y - y[ref]).detach().numpy()))
    return dict(at=st[:, 0:4], slew=st[:, 4:8], atg=st[:, 8:10], arc_delay=arc_delay, rc=rcr,
                plan=plan, decisions=decisions if want_decisions else None, blocks=blocks)


# --------------------------------------------------------------------------------------
# Backward propagation of required times and slack (Sec. 2.1 stage 4; Sec. 3.1.2).
# --------------------------------------------------------------------------------------
def backward(d, lv: Levelization, fwd, perturb=None) -> dict:
    """Required arrival time, slack, WNS and TNS (readings R8, R9). numpy float64.

    perturb: None (exact), or a function applied to each propagated required time (see
    forward)."""
    pt = perturb or (lambda v: v)
    plan = fwd["plan"]
    cons = d.cons
    P = d.n_pins
    at = fwd["at"].detach().numpy()
    delay = fwd["rc"]["delay"].detach().numpy()
    ad = fwd["arc_delay"]
    rat = np.empty((P, 4))
    rat[:, 0:2] = -np.inf
    rat[:, 2:4] = np.inf
    ep = plan.endpoints
    rat[ep, 0:2] = cons.hold
    rat[ep, 2:4] = cons.t_clk - cons.setup
    for l in range(plan.L - 1, -1, -1):
        drv, sinks, sd = plan.drv[l], plan.sinks[l], plan.sink_drv[l]
        # Net step: the driver needs its tightest sink, less the wire delay.
        req = pt(rat[sinks] - delay[sinks][:, None])
        rd = np.empty((len(drv), 4))
        rd[:, 0:2] = -np.inf
        rd[:, 2:4] = np.inf
        np.maximum.at(rd[:, 0:2], sd, req[:, 0:2])
        np.minimum.at(rd[:, 2:4], sd, req[:, 2:4])
        rat[drv] = rd
        if l == 0:
            continue
        # Cell step: each input's required time is the output's, less the arc delay.
        pins, mask, unate = plan.in_pins[l], plan.in_mask[l], plan.in_unate[l]
        for k in range(4):
            m, t = k // 2, k % 2
            tp = np.where(unate > 0, t, 1 - t)
            kp = 2 * m + tp
            val = pt(rat[drv, k][:, None] - ad[pins, k])
            rat[pins[mask], kp[mask]] = val[mask]
    slack = np.empty((P, 4))
    slack[:, 2:4] = rat[:, 2:4] - at[:, 2:4]
    slack[:, 0:2] = at[:, 0:2] - rat[:, 0:2]
    worst = np.minimum(slack[ep, 2], slack[ep, 3])
    wns = min(0.0, float(worst.min())) if len(ep) else 0.0
    tns = math.fsum(np.minimum(0.0, worst).tolist())
    return dict(rat=rat, slack=slack, wns=wns, tns=tns, endpoint_slack=worst, endpoints=ep)


# --------------------------------------------------------------------------------------
# Smoothed objective and its gradient (Sec. 3.2, Eq. 4; reading R10).
# --------------------------------------------------------------------------------------
def smoothed_objective(d, fwd, gamma: float) -> dict:
    ep = torch.from_numpy(fwd["plan"].endpoints)
    rat_late = d.cons.t_clk - d.cons.setup
    slack_g = rat_late - fwd["atg"][ep]                          # [E, 2]
    s = -lse(-slack_g, gamma, dim=1)                             # soft worst of rise/fall
    zeros = torch.zeros_like(s)
    tns_g = -lse(torch.stack([zeros, -s], dim=1), gamma, dim=1).sum()
    wns_g = -lse(torch.cat([torch.zeros(1, dtype=F64), -s]), gamma, dim=0)
    return dict(tns_g=tns_g, wns_g=wns_g, s=s)


def run(d, x=None, y=None, gamma: float = 10.0, grad: str | None = "tns", lv=None, plan=None, perturb=None):
    """Full oracle: forward, backward, smoothed objective and (optionally) its gradient.

    Returns numpy float64 arrays by original pin id.
    """
    lv = lv or levelize(d)
    xt = torch.tensor(np.asarray(d.x if x is None else x, np.float64), requires_grad=grad is not None)
    yt = torch.tensor(np.asarray(d.y if y is None else y, np.float64), requires_grad=grad is not None)
    fwd = forward(d, lv, xt, yt, gamma, plan=plan, perturb=perturb)
    bwd = backward(d, lv, fwd, perturb=perturb)
    obj = smoothed_objective(d, fwd, gamma)
    out = dict(at=fwd["at"].detach().numpy(), slew=fwd["slew"].detach().numpy(),
               atg=fwd["atg"].detach().numpy(), rat=bwd["rat"], slack=bwd["slack"],
               wns=bwd["wns"], tns=bwd["tns"], wns_g=float(obj["wns_g"].detach()), tns_g=float(obj["tns_g"].detach()),
               delay=fwd["rc"]["delay"].detach().numpy(), imp=fwd["rc"]["imp"].detach().numpy(),
               load_root=fwd["rc"]["load_root"].detach().numpy(), arc_delay=fwd["arc_delay"],
               endpoints=bwd["endpoints"], endpoint_slack=bwd["endpoint_slack"], lv=lv, plan=fwd["plan"])
    if grad is not None:
        target = obj["tns_g"] if grad == "tns" else obj["wns_g"]
        gx, gy = torch.autograd.grad(target, (xt, yt), allow_unused=True)
        out["dx"] = np.zeros(d.n_pins) if gx is None else gx.numpy()
        out["dy"] = np.zeros(d.n_pins) if gy is None else gy.numpy()
    return out


def objective_at(d, lv, plan, x: np.ndarray, y: np.ndarray, gamma: float, which: str = "tns"):
    """Smoothed objective value and decision fingerprint at the given coordinates (for FD)."""
    with torch.no_grad():
        fwd = forward(d, lv, torch.from_numpy(x), torch.from_numpy(y), gamma, plan=plan, want_decisions=True)
        obj = smoothed_objective(d, fwd, gamma)
    val = float(obj["tns_g"] if which == "tns" else obj["wns_g"])
    return val, fwd["decisions"]
