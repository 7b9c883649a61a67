"""Seeded synthetic netlists, NLDM libraries and placements for the levelized STA sweep.

This module draws inputs only: graph topology, cell types, pin capacitances, pin
coordinates, table values and constraints.  It computes no timing quantity (no
wire delay, no table lookup, no arrival or required time); both the FP64 oracle
and the GPU library take its arrays as given.

Workload shapes follow the paper's benchmark statistics (Table 1: superblue
designs with roughly 3 pins per net and up to 6.4M pins) and the synthetic
configurations of this project:

* ``CFG0``  1,000 gates with 1-4 inputs, 64 primary inputs, 64 flop endpoints,
  12 gate levels, fanout ``min(16, Geometric(0.4))`` (mean 2.5), 200 um box.
* ``CFG1``  200k gates, 2k primary inputs, 60 gate levels, heavy-tailed nets
  (70 % of nets have 2-3 pins, the rest Pareto alpha 1.5 up to 500 pins), 2000 um box.
* ``CFG2``  650k gates, 6.5k primary inputs, 90 gate levels, same net-size law,
  about 2.5M pins, 6000 um box (the size of superblue4, 2,497,940 pins).
* ``scaled_spec(P)``  designs of roughly ``P`` pins for batched and served runs.

Every array is produced from ``numpy.random.default_rng([260328381, cfg, stream])``.
Original pin, net and cell ids are random permutations, so the canonical
(levelized) order a timer builds is never the input order.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import math

import numpy as np

SEED_ROOT = 260328381

PIN_PI, PIN_CELL_IN, PIN_CELL_OUT, PIN_FF_D, PIN_PO = 0, 1, 2, 3, 4

LUT_N = 7
TYPES_PER_FANIN = 8


@dataclass(frozen=True)
class Spec:
    """Shape of one synthetic design."""

    name: str
    cfg_id: int
    n_gates: int
    n_pi: int
    n_levels: int          # gate levels; net levels run 0..n_levels
    n_ff: int              # flop (FF_D) endpoints; other leftover sinks become POs
    fanout: str            # "geom" or "mix"
    box_um: float
    geom_p: float = 0.4
    geom_cap: int = 16
    mix_p23: float = 0.7
    mix_alpha: float = 1.5
    mix_xm: float = 2.5
    mix_cap: int = 500     # max pins per net (driver included)
    fanin_max: int = 4
    back_q: float = 0.5    # geometric law of the level distance of non-critical inputs


CFG0 = Spec("cfg0", 0, 1000, 64, 12, 64, "geom", 200.0)
CFG1 = Spec("cfg1", 1, 200_000, 2000, 60, 2000, "mix", 2000.0, mix_xm=2.50)
CFG2 = Spec("cfg2", 2, 650_000, 6500, 90, 6500, "mix", 6000.0, mix_xm=2.24)


def scaled_spec(n_pins: int, cfg_id: int, box_um: float = 2000.0, name: str | None = None) -> Spec:
    """A design of roughly ``n_pins`` pins with the CFG1 net-size law.

    Gates = P / 3.85; gate levels = round(12 * (P / 4000) ** 0.31), which gives
    about 62 levels at 800k pins and 88 at 2.5M pins.
    """
    gates = max(16, int(round(n_pins / 3.85)))
    levels = max(2, int(round(12.0 * (n_pins / 4000.0) ** 0.31)))
    levels = min(levels, gates)
    pis = max(8, gates // 100)
    return Spec(name or f"p{n_pins}", cfg_id, gates, pis, levels, pis, "mix", box_um, mix_xm=2.50)


@dataclass
class Library:
    n_cell_types: int
    arc_offsets: np.ndarray   # int32 [T+1]
    arc_unate: np.ndarray     # int8 [n_arcs], +1 / -1
    slew_axis: np.ndarray     # float32 [7] ps
    load_axis: np.ndarray     # float32 [7] fF
    tables: np.ndarray        # float32 [n_arcs, 4, 7, 7]: delay-r, delay-f, slew-r, slew-f; [slew][load]

    @property
    def n_arcs(self) -> int:
        return int(self.arc_offsets[-1])


@dataclass
class Constraints:
    t_clk: float = 1000.0
    setup: float = 0.0
    hold: float = 0.0
    pi_at: float = 0.0
    pi_slew: float = 10.0
    r_per_um: float = 0.1
    c_per_um: float = 0.2


@dataclass
class Design:
    spec: Spec
    n_pins: int
    n_nets: int
    n_cells: int
    net_offsets: np.ndarray      # int32 [N+1]
    net_pins: np.ndarray         # int32 [P], driver first in each net
    cell_type: np.ndarray        # int32 [C]
    cell_in_offsets: np.ndarray  # int32 [C+1]
    cell_in_pins: np.ndarray     # int32 [A]
    cell_out_pin: np.ndarray     # int32 [C]
    pin_cap: np.ndarray          # float32 [P] fF
    pin_kind: np.ndarray         # int8 [P]
    x: np.ndarray                # float32 [P] um
    y: np.ndarray                # float32 [P] um
    lib: Library
    cons: Constraints
    gen_net_level: np.ndarray    # int32 [N], level the generator built each (original) net at
    stats: dict = field(default_factory=dict)
    pin_parent: np.ndarray | None = None   # int32 [P]: RC tree parent pin (-1 at drivers); None: stars

    @property
    def n_arcs(self) -> int:
        return int(self.cell_in_offsets[-1])


def _rng(cfg_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([SEED_ROOT, int(cfg_id), int(stream)])


def make_library(seed_stream: int = 0, noise_ps: float = 0.5, planar: bool = False) -> Library:
    """32 cell types (8 per fanin 1..4), one arc per input: 80 arcs.

    Table entries are ``a + b*slew + c*load + N(0, noise_ps)`` on 7-point
    log-spaced axes (slew 5..500 ps, load 1..200 fF); delay uses a in U[10,30],
    b in U[0.05,0.3], c in U[0.2,1.0]; slew uses a in U[3,10], b in U[0.02,0.15],
    c in U[0.5,2].  ``planar=True`` drops the noise.  Unateness is +1/-1 at random.
    """
    rng = _rng(99, seed_stream)
    n_types = 4 * TYPES_PER_FANIN
    fanin = np.repeat(np.arange(1, 5), TYPES_PER_FANIN)
    arc_offsets = np.zeros(n_types + 1, np.int32)
    arc_offsets[1:] = np.cumsum(fanin)
    n_arcs = int(arc_offsets[-1])
    slew_axis = np.geomspace(5.0, 500.0, LUT_N).astype(np.float32)
    load_axis = np.geomspace(1.0, 200.0, LUT_N).astype(np.float32)
    unate = np.where(rng.random(n_arcs) < 0.5, 1, -1).astype(np.int8)
    S = slew_axis.astype(np.float64)[:, None]
    Ld = load_axis.astype(np.float64)[None, :]
    tables = np.empty((n_arcs, 4, LUT_N, LUT_N), np.float64)
    for a in range(n_arcs):
        for t in range(4):
            if t < 2:
                ca, cb, cc = rng.uniform(10, 30), rng.uniform(0.05, 0.3), rng.uniform(0.2, 1.0)
            else:
                ca, cb, cc = rng.uniform(3, 10), rng.uniform(0.02, 0.15), rng.uniform(0.5, 2.0)
            noise = 0.0 if planar else rng.normal(0.0, noise_ps, (LUT_N, LUT_N))
            tables[a, t] = ca + cb * S + cc * Ld + noise
    return Library(n_types, arc_offsets, unate, slew_axis, load_axis, tables.astype(np.float32))


def _draw_fanout(spec: Spec, rng: np.random.Generator, n: int) -> np.ndarray:
    if spec.fanout == "geom":
        return np.minimum(spec.geom_cap, rng.geometric(spec.geom_p, n)).astype(np.int64)
    u = rng.random(n)
    small = rng.integers(2, 4, n)
    tail = np.floor(spec.mix_xm * rng.random(n) ** (-1.0 / spec.mix_alpha))
    tail = np.clip(tail, 4, spec.mix_cap)
    pins = np.where(u < spec.mix_p23, small, tail).astype(np.int64)
    return pins - 1


class _Pools:
    """Per-level pools of free fanout slots (a net id repeated once per slot)."""

    def __init__(self, rng, nets_by_level, fan):
        self.rng = rng
        self.nets_by_level = nets_by_level
        self.pool = []
        self.ptr = []
        for nets in nets_by_level:
            arr = np.repeat(nets, fan[nets])
            rng.shuffle(arr)
            self.pool.append(arr)
            self.ptr.append(0)
        self.extra = 0

    def take(self, level: int, n: int) -> np.ndarray:
        if n <= 0:
            return np.zeros(0, np.int64)
        p = self.ptr[level]
        avail = len(self.pool[level]) - p
        got = self.pool[level][p:p + min(n, avail)]
        self.ptr[level] = p + len(got)
        if len(got) < n:
            # Not enough free slots at this level: widen random nets of the level.
            more = self.rng.choice(self.nets_by_level[level], n - len(got))
            self.extra += n - len(got)
            got = np.concatenate([got, more])
        return got

    def leftovers(self) -> np.ndarray:
        return np.concatenate([pool[p:] for pool, p in zip(self.pool, self.ptr)])


def make_design(spec: Spec, stream: int = 0, lib: Library | None = None,
                cons: Constraints | None = None) -> Design:
    """Draw one design for ``spec`` (see module docstring for the recipe)."""
    rng = _rng(spec.cfg_id, stream)
    lib = lib or make_library()
    cons = cons or Constraints()
    G, L, n_pi = spec.n_gates, spec.n_levels, spec.n_pi
    if G < L:
        raise ValueError("need at least one gate per level")
    N = n_pi + G

    # Gates per level: as even as possible, remainder on random levels.
    per = np.full(L, G // L, np.int64)
    per[rng.choice(L, G % L, replace=False)] += 1
    gate_level = np.repeat(np.arange(1, L + 1), per)          # gates in level order
    net_level = np.concatenate([np.zeros(n_pi, np.int64), gate_level])
    level_start = np.concatenate([[0], np.cumsum(per)])        # gate index ranges
    nets_by_level = [np.arange(n_pi)] + [n_pi + np.arange(level_start[l], level_start[l + 1])
                                         for l in range(L)]

    fanin = rng.integers(1, spec.fanin_max + 1, G)
    fan = _draw_fanout(spec, rng, N)
    pools = _Pools(rng, nets_by_level, fan)

    in_off = np.zeros(G + 1, np.int64)
    in_off[1:] = np.cumsum(fanin)
    A = int(in_off[-1])
    in_src = np.empty(A, np.int64)
    for l in range(1, L + 1):
        g0, g1 = level_start[l - 1], level_start[l]
        k = fanin[g0:g1]
        first = in_off[g0:g1]
        # Input 0 of every gate comes from the level just below: levels are exact.
        in_src[first] = pools.take(l - 1, g1 - g0)
        # Other inputs: a level distance drawn from Geometric(back_q).
        n_other = int(k.sum() - (g1 - g0))
        if n_other:
            rep_gate = np.repeat(np.arange(g0, g1), k - 1)
            within = np.arange(n_other) - np.repeat(np.cumsum(k - 1) - (k - 1), k - 1)
            pos = in_off[rep_gate] + 1 + within
            tl = np.maximum(0, l - rng.geometric(spec.back_q, n_other))
            src = np.empty(n_other, np.int64)
            for t in np.unique(tl):
                m = tl == t
                src[m] = pools.take(int(t), int(m.sum()))
            in_src[pos] = src
    # Shuffle input order inside each gate, so the level-defining input is not always input 0.
    key = rng.random(A) + np.repeat(np.arange(G), fanin) * 2.0
    in_src = in_src[np.argsort(key, kind="stable")]

    # Free slots left over become endpoint sinks; exactly n_ff of them are flops.
    ep_net = pools.leftovers()
    if len(ep_net) < spec.n_ff:
        add = rng.choice(nets_by_level[L], spec.n_ff - len(ep_net))
        ep_net = np.concatenate([ep_net, add])
    ep_kind = np.full(len(ep_net), PIN_PO, np.int8)
    ep_kind[rng.choice(len(ep_net), spec.n_ff, replace=False)] = PIN_FF_D
    Ep = len(ep_net)

    # Pin records: drivers, cell inputs, endpoints.
    P = N + A + Ep
    rec_net = np.concatenate([np.arange(N), in_src, ep_net])
    rec_kind = np.concatenate([
        np.where(np.arange(N) < n_pi, PIN_PI, PIN_CELL_OUT).astype(np.int8),
        np.full(A, PIN_CELL_IN, np.int8),
        ep_kind,
    ])
    rec_is_sink = np.concatenate([np.zeros(N, bool), np.ones(A + Ep, bool)])
    pin_id = rng.permutation(P).astype(np.int64)              # original pin id of each record
    net_orig = rng.permutation(N).astype(np.int64)            # original net id of each generated net
    order = np.lexsort((rng.random(P), rec_is_sink, net_orig[rec_net]))
    net_pins = pin_id[order].astype(np.int32)
    counts = np.bincount(net_orig[rec_net], minlength=N)
    net_offsets = np.zeros(N + 1, np.int64)
    net_offsets[1:] = np.cumsum(counts)

    cell_orig = rng.permutation(G).astype(np.int64)           # original cell id of each gate
    inv_cell = np.argsort(cell_orig)                          # gate of each original cell
    ctype_gate = (fanin - 1) * TYPES_PER_FANIN + rng.integers(0, TYPES_PER_FANIN, G)
    cell_type = ctype_gate[inv_cell].astype(np.int32)
    fanin_c = fanin[inv_cell]
    cin_off = np.zeros(G + 1, np.int64)
    cin_off[1:] = np.cumsum(fanin_c)
    # Cell-input records are rec index N + (gate input slot).
    gate_of_slot = inv_cell.repeat(fanin_c)
    within = np.arange(A) - np.repeat(cin_off[:-1], fanin_c)
    slot = in_off[gate_of_slot] + within
    cell_in_pins = pin_id[N + slot].astype(np.int32)
    cell_out_pin = pin_id[n_pi + inv_cell].astype(np.int32)

    pin_kind = np.empty(P, np.int8)
    pin_kind[pin_id] = rec_kind
    pin_cap = np.zeros(P, np.float32)
    sink_pins = pin_id[N:]
    pin_cap[sink_pins] = rng.uniform(1.0, 5.0, A + Ep).astype(np.float32)
    x = rng.uniform(0.0, spec.box_um, P).astype(np.float32)
    y = rng.uniform(0.0, spec.box_um, P).astype(np.float32)

    gen_level = np.empty(N, np.int32)
    gen_level[net_orig] = net_level

    stats = dict(pins=P, nets=N, cells=G, arcs=A, endpoints=Ep,
                 ff=int(spec.n_ff), po=int(Ep - spec.n_ff), net_levels=L + 1,
                 extra_slots=int(pools.extra), mean_pins_per_net=P / N,
                 max_pins_per_net=int(counts.max()))
    return Design(spec, P, N, G, net_offsets.astype(np.int32), net_pins, cell_type,
                  cin_off.astype(np.int32), cell_in_pins, cell_out_pin, pin_cap, pin_kind,
                  x, y, lib, cons, gen_level, stats)


def jitter(d: Design, sigma_um: float, stream: int) -> tuple[np.ndarray, np.ndarray]:
    """Coordinates of one placement snapshot: x, y plus seeded N(0, sigma) noise."""
    rng = _rng(1000 + d.spec.cfg_id, stream)
    dx = rng.normal(0.0, sigma_um, d.n_pins)
    dy = rng.normal(0.0, sigma_um, d.n_pins)
    return (d.x + dx).astype(np.float32), (d.y + dy).astype(np.float32)


def batch_designs(n_designs: int = 16, lo: int = 10_000, hi: int = 400_000,
                  cfg_id: int = 3) -> list[Design]:
    """Designs with pin counts drawn log-uniform in [lo, hi]."""
    rng = _rng(cfg_id, 10_000)
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), n_designs)).astype(np.int64)
    return [make_design(scaled_spec(int(p), cfg_id * 100 + i), stream=0) for i, p in enumerate(sizes)]


def tiny_spec(n_gates: int, n_levels: int, n_pi: int = 4, seed: int = 0, box_um: float = 50.0,
              fanout_p: float = 0.5, fanout_cap: int = 4) -> Spec:
    """Small designs for brute-force checks (a few gates, a few levels)."""
    return Spec(f"tiny{seed}", 500 + seed, n_gates, n_pi, n_levels, min(2, n_pi), "geom",
                box_um, geom_p=fanout_p, geom_cap=fanout_cap)


def heap_trees(d: Design) -> Design:
    """The same design with an RC tree on every net instead of a star.

    Per net, the driver and then the sinks sorted by Manhattan distance from the driver
    (ties in net order) fill a binary heap: the k-th pin of that order hangs off the
    (k - 1) // 2-th, so trees branch in two and are about log2(pins) deep.
    """
    off = d.net_offsets.astype(np.int64)
    pins = d.net_pins.astype(np.int64)
    cnt = np.diff(off)
    net = np.repeat(np.arange(d.n_nets), cnt)
    pos = np.arange(len(pins)) - off[net]
    drv = pins[off[:-1]][net]
    x, y = d.x.astype(np.float64), d.y.astype(np.float64)
    dist = np.abs(x[pins] - x[drv]) + np.abs(y[pins] - y[drv])
    dist[pos == 0] = -1.0                       # the driver first
    order = np.lexsort((pos, dist, net))
    sp, sn = pins[order], net[order]
    rank = np.arange(len(pins)) - off[sn]
    sink = rank >= 1
    parent = np.full(d.n_pins, -1, np.int64)
    parent[sp[sink]] = sp[off[sn[sink]] + (rank[sink] - 1) // 2]
    return replace(d, pin_parent=parent.astype(np.int32))
