"""Hand-built and tiny designs for the tests (inputs only, no timing arithmetic)."""
from __future__ import annotations

import numpy as np

from gen.netlist import (Constraints, Design, Library, Spec, PIN_PI, PIN_CELL_IN, PIN_CELL_OUT,
                         PIN_FF_D, PIN_PO, make_library)


def build(nets, cells, kinds, caps, x, y, lib: Library | None = None, cons: Constraints | None = None,
          name: str = "hand") -> Design:
    """nets: list of pin lists (driver first); cells: list of (type, [input pins], output pin)."""
    lib = lib or make_library()
    cons = cons or Constraints()
    P = len(kinds)
    off = np.zeros(len(nets) + 1, np.int32)
    off[1:] = np.cumsum([len(n) for n in nets])
    net_pins = np.array([p for n in nets for p in n], np.int32)
    cin = np.zeros(len(cells) + 1, np.int32)
    cin[1:] = np.cumsum([len(c[1]) for c in cells])
    spec = Spec(name, 900, len(cells), sum(1 for k in kinds if k == PIN_PI), 1, 0, "geom", 1.0)
    return Design(spec, P, len(nets), len(cells), off, net_pins,
                  np.array([c[0] for c in cells], np.int32), cin,
                  np.array([p for c in cells for p in c[1]], np.int32),
                  np.array([c[2] for c in cells], np.int32),
                  np.asarray(caps, np.float32), np.asarray(kinds, np.int8),
                  np.asarray(x, np.float32), np.asarray(y, np.float32), lib, cons,
                  np.zeros(len(nets), np.int32), {})


def planar_library(seed: int = 0) -> Library:
    """The default library shape with planar tables a + b*slew + c*load, exact in float32.

    Axes are small integers and a, b, c are dyadic, so every table entry is stored
    without rounding and bilinear interpolation reproduces the plane exactly.
    """
    lib = make_library(seed_stream=seed, planar=True)
    rng = np.random.default_rng([seed, 17])
    xa = np.array([5, 10, 20, 50, 100, 200, 500], np.float64)
    ya = np.array([1, 2, 5, 10, 20, 50, 200], np.float64)
    tabs = np.empty_like(lib.tables, dtype=np.float64)
    for a in range(tabs.shape[0]):
        for t in range(4):
            ca = rng.integers(8, 64) / 2.0
            cb = rng.integers(1, 20) / 64.0
            cc = rng.integers(8, 64) / 64.0
            tabs[a, t] = ca + cb * xa[:, None] + cc * ya[None, :]
    assert np.array_equal(tabs.astype(np.float32).astype(np.float64), tabs)
    return Library(lib.n_cell_types, lib.arc_offsets, lib.arc_unate, xa.astype(np.float32),
                   ya.astype(np.float32), tabs.astype(np.float32))


def two_pin(L_um: float = 120.0, cpin: float = 3.0, lib=None, cons=None) -> Design:
    """PI pin 0 drives a 2-pin net whose sink (pin 1) is a primary output."""
    return build([[0, 1]], [], [PIN_PI, PIN_PO], [0.0, cpin], [0.0, L_um * 0.25], [0.0, L_um * 0.75],
                 lib=lib, cons=cons, name="two_pin")


def chain(n_gates: int, types, lib, L_um: float = 80.0, cpin: float = 2.0) -> Design:
    """PI -> gate_1 -> ... -> gate_n -> PO; every net has one sink at distance L_um."""
    kinds, caps, xs, ys, nets, cells = [], [], [], [], [], []

    def pin(kind, cap, x):
        kinds.append(kind)
        caps.append(cap)
        xs.append(x)
        ys.append(0.0)
        return len(kinds) - 1

    drv = pin(PIN_PI, 0.0, 0.0)
    pos = 0.0
    for g in range(n_gates):
        pos += L_um
        sink = pin(PIN_CELL_IN, cpin, pos)
        nets.append([drv, sink])
        out = pin(PIN_CELL_OUT, 0.0, pos)
        cells.append((types[g], [sink], out))
        drv = out
    pos += L_um
    po = pin(PIN_PO, cpin, pos)
    nets.append([drv, po])
    return build(nets, cells, kinds, caps, xs, ys, lib=lib, name="chain")


__all__ = ["build", "planar_library", "two_pin", "chain", "PIN_PI", "PIN_CELL_IN", "PIN_CELL_OUT",
           "PIN_FF_D", "PIN_PO"]


def wide_library(seed: int = 0) -> Library:
    """The default library plus two cell types of each fanin 5..8 (arcs appended)."""
    base = make_library(seed_stream=seed)
    rng = np.random.default_rng([seed, 23])
    fanins = [5, 5, 6, 6, 7, 7, 8, 8]
    n_new = sum(fanins)
    off = list(base.arc_offsets)
    for f in fanins:
        off.append(off[-1] + f)
    S = base.slew_axis.astype(np.float64)[:, None]
    Ld = base.load_axis.astype(np.float64)[None, :]
    tabs = np.empty((n_new, 4) + base.tables.shape[2:], np.float64)
    for a in range(n_new):
        for t in range(4):
            if t < 2:
                ca, cb, cc = rng.uniform(10, 30), rng.uniform(0.05, 0.3), rng.uniform(0.2, 1.0)
            else:
                ca, cb, cc = rng.uniform(3, 10), rng.uniform(0.02, 0.15), rng.uniform(0.5, 2.0)
            tabs[a, t] = ca + cb * S + cc * Ld + rng.normal(0.0, 0.5, S.shape[:1] + Ld.shape[1:])
    unate = np.concatenate([base.arc_unate, np.where(rng.random(n_new) < 0.5, 1, -1).astype(np.int8)])
    return Library(base.n_cell_types + len(fanins), np.array(off, np.int32), unate, base.slew_axis,
                   base.load_axis, np.concatenate([base.tables, tabs.astype(np.float32)]))


def wide_dag(n_levels: int = 8, gates_per_level: int = 40, n_pi: int = 12, seed: int = 0,
             box_um: float = 300.0) -> Design:
    """A random levelized DAG whose gates have 1-8 inputs (most 5-8), on wide_library()."""
    lib = wide_library(seed)
    rng = np.random.default_rng([seed, 31])
    fan_of_type = np.diff(lib.arc_offsets)
    kinds, nets, cells, levels = [], [], [], []

    def pin(kind):
        kinds.append(kind)
        return len(kinds) - 1

    for _ in range(n_pi):
        nets.append([pin(PIN_PI)])
        levels.append(0)
    for lv in range(1, n_levels + 1):
        prev = [i for i, l in enumerate(levels) if l == lv - 1]
        older = [i for i, l in enumerate(levels) if l < lv]
        for _ in range(gates_per_level):
            f = int(rng.choice([1, 2, 3, 4, 5, 6, 7, 8], p=[.05, .05, .05, .05, .2, .2, .2, .2]))
            f = min(f, len(older))
            typ = int(rng.choice(np.nonzero(fan_of_type == f)[0]))
            srcs = [int(rng.choice(prev))]
            rest = [n for n in older if n != srcs[0]]
            srcs += [int(v) for v in rng.choice(rest, size=f - 1, replace=False)] if f > 1 else []
            ins = []
            for n in srcs:
                p = pin(PIN_CELL_IN)
                nets[n].append(p)
                ins.append(p)
            out = pin(PIN_CELL_OUT)
            cells.append((typ, ins, out))
            nets.append([out])
            levels.append(lv)
    for n in nets:
        if len(n) == 1 or rng.random() < 0.2:
            n.append(pin(PIN_PO if rng.random() < 0.5 else PIN_FF_D))
    P = len(kinds)
    caps = np.where(np.asarray(kinds) == PIN_CELL_OUT, 0.0, rng.uniform(1, 5, P))
    caps = np.where(np.asarray(kinds) == PIN_PI, 0.0, caps)
    return build(nets, cells, kinds, caps, rng.uniform(0, box_um, P), rng.uniform(0, box_um, P),
                 lib=lib, name="wide")


def fanout_design(n_sinks=1300, n_buf=100, seed=3, via_cell=False):
    """A primary input driving one net of n_sinks sinks (n_buf of them 1-input cells whose
    outputs each drive a flop), placed at random: a net too big for one LDS chunk.  With
    via_cell the big net is driven by a 1-input cell fed by the primary input (the big net
    then sits at level 1, behind a cell step)."""
    lib = make_library()
    one_in = int(np.nonzero(np.diff(lib.arc_offsets) == 1)[0][0])
    rng = np.random.default_rng(seed)
    if via_cell:
        kinds, nets, cells = [PIN_PI, PIN_CELL_IN, PIN_CELL_OUT], [[0, 1], [2]], [(one_in, [1], 2)]
    else:
        kinds, nets, cells = [PIN_PI], [[0]], []
    big = nets[-1]
    for i in range(n_sinks):
        p = len(kinds)
        big.append(p)
        if i < n_buf:
            kinds += [PIN_CELL_IN, PIN_CELL_OUT, PIN_FF_D]
            cells.append((one_in, [p], p + 1))
            nets.append([p + 1, p + 2])
        else:
            kinds.append(PIN_PO)
    P = len(kinds)
    caps = np.where(np.isin(kinds, [PIN_PI, PIN_CELL_OUT]), 0.0, rng.uniform(1, 5, P)) if via_cell \
        else rng.uniform(1, 5, P)
    return build(nets, cells, kinds, caps, rng.uniform(0, 3000, P), rng.uniform(0, 3000, P), lib=lib)
