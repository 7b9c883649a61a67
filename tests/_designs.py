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
