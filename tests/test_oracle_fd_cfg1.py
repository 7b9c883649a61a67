"""The oracle's gradient at the 0.8M-pin workload's scale against central finite differences.

The smaller pins (tests/test_oracle_pins.py) check the gradient on a 4k-pin design in a
200 um box, where loads stay near the tables' range.  Here it is the 806k-pin design in a
2000 um box: root loads reach 1e5 fF, 500x past the last table column, so almost every
lookup extrapolates, and arrival times reach 1e5-1e6 ps.  100 seeded pins, both axes,
h = 1e-3 um, double precision throughout, the two sides' difference summed over endpoints
term by term (the total is too large to difference directly).  Tolerance 1e-4 |g| + 1e-3
ps/um plus the stencil's own rounding noise, from the first-order rounding bound of
oracle/sta_rounding.py: a pin near the inputs reaches tens of thousands of endpoint terms of
1e6-1e7 ps through chains of extrapolated tables whose slew gain exceeds 1, and their
double rounding over 2h can exceed the 1e-3 ps/um floor (moving h shows it: the central
difference of such a pin swings by +-1 ps/um at h = 1e-3 um and by +-20 at 2.5e-4, around
the analytic value).  The test prints how many stencils need that term.  A stencil whose two sides fall in different
table cells, pick a different slew arg max or flip the sign of a wire extent is not smooth
there and is skipped.  Each side recomputes only the levels from the pin's own net up: the
levels below cannot see the move (a net's coordinates reach its own level first).
"""
from __future__ import annotations

import math
import multiprocessing as mp
import os

import numpy as np
import pytest
import torch

from gen.netlist import CFG1, make_design
from oracle import sta_oracle as O
from oracle import sta_rounding as RB

GAMMA = 10.0
H = 1e-3
N_PINS = 100

_W = {}


def _init(sigma_ep):
    torch.set_num_threads(1)
    _W["sigma_ep"] = sigma_ep
    d = make_design(CFG1)
    lv = O.levelize(d)
    plan = O._Plan(d, lv)
    x = d.x.astype(np.float64)
    y = d.y.astype(np.float64)
    with torch.no_grad():
        base = O.forward(d, lv, torch.from_numpy(x), torch.from_numpy(y), GAMMA, plan=plan)
    _W.update(d=d, lv=lv, plan=plan, x=x, y=y, base=base)


def _objective_terms(x, y, start):
    """Each endpoint's term of TNS_g, -LSE(0, -s_e), and the decision fingerprint."""
    w = _W
    with torch.no_grad():
        f = O.forward(w["d"], w["lv"], torch.from_numpy(x), torch.from_numpy(y), GAMMA, plan=w["plan"],
                      want_decisions=True, base=w["base"], start_level=start)
        s = O.smoothed_objective(w["d"], f, GAMMA)["s"]
        terms = -O.lse(torch.stack([torch.zeros_like(s), -s], dim=1), GAMMA, dim=1)
    return terms.numpy(), f["decisions"]


def _stencil(task):
    p, axis = task
    w = _W
    start = int(w["lv"].level[w["lv"].net_of_pin[p]])
    xp, yp, xm, ym = w["x"].copy(), w["y"].copy(), w["x"].copy(), w["y"].copy()
    (xp if axis == 0 else yp)[p] += H
    (xm if axis == 0 else ym)[p] -= H
    tp, dp = _objective_terms(xp, yp, start)
    tm, dm = _objective_terms(xm, ym, start)
    smooth = len(dp) == len(dm) and all(np.array_equal(a, b) for a, b in zip(dp, dm))
    # The difference of the sums, taken term by term: TNS_g is about -3e11 ps here, whose
    # double-precision spacing (6e-5 ps) over 2h would alone be 0.03 ps/um of noise.  Each
    # term that moved still carries the rounding of its whole fan-in cone, at most
    # u * sigma of its endpoint's smoothed arrivals (u = 2^-53; a term's partials in them
    # are at most 1) plus its own, in each of the two sides: that is the stencil's noise.
    moved = tp != tm
    noise = 2 * 2.0 ** -53 * float((w["sigma_ep"][moved] + np.abs(tp[moved])).sum()) / (2 * H)
    return p, axis, math.fsum(tp - tm) / (2 * H), smooth, noise


@pytest.mark.slow
def test_gradient_matches_central_differences_at_0p8m_pins():
    d = make_design(CFG1)
    rng = np.random.default_rng([260328381, 1, 9001])
    pins = rng.choice(d.n_pins, N_PINS, replace=False)
    tasks = [(int(p), a) for p in pins for a in (0, 1)]
    ref = O.run(d, gamma=GAMMA, grad="tns")
    # first-order rounding bound of every endpoint's smoothed arrivals (both transitions)
    sigma_ep = RB.rounding_scales(d, ref)["atg_scale"][ref["plan"].endpoints].sum(axis=1)
    workers = max(1, min(8, len(os.sched_getaffinity(0))))
    with mp.get_context("spawn").Pool(workers, initializer=_init, initargs=(sigma_ep,)) as pool:
        fd = pool.map(_stencil, tasks, chunksize=1)
    checked, worst, noisy = 0, 0.0, 0
    for p, axis, v, smooth, noise in fd:
        if not smooth:
            continue
        an = ref["dx" if axis == 0 else "dy"][p]
        base = 1e-4 * abs(an) + 1e-3
        tol = base + noise
        worst = max(worst, abs(v - an) / tol)
        noisy += abs(v - an) > base
        assert abs(v - an) <= tol, (p, axis, v, an, noise)
        checked += 1
    ok = [(p, a, v, n) for p, a, v, s, n in fd if s]
    mags = np.abs([ref["dx" if a == 0 else "dy"][p] for p, a, _, _ in ok])
    rel = [abs(v - ref["dx" if a == 0 else "dy"][p]) / max(abs(ref["dx" if a == 0 else "dy"][p]), 1e-300)
           for p, a, v, _ in ok]
    print(f"{checked} of {len(tasks)} stencils smooth; |g| from {mags.min():.3g} to {mags.max():.3g} ps/um; "
          f"median relative error {np.median(rel):.3g}; {noisy} need the stencil's rounding noise "
          f"(largest {max(n for *_, n in ok):.3g} ps/um); worst {worst:.3g}x the tolerance")
    assert checked >= 150
    assert np.median(rel) <= 1e-5
