"""Pins of the FP64 oracle against closed forms, library routines, brute force and invariants.

None of these re-types an oracle formula: each checks the oracle against something
fixed independently of it (a closed form of the Elmore model, scipy's grid
interpolator and logsumexp, explicit enumeration of every path, finite differences,
or an invariant of the timing graph).
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch
from scipy.interpolate import RegularGridInterpolator
from scipy.special import logsumexp

from gen.netlist import CFG0, Constraints, make_design, make_library, tiny_spec
from oracle import sta_oracle as O
from oracle import sta_rounding as RB
from tests._designs import (PIN_CELL_IN, PIN_CELL_OUT, PIN_FF_D, PIN_PI, PIN_PO, build, chain,
                            planar_library, two_pin)

R, C = 0.1, 0.2


# ----------------------------------------------------------------------------- RC (Eq. 1-3)
@pytest.mark.parametrize("L_um,cpin", [(0.0, 2.0), (1.0, 1.0), (120.0, 3.0), (4321.5, 4.5)])
def test_two_pin_elmore_closed_form(L_um, cpin):
    # Distributed line driving a lumped load: t = r*c*L^2/2 + r*L*C_L (ohm*fF = 1e-3 ps).
    d = two_pin(L_um, cpin)
    out = O.run(d, grad=None)
    want = 1e-3 * (R * C * L_um ** 2 / 2 + R * L_um * cpin)
    assert out["delay"][1] == pytest.approx(want, rel=1e-12, abs=1e-15)
    # Eq. 1 at the root: the driver sees the whole wire plus the sink pin.
    assert out["load_root"][0] == pytest.approx(cpin + C * L_um, rel=1e-12)
    # Eq. 3 on a star leaf reduces to the delay itself.
    assert out["imp"][1] == pytest.approx(want, rel=1e-9, abs=1e-12)
    # Sink arrival and slew (wire step) for both modes and transitions.
    assert np.allclose(out["at"][1], d.cons.pi_at + want, rtol=1e-12)
    assert np.allclose(out["slew"][1], math.sqrt(d.cons.pi_slew ** 2 + want ** 2), rtol=1e-12)


def test_star_net_hand_example():
    # Driver at the origin, three sinks; lengths 30, 70 (=30+40), 100 um.
    d = build([[0, 1, 2, 3]], [], [PIN_PI, PIN_PO, PIN_PO, PIN_FF_D], [0.5, 1.0, 2.0, 4.0],
              [0.0, 30.0, 30.0, -60.0], [0.0, 0.0, 40.0, 40.0])
    out = O.run(d, grad=None)
    L = np.array([30.0, 70.0, 100.0])
    cp = np.array([1.0, 2.0, 4.0])
    assert out["load_root"][0] == pytest.approx(0.5 + np.sum(cp + C * L), rel=1e-12)
    want = 1e-3 * R * L * (cp + C * L / 2)
    assert np.allclose(out["delay"][1:], want, rtol=1e-12)
    assert np.allclose(out["imp"][1:], want, rtol=1e-9)


# ----------------------------------------------------------------------------- NLDM lookup
def _lut_np(tab, xa, ya, xv, yv):
    v, _, _ = O.lut(torch.from_numpy(tab), torch.from_numpy(xa), torch.from_numpy(ya),
                    torch.from_numpy(xv), torch.from_numpy(yv))
    return v.numpy()


def test_lut_matches_scipy_grid_interpolator():
    rng = np.random.default_rng(7)
    lib = make_library()
    xa = lib.slew_axis.astype(np.float64)
    ya = lib.load_axis.astype(np.float64)
    tab = rng.normal(50, 20, (7, 7))   # asymmetric on purpose: a transposed operand fails
    xv = np.concatenate([rng.uniform(0.5, 2000, 400), xa, [1e-3, 4000.0]])
    yv = np.concatenate([rng.uniform(0.1, 9000, 400), ya[::-1], [9000.0, 1e-3]])
    ref = RegularGridInterpolator((xa, ya), tab, method="linear", bounds_error=False,
                                  fill_value=None)(np.stack([xv, yv], 1))
    got = _lut_np(np.broadcast_to(tab, (len(xv), 7, 7)).copy(), xa, ya, xv, yv)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-9)


def test_lut_breakpoints_return_table_entries():
    lib = make_library()
    xa = lib.slew_axis.astype(np.float64)
    ya = lib.load_axis.astype(np.float64)
    tab = lib.tables[3, 1].astype(np.float64)
    ii, jj = np.meshgrid(np.arange(7), np.arange(7), indexing="ij")
    got = _lut_np(np.broadcast_to(tab, (49, 7, 7)).copy(), xa, ya, xa[ii.ravel()], ya[jj.ravel()])
    assert np.allclose(got, tab[ii.ravel(), jj.ravel()], rtol=0, atol=1e-10)


def test_lut_planar_tables_exact_with_extrapolation():
    lib = planar_library()
    xa = lib.slew_axis.astype(np.float64)
    ya = lib.load_axis.astype(np.float64)
    a, b, c = 13.0, 0.21, 0.77
    tab = a + b * xa[:, None] + c * ya[None, :]
    rng = np.random.default_rng(3)
    xv = rng.uniform(0.0, 5e4, 300)
    yv = rng.uniform(0.0, 1e5, 300)
    got = _lut_np(np.broadcast_to(tab, (300, 7, 7)).copy(), xa, ya, xv, yv)
    assert np.allclose(got, a + b * xv + c * yv, rtol=1e-11)


# ----------------------------------------------------------------------------- chain closed form
def test_inverter_buffer_chain_closed_form():
    # Planar tables make every lookup an exact plane, so a chain has a closed-form recursion.
    lib = planar_library(seed=4)
    n = 6
    types = [0, 1, 2, 3, 4, 5]            # fanin-1 types, arcs 0..5
    d = chain(n, types, lib, L_um=80.0, cpin=2.0)
    out = O.run(d, grad=None)
    xa = lib.slew_axis.astype(np.float64)
    ya = lib.load_axis.astype(np.float64)

    def plane(t):      # recover (a, b, c) of a planar table from three entries
        t = t.astype(np.float64)
        b = (t[1, 0] - t[0, 0]) / (xa[1] - xa[0])
        c = (t[0, 1] - t[0, 0]) / (ya[1] - ya[0])
        return t[0, 0] - b * xa[0] - c * ya[0], b, c

    wire = 1e-3 * (R * C * 80.0 ** 2 / 2 + R * 80.0 * 2.0)
    load = 2.0 + C * 80.0
    at = np.full(4, d.cons.pi_at)
    slew = np.full(4, d.cons.pi_slew)
    for g in range(n):
        at = at + wire
        slew = np.sqrt(slew ** 2 + wire ** 2)
        arc = lib.arc_offsets[types[g]]
        un = lib.arc_unate[arc]
        nat, nslew = np.empty(4), np.empty(4)
        for k in range(4):
            m, t = divmod(k, 2)
            kp = 2 * m + (t if un > 0 else 1 - t)
            ad, bd, cd = plane(lib.tables[arc, t])
            as_, bs, cs = plane(lib.tables[arc, 2 + t])
            nat[k] = at[kp] + ad + bd * slew[kp] + cd * load
            nslew[k] = as_ + bs * slew[kp] + cs * load
        at, slew = nat, nslew
    po = d.n_pins - 1
    assert np.allclose(out["at"][po], at + wire, rtol=1e-10)
    assert np.allclose(out["slew"][po], np.sqrt(slew ** 2 + wire ** 2), rtol=1e-10)


# ----------------------------------------------------------------------------- brute force paths
def _graph_maps(d, lv):
    off = d.net_offsets
    sinks = {int(lv.driver[n]): [int(p) for p in d.net_pins[off[n] + 1:off[n + 1]]] for n in range(d.n_nets)}
    drv_of = {int(p): int(lv.driver[lv.net_of_pin[p]]) for p in range(d.n_pins)}
    in_cell = {}
    for c in range(d.n_cells):
        ins = d.cell_in_pins[d.cell_in_offsets[c]:d.cell_in_offsets[c + 1]]
        for j, p in enumerate(ins):
            in_cell[int(p)] = (c, j)
    return sinks, drv_of, in_cell


def _all_arrivals(d, lv, out, p, k, sinks, drv_of):
    """Every path sum reaching condition k of pin p (explicit enumeration, no merging)."""
    kind = d.pin_kind[p]
    if kind == PIN_PI:
        return [d.cons.pi_at]
    if kind == PIN_CELL_OUT:
        c = int(lv.cell_of_out_pin[p])
        ins = d.cell_in_pins[d.cell_in_offsets[c]:d.cell_in_offsets[c + 1]]
        a0 = d.lib.arc_offsets[d.cell_type[c]]
        m, t = divmod(k, 2)
        res = []
        for j, q in enumerate(ins):
            tp = t if d.lib.arc_unate[a0 + j] > 0 else 1 - t
            res += [v + out["arc_delay"][q, k] for v in _all_arrivals(d, lv, out, int(q), 2 * m + tp, sinks, drv_of)]
        return res
    return [v + out["delay"][p] for v in _all_arrivals(d, lv, out, drv_of[p], k, sinks, drv_of)]


def _all_requireds(d, lv, out, p, k, sinks, in_cell):
    """Every (endpoint RAT - path delay) from condition k of pin p to an endpoint."""
    kind = d.pin_kind[p]
    m, t = divmod(k, 2)
    if kind in (PIN_FF_D, PIN_PO):
        return [d.cons.hold if m == 0 else d.cons.t_clk - d.cons.setup]
    if kind in (PIN_PI, PIN_CELL_OUT):
        res = []
        for s in sinks[p]:
            res += [v - out["delay"][s] for v in _all_requireds(d, lv, out, s, k, sinks, in_cell)]
        return res
    c, j = in_cell[p]
    arc = d.lib.arc_offsets[d.cell_type[c]] + j
    t_out = t if d.lib.arc_unate[arc] > 0 else 1 - t
    k_out = 2 * m + t_out
    o = int(d.cell_out_pin[c])
    return [v - out["arc_delay"][p, k_out] for v in _all_requireds(d, lv, out, o, k_out, sinks, in_cell)]


@pytest.mark.parametrize("seed", range(6))
def test_arrival_and_required_match_path_enumeration(seed):
    spec = tiny_spec(n_gates=9 + seed, n_levels=3 + seed % 3, n_pi=3, seed=seed)
    d = make_design(spec)
    lv = O.levelize(d)
    out = O.run(d, grad=None, lv=lv)
    sinks, drv_of, in_cell = _graph_maps(d, lv)
    for p in range(d.n_pins):
        for k in range(4):
            arr = _all_arrivals(d, lv, out, p, k, sinks, drv_of)
            want = max(arr) if k >= 2 else min(arr)
            assert out["at"][p, k] == pytest.approx(want, rel=1e-12, abs=1e-9)
            req = _all_requireds(d, lv, out, p, k, sinks, in_cell)
            if not req:
                assert out["rat"][p, k] == (math.inf if k >= 2 else -math.inf)
            else:
                want = min(req) if k >= 2 else max(req)
                assert out["rat"][p, k] == pytest.approx(want, rel=1e-12, abs=1e-9)


def test_critical_path_slack_property():
    # Every pin on a path to an endpoint has late slack >= the worst endpoint slack, and
    # the worst pin slack is attained at an endpoint.
    d = make_design(CFG0)
    out = O.run(d, grad=None)
    late = out["slack"][:, 2:4]
    ep_late = late[out["endpoints"]]
    assert np.min(late) == pytest.approx(np.min(ep_late), rel=1e-12)
    assert out["wns"] == pytest.approx(min(0.0, np.min(ep_late)), rel=1e-12)
    # slack is RAT - AT late and AT - RAT early, pin by pin.
    assert np.allclose(out["slack"][:, 2:], out["rat"][:, 2:] - out["at"][:, 2:])
    assert np.allclose(out["slack"][:, :2], out["at"][:, :2] - out["rat"][:, :2])


# ----------------------------------------------------------------------------- LSE (Eq. 4)
def test_lse_single_pair_and_scipy():
    g = 10.0
    x = torch.tensor([[3.0]], dtype=torch.float64)
    assert float(O.lse(x, g, 1)) == pytest.approx(3.0, abs=1e-12)
    x = torch.tensor([[5.0, 5.0]], dtype=torch.float64)
    assert float(O.lse(x, g, 1)) == pytest.approx(5.0 + g * math.log(2), rel=1e-14)
    rng = np.random.default_rng(0)
    v = rng.normal(1e5, 30, (50, 4))
    got = O.lse(torch.from_numpy(v), g, 1).numpy()
    assert np.allclose(got, g * logsumexp(v / g, axis=1), rtol=1e-14)


def test_smoothed_arrival_bounds_and_limit():
    d = make_design(CFG0)
    lv = O.levelize(d)
    out = O.run(d, grad=None, lv=lv, gamma=10.0)
    late = out["at"][:, 2:4]
    assert np.all(out["atg"] >= late - 1e-9)
    # Each LSE merge adds at most gamma*ln(fanin); depth bounds the accumulation.
    bound = 10.0 * math.log(4) * lv.n_levels
    assert np.all(out["atg"] - late <= bound)
    small = O.run(d, grad=None, lv=lv, gamma=1e-3)
    assert np.allclose(small["atg"], late, rtol=0, atol=1e-3 * math.log(4) * lv.n_levels + 1e-9)
    assert small["tns_g"] == pytest.approx(out["tns"], rel=1e-6)
    assert small["wns_g"] == pytest.approx(out["wns"], abs=0.05)


# ----------------------------------------------------------------------------- gradient
def test_two_pin_gradient_closed_form():
    cons = Constraints(t_clk=5.0)     # the sink violates
    d = two_pin(300.0, 2.0, cons=cons)
    g = 10.0
    out = O.run(d, grad="tns", gamma=g)
    L = 300.0
    D = 1e-3 * (R * C * L ** 2 / 2 + R * L * 2.0)
    s = (cons.t_clk - (cons.pi_at + D)) - g * math.log(2)      # soft worst of two equal transitions
    dD_dL = 1e-3 * (R * 2.0 + R * C * L)
    dT_dL = (1 / (1 + math.exp(s / g))) * (-dD_dL)
    assert out["tns_g"] == pytest.approx(-g * math.log1p(math.exp(-s / g)), rel=1e-12)
    assert out["dx"][1] == pytest.approx(dT_dL, rel=1e-10)     # x_s > x_d
    assert out["dy"][1] == pytest.approx(dT_dL, rel=1e-10)
    assert out["dx"][0] == pytest.approx(-dT_dL, rel=1e-10)


def test_gradient_translation_invariance_per_net():
    d = make_design(CFG0)
    out = O.run(d, grad="tns")
    net_sum_x = np.add.reduceat(out["dx"][d.net_pins], d.net_offsets[:-1])
    net_sum_y = np.add.reduceat(out["dy"][d.net_pins], d.net_offsets[:-1])
    scale = np.abs(out["dx"]).max()
    assert np.abs(net_sum_x).max() <= 1e-10 * scale
    assert np.abs(net_sum_y).max() <= 1e-10 * scale


@pytest.mark.parametrize("which", ["tns", "wns"])
def test_gradient_matches_central_differences(which):
    d = make_design(CFG0)
    lv = O.levelize(d)
    plan = O._Plan(d, lv)
    g = 10.0
    out = O.run(d, grad=which, gamma=g, lv=lv, plan=plan)
    rng = np.random.default_rng(11)
    pins = rng.choice(d.n_pins, 60, replace=False)
    h = 1e-3
    x0 = d.x.astype(np.float64)
    y0 = d.y.astype(np.float64)
    checked = 0
    for p in pins:
        for axis in (0, 1):
            xp, yp, xm, ym = x0.copy(), y0.copy(), x0.copy(), y0.copy()
            (xp if axis == 0 else yp)[p] += h
            (xm if axis == 0 else ym)[p] -= h
            fp, dp = O.objective_at(d, lv, plan, xp, yp, g, which)
            fm, dm = O.objective_at(d, lv, plan, xm, ym, g, which)
            if any(not np.array_equal(a, b) for a, b in zip(dp, dm)):
                continue   # the stencil crosses a table cell, an arg max or a sign: not smooth
            fd = (fp - fm) / (2 * h)
            an = out["dx" if axis == 0 else "dy"][p]
            assert abs(fd - an) <= 1e-4 * abs(an) + 1e-3, (p, axis, fd, an)
            checked += 1
    assert checked >= 80


# ----------------------------------------------------------------------------- levelization
def _longest_path_levels(d, lv):
    memo = {}
    preds = {}
    for n in range(d.n_nets):
        c = lv.cell_of_net[n]
        preds[n] = [] if c < 0 else [int(lv.net_of_pin[p]) for p in
                                     d.cell_in_pins[d.cell_in_offsets[c]:d.cell_in_offsets[c + 1]]]

    def depth(n):   # longest path from a PI-driven net, by plain recursion
        if n not in memo:
            memo[n] = 0 if not preds[n] else 1 + max(depth(m) for m in preds[n])
        return memo[n]
    return np.array([depth(n) for n in range(d.n_nets)])


@pytest.mark.parametrize("seed", range(8))
def test_levelize_matches_longest_path_and_canonical_rules(seed):
    d = make_design(tiny_spec(n_gates=10 + 3 * seed, n_levels=2 + seed % 5, n_pi=3, seed=seed))
    lv = O.levelize(d)
    assert np.array_equal(lv.level, _longest_path_levels(d, lv))
    assert np.array_equal(lv.level, d.gen_net_level)
    # nets by (level, pins of the net, original id); offsets delimit levels; pins net-major,
    # driver first, sinks in the input CSR order.
    size = np.diff(d.net_offsets)
    key = [(int(lv.level[n]), int(size[n]), int(n)) for n in lv.net_perm]
    assert key == sorted(key)
    assert lv.level_offsets[0] == 0 and lv.level_offsets[-1] == d.n_nets
    for l in range(lv.n_levels):
        seg = lv.net_perm[lv.level_offsets[l]:lv.level_offsets[l + 1]]
        assert len(seg) > 0 and np.all(lv.level[seg] == l)
    expect = [p for n in lv.net_perm for p in d.net_pins[d.net_offsets[n]:d.net_offsets[n + 1]]]
    assert lv.pin_perm.tolist() == expect
    assert sorted(lv.pin_perm.tolist()) == list(range(d.n_pins))


def test_levelize_rejects_cycle():
    # PI 0 -> net{0,1}; cell A: in 1 (and 5) -> out 2 -> net{2,3}; cell B: in 3 -> out 4 -> net{4,5}
    d = build([[0, 1], [2, 3], [4, 5]], [(8, [1, 5], 2), (0, [3], 4)],
              [PIN_PI, PIN_CELL_IN, PIN_CELL_OUT, PIN_CELL_IN, PIN_CELL_OUT, PIN_CELL_IN],
              [0, 1, 0, 1, 0, 1], [0, 1, 2, 3, 4, 5], [0] * 6)
    with pytest.raises(O.CycleError):
        O.levelize(d)


def test_generator_levels_are_exact_cfg0():
    d = make_design(CFG0)
    lv = O.levelize(d)
    assert lv.n_levels == CFG0.n_levels + 1
    assert np.array_equal(lv.level, d.gen_net_level)


# ----------------------------------------------------------------------------- conditioning
def test_fp32_noise_envelope_small_on_cfg0():
    # cfg0 stays inside the table range: float32-sized noise moves no arrival beyond 1e-6.
    d = make_design(CFG0)
    lv = O.levelize(d)
    ref = O.run(d, grad=None, lv=lv)
    r = O.run(d, grad=None, lv=lv, perturb=RB.fp32_rounding_noise(0))
    assert np.max(np.abs(r["at"] - ref["at"]) / np.maximum(np.abs(ref["at"]), 1.0)) < 1e-6
    assert not np.array_equal(r["at"], ref["at"])      # the perturbation is live


FAR = dict(cfg_id=77, box_um=4000.0)   # loads far past the table edge


@pytest.mark.parametrize("which", ["cfg0", "far_extrapolation"])
def test_rounding_scales_bound_float32_perturbation(which):
    # Lower pin: sigma is a first-order bound, so one rounding of relative size <= u at
    # every operation moves each value by at most u * sigma (up to second-order terms).
    from gen.netlist import scaled_spec
    d = make_design(CFG0 if which == "cfg0" else scaled_spec(20_000, **FAR))
    lv = O.levelize(d)
    plan = O._Plan(d, lv)
    ref = O.run(d, grad=None, lv=lv, plan=plan)
    sc = RB.rounding_scales(d, ref)
    u = RB.U32
    for seed in range(3):
        p = O.run(d, grad=None, lv=lv, plan=plan, perturb=RB.fp32_rounding_noise(seed))
        for k in ("at", "slew", "atg", "rat", "slack"):
            r, v = ref[k], p[k]
            fin = np.isfinite(r)
            assert np.array_equal(fin, np.isfinite(v)), k
            err = np.abs(v[fin] - r[fin])
            assert np.all(err <= 1.01 * u * sc[k + "_scale"][fin] + 1e-9), (k, np.max(err / (u * sc[k + "_scale"][fin])))


@pytest.mark.parametrize("which", ["cfg0", "far_extrapolation"])
def test_rounding_scales_reached_by_signed_rounding(which):
    # Upper pin: rounding every forward result down and every required time up by one
    # float32 unit (all errors of one sign) is a rounding pattern float32 could produce; it
    # moves the median value by about half its bound and the top percentile to it, so sigma
    # is not inflated.  A sigma with a spurious term (a doubled partial, a term counted
    # twice) would put these ratios near or below 0.5 and 0.25.
    from gen.netlist import scaled_spec
    d = make_design(CFG0 if which == "cfg0" else scaled_spec(20_000, **FAR))
    ref = O.run(d, grad=None)
    sc = RB.rounding_scales(d, ref)
    sg = RB.run_signed(d, lv=ref["lv"], plan=ref["plan"])
    for k in ("at", "slew", "atg", "rat", "slack"):
        s = sc[k + "_scale"]
        fin = np.isfinite(ref[k]) & (s > 0)
        ratio = np.abs(sg[k][fin] - ref[k][fin]) / (RB.U32 * s[fin])
        assert ratio.max() <= 1.0 + 1e-6, k                    # and it stays a bound
        assert np.median(ratio) >= 0.4 and np.quantile(ratio, 0.99) >= 0.8, (k, np.median(ratio))


def _gain_library(gain: float) -> "Library":
    """Planar tables without load dependence: delay = a + b slew, slew = a_s + gain * slew,
    the same for both output transitions, all coefficients dyadic so that every entry is
    exact in float32."""
    from gen.netlist import Library
    base = planar_library(seed=5)
    xa = base.slew_axis.astype(np.float64)
    rng = np.random.default_rng(9)
    tabs = np.empty(base.tables.shape, np.float64)
    for a in range(tabs.shape[0]):          # rise and fall alike, so all conditions share values
        tabs[a, 0:2] = rng.integers(8, 64) / 2.0 + rng.integers(1, 20) / 64.0 * xa[:, None]
        tabs[a, 2:4] = rng.integers(4, 16) / 2.0 + gain * xa[:, None]
    assert np.array_equal(tabs.astype(np.float32).astype(np.float64), tabs)
    return Library(base.n_cell_types, base.arc_offsets, base.arc_unate, base.slew_axis, base.load_axis,
                   tabs.astype(np.float32))


def test_rounding_scales_exact_on_amplifying_chain():
    # A chain of 12 single-input gates whose tables have slew gain 1.5 (slews run from 10 ps
    # to about 3e3 ps, far past the 500 ps axis end), co-located pins (no wire) and no load
    # dependence: every partial derivative is positive, so signed rounding reaches the
    # first-order bound exactly, and the slew bound has the closed form of a linear
    # recurrence: sigma(s_j) = gain * sigma(s'_(j-1)) + s_j at the gate output,
    # sigma(s'_j) = sigma(s_j) + s'_j at the next input (the sink slew's own rounding).
    gain = 1.5
    lib = _gain_library(gain)
    n = 12
    d = chain(n, [0, 1, 2, 3, 4, 5] * 2, lib, L_um=0.0, cpin=2.0)
    ref = O.run(d, grad=None)
    sc = RB.rounding_scales(d, ref)
    sg = RB.run_signed(d, lv=ref["lv"], plan=ref["plan"])
    for k in ("at", "slew", "atg", "rat"):
        s = sc[k + "_scale"]
        fin = np.isfinite(ref[k]) & (s > 0)
        ratio = np.abs(sg[k][fin] - ref[k][fin]) / (RB.U32 * s[fin])
        assert np.all(np.abs(ratio - 1.0) < 1e-5), (k, ratio.min(), ratio.max())
    fin = np.isfinite(ref["slack"])
    sl = np.abs(np.where(fin, ref["slack"], 0))
    ratio = np.abs(sg["slack"][fin] - ref["slack"][fin]) / (RB.U32 * (sc["slack_scale"][fin] - sl[fin]))
    assert np.all(np.abs(ratio - 1.0) < 1e-5)     # the final subtraction is not perturbed
    # Closed form of the slew bound along the chain (late rise of the primary output).
    po = d.n_pins - 1
    sig_in, s_in = 10.0, 10.0                      # PI sink: sqrt(10^2 + 0) rounded once
    sl_gate = ref["slew"]
    outs = d.cell_out_pin
    for j in range(n):
        s_out = sl_gate[outs[j], 2]
        kp_src = 2 if lib.arc_unate[lib.arc_offsets[d.cell_type[j]]] > 0 else 3
        assert np.isclose(s_in, ref["slew"][d.cell_in_pins[j], kp_src])
        sig_out = gain * sig_in + s_out
        sig_in, s_in = sig_out + s_out, s_out
    assert ref["slew"][po, 2] > 500.0 * 5                       # far past the table edge
    assert sc["slew_scale"][po, 2] == pytest.approx(sig_in, rel=1e-12)
    assert sig_in / ref["slew"][po, 2] > 2.5                    # amplified: sigma/slew ~ 1/(1-1/gain)


def test_wns_smoothed_counts_the_zero_member():
    # WNS_g = -LSE({0} u {-s_e}): with every endpoint's slack positive, the zero member is
    # the largest term.  A PI -> buffer -> FF design with the clock at 40 ps puts the
    # smoothed endpoint slack s at a few ps, so WNS_g = -gamma log(1 + exp(-s/gamma)), a
    # small negative number, where dropping {0} would give s itself (positive).
    lib = planar_library(seed=3)
    d = chain(1, [0], lib, L_um=30.0, cpin=2.0)
    d.pin_kind[-1] = PIN_FF_D
    d.cons = type(d.cons)(**{**d.cons.__dict__, "t_clk": 40.0})
    g = 10.0
    out = O.run(d, gamma=g, grad="wns")
    sl = out["slack"][d.n_pins - 1, 2:4]                         # late rise, fall slack at the FF
    assert np.all(sl > 0)
    s = -g * np.log(np.exp(-sl[0] / g) + np.exp(-sl[1] / g))     # soft worst of rise and fall
    assert 0 < s < 40
    assert out["wns_g"] == pytest.approx(-g * np.log1p(np.exp(-s / g)), rel=1e-12)
    assert out["wns"] == 0.0 and out["tns"] == 0.0
    # Two endpoints: both positive, WNS_g = -gamma log(1 + sum exp(-s_e / gamma)).
    d2 = chain(2, [0, 1], lib, L_um=30.0, cpin=2.0)
    d2 = _add_endpoint(d2, net_driver=int(d2.cell_out_pin[0]))
    d2.cons = type(d2.cons)(**{**d2.cons.__dict__, "t_clk": 80.0})
    out2 = O.run(d2, gamma=g, grad=None)
    ep = out2["endpoints"]
    sle = out2["slack"][ep][:, 2:4]
    assert len(ep) == 2 and np.all(sle > 0)
    se = -g * np.log(np.exp(-sle[:, 0] / g) + np.exp(-sle[:, 1] / g))
    assert out2["wns_g"] == pytest.approx(-g * np.log1p(np.exp(-se / g).sum()), rel=1e-12)


def _add_endpoint(d, net_driver: int):
    """Adds a flop D sink, co-located with the driver, to the net that `net_driver` drives."""
    from tests._designs import build
    nets = [list(d.net_pins[d.net_offsets[n]:d.net_offsets[n + 1]]) for n in range(d.n_nets)]
    new = d.n_pins
    for n in nets:
        if n[0] == net_driver:
            n.append(new)
    cells = [(int(d.cell_type[c]), list(d.cell_in_pins[d.cell_in_offsets[c]:d.cell_in_offsets[c + 1]]),
              int(d.cell_out_pin[c])) for c in range(d.n_cells)]
    kinds = list(d.pin_kind) + [PIN_FF_D]
    return build(nets, cells, kinds, list(d.pin_cap) + [2.0], list(d.x) + [float(d.x[net_driver])],
                 list(d.y) + [float(d.y[net_driver])], lib=d.lib, cons=d.cons)


@pytest.mark.parametrize("seed", range(3))
def test_wide_cells_match_path_enumeration(seed):
    # Cells of 5-8 inputs: the same explicit enumeration over every path.
    from tests._designs import wide_dag
    d = wide_dag(n_levels=3, gates_per_level=5, n_pi=9, seed=seed)
    lv = O.levelize(d)
    out = O.run(d, grad=None, lv=lv)
    sinks, drv_of, in_cell = _graph_maps(d, lv)
    assert np.diff(d.cell_in_offsets).max() >= 5
    for p in range(d.n_pins):
        for k in range(4):
            arr = _all_arrivals(d, lv, out, p, k, sinks, drv_of)
            want = max(arr) if k >= 2 else min(arr)
            assert out["at"][p, k] == pytest.approx(want, rel=1e-12, abs=1e-9)
            req = _all_requireds(d, lv, out, p, k, sinks, in_cell)
            if req:
                want = min(req) if k >= 2 else max(req)
                assert out["rat"][p, k] == pytest.approx(want, rel=1e-12, abs=1e-9)


# ----------------------------------------------------------------------------- RC trees (R13)
def _tree_moments_by_path_resistance(d, net):
    """Elmore delay and second moment of every pin of one net from the path-resistance
    form: Delay(u) = sum_k Rc(u, k) C_k and Beta(u) = sum_k Rc(u, k) C_k Delay(k), where
    Rc(u, k) is the resistance shared by the root-to-u and root-to-k paths and C_k the
    node capacitance (pin plus half of every segment touching it)."""
    pins = list(d.net_pins[d.net_offsets[net]:d.net_offsets[net + 1]])
    par = {p: int(d.pin_parent[p]) for p in pins}
    seg = {p: abs(float(d.x[p]) - float(d.x[par[p]])) + abs(float(d.y[p]) - float(d.y[par[p]]))
           for p in pins if par[p] >= 0}
    cap = {p: float(d.pin_cap[p]) for p in pins}
    for p, L in seg.items():
        cap[p] += 0.5 * C * L
        cap[par[p]] += 0.5 * C * L

    def path(p):
        out = []
        while par[p] >= 0:
            out.append(p)
            p = par[p]
        return set(out)
    paths = {p: path(p) for p in pins}
    rc = {(u, k): sum(R * seg[s] for s in paths[u] & paths[k]) for u in pins for k in pins}
    delay = {u: 1e-3 * sum(rc[u, k] * cap[k] for k in pins) for u in pins}
    beta = {u: 1e-3 * sum(rc[u, k] * cap[k] * delay[k] for k in pins) for u in pins}
    return pins, delay, beta, sum(cap.values())


def _tree_design(seed):
    from gen.netlist import heap_trees
    return heap_trees(make_design(tiny_spec(30, 4, n_pi=3, seed=seed, box_um=120.0, fanout_p=0.25,
                                            fanout_cap=12)))


@pytest.mark.parametrize("seed", [0, 1])
def test_tree_elmore_matches_path_resistance_form(seed):
    d = _tree_design(seed)
    lv = O.levelize(d)
    x = torch.from_numpy(d.x.astype(np.float64))
    y = torch.from_numpy(d.y.astype(np.float64))
    rcr = O.rc(d, lv, x, y)
    deep = 0
    for net in range(d.n_nets):
        pins, delay, beta, total = _tree_moments_by_path_resistance(d, net)
        assert float(rcr["load_root"][net]) == pytest.approx(total, rel=1e-12)   # Eq. 1 at the root
        for u in pins[1:]:
            assert float(rcr["delay"][u]) == pytest.approx(delay[u], rel=1e-11, abs=1e-15)
            assert float(rcr["beta"][u]) == pytest.approx(beta[u], rel=1e-11, abs=1e-18)
            arg = 2 * beta[u] - delay[u] ** 2
            assert float(rcr["imp"][u]) == pytest.approx(math.sqrt(max(arg, 0.0)), rel=1e-9, abs=1e-12)
        deep = max(deep, int(O.tree_depth(d.pin_parent.astype(np.int64))[pins].max()))
    assert deep >= 3                                   # trees deeper than a star were exercised


def test_tree_three_pin_chain_closed_form():
    # Driver -> a (40 um) -> b (60 um): Delay(b) = R1 (C_a + C_b) + R2 C_b with lumped node caps,
    # Delay(a) = R1 (C_a + C_b).
    from dataclasses import replace
    d = build([[0, 1, 2]], [], [PIN_PI, PIN_PO, PIN_FF_D], [0.5, 1.5, 3.0], [0.0, 40.0, 40.0],
              [0.0, 0.0, 60.0])
    d = replace(d, pin_parent=np.array([-1, 0, 1], np.int32))
    out = O.run(d, grad=None)
    R1, R2 = R * 40.0, R * 60.0
    Ca = 1.5 + 0.5 * C * 40.0 + 0.5 * C * 60.0
    Cb = 3.0 + 0.5 * C * 60.0
    assert out["delay"][1] == pytest.approx(1e-3 * R1 * (Ca + Cb), rel=1e-12)
    assert out["delay"][2] == pytest.approx(1e-3 * (R1 * (Ca + Cb) + R2 * Cb), rel=1e-12)
    assert out["load_root"][0] == pytest.approx(0.5 + C * 100.0 + 1.5 + 3.0, rel=1e-12)


def test_tree_of_depth_one_is_the_star():
    from dataclasses import replace
    d = make_design(CFG0)
    lv = O.levelize(d)
    star_tree = replace(d, pin_parent=np.where(lv.driver[lv.net_of_pin] == np.arange(d.n_pins), -1,
                                               lv.driver[lv.net_of_pin]).astype(np.int32))
    a = O.run(d, grad="tns")
    b = O.run(star_tree, grad="tns")
    for k in ("delay", "imp", "load_root", "at", "slew", "dx", "dy"):
        assert np.allclose(a[k], b[k], rtol=1e-12, atol=1e-12, equal_nan=True), k
    assert b["tns"] == pytest.approx(a["tns"], rel=1e-12)


def test_tree_gradient_matches_central_differences():
    d = _tree_design(2)
    lv = O.levelize(d)
    plan = O._Plan(d, lv)
    g = 10.0
    out = O.run(d, grad="tns", gamma=g, lv=lv, plan=plan)
    x0, y0 = d.x.astype(np.float64), d.y.astype(np.float64)
    h = 1e-3
    checked = 0
    for p in range(d.n_pins):
        for axis in (0, 1):
            xp, yp, xm, ym = x0.copy(), y0.copy(), x0.copy(), y0.copy()
            (xp if axis == 0 else yp)[p] += h
            (xm if axis == 0 else ym)[p] -= h
            fp, dp = O.objective_at(d, lv, plan, xp, yp, g)
            fm, dm = O.objective_at(d, lv, plan, xm, ym, g)
            if any(not np.array_equal(u, v) for u, v in zip(dp, dm)):
                continue
            an = out["dx" if axis == 0 else "dy"][p]
            assert abs((fp - fm) / (2 * h) - an) <= 1e-4 * abs(an) + 1e-3, (p, axis)
            checked += 1
    assert checked >= 40
