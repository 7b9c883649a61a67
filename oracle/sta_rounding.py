"""First-order rounding bounds for the oracle's values, and rounding experiments on it.

TEST INFRASTRUCTURE ONLY, like sta_oracle.py (which it reads and never changes): only the
tests and the benchmark's CPU baseline import this file; the GPU library shares nothing
with it.

The parity tests compare float32 GPU results with the float64 oracle.  Where a value is
well conditioned the stated bound max(1e-4 |ref|, 1e-3 ps) holds for any float32
evaluation.  Where the exact problem is ill conditioned at float32 resolution (sums of
large cancelling terms, chains of extrapolated tables whose slew gain exceeds 1), no
float32 evaluation can meet it, and the tests need a bound on what float32 rounding can do.
rounding_scales() computes that bound from the oracle's outputs alone:

Running error analysis (Wilkinson).  Every operation of the definitions rounds its result
once, with relative error at most u.  To first order in u the computed value of v then
differs from the exact one by at most u * sigma(v), where

    sigma(v) = sum over operands w of |d v / d w| * sigma(w)  +  |v|

(the |v| term is v's own rounding), sigma = 0 for exact inputs (coordinates, caps, table
entries and constraints are float32 numbers given to both sides), and a max or min merge
takes the largest sigma of its operands (a bound whichever operand is selected).  The
partial derivatives are those of the definitions: the bilinear table partials (the
oracle's lut_partials), 1 for sums and differences, a/sqrt(a^2+b^2) for the sink slew.  A
root load, wire delay and impulse each count as one rounded value of their own.

The experiments perturb every wire delay, impulse, root load, lookup, arrival, slew,
smoothed arrival and required time of the oracle (its `perturb` hook) by one float32-sized
relative error: at random (fp32_rounding_noise), or all of the same sign
(signed_rounding), which on a chain whose partial derivatives are all positive reaches the
first-order bound exactly.
"""
from __future__ import annotations

import numpy as np
import torch

from oracle import sta_oracle as O

U32 = 2.0 ** -24          # float32 unit roundoff


def fp32_rounding_noise(seed: int):
    """Multiplies each value by (1 + e), e uniform in +-2^-24: one float32-sized rounding."""
    gen = torch.Generator().manual_seed(seed)
    rng = np.random.default_rng([seed, 24])

    def p(v):
        if isinstance(v, np.ndarray):
            return v * (1 + rng.uniform(-U32, U32, v.shape))
        e = (torch.rand(v.shape, generator=gen, dtype=torch.float64) * 2 - 1) * U32
        return v * (1 + e)
    return p


def signed_rounding(sign: float):
    """Moves each finite value by sign * u * |value|: one rounding of the same sign everywhere."""
    def p(v):
        if isinstance(v, np.ndarray):
            return np.where(np.isfinite(v), v + sign * U32 * np.abs(v), v)
        return torch.where(torch.isfinite(v), v + sign * U32 * v.abs(), v)
    return p


def _exact_f32(v: float) -> bool:
    return float(np.float32(v)) == v


def rounding_scales(d, out) -> dict:
    """sigma for every value of an oracle result `out` (sta_oracle.run): arrays at_scale [P,4],
    slew_scale [P,4], atg_scale [P,2], rat_scale [P,4], slack_scale [P,4] by original pin id.
    Only late conditions have a smoothed arrival."""
    lv, plan = out["lv"], out["plan"]
    lib, cons = d.lib, d.cons
    P = d.n_pins
    at, slew, atg, rat, slack = out["at"], out["slew"], out["atg"], out["rat"], out["slack"]
    delay, imp, load_root, ad = out["delay"], out["imp"], out["load_root"], out["arc_delay"]
    xa = torch.from_numpy(lib.slew_axis.astype(np.float64))
    ya = torch.from_numpy(lib.load_axis.astype(np.float64))
    tables = torch.from_numpy(lib.tables.astype(np.float64))
    s_at, s_sl, s_g = np.zeros((P, 4)), np.zeros((P, 4)), np.zeros((P, 2))
    arc_sig = np.zeros((P, 4))            # sigma of the arc delay entered at each input, per output k
    # Primary inputs take the constraint values (exact float32 inputs): sigma 0.
    for l in range(plan.L):
        drv = plan.drv[l]
        if l > 0:
            pins, mask, arc, unate = plan.in_pins[l], plan.in_mask[l], plan.in_arc[l], plan.in_unate[l]
            lo = np.broadcast_to(load_root[lv.net_of_pin[drv]][:, None], pins.shape)
            lo_t = torch.from_numpy(np.array(lo))
            arc_t = torch.from_numpy(arc)
            c_at, c_sl, c_g = np.zeros((len(drv), 4)), np.zeros((len(drv), 4)), np.zeros((len(drv), 2))
            for k in range(4):
                m, t = k // 2, k % 2
                tp = np.where(unate > 0, t, 1 - t)
                kp = 2 * m + tp
                sl_in = slew[pins, kp]
                sl_t = torch.from_numpy(np.where(mask, sl_in, 1.0))
                dd_x, dd_y = (v.numpy() for v in O.lut_partials(tables[arc_t, t], xa, ya, sl_t, lo_t))
                ds_x, ds_y = (v.numpy() for v in O.lut_partials(tables[arc_t, 2 + t], xa, ya, sl_t, lo_t))
                sv = O.lut(tables[arc_t, 2 + t], xa, ya, sl_t, lo_t)[0].numpy()
                dv = np.where(mask, ad[pins, k], 0.0)
                sig_d = np.abs(dd_x) * s_sl[pins, kp] + np.abs(dd_y) * np.abs(lo) + np.abs(dv)
                sig_s = np.abs(ds_x) * s_sl[pins, kp] + np.abs(ds_y) * np.abs(lo) + np.abs(sv)
                cand = at[pins, kp] + dv
                c_at[:, k] = np.where(mask, s_at[pins, kp] + sig_d + np.abs(cand), 0.0).max(axis=1)
                c_sl[:, k] = np.where(mask, sig_s, 0.0).max(axis=1)
                if m == 1:
                    g = atg[pins, tp] + dv
                    c_g[:, t] = np.where(mask, s_g[pins, tp] + sig_d + np.abs(g), 0.0).max(axis=1) + np.abs(atg[drv, t])
                arc_sig[pins[mask], k] = sig_d[mask]
            s_at[drv], s_sl[drv], s_g[drv] = c_at, c_sl, c_g
        # Net step: sink = driver + wire delay; sink slew = sqrt(driver slew^2 + impulse^2).
        sinks = plan.sinks[l]
        dp = drv[plan.sink_drv[l]]
        w = np.abs(delay[sinks])[:, None]
        iv = np.abs(imp[sinks])[:, None]
        s_at[sinks] = s_at[dp] + w + np.abs(at[sinks])
        s_g[sinks] = s_g[dp] + w + np.abs(atg[sinks])
        sl_s = slew[sinks]
        s_sl[sinks] = np.where(sl_s > 0, (np.abs(slew[dp]) * s_sl[dp] + iv * iv) / np.where(sl_s > 0, sl_s, 1.0),
                               0.0) + sl_s
    # Required times, levels descending.  Endpoint values come from the constraints.
    rsc = np.zeros((P, 4))
    ep = plan.endpoints
    late = cons.t_clk - cons.setup
    if not _exact_f32(late) or float(np.float32(cons.t_clk) - np.float32(cons.setup)) != late:
        rsc[ep, 2:4] = abs(late)
    for l in range(plan.L - 1, -1, -1):
        drv, sinks, sd = plan.drv[l], plan.sinks[l], plan.sink_drv[l]
        req = rat[sinks] - delay[sinks][:, None]
        fin = np.isfinite(req)
        sv = np.where(fin, rsc[sinks] + np.abs(delay[sinks])[:, None] + np.abs(np.where(fin, req, 0.0)), 0.0)
        rd = np.zeros((len(drv), 4))
        np.maximum.at(rd, sd, sv)
        rsc[drv] = rd
        if l == 0:
            continue
        pins, mask, unate = plan.in_pins[l], plan.in_mask[l], plan.in_unate[l]
        for k in range(4):
            m, t = k // 2, k % 2
            kp = 2 * m + np.where(unate > 0, t, 1 - t)
            val = rat[pins, kp]
            vfin = mask & np.isfinite(val)
            vs = rsc[drv, k][:, None] + arc_sig[pins, k] + np.abs(np.where(vfin, val, 0.0))
            rsc[pins[vfin], kp[vfin]] = vs[vfin]
    s_slack = rsc + s_at + np.abs(np.where(np.isfinite(slack), slack, 0.0))
    return dict(at_scale=s_at, slew_scale=s_sl, atg_scale=s_g, rat_scale=rsc, slack_scale=s_slack)


def run_signed(d, gamma: float = 10.0, lv=None, plan=None) -> dict:
    """The oracle with every forward operation rounded by -u|v| and every backward one by
    +u|v| (no gradient).  On a design whose arc delays, slews and wire terms are all
    non-negative with non-negative partials, each forward error is then -u sigma and each
    required-time error +u sigma (first order): the bound is reached."""
    lv = lv or O.levelize(d)
    xt = torch.tensor(np.asarray(d.x, np.float64))
    yt = torch.tensor(np.asarray(d.y, np.float64))
    fwd = O.forward(d, lv, xt, yt, gamma, plan=plan, perturb=signed_rounding(-1.0))
    bwd = O.backward(d, lv, fwd, perturb=signed_rounding(+1.0))
    return dict(at=fwd["at"].numpy(), slew=fwd["slew"].numpy(), atg=fwd["atg"].numpy(), rat=bwd["rat"],
                slack=bwd["slack"])
