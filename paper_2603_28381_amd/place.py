"""Synthetic timing-driven placement loop (Sec. 3.3): cells move along the gradient of the
smoothed TNS of Eq. 4, with the forward sweep and its fused adjoint run every iteration.

This is the use the paper makes of the engine inside a global placer (Xplace 3.0), reduced to
its timing term: the placer's wirelength and density forces are replaced by a quadratic
anchor that keeps each cell near where it started.  Pins without a cell (primary inputs and
outputs, flop D pins) stay fixed; a cell's pins move together by the cell's displacement.
Everything outside the sweep (the per-cell gradient gather, the Adam step) is plain torch
on the device.
"""
from __future__ import annotations

import numpy as np
import torch

from .sta import Graph


class TimingDescent:
    """Gradient ascent of TNS_g over cell displacements.

    graph: a levelized Graph of the design; x0, y0: starting pin coordinates (original pin
    order, float32); cell_in_offsets, cell_in_pins, cell_out_pin: the netlist's cells (as given
    to sta_build_graph); lr: Adam step in um; anchor: weight of sum of squared displacements
    (ps per um^2) subtracted from TNS_g.
    """

    def __init__(self, graph: Graph, x0, y0, cell_in_offsets, cell_in_pins, cell_out_pin, gamma: float = 10.0,
                 lr: float = 0.5, anchor: float = 1e-3, device="cuda"):
        dev = torch.device(device)
        self.g, self.gamma, self.anchor = graph, float(gamma), float(anchor)
        P = graph.n_pins
        off = np.asarray(cell_in_offsets, np.int64)
        ins = np.asarray(cell_in_pins, np.int64)
        outp = np.asarray(cell_out_pin, np.int64)
        C = len(outp)
        fan = np.diff(off)
        F = int(fan.max()) if C else 0
        # Pins of each cell (output first, then inputs), padded with index P (a zero entry).
        idx = np.full((C, F + 1), P, np.int64)
        idx[:, 0] = outp
        for j in range(F):
            has = fan > j
            idx[has, j + 1] = ins[off[:-1][has] + j]
        cell = np.full(P, C, np.int64)              # C: no cell (fixed pin)
        cell[outp] = np.arange(C)
        cell[ins] = np.repeat(np.arange(C), fan)
        self.idx = torch.from_numpy(idx).to(dev)
        self.cell = torch.from_numpy(cell).to(dev)
        self.x0 = torch.as_tensor(np.asarray(x0, np.float32), device=dev)
        self.y0 = torch.as_tensor(np.asarray(y0, np.float32), device=dev)
        self.dxc = torch.zeros(C + 1, device=dev)      # last entry: the fixed pins, never moved
        self.dyc = torch.zeros(C + 1, device=dev)
        self.opt = torch.optim.Adam([self.dxc, self.dyc], lr=lr)
        self.state, self.ws = graph.new_state(dev), graph.new_workspace(dev)
        self.scal = torch.empty(4, dtype=torch.float64, device=dev)
        self.grads = {"dx": torch.empty(P, device=dev), "dy": torch.empty(P, device=dev)}
        self.zero = torch.zeros(1, device=dev)

    def coordinates(self) -> tuple[torch.Tensor, torch.Tensor]:
        return self.x0 + self.dxc[self.cell], self.y0 + self.dyc[self.cell]

    def step(self) -> torch.Tensor:
        """One iteration: STA and the TNS_g gradient at the current placement, then one Adam
        step of the cells.  Returns the device scalars (WNS, TNS, WNS_g, TNS_g) before the step."""
        x, y = self.coordinates()
        f = self.g.forward(x, y, gamma=self.gamma, smooth=True, state=self.state, scalars=self.scal)
        self.g.backward(x, y, f, rat=False, grad=True, pins=False, workspace=self.ws, out=self.grads)
        gx = torch.cat([self.grads["dx"], self.zero])[self.idx].sum(1)   # d TNS_g / d cell x
        gy = torch.cat([self.grads["dy"], self.zero])[self.idx].sum(1)
        self.cell_grad = (gx, gy)        # of this step's placement, kept for inspection
        C = self.idx.shape[0]
        self.dxc.grad = torch.cat([2.0 * self.anchor * self.dxc[:C] - gx, self.zero])
        self.dyc.grad = torch.cat([2.0 * self.anchor * self.dyc[:C] - gy, self.zero])
        self.opt.step()
        return self.scal.clone()

    def evaluate(self) -> torch.Tensor:
        x, y = self.coordinates()
        f = self.g.forward(x, y, gamma=self.gamma, smooth=True, state=self.state, scalars=self.scal)
        return f.scalars.clone()

    def run(self, iters: int) -> np.ndarray:
        """iters steps; rows 0..iters-1 are the scalars before each step, the last row after."""
        hist = [self.step() for _ in range(iters)]
        hist.append(self.evaluate())
        return torch.stack(hist).cpu().numpy()
