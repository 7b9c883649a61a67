"""Python binding of libsta (the C ABI in include/sta.h).

Argument marshalling only: every step of the timing sweep runs in the library's HIP
kernels.  PyTorch provides device memory and the stream.  The library must have been
built (``python -m paper_2603_28381_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsta.so")

STA_OK, STA_PENDING = 0, 1
STA_E_INVALID, STA_E_CYCLE, STA_E_NOMEM, STA_E_DEVICE = -1, -2, -3, -4
STA_E_BUSY, STA_E_STATE, STA_E_UNKNOWN_TICKET = -5, -6, -7

STA_SMOOTH = 1 << 0
STA_CANONICAL_IO = 1 << 1
STA_RAT = 1 << 2
STA_GRAD = 1 << 3
STA_GRAD_WNS = 1 << 4
STA_GRAPH = 1 << 5
STA_REQ_FWD, STA_REQ_FWD_BWD = 0, 1
STA_RC_GROUPS, STA_RC_CTE, STA_RC_THREAD = 0, 1, 2
STA_SNAP_OUTER, STA_SNAP_INNER = 0, 1
STA_LEVEL_GROUPS, STA_LEVEL_THREAD, STA_LEVEL_CTE = 0, 1, 2

EXPORTED = ["sta_build_graph", "sta_levelize", "sta_get_levelization", "sta_graph_upload",
            "sta_graph_info_get", "sta_graph_destroy", "sta_batch_create", "sta_batch_pin_map",
            "sta_forward", "sta_backward", "sta_backward_noalloc", "sta_get_schedule", "sta_set_schedule", "sta_tune",
            "sta_set_checkpointing", "sta_get_checkpointing", "sta_set_snapshots", "sta_set_snapshot_layout", "sta_server_create", "sta_server_add_design",
            "sta_submit", "sta_poll", "sta_wait", "sta_release", "sta_server_destroy", "sta_server_stats_get",
            "sta_server_set_max_merge", "sta_tune_cached",
            "sta_profile_enable", "sta_profile_read", "sta_last_error",
            "sta_version"]

KERNELS = ["rc", "fwd_level", "ep_partial", "ep_final", "expand", "ep_seed", "bwd_level", "recompute",
           "rc_adjoint"]

_P = ctypes.c_void_p
_I32P = ctypes.POINTER(ctypes.c_int32)


class StaNetlist(ctypes.Structure):
    _fields_ = [("n_pins", ctypes.c_int32), ("n_nets", ctypes.c_int32), ("n_cells", ctypes.c_int32),
                ("net_offsets", _P), ("net_pins", _P), ("cell_type", _P), ("cell_in_offsets", _P),
                ("cell_in_pins", _P), ("cell_out_pin", _P), ("pin_cap", _P), ("pin_kind", _P), ("pin_parent", _P)]


class StaLibrary(ctypes.Structure):
    _fields_ = [("n_cell_types", ctypes.c_int32), ("arc_offsets", _P), ("arc_unate", _P),
                ("slew_axis", _P), ("load_axis", _P), ("tables", _P)]


class StaConstraints(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in ("t_clk", "setup", "hold", "pi_at", "pi_slew",
                                              "r_per_um", "c_per_um")]


class StaGraphInfo(ctypes.Structure):
    _fields_ = [("n_pins", ctypes.c_int32), ("n_nets", ctypes.c_int32), ("n_cells", ctypes.c_int32),
                ("n_cell_inputs", ctypes.c_int32), ("n_endpoints", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("n_pi_nets", ctypes.c_int32),
                ("max_level_nets", ctypes.c_int32), ("fwd_state_bytes", ctypes.c_int64),
                ("bwd_workspace_bytes", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("n_designs", ctypes.c_int32), ("n_snapshots", ctypes.c_int32)]


class StaSchedule(ctypes.Structure):
    _fields_ = [("sweep_group_log2", ctypes.c_int32), ("flat_group_log2", ctypes.c_int32),
                ("heavy_sinks", ctypes.c_int32), ("rc_scheme", ctypes.c_int32),
                ("fwd_cell_lanes", ctypes.c_int32), ("level_scheme", ctypes.c_int32), ("lane_block", ctypes.c_int32)]


class StaServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int32), ("max_merge", ctypes.c_int32)]


class StaRequest(ctypes.Structure):
    _fields_ = [("design", ctypes.c_int32), ("kind", ctypes.c_int32), ("x", _P), ("y", _P),
                ("gamma_ps", ctypes.c_float)]


class StaResult(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_pins", ctypes.c_int32), ("scalars", ctypes.c_double * 4),
                ("dx", ctypes.POINTER(ctypes.c_float)), ("dy", ctypes.POINTER(ctypes.c_float)),
                ("queue_ms", ctypes.c_double), ("latency_ms", ctypes.c_double)]


class StaServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("captures", ctypes.c_int64), ("capture_ms", ctypes.c_double),
                ("sweeps", ctypes.c_int64), ("merged", ctypes.c_int64), ("slot_grows", ctypes.c_int64),
                ("grow_ms", ctypes.c_double), ("pinned_allocs", ctypes.c_int64), ("pinned_ms", ctypes.c_double)]


class StaFwdOut(ctypes.Structure):
    _fields_ = [("state", _P), ("at", _P), ("slew", _P), ("atg", _P), ("scalars", _P)]


class StaBwdOut(ctypes.Structure):
    _fields_ = [("workspace", _P), ("at", _P), ("slew", _P), ("rat", _P), ("slack", _P),
                ("dx", _P), ("dy", _P), ("grad_scale", ctypes.c_float), ("grad_scale_dev", _P)]


class StaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsta error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libsta.so once.  torch is imported first so the HIP runtime is shared."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libsta.so not built at {path}; run python -m paper_2603_28381_amd.build")
    lib = ctypes.CDLL(path)
    S = ctypes.c_int32
    lib.sta_build_graph.argtypes = [ctypes.POINTER(StaNetlist), ctypes.POINTER(StaLibrary),
                                    ctypes.POINTER(StaConstraints), ctypes.POINTER(_P)]
    lib.sta_build_graph.restype = S
    lib.sta_levelize.argtypes = [_P, _I32P]
    lib.sta_levelize.restype = S
    lib.sta_get_levelization.argtypes = [_P, _P, _P, _P, _P]
    lib.sta_get_levelization.restype = S
    lib.sta_graph_upload.argtypes = [_P]
    lib.sta_graph_upload.restype = S
    lib.sta_graph_info_get.argtypes = [_P, ctypes.POINTER(StaGraphInfo)]
    lib.sta_graph_info_get.restype = S
    lib.sta_graph_destroy.argtypes = [_P]
    lib.sta_graph_destroy.restype = None
    lib.sta_forward.argtypes = [_P, _P, _P, ctypes.POINTER(StaFwdOut), ctypes.c_uint32, ctypes.c_float, _P]
    lib.sta_forward.restype = S
    lib.sta_backward.argtypes = [_P, _P, _P, ctypes.POINTER(StaFwdOut), ctypes.POINTER(StaBwdOut),
                                 ctypes.c_uint32, ctypes.c_float, _P]
    lib.sta_backward.restype = S
    lib.sta_backward_noalloc.argtypes = lib.sta_backward.argtypes
    lib.sta_backward_noalloc.restype = S
    lib.sta_batch_create.argtypes = [ctypes.POINTER(_P), ctypes.c_int32, ctypes.POINTER(_P)]
    lib.sta_batch_create.restype = S
    lib.sta_batch_pin_map.argtypes = [_P, _P, _P]
    lib.sta_batch_pin_map.restype = S
    lib.sta_get_schedule.argtypes = [_P, ctypes.POINTER(StaSchedule)]
    lib.sta_get_schedule.restype = S
    lib.sta_set_schedule.argtypes = [_P, ctypes.POINTER(StaSchedule)]
    lib.sta_set_schedule.restype = S
    lib.sta_tune.argtypes = [_P, _P, _P, ctypes.c_float, ctypes.c_int32, ctypes.POINTER(StaSchedule), _P]
    lib.sta_tune.restype = S
    lib.sta_set_snapshots.argtypes = [_P, ctypes.c_int32]
    lib.sta_set_snapshots.restype = S
    lib.sta_set_snapshot_layout.argtypes = [_P, ctypes.c_int32]
    lib.sta_set_snapshot_layout.restype = S
    lib.sta_set_checkpointing.argtypes = [_P, ctypes.c_int32]
    lib.sta_set_checkpointing.restype = S
    lib.sta_get_checkpointing.argtypes = [_P, _I32P, _I32P, _I32P]
    lib.sta_get_checkpointing.restype = S
    lib.sta_server_create.argtypes = [ctypes.POINTER(StaServerConfig), ctypes.POINTER(_P)]
    lib.sta_server_create.restype = S
    lib.sta_server_add_design.argtypes = [_P, _P, _P, _P, _I32P]
    lib.sta_server_add_design.restype = S
    lib.sta_submit.argtypes = [_P, ctypes.POINTER(StaRequest), ctypes.POINTER(ctypes.c_uint64)]
    lib.sta_submit.restype = S
    for name in ("sta_poll", "sta_wait"):
        getattr(lib, name).argtypes = [_P, ctypes.c_uint64, ctypes.POINTER(StaResult)]
        getattr(lib, name).restype = S
    lib.sta_release.argtypes = [_P, ctypes.c_uint64]
    lib.sta_release.restype = S
    lib.sta_server_destroy.argtypes = [_P]
    lib.sta_server_destroy.restype = None
    lib.sta_server_stats_get.argtypes = [_P, ctypes.POINTER(StaServerStats)]
    lib.sta_server_stats_get.restype = S
    lib.sta_tune_cached.argtypes = [_P, ctypes.POINTER(StaSchedule)]
    lib.sta_tune_cached.restype = S
    lib.sta_server_set_max_merge.argtypes = [_P, ctypes.c_int32]
    lib.sta_server_set_max_merge.restype = S
    lib.sta_profile_enable.argtypes = [_P, ctypes.c_int32]
    lib.sta_profile_enable.restype = S
    lib.sta_profile_read.argtypes = [_P, _P, _P]
    lib.sta_profile_read.restype = S
    lib.sta_last_error.argtypes = []
    lib.sta_last_error.restype = ctypes.c_char_p
    lib.sta_version.argtypes = []
    lib.sta_version.restype = ctypes.c_int32
    _lib = lib
    return lib


def _check(code: int):
    if code != STA_OK:
        raise StaError(code, (_lib.sta_last_error() or b"").decode())


def _ptr(a) -> int | None:
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.data_ptr()
    return a.ctypes.data


def _stream_handle(stream=None) -> int | None:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream or None


def _dev_f32(a, device) -> torch.Tensor:
    t = torch.as_tensor(a)
    if t.dtype != torch.float32 or t.device != torch.device(device) or not t.is_contiguous():
        t = t.to(device=device, dtype=torch.float32).contiguous()
    return t


@dataclass
class Forward:
    """Result of Graph.forward: the opaque state plus the requested outputs."""
    state: torch.Tensor
    scalars: torch.Tensor          # float64 [4]: WNS, TNS, WNS_g, TNS_g
    at: torch.Tensor | None = None
    slew: torch.Tensor | None = None
    atg: torch.Tensor | None = None
    gamma: float = 10.0
    canonical: bool = False


class Graph:
    """A netlist handed to libsta: validated, levelized and (lazily) uploaded."""

    def __init__(self, netlist: dict, library: dict, constraints: dict):
        lib = load_library()
        self._keep = []

        def arr(v, dt):
            a = np.ascontiguousarray(v, dtype=dt)
            self._keep.append(a)
            return a.ctypes.data

        nl = StaNetlist(int(netlist["n_pins"]), int(netlist["n_nets"]), int(netlist["n_cells"]),
                        arr(netlist["net_offsets"], np.int32), arr(netlist["net_pins"], np.int32),
                        arr(netlist["cell_type"], np.int32), arr(netlist["cell_in_offsets"], np.int32),
                        arr(netlist["cell_in_pins"], np.int32), arr(netlist["cell_out_pin"], np.int32),
                        arr(netlist["pin_cap"], np.float32), arr(netlist["pin_kind"], np.int8),
                        None if netlist.get("pin_parent") is None else arr(netlist["pin_parent"], np.int32))
        lb = StaLibrary(int(library["n_cell_types"]), arr(library["arc_offsets"], np.int32),
                        arr(library["arc_unate"], np.int8), arr(library["slew_axis"], np.float32),
                        arr(library["load_axis"], np.float32), arr(library["tables"], np.float32))
        cs = StaConstraints(*[float(constraints[k]) for k in ("t_clk", "setup", "hold", "pi_at", "pi_slew",
                                                               "r_per_um", "c_per_um")])
        h = _P()
        _check(lib.sta_build_graph(ctypes.byref(nl), ctypes.byref(lb), ctypes.byref(cs), ctypes.byref(h)))
        self._keep = []
        self._h = h
        self.n_pins = int(netlist["n_pins"])

    @classmethod
    def from_design(cls, d) -> "Graph":
        """From a gen.netlist.Design (numpy arrays)."""
        nl = dict(n_pins=d.n_pins, n_nets=d.n_nets, n_cells=d.n_cells, net_offsets=d.net_offsets,
                  net_pins=d.net_pins, cell_type=d.cell_type, cell_in_offsets=d.cell_in_offsets,
                  cell_in_pins=d.cell_in_pins, cell_out_pin=d.cell_out_pin, pin_cap=d.pin_cap,
                  pin_kind=d.pin_kind, pin_parent=getattr(d, "pin_parent", None))
        lb = dict(n_cell_types=d.lib.n_cell_types, arc_offsets=d.lib.arc_offsets, arc_unate=d.lib.arc_unate,
                  slew_axis=d.lib.slew_axis, load_axis=d.lib.load_axis, tables=d.lib.tables)
        c = d.cons
        cs = dict(t_clk=c.t_clk, setup=c.setup, hold=c.hold, pi_at=c.pi_at, pi_slew=c.pi_slew,
                  r_per_um=c.r_per_um, c_per_um=c.c_per_um)
        return cls(nl, lb, cs)

    @classmethod
    def batch(cls, graphs: list["Graph"]) -> "Graph":
        """One graph sweeping several designs (or placement snapshots: repeat a graph)."""
        load_library()
        arr = (_P * len(graphs))(*[g._h.value for g in graphs])
        h = _P()
        _check(_lib.sta_batch_create(arr, len(graphs), ctypes.byref(h)))
        obj = cls.__new__(cls)
        obj._keep = []
        obj._h = h
        obj.n_pins = sum(g.n_pins for g in graphs)
        return obj

    def batch_pin_map(self) -> tuple[np.ndarray, np.ndarray]:
        """(design, pin) of every canonical pin of a levelized batch."""
        P = self.n_pins
        dsg = np.empty(P, np.int32)
        pin = np.empty(P, np.int32)
        _check(_lib.sta_batch_pin_map(self._h, dsg.ctypes.data, pin.ctypes.data))
        return dsg, pin

    @property
    def handle(self) -> int:
        return self._h.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.sta_graph_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def levelize(self) -> int:
        n = ctypes.c_int32()
        _check(_lib.sta_levelize(self._h, ctypes.byref(n)))
        return n.value

    def info(self) -> dict:
        i = StaGraphInfo()
        _check(_lib.sta_graph_info_get(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in StaGraphInfo._fields_}

    def levelization(self) -> dict:
        inf = self.info()
        level = np.empty(inf["n_nets"], np.int32)
        loff = np.empty(inf["n_levels"] + 1, np.int32)
        nperm = np.empty(inf["n_nets"], np.int32)
        pperm = np.empty(inf["n_pins"], np.int32)
        _check(_lib.sta_get_levelization(self._h, level.ctypes.data, loff.ctypes.data, nperm.ctypes.data,
                                         pperm.ctypes.data))
        return dict(level=level, level_offsets=loff, net_perm=nperm, pin_perm=pperm)

    def upload(self):
        _check(_lib.sta_graph_upload(self._h))

    def schedule(self) -> dict:
        sch = StaSchedule()
        _check(_lib.sta_get_schedule(self._h, ctypes.byref(sch)))
        return {k: getattr(sch, k) for k, _ in StaSchedule._fields_}

    def set_schedule(self, sweep_group_log2: int, flat_group_log2: int, heavy_sinks: int,
                     rc_scheme: int | str = 0, fwd_cell_lanes: int = 16, level_scheme: int | str = 0,
                     lane_block: int = 512):
        """rc_scheme: 0 / "groups" (lane groups, Alg. 1), 1 / "cte" (task pool, Alg. 2),
        2 / "thread" (one thread per net).  fwd_cell_lanes: 16, 8 or 4 lanes per cell in the
        forward level kernel.  level_scheme: 0 / "groups", 1 / "thread" (one thread per net
        and cell in every stage) or 2 / "cte" (the level kernels over a workgroup task pool).
        lane_block: threads per workgroup of the snapshot-lane backward level (256, 512, 1024)."""
        rc = {"groups": STA_RC_GROUPS, "cte": STA_RC_CTE, "thread": STA_RC_THREAD}.get(rc_scheme, rc_scheme)
        lv = {"groups": STA_LEVEL_GROUPS, "thread": STA_LEVEL_THREAD, "cte": STA_LEVEL_CTE}.get(level_scheme,
                                                                                               level_scheme)
        sch = StaSchedule(sweep_group_log2, flat_group_log2, heavy_sinks, int(rc), int(fwd_cell_lanes), int(lv),
                          int(lane_block))
        _check(_lib.sta_set_schedule(self._h, ctypes.byref(sch)))

    def tune(self, x, y, gamma: float = 10.0, reps: int = 3, stream=None) -> dict:
        """Time the candidate schedules (lane groups, then the RC mappings, then 8 and 4 lanes
        per forward cell, then the CTE and thread-per-net level schemes; with snapshot lanes the
        backward workgroup size) on these coordinates and keep the fastest."""
        dev = x.device if isinstance(x, torch.Tensor) and x.is_cuda else torch.device("cuda")
        x = _dev_f32(x, dev)
        y = _dev_f32(y, dev)
        sch = StaSchedule()
        _check(_lib.sta_tune(self._h, _ptr(x), _ptr(y), float(gamma), int(reps), ctypes.byref(sch),
                             _stream_handle(stream)))
        return {k: getattr(sch, k) for k, _ in StaSchedule._fields_}

    def tune_cached(self) -> dict | None:
        """Set the schedule sta_tune last found for this graph's shape bucket (pin count's
        power of two, snapshots, layout, checkpointing, trees, batch); None if there is none."""
        sch = StaSchedule()
        code = _lib.sta_tune_cached(self._h, ctypes.byref(sch))
        if code == STA_E_STATE and (_lib.sta_last_error() or b"").startswith(b"no tuned schedule"):
            return None
        _check(code)
        return {k: getattr(sch, k) for k, _ in StaSchedule._fields_}

    def set_snapshots(self, n: int):
        """Sweep n placement snapshots of this graph per call (per-call arrays gain a leading
        snapshot dimension)."""
        _check(_lib.sta_set_snapshots(self._h, int(n)))

    def set_snapshot_layout(self, inner: bool):
        """inner: every per-call array has the snapshot innermost ([pins][S]...), and the
        lanes of a wave take snapshots (STA_SNAP_INNER); else snapshots outermost."""
        _check(_lib.sta_set_snapshot_layout(self._h, STA_SNAP_INNER if inner else STA_SNAP_OUTER))
        self._inner = bool(inner)

    def _pin_shape(self, S: int, *tail) -> tuple:
        """Shape of a per-pin array of one call: [P, *tail], with the snapshots outermost or
        (snapshot-inner layout) right after the pin."""
        P = self.n_pins
        if S <= 1:
            return (P,) + tail
        return (P, S) + tail if getattr(self, "_inner", False) else (S, P) + tail

    def set_checkpointing(self, stride_levels: int = -1):
        """Per-level checkpointing of the arrival state: 0 off, < 0 picks ceil(sqrt(L-1))."""
        _check(_lib.sta_set_checkpointing(self._h, int(stride_levels)))

    def checkpointing(self) -> dict:
        k, slots, kept = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.sta_get_checkpointing(self._h, ctypes.byref(k), ctypes.byref(slots), ctypes.byref(kept)))
        return dict(stride_levels=k.value, record_slots=slots.value, kept_nets=kept.value)

    def profile(self, on: bool = True):
        _check(_lib.sta_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> dict:
        n = np.zeros(len(KERNELS), np.int64)
        ms = np.zeros(len(KERNELS), np.float64)
        _check(_lib.sta_profile_read(self._h, n.ctypes.data, ms.ctypes.data))
        return {k: (int(n[i]), float(ms[i])) for i, k in enumerate(KERNELS)}

    # ------------------------------------------------------------------ sweeps
    def new_state(self, device="cuda") -> torch.Tensor:
        return torch.empty(self.info()["fwd_state_bytes"], dtype=torch.uint8, device=device)

    def new_workspace(self, device="cuda") -> torch.Tensor:
        return torch.empty(self.info()["bwd_workspace_bytes"], dtype=torch.uint8, device=device)

    def forward(self, x, y, gamma: float = 10.0, smooth: bool = True, canonical: bool = False,
                pins: bool = False, state: torch.Tensor | None = None, scalars: torch.Tensor | None = None,
                stream=None, capture: bool = False, out: dict | None = None) -> Forward:
        dev = x.device if isinstance(x, torch.Tensor) and x.is_cuda else torch.device("cuda")
        x = _dev_f32(x, dev)
        y = _dev_f32(y, dev)
        inf = self.info()
        S, nd = inf["n_snapshots"], inf["n_designs"]
        lead = (S,) if S > 1 else ()
        state = self.new_state(dev) if state is None else state
        if scalars is None:
            scalars = torch.empty(lead + ((nd, 4) if nd > 1 else (4,)), dtype=torch.float64, device=dev)
        at = slew = atg = None
        if out is not None:
            at, slew, atg = out.get("at"), out.get("slew"), out.get("atg")
        elif pins:
            at = torch.empty(self._pin_shape(S, 4), dtype=torch.float32, device=dev)
            slew = torch.empty(self._pin_shape(S, 4), dtype=torch.float32, device=dev)
            atg = torch.empty(self._pin_shape(S, 2), dtype=torch.float32, device=dev) if smooth else None
        fo = StaFwdOut(_ptr(state), _ptr(at), _ptr(slew), _ptr(atg), _ptr(scalars))
        flags = ((STA_SMOOTH if smooth else 0) | (STA_CANONICAL_IO if canonical else 0)
                 | (STA_GRAPH if capture else 0))
        _check(_lib.sta_forward(self._h, _ptr(x), _ptr(y), ctypes.byref(fo), flags, float(gamma),
                                _stream_handle(stream)))
        return Forward(state, scalars, at, slew, atg, float(gamma), canonical)

    def backward(self, x, y, fwd: Forward, rat: bool = True, grad: bool = True, wns: bool = False,
                 pins: bool = True, grad_scale: float = 1.0, grad_scale_dev: torch.Tensor | None = None,
                 workspace: torch.Tensor | None = None, out: dict | None = None, stream=None,
                 capture: bool = False, noalloc: bool = False) -> dict:
        """noalloc: run sta_backward_noalloc, whose workspace is the library's fixed device
        array (no workspace tensor; outputs still come from `out` or are allocated here)."""
        dev = fwd.state.device
        x = _dev_f32(x, dev)
        y = _dev_f32(y, dev)
        S = self.info()["n_snapshots"]
        if noalloc and (workspace is not None or capture):
            raise ValueError("noalloc takes neither a workspace nor capture")
        ws = None if noalloc else (self.new_workspace(dev) if workspace is None else workspace)
        if out is None:
            out = {}
            if pins:
                for k in ("at", "slew"):
                    out[k] = torch.empty(self._pin_shape(S, 4), dtype=torch.float32, device=dev)
            if rat:
                out["rat"] = torch.empty(self._pin_shape(S, 4), dtype=torch.float32, device=dev)
                out["slack"] = torch.empty(self._pin_shape(S, 4), dtype=torch.float32, device=dev)
            if grad:
                out["dx"] = torch.empty(self._pin_shape(S), dtype=torch.float32, device=dev)
                out["dy"] = torch.empty(self._pin_shape(S), dtype=torch.float32, device=dev)
        bo = StaBwdOut(_ptr(ws), _ptr(out.get("at")), _ptr(out.get("slew")), _ptr(out.get("rat")),
                       _ptr(out.get("slack")), _ptr(out.get("dx")), _ptr(out.get("dy")), float(grad_scale),
                       _ptr(grad_scale_dev))
        fo = StaFwdOut(_ptr(fwd.state), None, None, None, None)
        flags = ((STA_RAT if rat else 0) | (STA_GRAD if grad else 0) | (STA_GRAD_WNS if wns else 0)
                 | (STA_CANONICAL_IO if fwd.canonical else 0) | (STA_GRAPH if capture else 0))
        call = _lib.sta_backward_noalloc if noalloc else _lib.sta_backward
        _check(call(self._h, _ptr(x), _ptr(y), ctypes.byref(fo), ctypes.byref(bo), flags, float(fwd.gamma),
                    _stream_handle(stream)))
        return out


class Server:
    """Serving loop of libsta: resident designs, admission against a device-memory budget
    and continuous batching of requests (the C server's scheduler thread runs them)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 8, queue_capacity: int = 4096, max_merge: int = 8):
        """max_merge: waiting requests of one design, kind and gamma swept together as
        snapshots of one launch sequence, at most (a power of two; 1 runs each alone)."""
        load_library()
        cfg = StaServerConfig(int(hbm_budget_bytes), int(max_slots), int(queue_capacity), int(max_merge))
        h = _P()
        _check(_lib.sta_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._graphs = []

    def add_design(self, graph: Graph, x, y) -> int:
        """Make a levelized graph resident with host coordinates (original pin order)."""
        xa = np.ascontiguousarray(x, dtype=np.float32)
        ya = np.ascontiguousarray(y, dtype=np.float32)
        i = ctypes.c_int32()
        _check(_lib.sta_server_add_design(self._h, graph.handle, xa.ctypes.data, ya.ctypes.data, ctypes.byref(i)))
        self._graphs.append(graph)
        return i.value

    def submit(self, design: int, grad: bool = False, x=None, y=None, gamma: float = 10.0) -> int:
        xa = ya = None
        if x is not None:
            xa = np.ascontiguousarray(x, dtype=np.float32)
            ya = np.ascontiguousarray(y, dtype=np.float32)
        r = StaRequest(int(design), STA_REQ_FWD_BWD if grad else STA_REQ_FWD,
                       None if xa is None else xa.ctypes.data, None if ya is None else ya.ctypes.data, float(gamma))
        t = ctypes.c_uint64()
        _check(_lib.sta_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        return t.value

    @staticmethod
    def _result(r: StaResult, grad: bool = True) -> dict:
        out = dict(scalars=np.array(r.scalars[:], np.float64), queue_ms=r.queue_ms, latency_ms=r.latency_ms,
                   kind=r.kind)
        if r.dx and grad:
            out["dx"] = np.ctypeslib.as_array(r.dx, (r.n_pins,)).copy()
            out["dy"] = np.ctypeslib.as_array(r.dy, (r.n_pins,)).copy()
        return out

    def poll(self, ticket: int) -> dict | None:
        r = StaResult()
        code = _lib.sta_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(r))
        if code == STA_PENDING:
            return None
        _check(code)
        return self._result(r)

    def wait(self, ticket: int, release: bool = True, grad: bool = True) -> dict:
        """Blocks until the request is done; grad=False leaves out the copy of its gradient."""
        r = StaResult()
        _check(_lib.sta_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(r)))
        out = self._result(r, grad)
        if release:
            self.release(ticket)
        return out

    def release(self, ticket: int):
        _check(_lib.sta_release(self._h, ctypes.c_uint64(ticket)))

    def set_max_merge(self, max_merge: int):
        """Waiting requests swept together as snapshots from now on, at most (1: each alone)."""
        _check(_lib.sta_server_set_max_merge(self._h, int(max_merge)))

    def stats(self) -> dict:
        st = StaServerStats()
        _check(_lib.sta_server_stats_get(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in StaServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.sta_server_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SmoothedSlack(torch.autograd.Function):
    """Smoothed TNS (or WNS) of a placement as a differentiable function of pin x, y.

    forward returns the float64 scalar TNS_g (WNS_g with which="wns"); backward runs the
    fused backward sweep of libsta and returns d/dx, d/dy scaled by the incoming gradient.
    On a batch of designs or several placement snapshots the scalar is the sum of the
    per-design (per-snapshot) objectives: the backward seeds every design and snapshot with
    the same incoming gradient, which is the gradient of that sum.
    """

    @staticmethod
    def forward(ctx, x, y, graph: Graph, gamma: float = 10.0, which: str = "tns"):
        fwd = graph.forward(x, y, gamma=gamma, smooth=True)
        ctx.graph, ctx.fwd, ctx.which = graph, fwd, which
        ctx.save_for_backward(x, y)
        return fwd.scalars[..., 3 if which == "tns" else 2].sum()

    @staticmethod
    def backward(ctx, g):
        x, y = ctx.saved_tensors
        gd = g.detach().to(torch.float64).reshape(1).contiguous()
        out = ctx.graph.backward(x, y, ctx.fwd, rat=False, grad=True, wns=ctx.which == "wns", pins=False,
                                 grad_scale_dev=gd)
        return out["dx"].to(x.dtype), out["dy"].to(y.dtype), None, None, None


def smoothed_tns(x, y, graph: Graph, gamma: float = 10.0) -> torch.Tensor:
    return SmoothedSlack.apply(x, y, graph, gamma, "tns")


def smoothed_wns(x, y, graph: Graph, gamma: float = 10.0) -> torch.Tensor:
    return SmoothedSlack.apply(x, y, graph, gamma, "wns")
