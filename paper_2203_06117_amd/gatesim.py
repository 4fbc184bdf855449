"""Python binding of libgatesim.so (the C ABI in include/gatesim.h).

Argument marshalling only: every step of the simulation runs in the HIP
library.  If the library is not built this module raises at import time;
there is no fallback.  PyTorch is used, when given, only for the stream and
for an optional caller-owned device arena.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GATESIM_LIBRARY names another build of the same library (same ABI)
LIB_PATH = os.environ.get("GATESIM_LIBRARY") or os.path.join(_HERE, "libgatesim.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
# PyTorch ships its own HIP runtime, whose libraries request it under an
# unversioned name.  Loading torch first makes this library bind to that
# same runtime (same soname); loading it after this library would put a
# second HIP runtime in the process, and one of them would see no device.
try:
    import torch  # noqa: F401
except ImportError:
    pass
_lib = C.CDLL(LIB_PATH)

GS_OK, GS_E_INVALID, GS_E_NOT_DAG, GS_E_NOMEM, GS_E_DEVICE, GS_E_STATE, GS_E_BUSY, GS_E_CAPACITY = \
    0, -1, -2, -3, -4, -5, -6, -7
SCHED_LEVELS, SCHED_GRAPH = 0, 1
REQ_WINDOW, REQ_EDIT = 0, 1

ARC_DTYPE = np.dtype([("gate", "<i4"), ("pin", "i1"), ("cond_pin", "i1"), ("cond_val", "i1"),
                      ("in_edge", "i1"), ("rise", "<i4"), ("fall", "<i4")])
assert ARC_DTYPE.itemsize == 16


class Options(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("hbm_budget", C.c_uint64),
                ("arena", C.c_void_p), ("arena_bytes", C.c_uint64), ("window_cycles", C.c_int32),
                ("lds_cap", C.c_int32), ("waves_per_block", C.c_int32), ("schedule", C.c_int32),
                ("timing", C.c_int32), ("tiles_per_wave", C.c_int32), ("autotune", C.c_int32),
                ("wire_transport", C.c_int32), ("release_dead", C.c_int32), ("reserved", C.c_int32 * 3)]


class DesignInfo(C.Structure):
    _fields_ = [("n_inputs", C.c_int32), ("n_gates", C.c_int32), ("n_levels", C.c_int32),
                ("max_pins", C.c_int32), ("n_fanin", C.c_int64), ("has_wires", C.c_int32),
                ("zero_delay", C.c_int32), ("max_delay_ps", C.c_int32), ("reserved", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("gate_eval_ms", C.c_double), ("expand_ms", C.c_double), ("wall_ms", C.c_double),
                ("gate_eval_launches", C.c_int64), ("windows", C.c_int64), ("window_retries", C.c_int64),
                ("gate_cycles", C.c_int64), ("spilled_lanes", C.c_int64), ("arena_words", C.c_int64),
                ("graph_launches", C.c_int64), ("unstaged_groups", C.c_int64), ("queue_overflows", C.c_int64),
                ("release_peak_words", C.c_int64), ("reserved", C.c_int64 * 2)]


class Tuning(C.Structure):
    _fields_ = [("lds_cap", C.c_int32), ("waves_per_block", C.c_int32), ("tiles_per_wave", C.c_int32),
                ("reserved", C.c_int32), ("trial_ms", C.c_double)]


class Job(C.Structure):
    _fields_ = [("design", C.c_int32), ("stim", C.c_int32), ("cycle_begin", C.c_int32), ("cycle_end", C.c_int32)]


class ArcEdit(C.Structure):
    _fields_ = [("gate", C.c_int32), ("pin", C.c_int8), ("cond_pin", C.c_int8), ("cond_val", C.c_int8),
                ("in_edge", C.c_int8), ("rise_ps", C.c_int32), ("fall_ps", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("design", C.c_int32), ("stim", C.c_int32), ("cycle_begin", C.c_int32),
                ("cycle_end", C.c_int32), ("n_edits", C.c_int32), ("edits", C.POINTER(ArcEdit))]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_nets", C.c_int32), ("tc", C.POINTER(C.c_int64)),
                ("t0", C.POINTER(C.c_int64)), ("t1", C.POINTER(C.c_int64)), ("ig", C.POINTER(C.c_int64)),
                ("gate_cycles", C.c_int64),
                ("t_submit_ns", C.c_uint64), ("t_admit_ns", C.c_uint64), ("t_done_ns", C.c_uint64)]


P = C.c_void_p
I32 = C.c_int32
_SIGS = {
    "gs_default_options": (None, [C.POINTER(Options)]),
    "gs_create": (I32, [C.POINTER(Options), C.POINTER(P)]),
    "gs_destroy": (I32, [P]),
    "gs_last_error": (C.c_char_p, [P]),
    "gs_load_cells": (I32, [P, I32, P, P]),
    "gs_load_netlist": (I32, [P, I32, I32, P, P, P, C.POINTER(I32)]),
    "gs_load_arcs": (I32, [P, I32, C.c_int64, P]),
    "gs_load_wires": (I32, [P, I32, P, P]),
    "gs_load_stimulus": (I32, [P, I32, I32, I32, P, P, P, C.POINTER(I32)]),
    "gs_segment_stimulus": (I32, [P, I32, I32, C.POINTER(I32)]),
    "gs_continuous_stimulus": (I32, [P, I32, I32, C.POINTER(I32)]),
    "gs_glitch_profile": (I32, [P, I32, I32, I32, I32, P]),
    "gs_cycle_profile": (I32, [P, I32, I32, I32, I32, P, P]),
    "gs_simulate": (I32, [P, I32, I32, I32, I32]),
    "gs_simulate_noalloc": (I32, [P, I32, I32, I32, I32]),
    "gs_read_saif": (I32, [P, I32, P, P, P, I32]),
    "gs_read_saif_ig": (I32, [P, I32, P, P, P, P, I32]),
    "gs_read_waveform": (I32, [P, I32, I32, I32, I32, C.POINTER(I32), P, I32, C.POINTER(I32)]),
    "gs_get_design_info": (I32, [P, I32, C.POINTER(DesignInfo)]),
    "gs_get_levels": (I32, [P, I32, P]),
    "gs_get_stats": (I32, [P, C.POINTER(Stats), I32]),
    "gs_check_netlist": (I32, [I32, P, I32, I32, P, P, P]),
    "gs_check_arcs": (I32, [I32, P, I32, P, C.c_int64, P]),
    "gs_check_stimulus": (I32, [I32, I32, I32, P, P, P]),
    "gs_simulate_batch": (I32, [P, I32, C.POINTER(Job)]),
    "gs_autotune": (I32, [P, I32, I32, I32, I32, C.POINTER(Tuning)]),
    "gs_serve_start": (I32, [P, I32, P, P, P, P, I32]),
    "gs_submit": (I32, [P, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "gs_poll": (I32, [P, C.c_uint64, I32, C.POINTER(Result)]),
    "gs_release": (I32, [P, C.c_uint64]),
    "gs_serve_stop": (I32, [P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTS = sorted(_SIGS)


class GateSimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def check_netlist(cell_pins, n_inputs, cell_of_gate, fanin_ptr, fanin_net) -> int:
    cp, cg, fp, fn = _c(cell_pins, np.uint8), _c(cell_of_gate, np.int32), _c(fanin_ptr, np.int64), _c(fanin_net, np.int32)
    return _lib.gs_check_netlist(len(cp), _p(cp), int(n_inputs), len(cg), _p(cg), _p(fp), _p(fn))


def check_arcs(cell_pins, cell_of_gate, arcs) -> int:
    cp, cg = _c(cell_pins, np.uint8), _c(cell_of_gate, np.int32)
    a = arcs_array(arcs)
    return _lib.gs_check_arcs(len(cp), _p(cp), len(cg), _p(cg), len(a), _p(a))


def check_stimulus(n_inputs, period, n_cycles, init, toggle_ptr, toggle_ps) -> int:
    i, tp, ts = _c(init, np.uint8), _c(toggle_ptr, np.int64), _c(toggle_ps, np.int64)
    return _lib.gs_check_stimulus(int(n_inputs), int(period), int(n_cycles), _p(i), _p(tp), _p(ts))


def last_error() -> str:
    return _lib.gs_last_error(None).decode()


def arcs_array(arcs) -> np.ndarray:
    """SoA dict (gate, pin, cond_pin, cond_val, rise, fall[, in_edge]) -> gs_arc records."""
    if isinstance(arcs, np.ndarray) and arcs.dtype == ARC_DTYPE:
        return np.ascontiguousarray(arcs)
    n = len(arcs["gate"])
    a = np.zeros(n, dtype=ARC_DTYPE)
    for k in ("gate", "pin", "cond_pin", "cond_val", "rise", "fall"):
        a[k] = arcs[k]
    a["in_edge"] = arcs["in_edge"] if "in_edge" in arcs else 0
    return a


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class GateSim:
    """One library context on one GPU."""

    def __init__(self, device: int = 0, stream=None, hbm_budget: int = 0, arena=None,
                 window_cycles: int = 0, lds_cap: int = 0, waves_per_block: int = 4,
                 schedule: int = SCHED_LEVELS, timing: bool = False, tiles_per_wave: int = 0,
                 autotune: bool = False, wire_transport: bool = False, release_dead: bool = False):
        o = Options()
        _lib.gs_default_options(C.byref(o))
        o.device = device
        o.stream = _stream_handle(stream)
        o.hbm_budget = hbm_budget
        self._arena = arena
        if arena is not None:
            o.arena = int(arena.data_ptr())
            o.arena_bytes = int(arena.numel() * arena.element_size())
        o.window_cycles = window_cycles
        o.lds_cap = lds_cap
        o.waves_per_block = waves_per_block
        o.schedule = schedule
        o.timing = 1 if timing else 0
        o.tiles_per_wave = tiles_per_wave
        o.autotune = 1 if autotune else 0
        o.wire_transport = 1 if wire_transport else 0
        o.release_dead = 1 if release_dead else 0
        h = P()
        st = _lib.gs_create(C.byref(o), C.byref(h))
        if st != GS_OK:
            raise GateSimError(st, last_error())
        self._h = h
        self.n_nets = {}

    # -- plumbing --------------------------------------------------------
    def _chk(self, st):
        if st != GS_OK:
            raise GateSimError(st, _lib.gs_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            _lib.gs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- loading ---------------------------------------------------------
    def load_cells(self, n_pins, truth):
        np_, tr = _c(n_pins, np.uint8), _c(truth, np.uint64)
        self._chk(_lib.gs_load_cells(self._h, len(np_), _p(np_), _p(tr)))

    def load_netlist(self, n_inputs, cell_of_gate, fanin_ptr, fanin_net) -> int:
        cg, fp, fn = _c(cell_of_gate, np.int32), _c(fanin_ptr, np.int64), _c(fanin_net, np.int32)
        d = I32()
        self._chk(_lib.gs_load_netlist(self._h, int(n_inputs), len(cg), _p(cg), _p(fp), _p(fn), C.byref(d)))
        self.n_nets[d.value] = int(n_inputs) + len(cg)
        return d.value

    def load_arcs(self, design, arcs):
        a = arcs_array(arcs)
        self._chk(_lib.gs_load_arcs(self._h, design, len(a), _p(a)))

    def load_wires(self, design, rise=None, fall=None):
        r = None if rise is None else _c(rise, np.int32)
        f = None if fall is None else _c(fall, np.int32)
        self._chk(_lib.gs_load_wires(self._h, design, _p(r), _p(f)))

    def load_stimulus(self, design, period, n_cycles, init, toggle_ptr, toggle_ps) -> int:
        i, tp, ts = _c(init, np.uint8), _c(toggle_ptr, np.int64), _c(toggle_ps, np.int64)
        s = I32()
        self._chk(_lib.gs_load_stimulus(self._h, design, int(period), int(n_cycles), _p(i), _p(tp), _p(ts),
                                        C.byref(s)))
        return s.value

    def glitch_profile(self, design, stim, cycle_begin, cycle_end) -> np.ndarray:
        """Simulates like ``simulate`` and returns the glitch toggles of every
        cycle of the range summed over all nets (int64 array)."""
        out = np.zeros(max(0, int(cycle_end) - int(cycle_begin)), dtype=np.int64)
        self._chk(_lib.gs_glitch_profile(self._h, int(design), int(stim), int(cycle_begin), int(cycle_end), _p(out)))
        return out

    def cycle_profile(self, design, stim, cycle_begin, cycle_end):
        """Simulates like ``simulate``; returns (glitch, late) per cycle of the
        range: glitch toggles over all nets, and nets whose activity reaches
        the end of the cycle (0 everywhere but the last cycle certifies that
        the cycle-by-cycle result equals a continuous run)."""
        n = max(0, int(cycle_end) - int(cycle_begin))
        glitch = np.zeros(n, dtype=np.int64)
        late = np.zeros(n, dtype=np.int64)
        self._chk(_lib.gs_cycle_profile(self._h, int(design), int(stim), int(cycle_begin), int(cycle_end),
                                        _p(glitch), _p(late)))
        return glitch, late

    def segment_stimulus(self, stim, segment_cycles) -> int:
        """A view of ``stim`` whose cycles are groups of ``segment_cycles``
        cycles, each simulated continuously (returns the new stimulus id)."""
        s = I32()
        self._chk(_lib.gs_segment_stimulus(self._h, int(stim), int(segment_cycles), C.byref(s)))
        return s.value

    def continuous_stimulus(self, stim, segment_cycles) -> int:
        """Like ``segment_stimulus`` (the same results), with one lane per
        cycle and the pending edge carried from cycle to cycle."""
        s = I32()
        self._chk(_lib.gs_continuous_stimulus(self._h, int(stim), int(segment_cycles), C.byref(s)))
        return s.value

    def load_work(self, work: dict, cells_loaded: bool = False):
        """Loads a workload dict (the seeded generator's format); returns (design, stim)."""
        n = work["netlist"]
        if not cells_loaded:
            self.load_cells(n["cell_pins"], n["cell_truth"])
        d = self.load_netlist(n["n_inputs"], n["cell_of_gate"], n["fanin_ptr"], n["fanin_net"])
        if work.get("wires") is not None:
            self.load_wires(d, work["wires"]["rise"], work["wires"]["fall"])
        self.load_arcs(d, work["arcs"])
        s = work["stimulus"]
        st = self.load_stimulus(d, s["period"], s["n_cycles"], s["init"], s["toggle_ptr"], s["toggle_ps"])
        return d, st

    # -- running ---------------------------------------------------------
    def simulate(self, design, stim, cycle_begin, cycle_end):
        self._chk(_lib.gs_simulate(self._h, design, stim, int(cycle_begin), int(cycle_end)))

    def simulate_noalloc(self, design, stim, cycle_begin, cycle_end):
        """gs_simulate_noalloc: the same result through the static device scratch."""
        self._chk(_lib.gs_simulate_noalloc(self._h, design, stim, int(cycle_begin), int(cycle_end)))

    def read_saif(self, design, reset=False, out=None):
        """TC, T0, T1 per net.  ``out``: three caller-owned int64 arrays of
        n_nets entries to fill instead of new ones (page-locked arrays let the
        copy run as one DMA)."""
        n = self.n_nets[design]
        if out is None:
            out = tuple(np.zeros(n, dtype=np.int64) for _ in range(3))
        for a in out:
            if a.dtype != np.int64 or a.shape != (n,) or not a.flags["C_CONTIGUOUS"] or not a.flags["WRITEABLE"]:
                raise ValueError(f"read_saif: out arrays must be writable contiguous int64[{n}]")
        tc, t0, t1 = out
        self._chk(_lib.gs_read_saif(self._h, design, _p(tc), _p(t0), _p(t1), 1 if reset else 0))
        return tc, t0, t1

    def read_saif_ig(self, design, reset=False):
        """TC, T0, T1 and glitch toggles (IG) per net."""
        n = self.n_nets[design]
        tc, t0, t1, ig = (np.zeros(n, dtype=np.int64) for _ in range(4))
        self._chk(_lib.gs_read_saif_ig(self._h, design, _p(tc), _p(t0), _p(t1), _p(ig), 1 if reset else 0))
        return tc, t0, t1, ig

    def read_waveform(self, design, stim, net, cycle, cap=65536):
        init, n = I32(), I32()
        buf = np.zeros(cap, dtype=np.int32)
        self._chk(_lib.gs_read_waveform(self._h, design, stim, int(net), int(cycle), C.byref(init), _p(buf), cap,
                                        C.byref(n)))
        return init.value, buf[: min(n.value, cap)].tolist(), n.value

    def design_info(self, design) -> DesignInfo:
        info = DesignInfo()
        self._chk(_lib.gs_get_design_info(self._h, design, C.byref(info)))
        return info

    def levels(self, design) -> np.ndarray:
        info = self.design_info(design)
        lv = np.zeros(info.n_gates, dtype=np.int32)
        self._chk(_lib.gs_get_levels(self._h, design, _p(lv)))
        return lv

    def stats(self, reset=False) -> dict:
        s = Stats()
        self._chk(_lib.gs_get_stats(self._h, C.byref(s), 1 if reset else 0))
        return {k: getattr(s, k) for k, _ in Stats._fields_ if k != "reserved"}

    def autotune(self, design, stim, cycle_begin, cycle_end) -> dict:
        t = Tuning()
        self._chk(_lib.gs_autotune(self._h, design, stim, int(cycle_begin), int(cycle_end), C.byref(t)))
        return {"lds_cap": t.lds_cap, "waves_per_block": t.waves_per_block, "tiles_per_wave": t.tiles_per_wave,
                "trial_ms": t.trial_ms}

    def simulate_batch(self, jobs):
        arr = (Job * len(jobs))(*[Job(*j) for j in jobs])
        self._chk(_lib.gs_simulate_batch(self._h, len(jobs), arr))

    # -- serving ---------------------------------------------------------
    def serve_start(self, resident, max_queue=4096):
        """resident: list of (design, stim, cycle_begin, n_cycles)."""
        n = len(resident)
        d = _c([r[0] for r in resident], np.int32)
        s = _c([r[1] for r in resident], np.int32)
        b = _c([r[2] for r in resident], np.int32)
        c = _c([r[3] for r in resident], np.int32)
        self._chk(_lib.gs_serve_start(self._h, n, _p(d), _p(s), _p(b), _p(c), int(max_queue)))

    def submit_window(self, design, stim, b, e) -> int:
        r = Request(REQ_WINDOW, design, stim, b, e, 0, None)
        t = C.c_uint64()
        self._chk(_lib.gs_submit(self._h, C.byref(r), C.byref(t)))
        return t.value

    def submit_edit(self, design, stim, edits) -> int:
        """edits: list of (gate, pin, cond_pin, cond_val, rise, fall[, in_edge])."""
        arr = (ArcEdit * max(1, len(edits)))(*[ArcEdit(e[0], e[1], e[2], e[3], e[6] if len(e) > 6 else 0, e[4], e[5])
                                               for e in edits])
        r = Request(REQ_EDIT, design, stim, 0, 0, len(edits), arr)
        t = C.c_uint64()
        self._chk(_lib.gs_submit(self._h, C.byref(r), C.byref(t)))
        return t.value

    def poll(self, ticket, wait=True):
        """Returns None while pending, else a dict with SAIF arrays and timestamps."""
        res = Result()
        st = _lib.gs_poll(self._h, C.c_uint64(ticket), 1 if wait else 0, C.byref(res))
        if st == GS_E_BUSY:
            return None
        self._chk(st)
        n = res.n_nets
        out = {"status": res.status, "gate_cycles": res.gate_cycles, "t_submit_ns": res.t_submit_ns,
               "t_admit_ns": res.t_admit_ns, "t_done_ns": res.t_done_ns}
        if res.status != GS_OK:
            out["error"] = _lib.gs_last_error(self._h).decode()
        if res.status == GS_OK:
            out["tc"] = np.ctypeslib.as_array(res.tc, shape=(n,)).copy()
            out["t0"] = np.ctypeslib.as_array(res.t0, shape=(n,)).copy()
            out["t1"] = np.ctypeslib.as_array(res.t1, shape=(n,)).copy()
            out["ig"] = np.ctypeslib.as_array(res.ig, shape=(n,)).copy()
        return out

    def release(self, ticket):
        self._chk(_lib.gs_release(self._h, C.c_uint64(ticket)))

    def serve_stop(self):
        self._chk(_lib.gs_serve_stop(self._h))
