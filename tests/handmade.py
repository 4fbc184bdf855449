"""Hand-built tiny workloads for pin tests (shared by oracle and GPU tests).

A workload is the same dict the seeded generator produces, written out by
hand so that the expected waveforms can be derived on paper.
"""
import numpy as np

from paper_2203_06117_amd import synth

CELL = {name: i for i, name in enumerate(synth.WIDE_NAMES)}


def work(n_inputs, gates, delays, toggles, init, period=1000, n_cycles=1, wires=None):
    """gates: list of (cell name, [fanin nets]); gate g drives net n_inputs + g.
    delays: list of arc tuples (gate, pin, cond_pin, cond_val, rise, fall
    [, in_edge]), or a (rise, fall) pair applied unconditionally to every pin.
    toggles: per input, list of absolute toggle times.  wires: None or a list
    of (rise, fall) per fanin slot in CSR order."""
    cog = np.array([CELL[c] for c, _ in gates], dtype=np.int32)
    fp = np.zeros(len(gates) + 1, dtype=np.int64)
    fp[1:] = np.cumsum([len(f) for _, f in gates])
    fn = np.array([n for _, f in gates for n in f], dtype=np.int32)
    if isinstance(delays, tuple):
        r, f = delays
        delays = [(g, j, -1, 0, r, f) for g, (_, fi) in enumerate(gates) for j in range(len(fi))]
    arcs = {
        "gate": np.array([a[0] for a in delays], dtype=np.int32),
        "pin": np.array([a[1] for a in delays], dtype=np.int8),
        "cond_pin": np.array([a[2] for a in delays], dtype=np.int8),
        "cond_val": np.array([a[3] for a in delays], dtype=np.int8),
        "rise": np.array([a[4] for a in delays], dtype=np.int32),
        "fall": np.array([a[5] for a in delays], dtype=np.int32),
        "in_edge": np.array([a[6] if len(a) > 6 else 0 for a in delays], dtype=np.int8),
    }
    tp = np.zeros(n_inputs + 1, dtype=np.int64)
    tp[1:] = np.cumsum([len(t) for t in toggles])
    ts = np.array([x for t in toggles for x in t], dtype=np.int64)
    w = None
    if wires is not None:
        w = {"rise": np.array([x[0] for x in wires], dtype=np.int32),
             "fall": np.array([x[1] for x in wires], dtype=np.int32)}
    net = {"n_inputs": n_inputs, "n_gates": len(gates), "cell_of_gate": cog,
           "fanin_ptr": fp, "fanin_net": fn, "cell_pins": synth.WIDE_PINS.copy(),
           "cell_truth": synth.WIDE_TRUTH.copy()}
    stim = {"period": period, "n_cycles": n_cycles, "init": np.array(init, dtype=np.uint8),
            "toggle_ptr": tp, "toggle_ps": ts}
    return {"name": "handmade", "netlist": net, "arcs": arcs, "wires": w, "stimulus": stim}
