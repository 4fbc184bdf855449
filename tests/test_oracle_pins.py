"""Pins for the oracle: closed forms, textbook functions and hand derivations.

Each test fixes the oracle to something other than itself: the Boolean
functions of the cell types, the arithmetic of delay chains, the closed form
of the inertial pulse filter, and small circuits worked out by hand from the
rules of GATSPI's Algorithm 1 (Section 3).
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from tests.handmade import work

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

TEXTBOOK = {
    "INV": lambda a: 1 - a,
    "BUF": lambda a: a,
    "NAND2": lambda a, b: 1 - (a & b),
    "NOR2": lambda a, b: 1 - (a | b),
    "AND3": lambda a, b, c: a & b & c,
    "XOR2": lambda a, b: a ^ b,
    "AOI21": lambda a1, a2, b: 1 - ((a1 & a2) | b),
    "MUX2": lambda i0, i1, s: i1 if s else i0,
    "AND4": lambda a, b, c, d: a & b & c & d,
    "OAI22": lambda a1, a2, b1, b2: 1 - ((a1 | a2) & (b1 | b2)),
    "AOI221": lambda a1, a2, b1, b2, c: 1 - ((a1 & a2) | (b1 & b2) | c),
    "AOI222": lambda a1, a2, b1, b2, c1, c2: 1 - ((a1 & a2) | (b1 & b2) | (c1 & c2)),
}


def run1(w, probes):
    return oracle.simulate(w, probes=probes)


@pytest.mark.parametrize("cell", list(TEXTBOOK))
def test_truth_tables_zero_delay(cell):
    """Every cell, every input vector, every pin toggling: zero-delay mode
    gives the textbook function before and after the toggle, one edge iff it
    changes, at the toggle time."""
    f = TEXTBOOK[cell]
    k = f.__code__.co_argcount
    for x in range(1 << k):
        for j in range(k):
            bits = [(x >> i) & 1 for i in range(k)]
            tog = [[5] if i == j else [] for i in range(k)]
            w = work(k, [(cell, list(range(k)))], (0, 0), tog, bits, period=100)
            r = run1(w, [(k, 0)])
            init, times, n = r["probes"][0]
            before = f(*bits)
            after_bits = list(bits)
            after_bits[j] ^= 1
            after = f(*after_bits)
            assert init == before, (cell, bits, j)
            assert times == ([5] if after != before else []), (cell, bits, j)


def test_inv_buf_chains():
    """Single edges through INV/BUF chains arrive after the summed stage
    delays, each stage using its rise or fall delay by the edge it makes."""
    rng = np.random.default_rng(7)
    for trial in range(40):
        n = int(rng.integers(1, 9))
        cells = [("INV" if rng.integers(2) else "BUF") for _ in range(n)]
        rise = rng.integers(1, 40, size=n).tolist()
        fall = rng.integers(1, 40, size=n).tolist()
        gates = [(c, [i]) for i, c in enumerate(cells)]
        arcs = [(i, 0, -1, 0, rise[i], fall[i]) for i in range(n)]
        period, C = 1000, 6
        init = int(rng.integers(2))
        tog = sorted(set(int(c * period + rng.integers(0, 200)) for c in range(C) if rng.integers(3)))
        w = work(1, gates, arcs, [tog], [init], period=period, n_cycles=C)
        probes = [(1 + i, c) for i in range(n) for c in range(C)]
        r = run1(w, probes)
        for c in range(C):
            v = (init + sum(1 for t in tog if t < c * period)) & 1
            edges = [t - c * period for t in tog if c * period <= t < (c + 1) * period]
            for i in range(n):
                out_v = v if cells[i] == "BUF" else 1 - v
                out_edges = []
                val = out_v
                for t in edges:
                    val ^= 1
                    out_edges.append(t + (rise[i] if val else fall[i]))
                pi = probes.index((1 + i, c))
                assert r["probes"][pi][0] == out_v
                assert r["probes"][pi][1] == out_edges, (trial, c, i)
                v, edges = out_v, out_edges
        assert r["ig"].tolist() == [0] * (n + 1)            # at most one toggle per cycle: nothing is a glitch


def _pulse_grid(cell, init):
    """One gate per (leading delay, trailing delay, width); returns the
    workload and the case list."""
    cases = [(dl, dt, wdt) for dl in range(1, 13) for dt in range(1, 13) for wdt in range(1, 15)]
    gates, arcs, tog = [], [], []
    n = len(cases)
    for g, (dl, dt, wdt) in enumerate(cases):
        gates.append((cell, [g]))
        out_rises_first = (init == 0) == (cell == "BUF")
        rise, fall = (dl, dt) if out_rises_first else (dt, dl)
        arcs.append((g, 0, -1, 0, rise, fall))
        tog.append([10, 10 + wdt])
    return work(n, gates, arcs, tog, [init] * n, period=100), cases


@pytest.mark.parametrize("cell", ["BUF", "INV"])
@pytest.mark.parametrize("init", [0, 1])
def test_gate_pulse_closed_form(cell, init):
    """A pulse of width w through a gate with leading-edge delay d_l and
    trailing-edge delay d_t survives iff w >= d_l and then has width
    w + d_t - d_l, starting at a + d_l."""
    w, cases = _pulse_grid(cell, init)
    n = len(cases)
    r = run1(w, [(n + g, 0) for g in range(n)])
    for g, (dl, dt, wdt) in enumerate(cases):
        _, times, _ = r["probes"][g]
        if wdt >= dl:
            assert times == [10 + dl, 10 + wdt + dt], (cell, init, dl, dt, wdt)
        else:
            assert times == [], (cell, init, dl, dt, wdt)


@pytest.mark.parametrize("init", [0, 1])
def test_wire_pulse_closed_form(init):
    """The interconnect filter obeys the same closed form with the wire's
    rise/fall delays; a BUF with unit delays behind it shifts the result by 1."""
    cases = [(dl, dt, wdt) for dl in range(1, 11) for dt in range(1, 11) for wdt in range(1, 13)]
    n = len(cases)
    gates = [("BUF", [g]) for g in range(n)]
    wires = []
    for dl, dt, wdt in cases:
        wires.append((dl, dt) if init == 0 else (dt, dl))
    w = work(n, gates, (1, 1), [[10, 10 + c[2]] for c in cases], [init] * n, period=100, wires=wires)
    r = run1(w, [(n + g, 0) for g in range(n)])
    for g, (dl, dt, wdt) in enumerate(cases):
        _, times, _ = r["probes"][g]
        if wdt >= dl:
            assert times == [11 + dl, 11 + wdt + dt]
        else:
            assert times == []


@pytest.mark.parametrize("init", [0, 1])
def test_wire_transport_closed_form(init):
    """Without the interconnect filter (the feature study's "no net delay",
    Algorithm 1 with its net-delay filtering lines deleted) a wire is a
    transport delay: a net pulse of width w whose leading edge takes d_l and
    trailing edge d_t arrives as a pin pulse of width w + d_t - d_l, starting
    at a + d_l, when that width is positive, and vanishes otherwise (a
    delayed trailing edge no later than the delayed leading one).  A BUF
    with unit delays behind it shifts the result by 1."""
    cases = [(dl, dt, wdt) for dl in range(1, 11) for dt in range(1, 11) for wdt in range(1, 13)]
    n = len(cases)
    gates = [("BUF", [g]) for g in range(n)]
    wires = [(dl, dt) if init == 0 else (dt, dl) for dl, dt, _ in cases]
    w = work(n, gates, (1, 1), [[10, 10 + c[2]] for c in cases], [init] * n, period=100, wires=wires)
    r = oracle.Oracle(w["netlist"], w["arcs"], w["wires"]).run(
        w["stimulus"], probes=[(n + g, 0) for g in range(n)], net_filter=False)
    for g, (dl, dt, wdt) in enumerate(cases):
        _, times, _ = r["probes"][g]
        if wdt + dt - dl > 0:
            assert times == [11 + dl, 11 + wdt + dt], (init, dl, dt, wdt)
        else:
            assert times == [], (init, dl, dt, wdt)


def test_wire_transport_keeps_every_pulse_in_flight():
    """A transport wire longer than the gaps between its net's edges holds
    several pin edges in flight at once; all of them arrive, shifted by the
    wire delay, where the inertial filter keeps none of the narrow pulses."""
    w = work(1, [("BUF", [0])], (1, 1), [[10, 20, 30, 45]], [0], period=200, wires=[(50, 50)])
    o = oracle.Oracle(w["netlist"], w["arcs"], w["wires"])
    r = o.run(w["stimulus"], probes=[(1, 0)], net_filter=False)
    assert r["probes"][0][1] == [61, 71, 81, 96]
    r = o.run(w["stimulus"], probes=[(1, 0)], net_filter=True)
    assert r["probes"][0][1] == []


def test_xor_glitch_generator():
    """One net through two buffers of delays a and b into an XOR2: a pulse
    of width |a-b| appears, filtered iff |a-b| is below the XOR's rise delay;
    equal delays switch both pins at once and give no edge."""
    for a, b, rx, fx in itertools.product(range(1, 7), range(1, 7), range(1, 6), range(1, 6)):
        gates = [("BUF", [0]), ("BUF", [0]), ("XOR2", [1, 2])]
        arcs = [(0, 0, -1, 0, a, a), (1, 0, -1, 0, b, b),
                (2, 0, -1, 0, rx, fx), (2, 1, -1, 0, rx, fx)]
        w = work(1, gates, arcs, [[10]], [0], period=100)
        r = run1(w, [(3, 0)])
        _, times, _ = r["probes"][0]
        lo, hi = min(a, b), max(a, b)
        if a == b or hi - lo < rx:
            assert times == [], (a, b, rx, fx)
            assert r["ig"][3] == 0
        else:
            assert times == [10 + lo + rx, 10 + hi + fx], (a, b, rx, fx)
            assert r["ig"][3] == 2 and r["tc"][3] == 2      # the whole pulse is a glitch
        assert r["ig"][:3].tolist() == [0, 0, 0]            # one functional edge on the input and buffers
        assert r["ig_cycle"].tolist() == [r["ig"][3]]       # the cycle's profile entry holds the pulse


def test_msi_min_delay():
    """Several pins switching at one time: the output edge takes the
    smallest of their arc delays (here the last pin in index order has the
    larger delay, so reading it literally would differ)."""
    for fa, fb in [(3, 7), (7, 3), (5, 5)]:
        arcs = [(0, 0, -1, 0, 20, fa), (0, 1, -1, 0, 20, fb)]
        w = work(2, [("NAND2", [0, 1])], arcs, [[10], [10]], [0, 0], period=100)
        init, times, _ = run1(w, [(2, 0)])["probes"][0]
        assert init == 1 and times == [10 + min(fa, fb)]
    # AND3 with its third pin held at 1
    arcs = [(0, 0, -1, 0, 9, 1), (0, 1, -1, 0, 4, 1), (0, 2, -1, 0, 2, 1)]
    w = work(3, [("AND3", [0, 1, 2])], arcs, [[10], [10], []], [0, 0, 1], period=100)
    assert run1(w, [(3, 0)])["probes"][0][:2] == (0, [14])
    # XOR2 with both pins switching together: no edge at all
    w = work(2, [("XOR2", [0, 1])], (3, 3), [[10], [10]], [0, 1], period=100)
    assert run1(w, [(2, 0)])["probes"][0][:2] == (1, [])


def test_conditional_delays():
    """SDF-style conditional arcs: pin A's delay depends on side pin B's
    value; B unconditional.  Cycles: A rises with B=0, A falls with B=0,
    B rises, A rises with B=1, A falls with B=1."""
    r0, f0, r1, f1, rb, fb = 11, 13, 17, 19, 5, 7
    arcs = [(0, 0, 1, 0, r0, f0), (0, 0, 1, 1, r1, f1), (0, 1, -1, 0, rb, fb)]
    T = 100
    togA = [10, 110, 310, 410]
    togB = [210]
    w = work(2, [("XOR2", [0, 1])], arcs, [togA, togB], [0, 0], period=T, n_cycles=5)
    r = run1(w, [(2, c) for c in range(5)])
    got = [p[:2] for p in r["probes"]]
    assert got == [(0, [10 + r0]),          # A 0->1, B=0: XOR rises, r0
                   (1, [10 + f0]),          # A 1->0, B=0: XOR falls, f0
                   (0, [10 + rb]),          # B 0->1: XOR rises via B
                   (1, [10 + f1]),          # A 0->1, B=1: XOR falls, f1
                   (0, [10 + r1])]          # A 1->0, B=1: XOR rises, r1


def test_conditional_uses_state_after_switching():
    """When the condition pin switches together with the arc's pin, the
    condition is read in the pin state after both switched."""
    # NAND2: pin 0 fall delay 30 when pin1 = 0, 4 when pin1 = 1; pin 1 fall 9
    arcs = [(0, 0, 1, 0, 50, 30), (0, 0, 1, 1, 50, 4), (0, 1, -1, 0, 50, 9)]
    w = work(2, [("NAND2", [0, 1])], arcs, [[10], [10]], [0, 0], period=100)
    assert run1(w, [(2, 0)])["probes"][0][:2] == (1, [14])


def test_input_edge_qualified_delays():
    """SDF IOPATH rows qualified by the input edge (posedge / negedge A):
    the delay row is picked by the input edge and the output edge
    separately.  XOR2 makes all four combinations reachable from pin A.
    Cycles: A rises with B=0, A falls with B=0, B rises, A rises with B=1,
    A falls with B=1."""
    ar, af, br, bf, rb, fb = 11, 13, 17, 19, 5, 7
    arcs = [(0, 0, -1, 0, ar, af, 1), (0, 0, -1, 0, br, bf, 2), (0, 1, -1, 0, rb, fb)]
    togA = [10, 110, 310, 410]
    w = work(2, [("XOR2", [0, 1])], arcs, [togA, [210]], [0, 0], period=100, n_cycles=5)
    got = [p[:2] for p in run1(w, [(2, c) for c in range(5)])["probes"]]
    assert got == [(0, [10 + ar]),          # A rises, output rises
                   (1, [10 + bf]),          # A falls, output falls
                   (0, [10 + rb]),          # via B
                   (1, [10 + af]),          # A rises, output falls
                   (0, [10 + br])]          # A falls, output rises


def test_specificity_order():
    """A record qualified by both a condition and an input edge beats one
    with a single qualifier, which beats an unqualified one; two records
    of the top matching specificity are an error, and so is a pin state
    that no record matches.  NAND2 pin 0, pin 1 held at 1, pin 0 rising
    then falling: the output falls, then rises."""
    base = [(0, 1, -1, 0, 50, 50)]
    def run_arcs(a):
        w = work(2, [("NAND2", [0, 1])], base + a, [[10, 110], []], [0, 1], period=100, n_cycles=2)
        return [p[:2] for p in run1(w, [(2, 0), (2, 1)])["probes"]]
    # unqualified only
    assert run_arcs([(0, 0, -1, 0, 21, 23)]) == [(1, [33]), (0, [31])]
    # a rising-input override beats it for the rising input only
    assert run_arcs([(0, 0, -1, 0, 21, 23), (0, 0, -1, 0, 31, 3, 1)]) == [(1, [13]), (0, [31])]
    # condition and edge together beat condition alone and edge alone
    cond = [(0, 0, 1, 0, 40, 40), (0, 0, 1, 1, 21, 23)]
    both = [(0, 0, 1, 0, 44, 44, 1), (0, 0, 1, 1, 61, 6, 1)]
    assert run_arcs(cond + [(0, 0, -1, 0, 31, 3, 1)] + both) == [(1, [16]), (0, [31])]
    # condition alone and edge alone both match pin 0 rising with pin 1 = 1
    with pytest.raises(oracle.OracleError, match="two arc records"):
        run_arcs(cond + [(0, 0, -1, 0, 31, 3, 1)])
    # records dominated everywhere by more specific ones may repeat
    assert run_arcs([(0, 0, -1, 0, 1, 1), (0, 0, -1, 0, 2, 2),
                     (0, 0, -1, 0, 21, 23, 1), (0, 0, -1, 0, 27, 29, 2)]) == [(1, [33]), (0, [37])]
    # nothing covers the falling input
    with pytest.raises(oracle.OracleError, match="no arc record"):
        run_arcs([(0, 0, -1, 0, 21, 23, 1)])


def test_continuous_segments():
    """Two cycles run as one segment: a BUF slower than the period lets
    its edge carry into the next cycle, where the input's return swallows
    it (t < W cancels the pending edge); run cycle by cycle, each cycle
    shows the edge instead.  A lone input edge: the output spends only the
    segment's last 30 ps at 1."""
    w = work(1, [("BUF", [0])], (150, 150), [[20, 120]], [0], period=100, n_cycles=2)
    iso = run1(w, [(1, 0), (1, 1)])
    assert [p[:2] for p in iso["probes"]] == [(0, [170]), (1, [170])]
    assert iso["tc"].tolist() == [2, 2] and iso["t1"].tolist() == [100, 100]
    seg = oracle.simulate(w, probes=[(1, 0), (0, 0)], segment_cycles=2)
    assert [p[:2] for p in seg["probes"]] == [(0, []), (0, [20, 120])]
    assert seg["tc"].tolist() == [2, 0] and seg["t1"].tolist() == [100, 0] and seg["t0"].tolist() == [100, 200]
    w = work(1, [("BUF", [0])], (150, 150), [[20]], [0], period=100, n_cycles=2)
    seg = oracle.simulate(w, probes=[(1, 0)], segment_cycles=2)
    assert seg["probes"][0][:2] == (0, [170])
    assert seg["tc"].tolist() == [1, 1] and seg["t1"].tolist() == [180, 30]
    assert run1(w, [])["t1"].tolist() == [180, 100]
    with pytest.raises(oracle.OracleError):
        oracle.simulate(w, segment_cycles=3)


def test_segment_input_glitches():
    """An input's glitch toggles in a continuous segment are its toggles in
    the segment less one when their number is odd (the net's value then
    changes across the segment).  Three-cycle segments of 100 ps: one toggle
    in a segment gives none, two give two, three give two, and toggles in
    different segments never pair; cycle by cycle the same toggles pair
    only within a cycle."""
    T = 100
    tog = [[255 * T + 50],                                      # segment 85: 1 toggle
           [100 * T + 30, 101 * T + 60, 255 * T + 40],          # segment 33: 2, segment 85: 1
           [255 * T + 10, 255 * T + 60, 256 * T + 20],          # segment 85: 3 (2 in cycle 255)
           [c * T + 35 for c in range(0, 261, 7)],              # one per segment at most
           [3 * T + 10, 3 * T + 20, 5 * T + 90]]                # segment 1: 3 (2 in cycle 3)
    w = work(5, [("BUF", [i]) for i in range(5)], (5, 5), tog, [0, 1, 0, 1, 0], period=T, n_cycles=261)
    seg = oracle.simulate(w, segment_cycles=3)
    assert seg["ig"][:5].tolist() == [0, 2, 2, 0, 2]
    assert seg["tc"][:5].tolist() == [1, 3, 3, 38, 3]
    iso = oracle.simulate(w)
    assert iso["ig"][:5].tolist() == [0, 0, 2, 0, 2]


def test_late_lanes():
    """A cycle ends quiescent unless a net's last edge, or its arrival at a
    fanout pin through the pin's wire, reaches the period."""
    w = work(1, [("BUF", [0])], (150, 150), [[20]], [0], period=100)
    assert oracle.simulate(w)["late_cycle"].tolist() == [1]          # the output edge at 170
    w = work(1, [("BUF", [0])], (50, 50), [[20]], [0], period=100)
    assert oracle.simulate(w)["late_cycle"].tolist() == [0]          # edge at 70
    w = work(1, [("BUF", [0])], (5, 5), [[20]], [0], period=100, wires=[(90, 60)])
    assert oracle.simulate(w)["late_cycle"].tolist() == [2]          # arrival 110, output edge 115
    w = work(1, [("BUF", [0])], (5, 5), [[20, 30]], [0], period=100, wires=[(90, 60)])
    assert oracle.simulate(w)["late_cycle"].tolist() == [0]          # the falling edge arrives at 90


def test_cycles_are_isolated():
    """Each cycle starts from the settled values; an edge later than the
    period still belongs to its cycle and is clipped out of T0/T1."""
    w = work(1, [("BUF", [0])], (150, 150), [[20]], [0], period=100, n_cycles=2)
    r = run1(w, [(1, 0), (1, 1)])
    assert r["probes"][0][:2] == (0, [170])
    assert r["probes"][1][:2] == (1, [])
    assert r["tc"].tolist() == [1, 1]
    assert r["t1"].tolist() == [80 + 100, 0 + 100]
    assert r["t0"].tolist() == [20, 100]


@pytest.mark.parametrize("path", sorted(f for f in os.listdir(GOLDEN) if f.endswith(".json")))
def test_golden_fixture(path):
    """Hand-derived waveforms stored under tests/golden (each file states its
    derivation and the passage it follows)."""
    with open(os.path.join(GOLDEN, path)) as fh:
        fx = json.load(fh)
    wires = [tuple(x) for x in fx["wires"]] if fx.get("wires") else None
    w = work(fx["n_inputs"], [tuple(g) for g in fx["gates"]], [tuple(a) for a in fx["arcs"]],
             fx["toggles"], fx["init"], period=fx["period"], n_cycles=fx["n_cycles"], wires=wires)
    probes = [(e["net"], e["cycle"]) for e in fx["expect"]]
    S = fx.get("segment_cycles", 1)                # cycles run as one continuous segment
    r = run1(w, probes) if S == 1 else oracle.simulate(w, probes=probes, segment_cycles=S)
    for e, p in zip(fx["expect"], r["probes"]):
        assert (p[0], p[1]) == (e["init"], e["times"]), e
