"""GPU parity over random combinations of the options that change how a run
is laid out, against the oracle, bit-exact: dead nets released or kept,
plain, single-lane segment and carried continuous views, windows, staging
caps, tiles per wave, waves per block, captured-graph rounds and cycle
sub-ranges, budgets that force windows to shrink and the arena to refill,
on random designs with every arc feature (wide cells, wires where the view
allows them), with sampled waveforms read back where the range runs as one
window; the same for batches, for the allocation-free entry point and for
serving (window and delay-edit requests from several threads).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2203_06117_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_06117_amd import gatesim
    return gatesim


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def draw_case(G, case, dense=False, extreme=False):
    rng = np.random.default_rng(12_000 + case)
    view = str(rng.choice(["plain", "plain", "segment", "carry", "carry"]))
    S = 1 if view == "plain" else int(rng.choice([2, 3, 8, 16, 64]))
    wide = bool(rng.random() < 0.25)
    gates = int(rng.integers(30, 800)) if rng.random() < 0.8 else int(rng.integers(800, 4000))
    if dense:
        gates = int(rng.integers(30, 500))
    C = S * int(rng.integers(2, max(3, 400 // S)))
    T = int(rng.integers(40, 700))
    if extreme:
        # periods far below the arc delays (every edge lands cycles later)
        # or near the largest period a segment may span (2^24 ps)
        T = int(rng.choice([1, 2, 5, 17, (1 << 24) // S - int(rng.integers(0, 1000))]))
    wires = view != "carry" and rng.random() < 0.4
    w = synth.small_random(12_000 + case, gates, int(rng.integers(16, 40)), min(gates, int(rng.integers(2, 30))),
                           C, T, float(rng.uniform(0.05, 0.6)), 1, int(rng.integers(2, 90)),
                           cond_frac=float(rng.choice([0.0, 0.2, 0.5])),
                           wire=(1, int(rng.integers(1, 30))) if wires else None,
                           extra=int(rng.choice([5, 6])) if dense else int(rng.choice([0, 0, 2, 4])),
                           extra_p=0.9 if dense else 0.4, skew=min(50, T - 1), wide=wide,
                           edge_frac=float(rng.choice([0.0, 0.3])))
    transport = wires and rng.random() < 0.3
    if transport:
        w["net_filter"] = False
    opt = {"release_dead": bool(rng.random() < 0.5), "wire_transport": transport}
    if rng.random() < 0.5:
        opt["window_cycles"] = int(rng.choice([37, 64, 100, 256]))
    if rng.random() < 0.5:
        opt["tiles_per_wave"] = int(rng.choice([1, 2, 3, 8, 16]))
    if rng.random() < 0.4:
        opt["lds_cap"] = int(rng.choice([4, 8, 16, 24, 32]))
    if rng.random() < 0.3:
        opt["waves_per_block"] = int(rng.choice([1, 2, 8]))
        if opt["waves_per_block"] == 8 and opt.get("lds_cap") == 32:
            opt["waves_per_block"] = 2              # 86 KB of LDS per block may exceed the device's limit
    if rng.random() < 0.3:
        opt["schedule"] = G.SCHED_GRAPH
    n = C // S
    b = int(rng.integers(0, n))
    e = int(rng.integers(b + 1, n + 1))
    if rng.random() < 0.2:
        # The budget holds window headers and arena: 144 B of chunk header and
        # lane ends per (net, 64-lane tile), a window's headers at most a
        # third of it.  0.5 to 2.5 times the range's headers splits every
        # range of more than one tile into windows; the floor leaves one tile
        # room for dense transitions.
        N = w["netlist"]["n_inputs"] + gates
        lanes = (e - b) * (1 if view == "segment" else S)
        hdr = N * 144 * ((lanes + 63) // 64)
        opt["hbm_budget"] = max(int(hdr * rng.uniform(0.5, 2.5)), N * 1500 + 65536)
    return w, view, S, wide, opt, b, e


@pytest.mark.parametrize("block", range(12))
def test_option_combinations(G, block):
    """Blocks 8 and 9 draw dense inputs (five or six extra toggles per cycle
    on most inputs), so that tile groups outgrow the fanin stage, lanes
    outgrow their output slots and queues overflow; blocks 10 and 11 draw
    periods of 1 to 17 ps or near 2^24 ps per segment."""
    budget_runs = 0
    dense = block in (8, 9)
    for case in range(block * 25, block * 25 + 25):
        w, view, S, wide, opt, b, e = draw_case(G, case, dense=dense, extreme=block >= 10)
        say("combo", case, view, S, wide, w["stimulus"]["n_cycles"], opt, (b, e))
        # the waveforms stay readable when the range runs as one window
        # (ranges here are shorter than the default window) and every net is kept
        readable = not (opt["release_dead"] or "window_cycles" in opt or "hbm_budget" in opt)
        rng = np.random.default_rng(case)
        N = w["netlist"]["n_inputs"] + w["netlist"]["n_gates"]
        probes = ([(int(n), int(k)) for n, k in zip(rng.integers(0, N, 40), rng.integers(b, e, 40))]
                  if readable else [])
        ref = oracle.simulate(w, b, e, probes=probes, segment_cycles=S)
        try:
            with G.GateSim(**opt) as sim:
                if wide:
                    sim.load_cells(synth.WIDE_PINS, synth.WIDE_TRUTH)
                d, s = sim.load_work(w, cells_loaded=wide)
                if view == "segment":
                    s = sim.segment_stimulus(s, S)
                elif view == "carry":
                    s = sim.continuous_stimulus(s, S)
                sim.simulate(d, s, b, e)
                tc, t0, t1, ig = sim.read_saif_ig(d)
                st = sim.stats()
                waves = [sim.read_waveform(d, s, n, k) for n, k in probes]
        except G.GateSimError as err:
            # a budget below what one window needs is refused, never run
            if "hbm_budget" in opt and err.status == G.GS_E_NOMEM:
                say("  refused:", err)
                continue
            raise
        if "hbm_budget" in opt:
            budget_runs += 1
            say("  windows", st["windows"], "retried", st["window_retries"])
        if dense:
            say("  unstaged groups", st["unstaged_groups"], "spilled lanes", st["spilled_lanes"],
                "queue overflows", st["queue_overflows"])
        for name, a, r in (("tc", tc, ref["tc"]), ("t0", t0, ref["t0"]), ("t1", t1, ref["t1"]), ("ig", ig, ref["ig"])):
            if not np.array_equal(a, r):
                bad = np.nonzero(a != r)[0]
                raise AssertionError(f"case {case} ({view}, S {S}, {opt}, cycles {b}..{e}): {name} differs on "
                                     f"{len(bad)} nets, first {bad[:8]} gpu {a[bad[:8]]} oracle {r[bad[:8]]}")
        for (n, k), gw, ow in zip(probes, waves, ref["probes"]):
            assert gw == ow, f"case {case} ({view}, S {S}, {opt}): waveform of net {n} in cycle {k}"
    say("block", block, "budget runs", budget_runs)


@pytest.mark.parametrize("block", range(8))
def test_batch_combinations(G, block):
    """Batches of two to six jobs drawn like the cases above (each its own
    design, view and cycle range) under one set of context options: every
    design's counts equal the oracle's for its job.  Block 6 draws dense
    inputs, block 7 extreme periods."""
    for bi in range(block * 5, block * 5 + 5):
        rng = np.random.default_rng(13_000 + bi)
        cases = [draw_case(G, 500 + 7 * bi + k, dense=block == 6, extreme=block == 7)
                 for k in range(int(rng.integers(2, 7)))]
        opt = {k: v for k, v in cases[0][4].items() if k != "hbm_budget"}
        opt["wire_transport"] = False
        jobs_desc = []
        say("batch", bi, opt, [(c[1], c[2], c[0]["netlist"]["n_gates"], (c[5], c[6])) for c in cases])
        with G.GateSim(**opt) as sim:
            sim.load_cells(synth.WIDE_PINS, synth.WIDE_TRUTH)     # a superset of every design's library
            jobs = []
            for w, view, S, wide, _, b, e in cases:
                w["net_filter"] = True
                d, s = sim.load_work(w, cells_loaded=True)
                if view == "segment":
                    s = sim.segment_stimulus(s, S)
                elif view == "carry":
                    s = sim.continuous_stimulus(s, S)
                jobs.append((d, s, b, e))
                jobs_desc.append((d, w, S, b, e))
            sim.simulate_batch(jobs)
            for d, w, S, b, e in jobs_desc:
                tc, t0, t1, ig = sim.read_saif_ig(d)
                ref = oracle.simulate(w, b, e, segment_cycles=S)
                for name, a, r in (("tc", tc, ref["tc"]), ("t0", t0, ref["t0"]), ("t1", t1, ref["t1"]),
                                   ("ig", ig, ref["ig"])):
                    assert np.array_equal(a, r), f"batch {bi} design {d} (S {S}, cycles {b}..{e}): {name}"


@pytest.mark.parametrize("block", range(5))
def test_noalloc_combinations(G, block):
    """The allocation-free entry point on cases drawn like the ones above
    (its scratch sets the window memory, and it keeps every net), called
    twice in a row on one context with other calls between: the oracle's
    counts each time.  Block 3 draws dense inputs, block 4 extreme periods."""
    for case in range(800 + block * 20, 800 + block * 20 + 20):
        w, view, S, wide, opt, b, e = draw_case(G, case, dense=block == 3, extreme=block == 4)
        opt.pop("hbm_budget", None)
        say("noalloc combo", case, view, S, wide, w["stimulus"]["n_cycles"], opt, (b, e))
        ref = oracle.simulate(w, b, e, segment_cycles=S)
        want = (ref["tc"], ref["t0"], ref["t1"], ref["ig"])
        with G.GateSim(**opt) as sim:
            if wide:
                sim.load_cells(synth.WIDE_PINS, synth.WIDE_TRUTH)
            d, s = sim.load_work(w, cells_loaded=wide)
            if view == "segment":
                s = sim.segment_stimulus(s, S)
            elif view == "carry":
                s = sim.continuous_stimulus(s, S)
            for rep in range(2):
                sim.simulate_noalloc(d, s, b, e)
                got = sim.read_saif_ig(d, reset=True)
                for name, a, r in zip(("tc", "t0", "t1", "ig"), got, want):
                    assert np.array_equal(a, r), f"case {case} ({view}, S {S}, {opt}, cycles {b}..{e}) call {rep}: {name}"
                sim.simulate(d, s, b, min(e, b + 1))         # a regular call between
                sim.read_saif_ig(d, reset=True)


@pytest.mark.parametrize("block", range(4))
def test_serve_combinations(G, block):
    """Serving under random context options (tiles per wave, caps, block
    shapes, transport wires): two or three resident designs with every arc
    feature, on plain or single-lane segment views, and sixteen window and
    delay-edit requests submitted from three threads; every result equals
    the oracle's for its range (an edit's: the resident range with the
    edited arcs)."""
    import threading
    from tests.test_gpu_serve import edited_arcs, random_edits
    for ci in range(block * 2, block * 2 + 2):
        rng = np.random.default_rng(14_000 + ci)
        opt = {"wire_transport": bool(rng.random() < 0.3)}
        if rng.random() < 0.5:
            opt["tiles_per_wave"] = int(rng.choice([1, 2, 4, 8]))
        if rng.random() < 0.4:
            opt["lds_cap"] = int(rng.choice([4, 8, 16, 24, 32]))
        if rng.random() < 0.3:
            opt["waves_per_block"] = int(rng.choice([1, 2, 8]))
            if opt["waves_per_block"] == 8 and opt.get("lds_cap") == 32:
                opt["waves_per_block"] = 2
        designs = []
        for k in range(int(rng.integers(2, 4))):
            S = int(rng.choice([1, 1, 1, 3, 8]))
            n_view = int(rng.integers(20, 200 // S + 21))
            T = int(rng.integers(60, 700))
            gates = int(rng.integers(50, 1500))
            wires = rng.random() < 0.4
            w = synth.small_random(14_000 + 10 * ci + k, gates, int(rng.integers(16, 40)),
                                   min(gates, int(rng.integers(2, 30))), S * n_view, T, float(rng.uniform(0.05, 0.5)),
                                   1, int(rng.integers(2, 90)), cond_frac=float(rng.choice([0.0, 0.2])),
                                   wire=(1, int(rng.integers(1, 30))) if wires else None,
                                   extra=int(rng.choice([0, 2])), extra_p=0.4, skew=min(50, T - 1),
                                   wide=bool(rng.random() < 0.3), edge_frac=float(rng.choice([0.0, 0.3])))
            w["net_filter"] = not (wires and opt["wire_transport"])
            rb = int(rng.integers(0, n_view - 1))
            designs.append((w, S, n_view, rb, int(rng.integers(1, n_view - rb + 1))))
        say("serve combo", ci, opt, [(d[0]["netlist"]["n_gates"], d[1], d[2], d[3], d[4]) for d in designs])
        plan = []
        for r in range(16):
            k = int(rng.integers(len(designs)))
            w, S, n_view, rb, rn = designs[k]
            if rng.random() < 0.5:
                b = int(rng.integers(0, n_view))
                plan.append(("w", k, (b, int(rng.integers(b + 1, n_view + 1)))))
            else:
                plan.append(("e", k, random_edits(rng, w, int(rng.integers(1, 12)))))
        sim = G.GateSim(**opt)
        started = False
        try:
            sim.load_cells(synth.WIDE_PINS, synth.WIDE_TRUTH)            # a superset of every design's library
            ids = []
            for w, S, n_view, rb, rn in designs:
                d, s = sim.load_work(w, cells_loaded=True)
                ids.append((d, sim.segment_stimulus(s, S) if S > 1 else s))
            sim.serve_start([(d, v, designs[k][3], designs[k][4]) for k, (d, v) in enumerate(ids)], max_queue=256)
            started = True
            tickets = [None] * len(plan)

            def worker(lo):
                for j in range(lo, len(plan), 3):
                    kind, k, arg = plan[j]
                    tickets[j] = (sim.submit_window(*ids[k], *arg) if kind == "w" else
                                  sim.submit_edit(*ids[k], arg))

            ths = [threading.Thread(target=worker, args=(lo,)) for lo in range(3)]
            for t in ths:
                t.start()
            for t in ths:
                t.join()
            for j, t in enumerate(tickets):
                r = sim.poll(t, wait=True)
                sim.release(t)
                assert r["status"] == 0, r.get("error")
                kind, k, arg = plan[j]
                w, S, n_view, rb, rn = designs[k]
                if kind == "w":
                    ref = oracle.simulate(w, arg[0], arg[1], segment_cycles=S)
                else:
                    ref = oracle.simulate(dict(w, arcs=edited_arcs(w["arcs"], arg)), rb, rb + rn, segment_cycles=S)
                for name in ("tc", "t0", "t1", "ig"):
                    assert np.array_equal(r[name], ref[name]), f"serve case {ci} request {j} ({kind}, design {k}): {name}"
        finally:
            if started:
                sim.serve_stop()
            sim.close()
