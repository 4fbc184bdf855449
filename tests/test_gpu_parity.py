"""GPU parity: the HIP library against the CPU oracle, bit-exact.

All results are integers (picosecond times, counts, SAIF sums), so the bar
is equality.  Cases cover hand-derived circuits, seeded random netlists with
wires, conditional and input-edge-qualified arcs, multi-edge inputs and
zero-delay mode, continuous segments, the per-cycle glitch profile, window
and tile invariance (ragged last tiles, window boundaries, forced arena
retries, forced on-chip staging overflow), the levelizer, error paths
(capacity overflow from inputs and from gates included), and the 1M-gate
workload in the launch configuration the benchmark times and in windows.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2203_06117_amd import synth
from tests.handmade import work

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_06117_amd import gatesim
    return gatesim


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_saif(G, w, b=0, e=None, probes=(), segment=1, **opt):
    C = w["stimulus"]["n_cycles"] // segment
    e = C if e is None else e
    with G.GateSim(**opt) as sim:
        d, s = sim.load_work(w)
        if segment > 1:
            s = sim.segment_stimulus(s, segment)
        sim.simulate(d, s, b, e)
        tc, t0, t1, ig = sim.read_saif_ig(d)
        waves = [sim.read_waveform(d, s, n, c) for n, c in probes]
        st = sim.stats()
    return tc, t0, t1, waves, st, ig


def assert_same(w, got, ref, tag=""):
    tc, t0, t1 = got[:3]
    cols = [("tc", tc, ref["tc"]), ("t0", t0, ref["t0"]), ("t1", t1, ref["t1"])]
    if len(got) > 5:
        cols.append(("ig", got[5], ref["ig"]))
    for name, a, b in cols:
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{tag}: {name} differs on {len(bad)} nets, first {bad[:8]} "
                                 f"gpu {a[bad[:8]]} oracle {b[bad[:8]]}")


def test_handmade_golden(G):
    for f in sorted(os.listdir(GOLDEN)):
        if not f.endswith(".json"):
            continue
        fx = json.load(open(os.path.join(GOLDEN, f)))
        wires = [tuple(x) for x in fx["wires"]] if fx.get("wires") else None
        w = work(fx["n_inputs"], [tuple(g) for g in fx["gates"]], [tuple(a) for a in fx["arcs"]],
                 fx["toggles"], fx["init"], period=fx["period"], n_cycles=fx["n_cycles"], wires=wires)
        say("golden", f)
        probes = [(x["net"], x["cycle"]) for x in fx["expect"]]
        S = fx.get("segment_cycles", 1)
        got = gpu_saif(G, w, probes=probes, segment=S)
        for x, (init, times, n) in zip(fx["expect"], got[3]):
            assert (init, times) == (x["init"], x["times"]), (f, x)
        assert_same(w, got, oracle.simulate(w, segment_cycles=S), f)


@pytest.mark.parametrize("cell", ["BUF", "INV"])
def test_pulse_grid(G, cell):
    """The inertial closed-form grid (every leading/trailing delay and width)."""
    cases = [(dl, dt, wd) for dl in range(1, 13) for dt in range(1, 13) for wd in range(1, 15)]
    n = len(cases)
    gates, arcs, tog = [], [], []
    for g, (dl, dt, wd) in enumerate(cases):
        gates.append((cell, [g]))
        rise, fall = (dl, dt) if cell == "BUF" else (dt, dl)
        arcs.append((g, 0, -1, 0, rise, fall))
        tog.append([10 + 100 * c + (wd if c % 2 else 0) for c in range(2)] + [210, 210 + wd])
    w = work(n, gates, arcs, tog, [0] * n, period=100, n_cycles=3)
    say("pulse grid", cell, n)
    got = gpu_saif(G, w)
    assert_same(w, got, oracle.simulate(w), cell)


@pytest.mark.parametrize("mode", ["plain", "wires", "cond", "wires+cond", "zero", "multi-edge", "wires+cond+edges",
                                  "transport-wires", "transport-wires+cond+edges"])
def test_random_small(G, mode):
    for seed in range(20):
        rng = np.random.default_rng(seed + 100)
        gates = int(rng.integers(50, 900))
        levels = int(rng.integers(2, 30))
        C = int(rng.integers(1, 200))
        T = int(rng.integers(60, 600))
        zero = mode == "zero"
        w = synth.small_random(seed + 7000, gates, int(rng.integers(3, 40)), min(levels, gates), C, T,
                               float(rng.uniform(0.05, 0.6)), 0 if zero else 1, 0 if zero else int(rng.integers(2, 80)),
                               cond_frac=0.3 if "cond" in mode else 0.0,
                               wire=(1, int(rng.integers(1, 25))) if "wires" in mode else None,
                               extra=3 if mode in ("multi-edge", "wires", "transport-wires") else 0, extra_p=0.3,
                               skew=min(50, T - 1), edge_frac=0.4 if "edges" in mode else 0.0)
        transport = "transport" in mode
        if transport:
            w["net_filter"] = False
        say("random", mode, seed, gates, levels, C, T)
        got = gpu_saif(G, w, window_cycles=int(rng.choice([0, 64, 100, 37])), wire_transport=transport)
        assert_same(w, got, oracle.simulate(w), f"{mode} seed {seed}")


@pytest.mark.parametrize("S", [2, 7, 16, 64])
def test_continuous_segments(G, S):
    """Cycles grouped into continuous segments of S cycles on netlists whose
    depth spans several periods, so edges and pending events cross cycle
    boundaries: SAIF, glitch counts and sampled waveforms equal the oracle's
    segment run, whole and in windows, and differ from the cycle-by-cycle
    run."""
    n_segs = 70 if S < 64 else 20
    for seed in range(3):
        rng = np.random.default_rng(seed + 8100)
        T = int(rng.integers(80, 300))
        w = synth.small_random(seed + 8100, 700, 24, 20, S * n_segs, T, 0.3, 2, 60, cond_frac=0.2,
                               wire=(1, 10) if seed % 2 else None, extra=1, extra_p=0.3, skew=min(50, T - 1),
                               edge_frac=0.2)
        N = 24 + 700
        probes = [(int(n), int(k)) for n, k in zip(rng.integers(0, N, 200), rng.integers(0, n_segs, 200))]
        ref = oracle.simulate(w, probes=probes, segment_cycles=S)
        for opt in (dict(), dict(window_cycles=37, tiles_per_wave=3)):
            say("segments", S, seed, T, opt)
            pr = probes if not opt else ()            # only the last window stays resident
            got = gpu_saif(G, w, probes=pr, segment=S, **opt)
            assert_same(w, got, ref, f"S {S} seed {seed} {opt}")
            for (n, k), gw, ow in zip(pr, got[3], ref["probes"]):
                assert gw == ow, (n, k)
        iso = oracle.simulate(w)
        assert not np.array_equal(iso["t1"], ref["t1"])


@pytest.mark.parametrize("opt", [dict(), dict(window_cycles=37), dict(window_cycles=100, hbm_budget=1_900_000),
                                 dict(schedule=1)])
def test_glitch_profile(G, opt):
    """Per-cycle glitch toggles over all nets against the oracle's profile,
    for a sub-range run whole, in windows, split by a tight budget and from
    captured graphs; the profile sums to the per-net glitch counts.  With
    default options also on a continuous-segment view (one entry per
    segment)."""
    w = synth.small_random(95, 1500, 40, 25, 300, 500, 0.4, 2, 70, cond_frac=0.2, extra=2, extra_p=0.3,
                           edge_frac=0.2)
    b, e = 13, 290
    ref = oracle.simulate(w, b, e)
    say("profile", opt)
    with G.GateSim(**opt) as sim:
        d, s = sim.load_work(w)
        prof = sim.glitch_profile(d, s, b, e)
        tc, t0, t1, ig = sim.read_saif_ig(d, reset=True)
        assert len(prof) == e - b and prof.any()
        assert np.array_equal(prof, ref["ig_cycle"])
        assert prof.sum() == ig.sum()
        assert_same(w, (tc, t0, t1, [], {}, ig), ref, f"profile {opt}")
        assert len(sim.glitch_profile(d, s, 5, 5)) == 0
        if not opt:
            v = sim.segment_stimulus(s, 5)
            sim.read_saif_ig(d, reset=True)
            prof = sim.glitch_profile(d, v, 2, 60)
            assert np.array_equal(prof, oracle.simulate(w, 2, 60, segment_cycles=5)["ig_cycle"])


@pytest.mark.parametrize("opt", [dict(), dict(window_cycles=37, tiles_per_wave=3)])
def test_late_nets(G, opt):
    """Per-cycle counts of nets whose activity reaches the end of the cycle,
    with the glitch totals, against the oracle: short periods (most cycles
    late), long ones (none), with and without wires, and on a segment view;
    where no cycle but the last is late, the run equals a continuous one."""
    for seed, T, wire in ((11, 120, None), (12, 150, (1, 30)), (13, 4000, None), (14, 4000, (1, 30))):
        w = synth.small_random(seed + 8200, 800, 24, 20, 140, T, 0.3, 2, 60, cond_frac=0.2, wire=wire,
                               extra=1 if T < 1000 else 0, extra_p=0.3, skew=min(50, T - 1), edge_frac=0.2)
        ref = oracle.simulate(w, 3, 131)
        say("late", seed, T, wire, opt)
        with G.GateSim(**opt) as sim:
            d, s = sim.load_work(w)
            glitch, late = sim.cycle_profile(d, s, 3, 131)
            tc, t0, t1, ig = sim.read_saif_ig(d, reset=True)
            assert np.array_equal(late, ref["late_cycle"]), (seed, np.nonzero(late != ref["late_cycle"])[0][:5])
            assert np.array_equal(glitch, ref["ig_cycle"]), seed
            assert_same(w, (tc, t0, t1, [], {}, ig), ref, f"late {seed}")
            if T < 1000:
                assert late.sum() > 0
            else:
                assert late[:-1].sum() == 0
                cont = oracle.simulate(w, segment_cycles=140)
                full = oracle.simulate(w)
                for k in ("tc", "t0", "t1"):
                    assert np.array_equal(full[k], cont[k]), k
            if not opt and seed == 12:
                v = sim.segment_stimulus(s, 7)
                glitch, late = sim.cycle_profile(d, v, 0, 20)
                r7 = oracle.simulate(w, 0, 20, segment_cycles=7)
                assert np.array_equal(late, r7["late_cycle"]) and np.array_equal(glitch, r7["ig_cycle"])


def test_random_feature_mix(G):
    """Forty small designs, each drawing its own mix of every feature
    (conditional and input-edge-qualified arcs, wires, cells of up to six
    pins, multi-edge inputs, continuous segments) and of launch options
    (window, tiles per wave, staging cap, block shape, schedule); SAIF, glitch
    toggles, the per-cycle profile and late counts all equal the oracle's."""
    for case in range(40):
        rng = np.random.default_rng(9000 + case)
        wide = bool(rng.random() < 0.3)
        gates = int(rng.integers(20, 600))
        S = int(rng.choice([1, 1, 2, 3, 8]))
        C = S * int(rng.integers(3, 90))
        T = int(rng.integers(40, 900))
        w = synth.small_random(9000 + case, gates, int(rng.integers(8, 30)), min(gates, int(rng.integers(2, 25))), C, T,
                               float(rng.uniform(0.05, 0.6)), 1, int(rng.integers(2, 80)),
                               cond_frac=float(rng.choice([0.0, 0.2, 0.5])),
                               wire=(1, int(rng.integers(1, 30))) if rng.random() < 0.4 else None,
                               extra=int(rng.choice([0, 0, 2])), extra_p=0.3, skew=min(50, T - 1), wide=wide,
                               edge_frac=float(rng.choice([0.0, 0.3])))
        opt = {}
        if rng.random() < 0.5:
            opt["window_cycles"] = int(rng.choice([17, 64, 100]))
        if rng.random() < 0.5:
            opt["tiles_per_wave"] = int(rng.choice([1, 2, 3, 8, 16]))
        if rng.random() < 0.4:
            opt["lds_cap"] = int(rng.choice([4, 8, 16, 32]))
        if rng.random() < 0.3:
            opt["waves_per_block"] = int(rng.choice([1, 2, 8]))
            if opt["waves_per_block"] == 8 and opt.get("lds_cap") == 32:
                opt["waves_per_block"] = 2          # 86 KB of LDS per block may exceed the device's limit
        if rng.random() < 0.3:
            opt["schedule"] = G.SCHED_GRAPH
        n = C // S
        b = int(rng.integers(0, n))
        e = int(rng.integers(b + 1, n + 1))
        say("mix", case, gates, C, T, S, wide, opt, (b, e))
        ref = oracle.simulate(w, b, e, segment_cycles=S)
        with G.GateSim(**opt) as sim:
            if wide:
                sim.load_cells(synth.WIDE_PINS, synth.WIDE_TRUTH)
            d, s = sim.load_work(w, cells_loaded=wide)
            if S > 1:
                s = sim.segment_stimulus(s, S)
            glitch, late = sim.cycle_profile(d, s, b, e)
            tc, t0, t1, ig = sim.read_saif_ig(d)
        assert_same(w, (tc, t0, t1, [], {}, ig), ref, f"mix {case}")
        assert np.array_equal(glitch, ref["ig_cycle"]), case
        assert np.array_equal(late, ref["late_cycle"]), case


def test_tiny_config_waveforms(G):
    """2,000 gates x 100 cycles: all SAIF counts plus a sample of full
    waveforms (the analog of the paper's spot-checks)."""
    w = synth.tiny()
    rng = np.random.default_rng(0)
    N = 64 + 2000
    probes = [(int(n), int(c)) for n, c in zip(rng.integers(0, N, 400), rng.integers(0, 100, 400))]
    ref = oracle.simulate(w, probes=probes)
    got = gpu_saif(G, w, probes=probes)
    assert_same(w, got, ref, "tiny")
    for (n, c), (gi, gt, gn), (oi, ot, on) in zip(probes, got[3], ref["probes"]):
        assert (gi, gt, gn) == (oi, ot, on), (n, c)


@pytest.mark.parametrize("opt", [dict(window_cycles=64), dict(window_cycles=37), dict(window_cycles=100),
                                 dict(lds_cap=4), dict(lds_cap=32, waves_per_block=1),
                                 dict(waves_per_block=8, lds_cap=8), dict(window_cycles=300, hbm_budget=1_900_000),
                                 dict(tiles_per_wave=1), dict(tiles_per_wave=3), dict(tiles_per_wave=16, lds_cap=16)])
def test_invariance(G, opt):
    """Same SAIF for every window size, staging cap, block shape and for a
    budget so small that windows shrink and the transition arena refills."""
    w = synth.small_random(42, 1500, 40, 40, 300, 500, 0.4, 2, 70, cond_frac=0.2, extra=2, extra_p=0.3)
    say("invariance", opt)
    got = gpu_saif(G, w, **opt)
    assert_same(w, got, oracle.simulate(w), str(opt))
    if opt.get("hbm_budget"):
        assert got[4]["window_retries"] > 0


def test_transport_wires_dense(G):
    """Wire delays without the net-delay filter on inputs with several
    toggles per cycle: the per-tile walk from the arena (unstaged groups),
    its spill path, and the staged paths all keep every pulse whose delayed
    width is positive."""
    w = synth.small_random(78, 600, 16, 12, 200, 2000, 0.9, 2, 60, cond_frac=0.2, extra=6, extra_p=0.9,
                           wire=(1, 40), edge_frac=0.3)
    w["net_filter"] = False
    ref = oracle.simulate(w)
    for opt in (dict(lds_cap=8), dict(tiles_per_wave=2, lds_cap=4), dict()):
        say("transport dense", opt)
        got = gpu_saif(G, w, wire_transport=True, **opt)
        assert_same(w, got, ref, f"transport dense {opt}")
        assert got[4]["unstaged_groups"] > 0


def test_dense_activity(G):
    """Inputs with about six toggles per cycle: tile groups carry more fanin
    words than the on-chip stage holds, so waves walk the arena directly, and
    output lists outgrow the LDS staging; both paths must match the oracle."""
    w = synth.small_random(77, 600, 16, 12, 200, 2000, 0.9, 2, 60, cond_frac=0.2, extra=6, extra_p=0.9,
                           edge_frac=0.3)
    for opt in (dict(lds_cap=8), dict(tiles_per_wave=2, lds_cap=4), dict()):
        say("dense", opt)
        got = gpu_saif(G, w, **opt)
        assert_same(w, got, oracle.simulate(w), f"dense {opt}")
        assert got[4]["unstaged_groups"] > 0
        if opt:                                   # the automatic cap (32 here) may leave no lane over it
            assert got[4]["spilled_lanes"] > 0


def test_cap_24_spills(G):
    """The cap the library picks for glitch-heavy rounds (24 staged edges per
    lane): inputs with about thirteen toggles per cycle give gate outputs up
    to 39 edges in a cycle (512 (net, cycle) lists above 24, from the
    oracle's probes), so lanes take the spill path; every tile and block
    shape must match the oracle."""
    w = synth.small_random(83, 300, 16, 8, 128, 2000, 0.9, 2, 30, cond_frac=0.2, extra=12, extra_p=1.0,
                           edge_frac=0.3)
    probes = [(n, c) for n in range(16, 316) for c in range(128)]
    ref = oracle.simulate(w, probes=probes)
    ln = np.array([p[2] for p in ref["probes"]])
    assert (ln > 24).sum() > 0, ln.max()
    for opt in (dict(lds_cap=24), dict(lds_cap=24, tiles_per_wave=1), dict(lds_cap=24, tiles_per_wave=3),
                dict(lds_cap=24, waves_per_block=8), dict(lds_cap=24, window_cycles=64)):
        say("cap 24", opt)
        got = gpu_saif(G, w, **opt)
        assert_same(w, got, ref, f"cap 24 {opt}")
        assert got[4]["spilled_lanes"] > 0


def tile_fanin_words(w, ref_probes, n_nets, n_cycles):
    """Fanin words of every (gate, 64-cycle tile): the transitions of its pin
    nets over the tile, from the oracle's probe lengths."""
    ln = np.array([p[2] for p in ref_probes], dtype=np.int64).reshape(n_nets, n_cycles)
    nt = (n_cycles + 63) // 64
    per_tile = np.zeros((n_nets, nt), dtype=np.int64)
    for t in range(nt):
        per_tile[:, t] = ln[:, t * 64:(t + 1) * 64].sum(1)
    fp = np.asarray(w["netlist"]["fanin_ptr"])
    fn = np.asarray(w["netlist"]["fanin_net"])
    return np.array([per_tile[fn[fp[g]:fp[g + 1]]].sum(0) for g in range(len(fp) - 1)])


@pytest.mark.parametrize("wires", [False, True])
def test_tile_stage_mix(G, wires):
    """Tile groups too large for the 512-word fanin stage, at the caps that
    dense designs take: each tile whose fanin fits the stage is staged alone
    and walked from LDS, each larger one is walked from the arena, in the
    same group.  The design has tiles of both kinds (up to three times the
    stage); every tile shape and block shape must match the oracle, with
    interconnect delays filtered or transported."""
    w = synth.small_random(79, 500, 16, 10, 192, 2000, 0.9, 2, 60, cond_frac=0.2, extra=5, extra_p=0.8,
                           edge_frac=0.3, wire=(1, 30) if wires else None)
    n_nets, C = 16 + 500, 192
    probes = [(n, c) for n in range(n_nets) for c in range(C)]
    runs = [("filtered", True)] + ([("transport", False)] if wires else [])
    for name, flt in runs:
        w["net_filter"] = flt
        ref = oracle.Oracle(w["netlist"], w["arcs"], w["wires"]).run(w["stimulus"], probes=probes, probe_cap=1,
                                                                       net_filter=flt)
        fw = tile_fanin_words(w, ref["probes"], n_nets, C)
        classes = ((fw <= 512).sum(), (fw > 512).sum(), (fw > 1024).sum())
        say("tile stage", name, "tiles by fanin words (<=512, >512, >1024):", classes)
        assert min(classes) > 0, classes
        for opt in (dict(lds_cap=32), dict(lds_cap=32, tiles_per_wave=1), dict(lds_cap=32, tiles_per_wave=3),
                    dict(lds_cap=32, waves_per_block=2), dict(lds_cap=16)):
            say("tile stage", name, opt)
            got = gpu_saif(G, w, wire_transport=not flt, **opt)
            assert_same(w, got, ref, f"tile stage {name} {opt}")
            assert got[4]["unstaged_groups"] > 0


def test_queue_overflow(G):
    """Inputs with about two toggles in nearly every cycle: single-pin gates
    fed by them have two pin events in most lanes, so their staged tile
    groups queue more lanes than the compacted walk holds and take the
    per-tile walk instead, beside groups of the compacted path and unstaged
    groups; every path must match the oracle."""
    for wire in (None, (1, 20)):
        w = synth.small_random(91, 400, 24, 4, 256, 1000, 0.95, 5, 60, cond_frac=0.2, extra=1, extra_p=0.95,
                               wire=wire)
        ref = oracle.simulate(w)
        for opt in (dict(), dict(tiles_per_wave=2), dict(lds_cap=4)):
            say("queue overflow", wire, opt)
            got = gpu_saif(G, w, **opt)
            assert_same(w, got, ref, f"queue overflow {wire} {opt}")
            if opt.get("tiles_per_wave", 8) >= 4:        # groups of 2 tiles have only 128 lanes
                assert got[4]["queue_overflows"] > 0


def test_exact_arena(G):
    """Output chunks reserve exactly their words on the compacted path, in
    unstaged groups (the dense-activity case) and in stimulus expansion;
    the per-tile walk of staged groups reserves their fanin bound (at most
    kStageWords per group) up front.  One window's arena use is at least its
    transitions and at most 1% more."""
    w = synth.small_random(79, 3000, 40, 30, 512, 1500, 0.9, 2, 60, cond_frac=0.2, extra=6, extra_p=0.9,
                           edge_frac=0.3)
    ref = oracle.simulate(w)
    for opt in (dict(window_cycles=512), dict(window_cycles=512, tiles_per_wave=1), dict(window_cycles=512,
                                                                                         lds_cap=4)):
        say("exact arena", opt)
        got = gpu_saif(G, w, **opt)
        assert_same(w, got, ref, f"exact arena {opt}")
        assert got[4]["unstaged_groups"] > 0
        words, trans = got[4]["arena_words"], int(ref["tc"].sum())
        assert trans <= words <= 1.01 * trans, (words, trans)


def test_learned_density(G):
    """A design whose logic multiplies its inputs' toggles (ripple-carry-like
    XOR/MUX chains, about 1.07 transitions per net and cycle from 0.3 input
    toggles): the first run sizes the staging cap from the inputs, the second
    from the density the first observed; both equal the oracle, and the
    second re-walks no more lanes."""
    w = synth.glitchy(seed=21, n_gates=20000, n_inputs=400, n_levels=60, n_cycles=128)
    ref = oracle.simulate(w)
    spilled = []
    with G.GateSim() as sim:
        d, s = sim.load_work(w)
        for run in range(2):
            say("learned density, run", run)
            sim.stats(reset=True)
            sim.simulate(d, s, 0, 128)
            spilled.append(sim.stats()["spilled_lanes"])
            tc, t0, t1, ig = sim.read_saif_ig(d, reset=True)
            assert_same(w, (tc, t0, t1, [], {}, ig), ref, f"run {run}")
    assert spilled[1] <= spilled[0], spilled


@pytest.mark.parametrize("opt", [dict(), dict(tiles_per_wave=3), dict(lds_cap=4, waves_per_block=2)])
def test_wide_cells(G, opt):
    """Cells of four to six pins (no delay lookup table; arc delays chosen per
    event, two tiles per staging group) mixed with the base cells, with
    conditional arcs and glitchy inputs, with and without wire delays (with
    wires also with input-edge-qualified arcs)."""
    for wire in (None, (1, 6)):
        w = synth.small_random(91, 1500, 40, 20, 200, 600, 0.3, 2, 60, cond_frac=0.2, extra=2, extra_p=0.3,
                               wide=True, wire=wire, edge_frac=0.3 if wire else 0.0)
        say("wide", opt, wire)
        rng = np.random.default_rng(5)
        N = 40 + 1500
        probes = [(int(n), int(c)) for n, c in zip(rng.integers(40, N, 200), rng.integers(0, 200, 200))]
        ref = oracle.simulate(w, probes=probes)
        got = gpu_saif(G, w, probes=probes, **opt)
        assert_same(w, got, ref, f"wide {opt} {wire}")
        for (n, c), g_, o_ in zip(probes, got[3], ref["probes"]):
            assert g_ == o_, (n, c)


def test_long_period(G):
    """The longest allowed period: a wave's T1 sum over its tiles passes 2^32
    picoseconds, so the per-wave reductions must not wrap."""
    T = (1 << 24) - 1
    w = synth.small_random(93, 400, 12, 10, 300, T, 0.5, 5, 60, cond_frac=0.2, extra=2, extra_p=0.3)
    ref = oracle.simulate(w)
    assert int(ref["t1"].max()) > (1 << 32)
    for opt in (dict(), dict(tiles_per_wave=16)):
        assert_same(w, gpu_saif(G, w, **opt), ref, f"long period {opt}")


def test_cycle_subranges(G):
    """Accumulating disjoint sub-ranges equals the whole range; a range can
    start and end anywhere (ragged tiles on both sides)."""
    w = synth.small_random(9, 800, 30, 20, 260, 700, 0.3, 3, 60, cond_frac=0.2)
    ref = oracle.simulate(w)
    with G.GateSim(window_cycles=90) as sim:
        d, s = sim.load_work(w)
        for b, e in ((0, 1), (1, 63), (63, 64), (64, 200), (200, 200), (200, 260)):
            sim.simulate(d, s, b, e)
        got = sim.read_saif(d)
    assert_same(w, got, ref, "subranges")


def test_levelizer_matches_oracle(G):
    w = synth.small_random(13, 3000, 50, 60, 2, 100, 0.3, 1, 5)
    o = oracle.Oracle(w["netlist"], w["arcs"])
    with G.GateSim() as sim:
        d, s = sim.load_work(w)
        lv = sim.levels(d)
        info = sim.design_info(d)
    exp = np.array([o.level(50 + g) for g in range(3000)])
    assert np.array_equal(lv, exp)
    assert info.n_levels == exp.max()


def test_errors(G):
    with G.GateSim() as sim:
        sim.load_cells(synth.CELL_PINS, synth.CELL_TRUTH)
        # a two-gate loop: NAND2(in, g1) -> g0 ; BUF(g0) -> g1
        with pytest.raises(G.GateSimError) as e:
            sim.load_netlist(1, [synth.NAND2, synth.BUF], [0, 2, 3], [0, 2, 1])
        assert e.value.status == G.GS_E_NOT_DAG
        w = synth.small_random(3, 100, 8, 5, 10, 200, 0.3, 2, 9)
        d, s = sim.load_work(w, cells_loaded=True)
        with pytest.raises(G.GateSimError) as e:
            sim.simulate(d, s, 5, 11)
        assert e.value.status == G.GS_E_INVALID
        with pytest.raises(G.GateSimError) as e:
            sim.read_waveform(d, s, 3, 0)
        assert e.value.status == G.GS_E_STATE
        n = w["netlist"]
        d2 = sim.load_netlist(n["n_inputs"], n["cell_of_gate"], n["fanin_ptr"], n["fanin_net"])
        s2 = sim.load_stimulus(d2, 200, 10, w["stimulus"]["init"], w["stimulus"]["toggle_ptr"],
                               w["stimulus"]["toggle_ps"])
        with pytest.raises(G.GateSimError) as e:
            sim.simulate(d2, s2, 0, 10)                       # no arcs yet
        assert e.value.status == G.GS_E_STATE
        sim.simulate(d, s, 0, 0)                              # empty range is fine


def test_capacity_errors(G):
    """More than 32,767 transitions in one (net, 64-cycle tile) is reported
    as GS_E_CAPACITY, from the expansion (one input with 520 toggles per
    cycle) and from a gate (an XOR2 of two inputs toggling on alternate
    picoseconds, 624 output edges per cycle); the chunk is written empty,
    nothing is committed, and the context keeps working."""
    T, C = 1000, 64
    heavy = [[c * T + t for c in range(C) for t in range(520)]]
    w = work(1, [("BUF", [0])], (1, 1), heavy, [0], period=T, n_cycles=C)
    even = [c * T + t for c in range(C) for t in range(0, 624, 2)]
    odd = [c * T + t for c in range(C) for t in range(1, 624, 2)]
    w2 = work(2, [("XOR2", [0, 1])], (1, 1), [even, odd], [0, 0], period=T, n_cycles=C)
    ok = synth.small_random(5, 300, 16, 12, 150, 400, 0.3, 3, 40, cond_frac=0.2)
    with G.GateSim() as sim:
        sim.load_cells(synth.WIDE_PINS, synth.WIDE_TRUTH)
        for case, ww in (("input", w), ("gate", w2)):
            say("capacity", case)
            d, s = sim.load_work(ww, cells_loaded=True)
            with pytest.raises(G.GateSimError) as e:
                sim.simulate(d, s, 0, C)
            assert e.value.status == G.GS_E_CAPACITY, case
            tc, t0, t1 = sim.read_saif(d)
            assert not tc.any() and not t1.any(), case
        d, s = sim.load_work(ok, cells_loaded=True)
        sim.simulate(d, s, 0, 150)
        tc, t0, t1, ig = sim.read_saif_ig(d)
    assert_same(ok, (tc, t0, t1, [], {}, ig), oracle.simulate(ok), "after capacity errors")


def test_entry_point_errors(G):
    """Segment views and the glitch profile reject what they cannot do."""
    w = synth.small_random(3, 100, 8, 5, 10, 200, 0.3, 2, 9)
    with G.GateSim() as sim:
        d, s = sim.load_work(w)
        for seg in (0, 3, 11):                                # 10 cycles: not a positive divisor
            with pytest.raises(G.GateSimError) as e:
                sim.segment_stimulus(s, seg)
            assert e.value.status == G.GS_E_INVALID, seg
        st = w["stimulus"]
        s3 = sim.load_stimulus(d, 1 << 23, 4, st["init"], np.zeros(9, dtype=np.int64), np.zeros(0, dtype=np.int64))
        with pytest.raises(G.GateSimError) as e:
            sim.segment_stimulus(s3, 4)                       # 2^25 ps segments
        assert e.value.status == G.GS_E_INVALID
        v = sim.segment_stimulus(s3, 2)                       # 2^24 ps is allowed
        with pytest.raises(G.GateSimError) as e:
            sim.simulate(d, v, 0, 3)                          # the view has 2 cycles
        assert e.value.status == G.GS_E_INVALID
        with pytest.raises(G.GateSimError) as e:
            sim.glitch_profile(d, s, 4, 12)
        assert e.value.status == G.GS_E_INVALID
        with pytest.raises(G.GateSimError) as e:
            sim.glitch_profile(d, 99, 0, 2)
        assert e.value.status == G.GS_E_INVALID


def test_edge_cases(G):
    # inputs that never toggle, a gate-free design, single-cycle stimulus
    w = synth.small_random(21, 400, 12, 10, 1, 300, 0.0, 2, 40)
    assert_same(w, gpu_saif(G, w), oracle.simulate(w), "no toggles")
    w = work(3, [], [], [[5, 50], [], [7]], [0, 1, 1], period=100, n_cycles=1)
    assert_same(w, gpu_saif(G, w), oracle.simulate(w), "no gates")
    # a toggle at local time 0 and at the last picosecond of a cycle
    w = work(2, [("XOR2", [0, 1]), ("NAND2", [0, 2])], (7, 5), [[0, 99, 100], [199]], [0, 1], period=100, n_cycles=2)
    assert_same(w, gpu_saif(G, w), oracle.simulate(w), "boundary toggles")


def test_scale_bench_launch(G):
    """The 1M-gate workload exactly as the benchmark launches it: all 10,000
    cycles in one window, default tiles, staging and options.  Ten cycles
    spread over the run are re-simulated by the oracle; the GPU's waveforms
    of 60 nets in each and its per-cycle glitch and late-net totals must
    equal the oracle's, and T0 + T1 = C x T for every net."""
    w = synth.scale()
    C, T = w["stimulus"]["n_cycles"], w["stimulus"]["period"]
    N = 20_000 + 1_000_000
    rng = np.random.default_rng(4)
    cycles = sorted(int(c) for c in rng.choice(C, 10, replace=False))
    nets = [int(n) for n in rng.integers(0, N, 60)]
    say("scale launch: gpu")
    with G.GateSim() as sim:
        d, s = sim.load_work(w)
        prof, late = sim.cycle_profile(d, s, 0, C)
        tc, t0, t1 = sim.read_saif(d)
        waves = {(n, c): sim.read_waveform(d, s, n, c) for c in cycles for n in nets}
    assert np.all(t0 + t1 == C * T)
    o = oracle.Oracle(w["netlist"], w["arcs"])
    for c in cycles:
        say("scale launch: oracle cycle", c)
        ref = o.run(w["stimulus"], c, c + 1, probes=[(n, c) for n in nets])
        assert int(prof[c]) == int(ref["ig_cycle"][0]), c
        assert int(late[c]) == int(ref["late_cycle"][0]), c
        for n, pr in zip(nets, ref["probes"]):
            assert waves[(n, c)] == pr, (n, c)


def test_scale_config_sample(G):
    """The 1M-gate workload in 1,000-cycle windows from cycle 0 (default tile
    and staging).  The GPU runs cycles [0, 990) and [0, 1010); under cycle
    isolation their SAIF difference is cycles 990..1009, which straddle the
    first window boundary and are compared net by net with the oracle, plus
    a waveform sample from the resident second window and the per-cycle
    glitch profile of those cycles."""
    w = synth.scale(n_cycles=1100)
    b, e = 990, 1010
    N = 20_000 + 1_000_000
    rng = np.random.default_rng(1)
    probes = [(int(n), int(c)) for n, c in zip(rng.integers(0, N, 200), rng.integers(1000, 1010, 200))]
    say("scale: oracle")
    ref = oracle.simulate(w, b, e, probes=probes)
    say("scale: gpu")
    with G.GateSim(window_cycles=1000) as sim:
        d, s = sim.load_work(w)
        sim.simulate(d, s, 0, b)
        lo = sim.read_saif(d, reset=True)
        prof = sim.glitch_profile(d, s, 0, e)
        hi = sim.read_saif(d, reset=True)
        waves = [sim.read_waveform(d, s, n, c) for n, c in probes]
    got = tuple(h - l for h, l in zip(hi, lo))
    assert_same(w, got, ref, "scale")
    assert np.array_equal(prof[b:e], ref["ig_cycle"])
    for (n, c), g_, o_ in zip(probes, waves, ref["probes"]):
        assert g_ == o_, (n, c)


def test_glitchy_config_sample(G):
    """The 8M-gate glitch-heavy workload (30% ripple-carry-like XOR/MUX
    chains, 2,000 cycles) with windows sized by the planner to fit memory:
    the SAIF difference of GPU runs over [0, 999) and [0, 1000) is cycle
    999, compared net by net with the oracle; lanes above the on-chip
    staging cap take the spill path."""
    w = synth.glitchy()
    N = 150_000 + 8_000_000
    rng = np.random.default_rng(2)
    probes = [(int(n), 999) for n in rng.integers(150_000, N, 200)]
    say("glitchy: oracle")
    ref = oracle.simulate(w, 999, 1000, probes=probes)
    say("glitchy: gpu")
    with G.GateSim() as sim:
        d, s = sim.load_work(w)
        sim.simulate(d, s, 0, 999)
        lo = sim.read_saif(d, reset=True)
        sim.simulate(d, s, 0, 1000)
        hi = sim.read_saif(d, reset=True)
        waves = [sim.read_waveform(d, s, n, c) for n, c in probes]
        st = sim.stats()
    got = tuple(h - l for h, l in zip(hi, lo))
    assert_same(w, got, ref, "glitchy")
    for (n, c), g_, o_ in zip(probes, waves, ref["probes"]):
        assert g_ == o_, (n, c)
    assert st["spilled_lanes"] > 0
