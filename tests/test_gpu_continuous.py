"""GPU parity of continuous views: segments of S cycles simulated as one
continuous run, with one lane per cycle and the pending output edge carried
from each cycle into the next (Section 1's re-simulation, Section 3's cycle
parallelism), against the oracle's segment run, bit-exact.

The netlists are several periods deep (levels x delays well beyond the
period), so most segments have edges and pending events that cross cycle
boundaries.  The single-lane segment view (gs_segment_stimulus) computes the
same results another way and is compared where the oracle would be slow.
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


def run_view(G, w, S, b=0, e=None, probes=(), carry=True, noalloc=False, **opt):
    with G.GateSim(**opt) as sim:
        d, s = sim.load_work(w)
        v = sim.continuous_stimulus(s, S) if carry else sim.segment_stimulus(s, S)
        e = w["stimulus"]["n_cycles"] // S if e is None else e
        if noalloc:
            sim.simulate_noalloc(d, v, b, e)
        else:
            sim.simulate(d, v, b, e)
        tc, t0, t1, ig = sim.read_saif_ig(d)
        waves = [sim.read_waveform(d, v, n, c) for n, c in probes]
        st = sim.stats()
    return {"tc": tc, "t0": t0, "t1": t1, "ig": ig, "waves": waves, "stats": st}


def assert_same(got, ref, tag):
    for name in ("tc", "t0", "t1", "ig"):
        a, b = got[name], ref[name]
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{tag}: {name} differs on {len(bad)} nets, first {bad[:8]} "
                                 f"gpu {a[bad[:8]]} oracle {b[bad[:8]]}")


def deep(seed, n_gates, n_inputs, levels, cycles, wide=False, zero=False):
    """A netlist whose depth spans several periods: 2-60 ps arcs over
    `levels` levels against a 80-300 ps period; conditional and
    input-edge-qualified arcs, inputs with several edges per cycle."""
    rng = np.random.default_rng(seed)
    T = int(rng.integers(80, 300))
    return synth.small_random(seed, n_gates, n_inputs, levels, cycles, T, 0.3, 0 if zero else 2, 0 if zero else 60,
                              cond_frac=0.0 if zero else 0.2, extra=1, extra_p=0.3, skew=min(50, T - 1),
                              wide=wide, edge_frac=0.0 if zero else 0.2)


@pytest.mark.parametrize("S", [2, 7, 16, 64, 100])
def test_carry_matches_oracle(G, S):
    """SAIF, glitch counts and sampled segment waveforms equal the oracle's
    segment run, whole and in windows (37 cycles rounded down to whole
    segments; 3 tiles per wave where segments tile 64 cycles)."""
    n_segs = max(4, 1400 // S)
    for seed in range(3):
        w = deep(seed + 9100, 700, 24, 20, S * n_segs)
        N = 24 + 700
        rng = np.random.default_rng(seed)
        probes = [(int(n), int(k)) for n, k in zip(rng.integers(0, N, 150), rng.integers(0, n_segs, 150))]
        ref = oracle.simulate(w, probes=probes, segment_cycles=S)
        for opt in (dict(), dict(window_cycles=37, tiles_per_wave=3)):
            say("carry", S, seed, w["stimulus"]["period"], opt)
            pr = probes if not opt else ()            # only the last window stays resident
            got = run_view(G, w, S, probes=pr, **opt)
            assert_same(got, ref, f"S {S} seed {seed} {opt}")
            for (n, k), gw, ow in zip(pr, got["waves"], ref["probes"]):
                assert gw == ow, (n, k)
        iso = oracle.simulate(w)
        assert not np.array_equal(iso["t1"], ref["t1"])    # the segments do cross cycle boundaries


def test_carry_input_glitches_across_expansion_groups(G):
    """Regression: the stimulus expansion counts an input's glitch toggles
    per group of four 64-cycle tiles, and a segment can end in a group that
    holds none of its toggles (S = 3, segment 85 = cycles 255-257 straddles
    the groups at cycle 256, and the last group, cycles 256-260, is short).
    That group's share is negative and must subtract.  Input 0 toggles once
    in that segment (IG 0), input 1 twice in segment 33 and once in segment
    85 (IG 2), input 2 twice before cycle 256 and once after it, all in
    segment 85 (IG 2); input 3 toggles every seventh cycle."""
    from tests.handmade import work
    T, C, S = 100, 261, 3
    tog = [[255 * T + 50],
           [100 * T + 30, 101 * T + 60, 255 * T + 40],
           [255 * T + 10, 255 * T + 60, 256 * T + 20],
           [c * T + 35 for c in range(0, C, 7)]]
    w = work(4, [("BUF", [i]) for i in range(4)], (5, 5), tog, [0, 1, 0, 1], period=T, n_cycles=C)
    ref = oracle.simulate(w, segment_cycles=S)
    assert ref["ig"][:3].tolist() == [0, 2, 2]
    for opt in (dict(), dict(noalloc=True), dict(tiles_per_wave=1)):
        say("carry input glitches", opt)
        assert_same(run_view(G, w, S, **opt), ref, f"input glitches {opt}")
    assert_same(run_view(G, w, S, 1, C // S), oracle.simulate(w, 1, C // S, segment_cycles=S), "from segment 1")


@pytest.mark.parametrize("S", [16, 50])
def test_carry_wide_cells(G, S):
    """Cells of four to six pins (delays read per pin, not from the table)."""
    for seed in range(2):
        w = deep(seed + 9200, 500, 30, 15, S * 12, wide=True)
        say("carry wide", S, seed)
        assert_same(run_view(G, w, S, window_cycles=2 * S), oracle.simulate(w, segment_cycles=S), f"wide {S} {seed}")


def test_carry_subranges_and_zero_delay(G):
    """Segment sub-ranges accumulate to the whole range; zero-delay designs
    (nothing is ever pending at a cycle's end) equal their isolated run."""
    S = 10
    w = deep(9300, 600, 20, 18, S * 30)
    ref = oracle.simulate(w, segment_cycles=S)
    with G.GateSim() as sim:
        d, s = sim.load_work(w)
        v = sim.continuous_stimulus(s, S)
        for b, e in ((0, 7), (7, 8), (8, 30)):
            sim.simulate(d, v, b, e)
        tc, t0, t1, ig = sim.read_saif_ig(d)
    assert_same({"tc": tc, "t0": t0, "t1": t1, "ig": ig}, ref, "sub-ranges")
    z = deep(9301, 600, 20, 18, S * 30, zero=True)
    assert_same(run_view(G, z, S), oracle.simulate(z, segment_cycles=S), "zero delay")


def test_carry_equals_segment_view(G):
    """A 6,000-gate, 60-level design over 1,000-cycle segments: the
    cycle-parallel view equals the single-lane segment view exactly, and the
    oracle on the first segment."""
    S = 1000
    w = deep(9400, 6000, 200, 60, 2 * S)
    a = run_view(G, w, S)
    b = run_view(G, w, S, carry=False)
    assert_same(a, b, "carry vs single lane")
    say("carry 6k gates, oracle on segment 0")
    assert_same(run_view(G, w, S, 0, 1), oracle.simulate(w, 0, 1, segment_cycles=S), "segment 0")


def test_carry_20k_gates_1000_cycles(G):
    """20k gates over 80 levels of 5-60 ps arcs (several 400 ps periods
    deep), one 1,000-cycle segment, bit-exact against the oracle's segment
    run (about 40 s of oracle time)."""
    S = 1000
    w = synth.small_random(9500, 20_000, 400, 80, S, 400, 0.2, 5, 60, cond_frac=0.1, extra=1, extra_p=0.2,
                           skew=50, edge_frac=0.1)
    say("carry 20k gates: oracle")
    ref = oracle.simulate(w, segment_cycles=S)
    say("carry 20k gates: gpu")
    got = run_view(G, w, S)
    assert_same(got, ref, "20k")


def test_carry_noalloc_and_batch(G):
    """The allocation-free entry point and a batch mixing continuous views,
    single-lane views and plain stimuli give each job its own result."""
    S = 32
    ws = [deep(9600 + i, 400 + 200 * i, 16, 14, S * 20) for i in range(3)]
    refs = [oracle.simulate(ws[0], segment_cycles=S), oracle.simulate(ws[1], segment_cycles=S),
            oracle.simulate(ws[2])]
    assert_same(run_view(G, ws[0], S, noalloc=True), refs[0], "noalloc")
    with G.GateSim() as sim:
        ids = [sim.load_work(x) for x in ws]
        v0 = sim.continuous_stimulus(ids[0][1], S)
        v1 = sim.segment_stimulus(ids[1][1], S)
        sim.simulate_batch([(ids[0][0], v0, 0, 20), (ids[2][0], ids[2][1], 0, S * 20), (ids[1][0], v1, 0, 20)])
        for (d, _), ref, tag in zip(ids, refs, ("carry", "single lane", "plain")):
            tc, t0, t1, ig = sim.read_saif_ig(d)
            assert_same({"tc": tc, "t0": t0, "t1": t1, "ig": ig}, ref, f"batch {tag}")


def test_carry_errors(G):
    """Designs with interconnect delays, the cycle profile, tuning and views
    of views are refused; a segment larger than the budget is GS_E_NOMEM."""
    w = synth.small_random(9700, 200, 10, 8, 64, 200, 0.3, 2, 40, wire=(1, 10))
    with G.GateSim() as sim:
        d, s = sim.load_work(w)
        v = sim.continuous_stimulus(s, 8)
        with pytest.raises(G.GateSimError):
            sim.simulate(d, v, 0, 8)                    # interconnect delays
    w = deep(9701, 200, 10, 8, 64)
    with G.GateSim() as sim:
        d, s = sim.load_work(w)
        v = sim.continuous_stimulus(s, 8)
        for bad in (lambda: sim.cycle_profile(d, v, 0, 8), lambda: sim.autotune(d, v, 0, 8),
                    lambda: sim.continuous_stimulus(v, 2), lambda: sim.segment_stimulus(v, 2),
                    lambda: sim.continuous_stimulus(s, 7), lambda: sim.simulate(d, v, 0, 9)):
            with pytest.raises(G.GateSimError):
                bad()
    w = deep(9702, 3000, 20, 20, 2048)
    with G.GateSim(hbm_budget=3_000_000) as sim:
        d, s = sim.load_work(w)
        v = sim.continuous_stimulus(s, 2048)
        with pytest.raises(G.GateSimError) as e:
            sim.simulate(d, v, 0, 1)
        assert e.value.status == G.GS_E_NOMEM
