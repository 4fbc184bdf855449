"""GPU parity with dead nets released (gs_options.release_dead): a net's
transitions are kept only until the last level that reads them, the window's
arena being split into one region per such level and regions reused once
their level has run.  Results must equal the oracle's bit for bit; a budget
that holds the regions' peak but not every net's transitions must run with
release and fail without it.
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


def run(G, w, b=0, e=None, **opt):
    e = w["stimulus"]["n_cycles"] if e is None else e
    with G.GateSim(**opt) as sim:
        d, s = sim.load_work(w)
        sim.simulate(d, s, b, e)
        tc, t0, t1, ig = sim.read_saif_ig(d)
        st = sim.stats()
    return {"tc": tc, "t0": t0, "t1": t1, "ig": ig, "stats": st}


def assert_same(got, ref, tag):
    for name in ("tc", "t0", "t1", "ig"):
        a, b = got[name], ref[name]
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{tag}: {name} differs on {len(bad)} nets, first {bad[:8]} "
                                 f"gpu {a[bad[:8]]} oracle {b[bad[:8]]}")


@pytest.mark.parametrize("mode", ["plain", "cond+edges", "wires", "multi-edge", "wide"])
def test_release_matches_oracle(G, mode):
    """Random designs of every feature, whole and in windows (several windows
    share a round and so a region plan), against the oracle."""
    for seed in range(4):
        rng = np.random.default_rng(seed + 9800)
        gates = int(rng.integers(100, 1500))
        levels = int(rng.integers(3, 40))
        C = int(rng.integers(64, 400))
        T = int(rng.integers(80, 500))
        n_in = int(rng.integers(4, 40))
        if mode == "wide":
            n_in = max(n_in, 16)                         # room for six distinct fanins
        w = synth.small_random(seed + 9800, gates, n_in, min(levels, gates), C, T,
                               float(rng.uniform(0.1, 0.6)), 1, int(rng.integers(2, 80)),
                               cond_frac=0.3 if "cond" in mode else 0.0,
                               wire=(1, int(rng.integers(1, 25))) if mode == "wires" else None,
                               extra=3 if mode == "multi-edge" else 0, extra_p=0.4, skew=min(50, T - 1),
                               wide=mode == "wide", edge_frac=0.3 if "edges" in mode else 0.0)
        ref = oracle.simulate(w)
        for opt in (dict(), dict(window_cycles=int(rng.choice([64, 100, 37])))):
            say("release", mode, seed, gates, levels, C, T, opt)
            got = run(G, w, release_dead=True, **opt)
            assert_same(got, ref, f"{mode} seed {seed} {opt}")


def test_release_reuses_space(G):
    """On a 20,000-gate design 60 levels deep the regions' peak stays below
    the transitions the window stores, the waveform readback is refused, and
    a second call (learned region densities) needs no retry."""
    w = synth.small_random(9900, 20_000, 300, 60, 256, 400, 0.4, 2, 60, cond_frac=0.1, extra=2, extra_p=0.4,
                           skew=50)
    ref = oracle.simulate(w)
    with G.GateSim(release_dead=True) as sim:
        d, s = sim.load_work(w)
        sim.simulate(d, s, 0, 256)
        tc, t0, t1, ig = sim.read_saif_ig(d, reset=True)
        assert_same({"tc": tc, "t0": t0, "t1": t1, "ig": ig}, ref, "first call")
        with pytest.raises(G.GateSimError) as e:
            sim.read_waveform(d, s, 300, 0)
        assert e.value.status == G.GS_E_STATE
        with pytest.raises(G.GateSimError):
            sim.cycle_profile(d, s, 0, 8)
        sim.stats(reset=True)
        sim.simulate(d, s, 0, 256)
        tc, t0, t1, ig = sim.read_saif_ig(d, reset=True)
        st = sim.stats()
    assert_same({"tc": tc, "t0": t0, "t1": t1, "ig": ig}, ref, "second call")
    say("release: stored", st["arena_words"], "peak", st["release_peak_words"], "retries", st["window_retries"])
    assert st["window_retries"] == 0
    assert 0 < st["release_peak_words"] < st["arena_words"]


def test_release_fits_where_every_net_does_not(G):
    """A 64-cycle window (which cannot be split) of a glitch-heavy design,
    under a budget that holds its chunk headers and the regions' peak but not
    the transitions of every net: GS_E_NOMEM without release, bit-exact
    against the oracle with it."""
    w = synth.small_random(9950, 12_000, 200, 50, 64, 300, 0.5, 2, 40, extra=3, extra_p=0.6, skew=50)
    N = 200 + 12_000
    hdr = N * 1 * (16 + 64 * 2)
    full = run(G, w)
    rel = run(G, w, release_dead=True)
    assert rel["stats"]["window_retries"] == 0
    peak, stored = rel["stats"]["release_peak_words"], full["stats"]["arena_words"]
    budget = hdr + int(peak * 4 * 1.02) + 4096
    say("release: headers", hdr, "stored words", stored, "peak words", peak, "budget", budget)
    assert budget < hdr + stored * 4, "the design does not need release"
    with pytest.raises(G.GateSimError) as e:
        run(G, w, hbm_budget=budget)
    assert e.value.status == G.GS_E_NOMEM
    ref = oracle.simulate(w)
    got = run(G, w, hbm_budget=budget, release_dead=True)
    assert_same(got, ref, "tight budget")


def test_release_with_continuous_views_and_graphs(G):
    """Release combined with a cycle-parallel continuous view (carried
    edges), with captured-graph rounds replayed for several windows, and
    with transport wires."""
    w = synth.small_random(9960, 900, 20, 24, 16 * 24, 150, 0.35, 2, 50, cond_frac=0.2, extra=1, extra_p=0.3,
                           skew=50, edge_frac=0.2)
    with G.GateSim(release_dead=True, window_cycles=64) as sim:
        d, s = sim.load_work(w)
        v = sim.continuous_stimulus(s, 16)
        sim.simulate(d, v, 0, 24)
        tc, t0, t1, ig = sim.read_saif_ig(d)
    assert_same({"tc": tc, "t0": t0, "t1": t1, "ig": ig}, oracle.simulate(w, segment_cycles=16), "continuous")
    ref = oracle.simulate(w)
    got = run(G, w, release_dead=True, window_cycles=64, schedule=G.SCHED_GRAPH)
    assert_same(got, ref, "graphs")
    assert got["stats"]["graph_launches"] > 0
    wt = synth.small_random(9961, 700, 20, 20, 200, 300, 0.4, 1, 40, wire=(1, 20), extra=3, extra_p=0.5, skew=50)
    wt["net_filter"] = False
    assert_same(run(G, wt, release_dead=True, wire_transport=True), oracle.simulate(wt), "transport wires")
