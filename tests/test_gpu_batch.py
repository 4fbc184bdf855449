"""GPU parity of the batched schedule, captured-graph replays and the
autotuner, each checked bit-exactly against the oracle."""
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


def same(got, ref, tag):
    for name, a, b in zip(("tc", "t0", "t1", "ig"), got, (ref["tc"], ref["t0"], ref["t1"], ref["ig"])):
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{tag}: {name} differs on {len(bad)} nets, first {bad[:6]}")


def uneven_jobs(n, seed0=400, gmax=3000, wide_every=0):
    """Uneven instances shaped like the batched workload, scaled to oracle size
    (every ``wide_every``-th one drawing four- to six-pin cells as well)."""
    works = []
    rng = np.random.default_rng(seed0)
    for i in range(n):
        g = int(np.exp(rng.uniform(np.log(200), np.log(gmax))))
        inputs = max(3, g // 50)
        levels = max(2, int(round(6 + 20 * np.log(g / 200) / np.log(gmax / 200))))
        cycles = int(np.exp(rng.uniform(np.log(20), np.log(300))))
        p = float(rng.uniform(0.05, 0.3))
        wide = wide_every > 0 and i % wide_every == 1
        inputs = max(inputs, 8) if wide else inputs
        works.append(synth.small_random(seed0 + i, g, inputs, min(levels, g), cycles, 800, p, 5, 80, cond_frac=0.1,
                                        wide=wide, edge_frac=0.3 if i % 3 == 2 else 0.0))
    return works


def test_graph_replays(G):
    """Windows of one shape replay one captured graph; every replay is
    compared with the oracle, with unrelated eager GPU work in between."""
    import torch
    w = synth.small_random(31, 1200, 30, 25, 330, 600, 0.3, 3, 60, cond_frac=0.2, extra=1, extra_p=0.2)
    with G.GateSim(window_cycles=64, schedule=G.SCHED_GRAPH) as sim:
        d, s = sim.load_work(w)
        o = oracle.Oracle(w["netlist"], w["arcs"])
        for b in range(0, 330, 64):
            e = min(330, b + 64)
            sim.simulate(d, s, b, e)
            got = sim.read_saif_ig(d, reset=True)
            x = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
            assert float(x.sum().item()) > 0
            torch.cuda.synchronize()
            same(got, o.run(w["stimulus"], b, e), f"window {b}")
        st = sim.stats()
    assert st["graph_launches"] == 6


def test_batch_uneven_instances(G):
    works = uneven_jobs(10, wide_every=3)
    with G.GateSim() as sim:
        sim.load_cells(synth.WIDE_PINS, synth.WIDE_TRUTH)         # a superset of every instance's library
        ids = []
        for w in works:
            ids.append(sim.load_work(w, cells_loaded=True))
        jobs = [(d, s, 0, w["stimulus"]["n_cycles"]) for (d, s), w in zip(ids, works)]
        say("batch", [w["netlist"]["n_gates"] for w in works])
        sim.simulate_batch(jobs)
        for (d, s), w in zip(ids, works):
            same(sim.read_saif_ig(d), oracle.simulate(w), f"design {d}")


def test_batch_segmented_stimuli(G):
    """Jobs on continuous-segment views of their stimuli (segments of 4 and
    10 cycles) batched with a plain job: every design matches the oracle's
    segment run."""
    works = uneven_jobs(3, seed0=700, gmax=1500)
    seg = [4, 10, 1]
    for w, S in zip(works, seg):
        C = w["stimulus"]["n_cycles"]
        w["stimulus"] = synth.make_stimulus(700 + S, w["netlist"]["n_inputs"], max(S, C - C % S), 800, 0.2, skew=50)
    with G.GateSim() as sim:
        ids = [sim.load_work(w, cells_loaded=i > 0) for i, w in enumerate(works)]
        jobs = []
        for (d, s), w, S in zip(ids, works, seg):
            v = sim.segment_stimulus(s, S) if S > 1 else s
            jobs.append((d, v, 0, w["stimulus"]["n_cycles"] // S))
        sim.simulate_batch(jobs)
        for (d, s), w, S in zip(ids, works, seg):
            same(sim.read_saif_ig(d), oracle.simulate(w, segment_cycles=S), f"design {d} S {S}")


def test_batch_repeated_design_and_ranges(G):
    """One design in several jobs with different cycle ranges: the counts add up."""
    w = synth.small_random(77, 900, 20, 18, 200, 500, 0.3, 3, 50, cond_frac=0.1)
    with G.GateSim(schedule=G.SCHED_GRAPH) as sim:
        d, s = sim.load_work(w)
        jobs = [(d, s, 0, 70), (d, s, 70, 71), (d, s, 71, 200)]
        for rep in range(3):
            sim.simulate_batch(jobs)
            same(sim.read_saif_ig(d, reset=True), oracle.simulate(w), f"replay {rep}")


def test_batch_tight_budget(G):
    """A budget that holds only part of the batch: rounds are split and
    windows halved, results unchanged."""
    works = uneven_jobs(6, seed0=500, gmax=1500)
    with G.GateSim(hbm_budget=3_000_000) as sim:
        ids = [sim.load_work(w, cells_loaded=i > 0) for i, w in enumerate(works)]
        sim.simulate_batch([(d, s, 0, w["stimulus"]["n_cycles"]) for (d, s), w in zip(ids, works)])
        for (d, s), w in zip(ids, works):
            same(sim.read_saif_ig(d), oracle.simulate(w), f"design {d}")


def test_autotune_keeps_results(G):
    w = synth.small_random(88, 2500, 40, 30, 150, 800, 0.2, 5, 80, cond_frac=0.1)
    with G.GateSim(autotune=True) as sim:
        d, s = sim.load_work(w)
        t = sim.autotune(d, s, 0, 128)
        say("autotune", t)
        assert t["lds_cap"] in (8, 16) and t["tiles_per_wave"] >= 1
        tc, t0, t1 = sim.read_saif(d)
        assert not tc.any() and not t1.any()                  # nothing committed while tuning
        sim.simulate_batch([(d, s, 0, 150)])
        same(sim.read_saif_ig(d), oracle.simulate(w), "after autotune")
