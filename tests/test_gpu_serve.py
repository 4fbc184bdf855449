"""GPU tests of the serving loop (continuous batching of re-simulation
requests): window requests and delay-edit cone re-simulation are checked
against the oracle, and every request's result is identical alone and in a
concurrent mix."""
import sys
import threading

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
    for name, a, b in zip(("tc", "t0", "t1", "ig"), got, ref):
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{tag}: {name} differs on {len(bad)} nets, first {bad[:6]}")


def edited_arcs(arcs, edits):
    a = {k: v.copy() for k, v in arcs.items()}
    for g, p, cp, cv, r, f, ie in edits:
        m = (a["gate"] == g) & (a["pin"] == p) & (a["cond_pin"] == cp) & (a["in_edge"] == ie)
        if cp >= 0:
            m &= a["cond_val"] == cv
        assert m.sum() == 1
        a["rise"][m] = r
        a["fall"][m] = f
    return a


def random_edits(rng, w, n):
    arcs = w["arcs"]
    idx = rng.choice(len(arcs["gate"]), size=n, replace=False)
    out = []
    for i in idx:
        r = max(1, int(round(arcs["rise"][i] * (1 + rng.uniform(-0.2, 0.2)))))
        f = max(1, int(round(arcs["fall"][i] * (1 + rng.uniform(-0.2, 0.2)))))
        out.append((int(arcs["gate"][i]), int(arcs["pin"][i]), int(arcs["cond_pin"][i]), int(arcs["cond_val"][i]), r, f,
                    int(arcs["in_edge"][i])))
    return out


@pytest.fixture(scope="module")
def served(G):
    # the second design has input-edge-qualified arcs, the third four- to six-pin cells and both
    works = [synth.small_random(600 + i, g, max(8, g // 50), lv, 400, 800, 0.2, 5, 80, cond_frac=0.1, wide=i == 2,
                                edge_frac=0.3 if i else 0.0)
             for i, (g, lv) in enumerate(((3000, 30), (1200, 20), (600, 12)))]
    sim = G.GateSim()
    sim.load_cells(synth.WIDE_PINS, synth.WIDE_TRUTH)
    ids = [sim.load_work(w, cells_loaded=True) for w in works]
    resident = [(d, s, 100, 150) for d, s in ids]
    sim.serve_start(resident, max_queue=1000)
    yield sim, works, ids, resident
    sim.serve_stop()
    sim.close()


def result_of(sim, t):
    r = sim.poll(t, wait=True)
    sim.release(t)
    assert r["status"] == 0, r.get("error")
    return r


def test_window_requests(served):
    sim, works, ids, _ = served
    rng = np.random.default_rng(1)
    reqs = []
    for k in range(12):
        i = int(rng.integers(len(works)))
        b = int(rng.integers(0, 350))
        e = int(rng.integers(b + 1, min(400, b + 120) + 1))
        reqs.append((i, b, e, sim.submit_window(*ids[i], b, e)))
    for i, b, e, t in reqs:
        r = result_of(sim, t)
        ref = oracle.simulate(works[i], b, e)
        same((r["tc"], r["t0"], r["t1"], r["ig"]), (ref["tc"], ref["t0"], ref["t1"], ref["ig"]), f"window {i} [{b},{e})")
        assert r["t_submit_ns"] <= r["t_admit_ns"] <= r["t_done_ns"]


def test_edit_requests(served):
    sim, works, ids, resident = served
    rng = np.random.default_rng(2)
    for k in range(8):
        i = k % len(works)
        edits = random_edits(rng, works[i], int(rng.integers(1, 30)))
        r = result_of(sim, sim.submit_edit(*ids[i], edits))
        w2 = dict(works[i], arcs=edited_arcs(works[i]["arcs"], edits))
        _, _, b, n = resident[i]
        ref = oracle.simulate(w2, b, b + n)
        same((r["tc"], r["t0"], r["t1"], r["ig"]), (ref["tc"], ref["t0"], ref["t1"], ref["ig"]), f"edit {k}")
        assert r["gate_cycles"] <= works[i]["netlist"]["n_gates"] * n


def test_alone_equals_mix(served):
    """Each request's result is the same when it runs alone and when it runs
    concurrently with others submitted from several threads; in the mixed
    phase requests are on the device together (a request is admitted before
    another one has finished)."""
    sim, works, ids, _ = served
    rng = np.random.default_rng(3)
    plan = []
    for k in range(24):
        i = int(rng.integers(len(works)))
        if k % 2:
            b = int(rng.integers(0, 300))
            plan.append(("w", i, (b, b + int(rng.integers(1, 100)))))
        else:
            plan.append(("e", i, random_edits(rng, works[i], int(rng.integers(1, 20)))))

    def submit(p):
        kind, i, arg = p
        return sim.submit_window(*ids[i], *arg) if kind == "w" else sim.submit_edit(*ids[i], arg)

    alone = []
    for p in plan:
        r = result_of(sim, submit(p))
        alone.append((r["tc"], r["t0"], r["t1"], r["ig"]))
    tickets = [None] * len(plan)

    def worker(lo):
        for j in range(lo, len(plan), 4):
            tickets[j] = submit(plan[j])

    ths = [threading.Thread(target=worker, args=(lo,)) for lo in range(4)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    spans = []
    for j, t in enumerate(tickets):
        r = result_of(sim, t)
        same((r["tc"], r["t0"], r["t1"], r["ig"]), alone[j], f"request {j}")
        spans.append((r["t_admit_ns"], r["t_done_ns"]))
    # pairs of requests whose [admit, done] intervals overlap: both were
    # admitted and neither had finished
    overlap = sum(1 for a in range(len(spans)) for b in range(a + 1, len(spans))
                  if spans[a][0] < spans[b][1] and spans[b][0] < spans[a][1])
    say("alone == mix: overlapping request pairs", overlap)
    assert overlap >= 4, spans


def test_bad_edit_is_rejected(served):
    sim, works, ids, _ = served
    a = works[0]["arcs"]
    i = int(np.nonzero(a["cond_pin"] < 0)[0][0])
    t = sim.submit_edit(*ids[0], [(int(a["gate"][i]), int(a["pin"][i]), 0 if a["pin"][i] else 1, 1, 5, 5)])
    r = sim.poll(t, wait=True)
    sim.release(t)
    assert r["status"] != 0
    # the first design has no input-edge-qualified records to edit
    t = sim.submit_edit(*ids[0], [(int(a["gate"][i]), int(a["pin"][i]), -1, 0, 5, 5, 1)])
    r = sim.poll(t, wait=True)
    sim.release(t)
    assert r["status"] != 0


def test_segment_view_served(G):
    """A continuous-segment view of a stimulus is served like any other:
    window and delay-edit requests on 5-cycle segments match the oracle's
    segment runs (the serving loop keeps the single-cycle staging cap, so
    long lanes take the spill path)."""
    S = 5
    w = synth.small_random(640, 900, 20, 15, 200, 300, 0.3, 3, 70, cond_frac=0.1, edge_frac=0.2)
    sim = G.GateSim()
    started = False
    try:
        d, s = sim.load_work(w)
        v = sim.segment_stimulus(s, S)
        sim.serve_start([(d, v, 0, 40)], max_queue=64)
        started = True
        say("segment view served")
        tw = sim.submit_window(d, v, 3, 29)
        edits = random_edits(np.random.default_rng(3), w, 12)
        te = sim.submit_edit(d, v, edits)
        r = result_of(sim, tw)
        ref = oracle.simulate(w, 3, 29, segment_cycles=S)
        same((r["tc"], r["t0"], r["t1"], r["ig"]), (ref["tc"], ref["t0"], ref["t1"], ref["ig"]), "segment window")
        r = result_of(sim, te)
        ref = oracle.simulate(dict(w, arcs=edited_arcs(w["arcs"], edits)), 0, 40, segment_cycles=S)
        same((r["tc"], r["t0"], r["t1"], r["ig"]), (ref["tc"], ref["t0"], ref["t1"], ref["ig"]), "segment edit")
    finally:
        if started:
            sim.serve_stop()
        sim.close()
