"""The allocation-free entry point against gs_simulate, bit-exact.

gs_simulate_noalloc takes every per-call device buffer from a static scratch
array per GPU.  Its SAIF counts must equal gs_simulate's on the same inputs:
on two calls in a row (the second on a smaller design, so that it runs over
what the first left in the scratch), on a design whose windows the scratch
splits, and when regular calls come before and after it on one context.  A
design whose 64-cycle window cannot fit is rejected before any launch.
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


def run(G, w, noalloc, b=0, e=None, **opt):
    e = w["stimulus"]["n_cycles"] if e is None else e
    with G.GateSim(**opt) as sim:
        d, s = sim.load_work(w)
        (sim.simulate_noalloc if noalloc else sim.simulate)(d, s, b, e)
        return sim.read_saif_ig(d)


def same(a, b, tag):
    for name, x, y in zip(("tc", "t0", "t1", "ig"), a, b):
        if not np.array_equal(x, y):
            bad = np.nonzero(x != y)[0]
            raise AssertionError(f"{tag}: {name} differs on {len(bad)} nets, first {bad[:8]}")


def test_two_calls_second_smaller(G):
    big = synth.small_random(501, 3000, 60, 30, 700, 700, 0.3, 3, 60, cond_frac=0.2, wire=(1, 12),
                             extra=1, extra_p=0.3, edge_frac=0.2)
    small = synth.small_random(502, 300, 16, 12, 150, 400, 0.3, 3, 40, cond_frac=0.2)
    for tag, w in (("first, 3000 gates", big), ("second, 300 gates", small)):
        say("noalloc", tag)
        got = run(G, w, True)
        want = run(G, w, False)
        same(got, want, tag)
        ref = oracle.simulate(w)
        same(got, (ref["tc"], ref["t0"], ref["t1"], ref["ig"]), tag + " vs oracle")


def test_windows_split_by_scratch(G):
    # 60,000 gates: a 64-cycle window's headers take 8.6 MB, so the scratch
    # runs the 600 cycles as several windows
    w = synth.small_random(503, 60000, 600, 40, 600, 800, 0.2, 5, 60, cond_frac=0.1)
    say("noalloc: windows split by the scratch")
    same(run(G, w, True), run(G, w, False), "split windows")


def test_between_regular_calls(G):
    w = synth.small_random(504, 1200, 30, 20, 400, 600, 0.3, 3, 50, cond_frac=0.2, extra=1, extra_p=0.2)
    ref = oracle.simulate(w)
    refs = (ref["tc"], ref["t0"], ref["t1"], ref["ig"])
    with G.GateSim() as sim:
        d, s = sim.load_work(w)
        say("regular, then noalloc, then regular on one context")
        sim.simulate(d, s, 0, 400)
        same(sim.read_saif_ig(d, reset=True), refs, "regular before")
        sim.simulate_noalloc(d, s, 0, 400)
        same(sim.read_saif_ig(d, reset=True), refs, "noalloc")
        sim.simulate(d, s, 0, 250)
        sim.simulate_noalloc(d, s, 250, 400)
        same(sim.read_saif_ig(d, reset=True), refs, "split between the two calls")


def test_too_large_is_rejected(G):
    # 250,000 nets: one 64-cycle window needs 36 MB of headers and lane ends,
    # more than half of the scratch
    w = synth.small_random(505, 249000, 1000, 20, 64, 800, 0.2, 5, 60)
    with G.GateSim() as sim:
        d, s = sim.load_work(w)
        with pytest.raises(G.GateSimError) as ei:
            sim.simulate_noalloc(d, s, 0, 64)
        assert ei.value.status == G.GS_E_NOMEM
        assert "static scratch" in str(ei.value)
        sim.simulate(d, s, 0, 64)                 # the context still works
