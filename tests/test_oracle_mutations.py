"""Strength of the oracle's pins: deliberately broken copies of oracle.c.

Each mutant below breaks one rule of the oracle in one place (a tie, a
threshold, a delay choice, the same-time order, the settled start, SDF
precedence, SAIF clipping, the glitch and late counts).  The mutant is
compiled to its own library and the oracle's CPU pin and brute-force tests
are run against it in a separate process; every mutant must make at least
one of them fail.  The unmodified source runs through the same harness as
the control and must pass.  CPU only.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, text in oracle.c, replacement)
MUTANTS = [
    ("msi-largest-delay", "if (dl < 0 || x < dl) dl = x;", "if (dl < 0 || x > dl) dl = x;"),
    ("msi-pre-switch-state", "int64_t x = d->dtab[d->dtab_ptr[s] + 2 * st + y];",
     "int64_t x = d->dtab[d->dtab_ptr[s] + 2 * (st ^ sw_mask[g]) + y];"),
    ("output-edge-delays-swapped", "d->dtab[base + 2 * st + 0] = arc_fall[a];",
     "d->dtab[base + 2 * st + 0] = arc_rise[a];"),
    ("same-time-order-reversed", "return a->kind < b->kind;", "return a->kind > b->kind;"),
    ("t0-t1-not-clipped", "int64_t lo = prev < T ? prev : T, hi = end < T ? end : T;",
     "int64_t lo = prev, hi = end;"),
    ("wire-filter-off", "(net_filter ? ev.t < arc_pend_t[s] :", "(net_filter ? 0 :"),
    ("wire-filter-tie-cancels", "(net_filter ? ev.t < arc_pend_t[s] :", "(net_filter ? ev.t <= arc_pend_t[s] :"),
    ("transport-tie-keeps", "ev.t + delta <= arc_pend_t[s])", "ev.t + delta < arc_pend_t[s])"),
    ("wire-delay-direction-swapped", "int64_t delta = v ? d->wire_r[s] : d->wire_f[s];",
     "int64_t delta = v ? d->wire_f[s] : d->wire_r[s];"),
    ("gate-filter-off", "int32_t z = pending ? (cur ^ 1) : cur;", "int32_t z = cur;"),
    ("settle-skipped", "net_val[I + g] = (int32_t)((d->truth[g] >> st) & 1);", "net_val[I + g] = 0;"),
    ("input-start-parity-ignored", "net_val[i] = (init[i] ^ (int32_t)((tcur[i] - toggle_ptr[i]) & 1)) & 1;",
     "net_val[i] = init[i] & 1;"),
    ("specificity-ignored", "if (filled[base + 2 * st] > pass + 1) continue;   /* a more specific record holds it */",
     ""),
    ("input-edge-qualifier-inverted", "if (edge == 1 && !((st >> j) & 1)) continue;",
     "if (edge == 1 && ((st >> j) & 1)) continue;"),
    ("glitch-count-without-parity", "if (ig) ig[n] += (b - a) - ((b - a) & 1);", "if (ig) ig[n] += (b - a);"),
    ("glitch-profile-shifted", "if (ig_cycle) ig_cycle[c - cycle_begin] +=", "if (ig_cycle) ig_cycle[c - cycle_begin + 1] +="),
    ("late-threshold-strict", "if (reach >= T) late_cycle[c - cycle_begin]++;",
     "if (reach > T) late_cycle[c - cycle_begin]++;"),
    ("late-ignores-wires", "int64_t r = last + (v_end ? d->wire_r[s] : d->wire_f[s]);", "int64_t r = last;"),
]

TESTS = ["tests/test_oracle_pins.py", "tests/test_oracle_brute.py"]


def _run(name, text, tmp):
    src = open(SRC).read()
    if text is not None:
        assert src.count(text[0]) == 1, f"{name}: the mutated text must occur exactly once"
        src = src.replace(text[0], text[1])
    path = os.path.join(tmp, name + ".c")
    with open(path, "w") as f:
        f.write(src)
    lib = oracle.compile_oracle(path, os.path.join(tmp, name + ".so"))
    env = dict(os.environ, GATESIM_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] + TESTS,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    return name, r.returncode, r.stdout[-2000:]


def test_every_mutant_is_caught(tmp_path):
    jobs = [("control", None)] + [(n, (a, b)) for n, a, b in MUTANTS]
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda j: _run(j[0], j[1], str(tmp_path)), jobs))
    control = results[0]
    assert control[1] == 0, "the unmodified oracle fails its own pins:\n" + control[2]
    survivors = [n for n, rc, _ in results[1:] if rc == 0]
    assert not survivors, f"mutants no pin rejects: {survivors}"
    # a failure must come from an assertion or the oracle's own
    # consistency check, not from a crash of the test process
    crashed = [n for n, rc, _ in results[1:] if rc not in (1,)]
    assert not crashed, f"mutants that crashed instead of failing a test: {crashed}"
