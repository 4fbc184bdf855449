"""Seeded synthetic workloads: netlists, delay arcs and stimuli.

This module only draws inputs.  It holds none of the simulation method's
arithmetic and is shared, unchanged, by the CPU oracle harness and by the HIP
path's harness so both sides see byte-identical arrays.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  Output i of a SplitMix64
stream seeded with s is mix(s + (i + 1) * gamma), so the stream is used with
random access: every purpose gets its own stream seed and every draw is
addressed by an integer counter.  That keeps generation vectorised in numpy and
independent of evaluation order.

Workload shapes follow the paper's benchmark range (gate counts from 1k to
about 2.3M, activity from sparse functional tests to scan, Section 4, Table 2)
with the cell mix, levels, delays and toggle rates of the configurations this
library is measured on; the paper's own netlists are not available, so these
synthetic designs stand in for them.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def _seed_of(seed: int, tag: str) -> np.uint64:
    h = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    for ch in tag.encode():
        with np.errstate(over="ignore"):
            h = _mix(np.array([h ^ np.uint64(ch)], dtype=np.uint64))[0] + _GAMMA
    return np.uint64(h)


class Stream:
    """Random-access SplitMix64 stream for one purpose of one workload."""

    def __init__(self, seed: int, tag: str):
        self.base = _seed_of(seed, tag)

    def u64(self, idx) -> np.ndarray:
        idx = np.asarray(idx, dtype=np.uint64)
        with np.errstate(over="ignore"):
            return _mix(self.base + (idx + np.uint64(1)) * _GAMMA)

    def below(self, idx, n) -> np.ndarray:
        """Integers in [0, n) (n may be an array, each < 2**32)."""
        hi = self.u64(idx) >> np.uint64(32)
        return ((hi * np.asarray(n, dtype=np.uint64)) >> np.uint64(32)).astype(np.int64)

    def unit(self, idx) -> np.ndarray:
        """Floats in [0, 1) with 53 random bits."""
        return (self.u64(idx) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# ---------------------------------------------------------------------------
# Cell library: the eight cell types of the measured configurations.
# Truth bit b is the output for input index b, pin 0 being the least
# significant bit of b.
# ---------------------------------------------------------------------------
CELL_NAMES = ["INV", "BUF", "NAND2", "NOR2", "AND3", "XOR2", "AOI21", "MUX2"]
CELL_PINS = np.array([1, 1, 2, 2, 3, 2, 3, 3], dtype=np.uint8)
CELL_TRUTH = np.array([0x1, 0x2, 0x7, 0x1, 0x80, 0x6, 0x07, 0xCA], dtype=np.uint64)
INV, BUF, NAND2, NOR2, AND3, XOR2, AOI21, MUX2 = range(8)


def _truth(k: int, f) -> int:
    """Truth bits of a k-pin cell: bit s is f(pin values), pin j = bit j of s."""
    return sum(1 << s for s in range(1 << k) if f(*[(s >> j) & 1 for j in range(k)]))


# The base library plus cells of four to six pins (same indices for the base
# cells), for netlists that exercise wide gates.
WIDE_NAMES = CELL_NAMES + ["AND4", "OAI22", "AOI221", "AOI222"]
WIDE_PINS = np.append(CELL_PINS, np.array([4, 4, 5, 6], dtype=np.uint8)).astype(np.uint8)
WIDE_TRUTH = np.append(CELL_TRUTH, np.array([
    _truth(4, lambda a, b, c, d: a & b & c & d),
    _truth(4, lambda a, b, c, d: 1 - ((a | b) & (c | d))),
    _truth(5, lambda a, b, c, d, e: 1 - ((a & b) | (c & d) | e)),
    _truth(6, lambda a, b, c, d, e, f: 1 - ((a & b) | (c & d) | (e & f))),
], dtype=np.uint64)).astype(np.uint64)


def make_netlist(seed: int, n_gates: int, n_inputs: int, n_levels: int,
                 cell_probs=None, fanout_mean: float = 2.5,
                 arith_frac: float = 0.0, shuffle: bool = True, wide: bool = False) -> dict:
    """Random levelized DAG.

    Gates are split evenly over ``n_levels`` levels.  Pin 0 of a level-l gate
    is drawn from the nets of level l-1 (inputs are level 0), which fixes the
    gate's level; the other pins are drawn from all nets of levels < l.  Each
    net carries a geometric fanout budget (support >= 1, mean
    ``fanout_mean``) and nets are drawn with probability proportional to it.
    A gate's fanin nets are distinct.  With ``arith_frac`` > 0 that fraction
    of the gates is instead laid out as ripple-carry adder slices (XOR2 sum,
    MUX2 carry select, AND3/AOI21 side logic) chained across consecutive
    levels, giving deep reconvergent XOR/MUX cones.  Gate ids are a random
    permutation of the level order unless ``shuffle`` is False.  ``wide``
    draws cells from the library with four- to six-pin cells as well.
    """
    G, I, L = int(n_gates), int(n_inputs), int(n_levels)
    if G < L or L < 1 or I < 3:
        raise ValueError("need n_gates >= n_levels >= 1 and n_inputs >= 3")
    s_cell = Stream(seed, "cell")
    s_budget = Stream(seed, "budget")
    s_pick = Stream(seed, "pick")
    s_perm = Stream(seed, "perm")

    per = np.full(L, G // L, dtype=np.int64)
    per[: G % L] += 1
    lvl_start = np.concatenate([[0], np.cumsum(per)])           # level-order gate index range per level
    level_of_q = np.repeat(np.arange(1, L + 1, dtype=np.int64), per)

    lib_pins, lib_truth = (WIDE_PINS, WIDE_TRUTH) if wide else (CELL_PINS, CELL_TRUTH)
    n_cells = len(lib_pins)
    q = np.arange(G, dtype=np.int64)
    if cell_probs is None:
        cell = s_cell.below(q, n_cells).astype(np.int32)
    else:
        cp = np.cumsum(np.asarray(cell_probs, dtype=np.float64))
        cp /= cp[-1]
        cell = np.searchsorted(cp, s_cell.unit(q), side="right").astype(np.int32)
        cell = np.minimum(cell, n_cells - 1)

    # arithmetic-like chains: overwrite the cell of a fraction of gates so
    # that chains of (XOR2 sum, MUX2 carry) pairs walk up consecutive levels
    arith = np.zeros(G, dtype=bool)
    if arith_frac > 0.0:
        a = s_cell.unit(q + np.int64(G)) < arith_frac
        arith = a
        pat = np.array([XOR2, MUX2, XOR2, MUX2, AND3, XOR2, AOI21, MUX2], dtype=np.int32)
        cell = np.where(arith, pat[(q % 8)], cell)

    k = lib_pins[cell].astype(np.int64)

    n_nets = I + G
    m = np.arange(n_nets, dtype=np.int64)
    u = s_budget.unit(m)
    p = 1.0 / fanout_mean
    budget = 1 + np.floor(np.log1p(-u) / np.log1p(-p)).astype(np.int64)
    cum = np.cumsum(budget)                                        # over level-order nets

    # level-order net index range of each level (level 0 = inputs)
    net_lo = np.concatenate([[0], I + lvl_start[:-1]])              # indexed by level 0..L-1
    net_hi = np.concatenate([[I], I + lvl_start[1:]])

    def draw(lo_net, hi_net, ctr):
        lo_c = np.where(lo_net > 0, cum[np.maximum(lo_net - 1, 0)], 0)
        hi_c = cum[hi_net - 1]
        r = lo_c + (s_pick.unit(ctr) * (hi_c - lo_c)).astype(np.int64)
        r = np.minimum(r, hi_c - 1)
        return np.searchsorted(cum, r, side="right")

    maxk = 3 if k.max() <= 3 else int(k.max())
    fan = np.full((G, maxk), -1, dtype=np.int64)
    lv = level_of_q
    fan[:, 0] = draw(net_lo[lv - 1], net_hi[lv - 1], q * 1024)
    # arithmetic chains take their side inputs from the previous two levels,
    # which keeps the reconvergence local and the cones deep
    side_lo = np.where(arith, net_lo[np.maximum(lv - 2, 0)], 0)
    for j in range(1, maxk):
        has = k > j
        fan[has, j] = draw(side_lo[has], net_hi[lv[has] - 1], q[has] * 1024 + j)
    for rnd in range(1, 64):
        bad = np.zeros(G, dtype=bool)
        for j in range(1, maxk):
            for i in range(j):
                bad_j = (k > j) & (fan[:, j] == fan[:, i])
                if bad_j.any():
                    idx = np.nonzero(bad_j)[0]
                    fan[idx, j] = draw(np.where(arith[idx], side_lo[idx], 0),
                                       net_hi[lv[idx] - 1], idx * 1024 + j + 8 * rnd)
                    bad |= bad_j
        if not bad.any():
            break
    else:
        raise RuntimeError("could not draw distinct fanins")

    if shuffle:
        perm = np.argsort(s_perm.u64(q), kind="stable")             # level-order q -> gate id
        gate_of_q = np.empty(G, dtype=np.int64)
        gate_of_q[perm] = q
    else:
        gate_of_q = q.copy()
    net_of_m = np.concatenate([np.arange(I, dtype=np.int64), I + gate_of_q])

    order = np.argsort(gate_of_q, kind="stable")                    # gate id -> level-order q
    kk = k[order]
    fanin_ptr = np.zeros(G + 1, dtype=np.int64)
    fanin_ptr[1:] = np.cumsum(kk)
    ff = fan[order]
    sel = np.arange(maxk)[None, :] < kk[:, None]
    fanin_net = net_of_m[ff[sel]].astype(np.int32)
    return {
        "n_inputs": I,
        "n_gates": G,
        "cell_of_gate": cell[order].astype(np.int32),
        "fanin_ptr": fanin_ptr,
        "fanin_net": fanin_net,
        "level_hint": level_of_q[order].astype(np.int32),
        "cell_pins": lib_pins.copy(),
        "cell_truth": lib_truth.copy(),
    }


def make_arcs(seed: int, net: dict, lo: int, hi: int, cond_frac: float = 0.0, edge_frac: float = 0.0) -> dict:
    """Per-(gate, pin) rise/fall delays, i.i.d. U{lo..hi} picoseconds.

    ``cond_frac`` of all gates (drawn among cells with at least two pins)
    carry SDF-style conditional delays: one pin's arc is replaced by two
    records keyed on one other pin of the same gate (value 0 and value 1),
    each with its own rise/fall pair.

    ``edge_frac`` of all fanin slots get input-edge-qualified records
    (``in_edge`` 1: rising input, 2: falling input), mixed three ways: an
    unconditional slot either splits its record into a rising- and a
    falling-input record, or keeps it and gains one record for one input
    edge that overrides it there; a conditional slot gains one record with
    both its condition (one value) and an input edge.
    """
    G = net["n_gates"]
    fp = net["fanin_ptr"]
    k = np.diff(fp)
    s = Stream(seed, "arcs")
    g = np.arange(G, dtype=np.int64)
    multi = k >= 2
    frac_multi = max(multi.mean(), 1e-12)
    has_cond = multi & (s.unit(g * 8 + 7) < min(1.0, cond_frac / frac_multi))
    cpin = np.where(has_cond, s.below(g * 8 + 6, np.maximum(k, 1)), -1)
    qraw = s.below(g * 8 + 5, np.maximum(k - 1, 1))
    qpin = np.where(has_cond, qraw + (qraw >= cpin), -1)

    slot_gate = np.repeat(g, k)
    slot_pin = np.arange(fp[-1], dtype=np.int64) - fp[slot_gate]
    slot_is_cond = slot_pin == cpin[slot_gate]
    n_slots = int(fp[-1])
    sl = np.arange(n_slots, dtype=np.int64)
    span = hi - lo + 1
    r0 = lo + s.below(sl * 4 + 0 + 1_000_000_000_000, span)
    f0 = lo + s.below(sl * 4 + 1 + 1_000_000_000_000, span)
    r1 = lo + s.below(sl * 4 + 2 + 1_000_000_000_000, span)
    f1 = lo + s.below(sl * 4 + 3 + 1_000_000_000_000, span)

    uncond = ~slot_is_cond
    cond_idx = np.nonzero(slot_is_cond)[0]
    n_arcs = int(uncond.sum()) + 2 * len(cond_idx)
    gate = np.empty(n_arcs, dtype=np.int32)
    pin = np.empty(n_arcs, dtype=np.int8)
    cp = np.empty(n_arcs, dtype=np.int8)
    cv = np.empty(n_arcs, dtype=np.int8)
    rise = np.empty(n_arcs, dtype=np.int32)
    fall = np.empty(n_arcs, dtype=np.int32)
    nu = int(uncond.sum())
    gate[:nu] = slot_gate[uncond]
    pin[:nu] = slot_pin[uncond]
    cp[:nu] = -1
    cv[:nu] = 0
    rise[:nu] = r0[uncond]
    fall[:nu] = f0[uncond]
    for half, (rr, ff, val) in enumerate(((r0, f0, 0), (r1, f1, 1))):
        a = nu + half * len(cond_idx)
        b = a + len(cond_idx)
        gate[a:b] = slot_gate[cond_idx]
        pin[a:b] = slot_pin[cond_idx]
        cp[a:b] = qpin[slot_gate[cond_idx]]
        cv[a:b] = val
        rise[a:b] = rr[cond_idx]
        fall[a:b] = ff[cond_idx]
    in_edge = np.zeros(n_arcs, dtype=np.int8)
    if edge_frac > 0:
        e0 = 3_000_000_000_000
        sel = s.unit(sl * 4 + e0) < edge_frac
        split = (s.below(sl * 4 + 1 + e0, 2) == 0) & uncond
        which = 1 + s.below(sl * 4 + 2 + e0, 2)
        val = s.below(sl * 4 + 3 + e0, 2)
        xr = lo + s.below(sl * 4 + 0 + 2 * e0, span)
        xf = lo + s.below(sl * 4 + 1 + 2 * e0, span)
        rec_of_slot = np.cumsum(uncond) - 1         # unconditional record of each unconditional slot
        in_edge[rec_of_slot[sel & split]] = 1
        add = np.nonzero(sel)[0]
        gate = np.concatenate([gate, slot_gate[add].astype(np.int32)])
        pin = np.concatenate([pin, slot_pin[add].astype(np.int8)])
        cp = np.concatenate([cp, np.where(slot_is_cond[add], qpin[slot_gate[add]], -1).astype(np.int8)])
        cv = np.concatenate([cv, np.where(slot_is_cond[add], val[add], 0).astype(np.int8)])
        in_edge = np.concatenate([in_edge, np.where(split[add], 2, which[add]).astype(np.int8)])
        rise = np.concatenate([rise, xr[add].astype(np.int32)])
        fall = np.concatenate([fall, xf[add].astype(np.int32)])
    return {"gate": gate, "pin": pin, "cond_pin": cp, "cond_val": cv, "in_edge": in_edge,
            "rise": rise, "fall": fall}


def make_wires(seed: int, net: dict, lo: int, hi: int) -> dict:
    """Per-fanin-slot interconnect rise/fall delays, i.i.d. U{lo..hi}."""
    n = int(net["fanin_ptr"][-1])
    s = Stream(seed, "wires")
    i = np.arange(n, dtype=np.int64)
    span = hi - lo + 1
    return {"rise": (lo + s.below(2 * i, span)).astype(np.int32),
            "fall": (lo + s.below(2 * i + 1, span)).astype(np.int32)}


def make_stimulus(seed: int, n_inputs: int, n_cycles: int, period: int, p: float,
                  skew: int = 50, extra: int = 0, extra_p: float = 0.0,
                  chunk: int = 512) -> dict:
    """Clocked input waveforms (absolute picoseconds).

    Each input starts at a Bernoulli(0.5) value.  In every cycle it toggles
    with probability ``p`` at c*period + U{0..skew}.  For test workloads,
    ``extra`` further candidate toggles per (input, cycle), each present with
    probability ``extra_p`` at c*period + U{0..period-1}, give multi-edge
    and glitchy inputs; coinciding times are merged.
    """
    I, C, T = int(n_inputs), int(n_cycles), int(period)
    if not (0 <= skew < T):
        raise ValueError("skew must lie in [0, period)")
    s_init = Stream(seed, "init")
    s_tog = Stream(seed, "toggle")
    s_skew = Stream(seed, "skew")
    s_ex = Stream(seed, "extra")
    init = (s_init.below(np.arange(I), 2)).astype(np.uint8)
    counts = np.zeros(I, dtype=np.int64)
    parts = []
    nslot = 1 + extra
    for i0 in range(0, I, chunk):
        i1 = min(I, i0 + chunk)
        ii = np.arange(i0, i1, dtype=np.int64)[:, None]
        cc = np.arange(C, dtype=np.int64)[None, :]
        ctr = ii * C + cc
        base = (cc * T).astype(np.int64)
        tog = s_tog.unit(ctr) < p
        t0 = np.where(tog, base + s_skew.below(ctr, skew + 1), -1)
        if extra == 0:
            times = t0[:, :, None]
        else:
            cols = [t0]
            for e in range(extra):
                ce = ctr * extra + e
                pres = s_ex.unit(ce) < extra_p
                cols.append(np.where(pres, base + s_ex.below(ce + (1 << 40), T), -1))
            times = np.stack(cols, axis=2)
            times.sort(axis=2)
            dup = np.zeros_like(times, dtype=bool)
            dup[:, :, 1:] = times[:, :, 1:] == times[:, :, :-1]
            times = np.where(dup, -1, times)
            times.sort(axis=2)
        flat = times.reshape(i1 - i0, C * nslot)
        valid = flat >= 0
        counts[i0:i1] = valid.sum(axis=1)
        parts.append(flat[valid])                                    # row-major: input, then time
    toggle_ptr = np.zeros(I + 1, dtype=np.int64)
    toggle_ptr[1:] = np.cumsum(counts)
    toggle_ps = np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64)
    return {"period": T, "n_cycles": C, "init": init,
            "toggle_ptr": toggle_ptr, "toggle_ps": toggle_ps.astype(np.int64)}


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------
def tiny(seed: int = 1) -> dict:
    """2,000 gates, 64 inputs, 24 levels, delays U{5..60}, 100 cycles of 1000 ps, p = 0.2."""
    net = make_netlist(seed, 2000, 64, 24)
    return {"name": "tiny-2k", "netlist": net, "arcs": make_arcs(seed, net, 5, 60, 0.0),
            "wires": None, "stimulus": make_stimulus(seed, 64, 100, 1000, 0.2, skew=50)}


def scale(seed: int = 2, n_cycles: int = 10_000) -> dict:
    """1,000,000 gates, 20,000 inputs, 120 levels, delays U{5..80}, 10% COND cells,
    cycles of 800 ps with input toggle probability 0.15."""
    net = make_netlist(seed, 1_000_000, 20_000, 120)
    return {"name": "scale-1M", "netlist": net, "arcs": make_arcs(seed, net, 5, 80, 0.10),
            "wires": None, "stimulus": make_stimulus(seed, 20_000, n_cycles, 800, 0.15, skew=50)}


def glitchy(seed: int = 3, n_gates: int = 8_000_000, n_inputs: int = 150_000,
            n_levels: int = 200, n_cycles: int = 2000) -> dict:
    """Glitch-heavy large design: 30% of gates in ripple-carry-like XOR/MUX
    chains, delays U{3..120}, 10% COND cells, 1000 ps cycles, p = 0.3."""
    net = make_netlist(seed, n_gates, n_inputs, n_levels, arith_frac=0.30)
    return {"name": "glitchy", "netlist": net, "arcs": make_arcs(seed, net, 3, 120, 0.10),
            "wires": None, "stimulus": make_stimulus(seed, n_inputs, n_cycles, 1000, 0.3, skew=50)}


def small_random(seed: int, n_gates: int, n_inputs: int, n_levels: int, n_cycles: int,
                 period: int, p: float, dlo: int, dhi: int, cond_frac: float = 0.0,
                 wire: tuple | None = None, extra: int = 0, extra_p: float = 0.0,
                 skew: int = 50, wide: bool = False, edge_frac: float = 0.0) -> dict:
    """Parametric small workload used by parity and property tests."""
    net = make_netlist(seed, n_gates, n_inputs, n_levels, wide=wide)
    wires = make_wires(seed, net, wire[0], wire[1]) if wire else None
    return {"name": f"rand-{seed}", "netlist": net,
            "arcs": make_arcs(seed, net, dlo, dhi, cond_frac, edge_frac), "wires": wires,
            "stimulus": make_stimulus(seed, n_inputs, n_cycles, period, p, skew=skew,
                                      extra=extra, extra_p=extra_p)}


def batched(seed: int = 4, n: int = 64) -> list:
    """Uneven independent instances: gates log-uniform in [1e4, 5e5],
    inputs = gates / 50, levels 24 + 96 ln(G/1e4) / ln 50, cycles
    log-uniform in [200, 5000], toggle p uniform in [0.05, 0.3], delays
    5-80 ps with 10% COND cells, 800 ps cycles; instance i uses seed 400 + i."""
    s = Stream(seed, "batch-shapes")
    i = np.arange(n, dtype=np.int64)
    G = np.exp(np.log(1e4) + s.unit(4 * i) * (np.log(5e5) - np.log(1e4))).astype(np.int64)
    C = np.exp(np.log(200) + s.unit(4 * i + 1) * (np.log(5000) - np.log(200))).astype(np.int64)
    P = 0.05 + 0.25 * s.unit(4 * i + 2)
    out = []
    for k in range(n):
        g = int(G[k])
        L = int(round(24 + 96 * np.log(g / 1e4) / np.log(50)))
        net = make_netlist(400 + k, g, max(3, g // 50), L)
        out.append({"name": f"batch-{k}", "netlist": net, "arcs": make_arcs(400 + k, net, 5, 80, 0.10),
                    "wires": None,
                    "stimulus": make_stimulus(400 + k, max(3, g // 50), int(C[k]), 800, float(P[k]), skew=50)})
    return out


def served_designs(seed: int = 5, scale_cycles: int = 4000, small_cycles: int = 2500) -> list:
    """The 1M-gate design plus eight designs of 5e4-2e5 gates (log-uniform,
    seeds 501..508) with delays 5-80 ps and 10% COND cells, 800 ps cycles,
    toggle probability 0.15."""
    s = Stream(seed, "served-shapes")
    out = [scale(2, n_cycles=scale_cycles)]
    for k in range(8):
        g = int(np.exp(np.log(5e4) + float(s.unit(np.array([k]))[0]) * (np.log(2e5) - np.log(5e4))))
        L = int(round(24 + 96 * np.log(g / 1e4) / np.log(50)))
        net = make_netlist(501 + k, g, max(3, g // 50), L)
        out.append({"name": f"served-{k}", "netlist": net, "arcs": make_arcs(501 + k, net, 5, 80, 0.10),
                    "wires": None,
                    "stimulus": make_stimulus(501 + k, max(3, g // 50), small_cycles, 800, 0.15, skew=50)})
    return out
