"""Brute-force checker for the oracle — TEST INFRASTRUCTURE ONLY.

A second, independently written model of the same semantics, used only on
tiny netlists.  Where ``oracle.c`` is an event queue over the whole netlist,
this module works gate by gate on a 1 ps time grid, the way GATSPI's
Algorithm 1 walks one gate's input waveforms:

1. Each net's waveform in one cycle is a list of 0/1 samples at
   t = -1, 0, 1, ..., H (t = -1 holds the value before the cycle's first
   event, i.e. the zero-delay settled value).
2. A fanin arc turns the driving net's change list into the pin's change
   list with the interconnect inertial rule of Algorithm 1: walking the
   net's changes in order, a change at e_k followed by one at e_(k+1) with
   e_(k+1) - e_k < delta(e_k) drops both; otherwise the pin changes at
   e_k + delta(e_k), delta chosen by the value the net changes to.  With
   ``net_filter`` False in the work dict (the feature study's wire delays
   without that filter) every change arrives at e_k + delta(e_k), kept on a
   stack: an arrival no later than the stack's top cancels it and is itself
   dropped (a pulse of non-positive delayed width).
3. The gate's zero-delay response y(t) = truth[pins(t)] is sampled at every
   picosecond.  At each t where y changes, the pins that switched at t give
   the arc delay: the smallest over those pins of the arc's delay for the new
   output edge, looked up in the pin state at t (SDF conditional records
   take precedence over unconditional ones).
4. Algorithm 1's output filter (PATHPULSEPERCENT = 100): walking y's
   changes, a change at u while the previously scheduled output edge W is
   still ahead (u < W) cancels that edge and schedules nothing; otherwise an
   edge is scheduled at u + delay.

Cycles are independent: inputs hold their pre-cycle values at t = -1 and
toggle at their cycle-local times.  Gates are processed in topological
order.  Pure Python loops; for netlists of a few gates and short horizons.
"""
from __future__ import annotations


def _levels(n_inputs, n_gates, fanin_ptr, fanin_net):
    lvl = [0] * n_inputs + [None] * n_gates
    changed = True
    while changed:
        changed = False
        for g in range(n_gates):
            if lvl[n_inputs + g] is not None:
                continue
            ins = [lvl[fanin_net[s]] for s in range(fanin_ptr[g], fanin_ptr[g + 1])]
            if all(x is not None for x in ins):
                lvl[n_inputs + g] = 1 + max(ins) if ins else 1
                changed = True
    if any(x is None for x in lvl):
        raise ValueError("combinational cycle")
    return lvl


def _arc_delay(arcs_of_pin, pin, state, rising):
    # records are (cond_pin, cond_val, in_edge, rise, fall); the pin's own bit
    # in the post-switch state tells whether its input edge was a rise
    in_rise = (state >> pin) & 1
    ok = []
    for cp, cv, ie, r, f in arcs_of_pin:
        if cp >= 0 and ((state >> cp) & 1) != cv:
            continue
        if (ie == 1 and not in_rise) or (ie == 2 and in_rise):
            continue
        ok.append(((cp >= 0) + (ie != 0), r, f))
    top = max((x[0] for x in ok), default=-1)
    pick = [x for x in ok if x[0] == top]
    if len(pick) != 1:
        raise ValueError("arc records do not select exactly one delay")
    return pick[0][1] if rising else pick[0][2]


def _changes(samples):
    """Times t >= 0 where samples (indexed t+1) differ from the previous sample."""
    return [t for t in range(0, len(samples) - 1) if samples[t + 1] != samples[t]]


def _samples(v0, change_times, H):
    out = []
    v = v0
    ch = set(change_times)
    out.append(v0)                       # t = -1
    for t in range(0, H + 1):
        if t in ch:
            v ^= 1
        out.append(v)
    return out


def _wire(net_samples, dr, df, H, net_filter=True):
    v0 = net_samples[0]
    e = _changes(net_samples)
    if not net_filter:
        # transport delay: every change arrives at e + delta; a pulse whose
        # delayed end is no later than its delayed start vanishes, which may
        # expose an older arrival to the next change
        out = []
        for t in e:
            a = t + (dr if net_samples[t + 1] else df)
            if out and out[-1] >= a:
                out.pop()
            else:
                out.append(a)
        return _samples(v0, out, H)
    out = []
    k = 0
    while k < len(e):
        val_after = net_samples[e[k] + 1]
        d = dr if val_after else df
        if k + 1 < len(e) and e[k + 1] - e[k] < d:
            k += 2
            continue
        out.append(e[k] + d)
        k += 1
    return _samples(v0, out, H)


def simulate(work: dict, cycle_begin: int = 0, cycle_end: int | None = None, horizon: int | None = None,
             segment_cycles: int = 1):
    """Returns (tc, t0, t1, waves) with waves[(net, cycle)] = (init, [times]).

    segment_cycles S: every S cycles form one interval simulated from its
    settled start (cycles and times in the results then count intervals)."""
    net = work["netlist"]
    arcs = work["arcs"]
    wires = work.get("wires")
    stim = work["stimulus"]
    if segment_cycles > 1:
        assert int(stim["n_cycles"]) % segment_cycles == 0
        stim = dict(stim, period=int(stim["period"]) * segment_cycles,
                    n_cycles=int(stim["n_cycles"]) // segment_cycles)
    I, G = int(net["n_inputs"]), int(net["n_gates"])
    fp = [int(x) for x in net["fanin_ptr"]]
    fn = [int(x) for x in net["fanin_net"]]
    cell = [int(x) for x in net["cell_of_gate"]]
    truth = [int(x) for x in net["cell_truth"]]
    T = int(stim["period"])
    C = int(stim["n_cycles"]) if cycle_end is None else cycle_end
    lvl = _levels(I, G, fp, fn)
    order = sorted(range(G), key=lambda g: lvl[I + g])
    by_pin = {}
    for a in range(len(arcs["gate"])):
        key = (int(arcs["gate"][a]), int(arcs["pin"][a]))
        ie = int(arcs["in_edge"][a]) if "in_edge" in arcs else 0
        by_pin.setdefault(key, []).append((int(arcs["cond_pin"][a]), int(arcs["cond_val"][a]), ie,
                                           int(arcs["rise"][a]), int(arcs["fall"][a])))
    wr = [int(x) for x in wires["rise"]] if wires is not None else [0] * fp[-1]
    wf = [int(x) for x in wires["fall"]] if wires is not None else [0] * fp[-1]
    dmax = max([max(int(r), int(f)) for r, f in zip(arcs["rise"], arcs["fall"])] + [0])
    wmax = max(wr + wf + [0])
    L = max(lvl)
    H = horizon if horizon is not None else T + (L + 1) * (dmax + wmax) + 2

    N = I + G
    tc = [0] * N
    t0 = [0] * N
    t1 = [0] * N
    waves = {}
    tp = [int(x) for x in stim["toggle_ptr"]]
    ts = [int(x) for x in stim["toggle_ps"]]
    for c in range(cycle_begin, C):
        S = [None] * N
        for i in range(I):
            before = sum(1 for k in range(tp[i], tp[i + 1]) if ts[k] < c * T)
            v0 = (int(stim["init"][i]) + before) & 1
            loc = [ts[k] - c * T for k in range(tp[i], tp[i + 1]) if c * T <= ts[k] < (c + 1) * T]
            S[i] = _samples(v0, loc, H)
        for g in order:
            k = fp[g + 1] - fp[g]
            pins = [_wire(S[fn[s]], wr[s], wf[s], H, work.get("net_filter", True)) for s in range(fp[g], fp[g + 1])]
            def state(ix):
                return sum(pins[j][ix] << j for j in range(k))
            y = [(truth[cell[g]] >> state(ix)) & 1 for ix in range(H + 2)]
            sched = []          # scheduled, not cancelled output edges
            for u in _changes(y):
                if sched and u < sched[-1]:
                    sched.pop()
                    continue
                st = state(u + 1)
                sw = [j for j in range(k) if pins[j][u + 1] != pins[j][u]]
                d = min(_arc_delay(by_pin[(g, j)], j, st, y[u + 1] == 1) for j in sw)
                sched.append(u + d)
            if sched and sched[-1] > H:
                raise ValueError("horizon too short")
            S[I + g] = _samples(y[0], sched, H)
        for n in range(N):
            ch = _changes(S[n])
            tc[n] += len(ch)
            t1[n] += sum(S[n][t + 1] for t in range(0, T))
            t0[n] += sum(1 - S[n][t + 1] for t in range(0, T))
            waves[(n, c)] = (S[n][0], ch)
    return tc, t0, t1, waves
