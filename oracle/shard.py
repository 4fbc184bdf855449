"""Times the oracle on one cycle range of the 1M-gate synthetic workload —
TEST INFRASTRUCTURE ONLY (the benchmark's CPU baseline runs one process of
this per host core, each on its own range; under cycle isolation the ranges
are independent, so their SAIF counts add up to the whole run's).

    python -m oracle.shard BEGIN END

prints one JSON line: the range, the oracle's wall time for it (workload
generation excluded) and the range's TC total.
"""
from __future__ import annotations

import json
import sys
import time


def main(argv):
    begin, end = int(argv[1]), int(argv[2])
    import oracle
    from paper_2203_06117_amd import synth
    w = synth.scale(n_cycles=max(end, 1))
    o = oracle.Oracle(w["netlist"], w["arcs"], w.get("wires"))
    t = time.perf_counter()
    r = o.run(w["stimulus"], begin, end)
    sec = time.perf_counter() - t
    print(json.dumps({"begin": begin, "end": end, "seconds": sec,
                      "gate_cycles": int(w["netlist"]["n_gates"]) * (end - begin), "tc_sum": int(r["tc"].sum())}),
          flush=True)


if __name__ == "__main__":
    main(sys.argv)
