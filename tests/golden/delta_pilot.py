"""Oracle pilot that fixes delta in the random-network formulas.

The random-network workloads check
  (X0 >= x0_0 - d) U[0,100] ((X1 <= x0_1 + d) U[0,100] (X2 >= x0_2 + d & X3 <= x0_3 - d))
(nested bounded until, Sec. 3.1).  The offset d sets how hard the formula is
to satisfy.  This script picks it once per network, with the CPU oracle only:
trajectories 0..999 of seed 1, model 0, 10^5-event cap.

Rule: the smallest d in 1, 2, 5, 10, 20, 50, 100 with 0.2 <= p_hat <= 0.8 and
under 1 % of trajectories stopped by the cap.  The list is scanned upwards
and the scan ends at the first d with p_hat < 0.2.  If no listed d
qualifies, the integers strictly between the last listed d with p_hat > 0.8
and that first d with p_hat < 0.2 are scanned upwards in the same way.  If
still none qualifies, the network is recorded as not qualifying and the
scanned d with p_hat nearest 0.5 (the smaller on a tie) is used, among the
ones under the truncation limit when there are any.

Usage: python tests/golden/delta_pilot.py [c3|c4|all]
writes configs/c3.json and/or configs/c4_networks.json.
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

LIST = (1, 2, 5, 10, 20, 50, 100)
P_LO, P_HI, TRUNC_MAX = 0.2, 0.8, 0.01
N_PILOT, SEED, CAP = 1000, 1, 100_000


def choose_delta(run):
    """run(d) -> (p_hat, truncated fraction).  Returns (d, qualifies, tried)
    with tried = [(d, p_hat, truncated fraction), ...] in scan order."""
    tried = []

    def ok(p, tr):
        return P_LO <= p <= P_HI and tr < TRUNC_MAX

    above = None     # last listed d with p_hat > P_HI
    below = None     # first listed d with p_hat < P_LO
    for d in LIST:
        p, tr = run(d)
        tried.append((d, p, tr))
        if ok(p, tr):
            return d, True, tried
        if p > P_HI:
            above = d
        if p < P_LO:
            below = d
            break
    if above is not None and below is not None:
        for d in range(above + 1, below):
            p, tr = run(d)
            tried.append((d, p, tr))
            if ok(p, tr):
                return d, True, tried
            if p < P_LO:
                break
    pool = [t for t in tried if t[2] < TRUNC_MAX] or tried
    best = min(pool, key=lambda t: (abs(t[1] - 0.5), t[0]))
    return best[0], False, tried


def pilot(net, species=(0, 1, 2, 3), threads=None, log=None):
    import numpy as np
    import oracle
    from paper_0912_2551_amd import workloads as W

    def run(d):
        t0 = time.perf_counter()
        f = oracle.parse(W.nested_until_formula(net, d, species), net)
        ev, vd, rs = oracle.trajectories(net, f, 0, N_PILOT, seed=SEED, max_events=CAP,
                                         threads=threads)
        p = float(vd.mean())
        tr = float((rs == oracle.R_CAP).mean())
        if log:
            log(f"  d={d}: p_hat={p:.3f} truncated={tr:.3f} mean events={float(np.mean(ev)):.0f} "
                f"({time.perf_counter() - t0:.1f} s)")
        return p, tr

    d, qual, tried = choose_delta(run)
    return {"delta": d, "qualifies": qual,
            "pilot": [{"delta": a, "p_hat": p, "truncated": tr} for a, p, tr in tried]}


def write_c3(log=print):
    from paper_0912_2551_amd import workloads as W
    net = W.c3_network()
    log(f"C3 {net.label}")
    rec = pilot(net, log=log)
    rec.update({"network": net.label, "species": [0, 1, 2, 3], "pilot_trajectories": N_PILOT,
                "pilot_seed": SEED, "cap": CAP,
                "formula": W.nested_until_formula(net, rec["delta"], (0, 1, 2, 3))})
    with open(os.path.join(ROOT, "configs", "c3.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")


def write_c4(log=print):
    from paper_0912_2551_amd import workloads as W
    out = []
    for q, net in enumerate(W.c4_random_networks()):
        log(f"C4 network {q}: {net.label}")
        rec = pilot(net, log=log)
        rec["network"] = net.label
        out.append(rec)
    doc = {"pilot_trajectories": N_PILOT, "pilot_seed": SEED, "cap": CAP, "species": [0, 1, 2, 3],
           "networks": out}
    with open(os.path.join(ROOT, "configs", "c4_networks.json"), "w") as fh:
        json.dump(doc, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    log = lambda s: print(s, flush=True)  # noqa: E731
    if what in ("c3", "all"):
        write_c3(log)
    if what in ("c4", "all"):
        write_c4(log)
