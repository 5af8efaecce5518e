"""Oracle values for the batched sweep at its full configuration.

Writes, with the CPU oracle only:
  tests/golden/c4_expected.json   every job of the sweep (512 Michaelis-Menten
      rate sets and 64 random networks, each an iterative 95% +-0.01 Wilson
      estimate, Fig. 2): n, successes, SSA events, truncated trajectories,
      batches, p_hat and the Wilson interval (eq. 3);
  tests/golden/c4_trajectories.npz   per-trajectory (events, verdict | reason << 1)
      of indices 0..1023 for eight of the random networks, chosen to span
      their sizes (8..128 species).

Usage: python tests/golden/c4_expected.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
N_TRAJ = 1024


def per_trajectory_networks(nets):
    """Eight networks spanning the sizes: positions 0, 9, ..., 63 of the
    networks sorted by species count (stable)."""
    order = sorted(range(len(nets)), key=lambda q: (nets[q].S, q))
    return [order[int(round(k * (len(order) - 1) / 7))] for k in range(8)]


def main():
    import oracle
    from paper_0912_2551_amd import workloads as W
    jobs = W.c4_jobs()
    out = []
    t_all = time.perf_counter()
    for k, (net, text, kw) in enumerate(jobs):
        t0 = time.perf_counter()
        o = oracle.estimate(net, text, confidence=kw["confidence"], eps=kw["half_width"], seed=kw["seed"],
                            model_id=kw["model_id"], max_events=kw.get("max_events", 0))
        out.append({"job": k, "label": net.label, "model_id": kw["model_id"], "n": o["n"],
                    "successes": o["successes"], "events": o["events"], "truncated": o["truncated"],
                    "batches": len(o["bounds"]), "p_hat": o["p_hat"], "lo": o["lo"], "hi": o["hi"]})
        if k >= 512 or k % 64 == 0:
            print(f"job {k} {net.label}: n={o['n']} p_hat={o['p_hat']:.4f} batches={len(o['bounds'])} "
                  f"events={o['events']} ({time.perf_counter() - t0:.1f} s)", flush=True)
    nets = [net for net, _, _ in jobs[512:]]
    sel = per_trajectory_networks(nets)
    arrays = {}
    for q in sel:
        net, text, kw = jobs[512 + q]
        ev, vd, rs = oracle.trajectories(net, oracle.parse(text, net), 0, N_TRAJ, seed=kw["seed"],
                                         model_id=kw["model_id"], max_events=kw["max_events"])
        arrays[f"events_{q}"] = ev
        arrays[f"vr_{q}"] = (vd | (rs << 1)).astype(np.uint8)
        print(f"network {q} ({net.label}): {N_TRAJ} trajectories, {int(ev.sum())} events", flush=True)
    doc = {"configuration": "95% Wilson +-0.01 per job, seed 1, model ids 0..575, cap 10^5 for the networks",
           "jobs": out, "per_trajectory_networks": sel, "per_trajectory_count": N_TRAJ}
    with open(os.path.join(HERE, "c4_expected.json"), "w") as fh:
        json.dump(doc, fh, indent=0)
        fh.write("\n")
    np.savez_compressed(os.path.join(HERE, "c4_trajectories.npz"), **arrays)
    print(f"done in {time.perf_counter() - t_all:.0f} s", flush=True)


if __name__ == "__main__":
    main()
