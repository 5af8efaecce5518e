"""The oracle pilot that fixes the offset d of the random-network formulas
(tests/golden/delta_pilot.py): its selection rule on made-up pilot results,
and the frozen configuration files against the rule and the oracle."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_0912_2551_amd import workloads as W

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import delta_pilot as DP  # noqa: E402


def _runner(table, trunc=None):
    seen = []

    def run(d):
        seen.append(d)
        return table(d), (trunc(d) if trunc else 0.0)
    return run, seen


def test_rule_first_listed_delta_in_range():
    run, seen = _runner(lambda d: {1: 0.99, 2: 0.95, 5: 0.7}.get(d, 0.1))
    d, ok, _ = DP.choose_delta(run)
    assert (d, ok) == (5, True) and seen == [1, 2, 5]


def test_rule_refines_between_listed_deltas():
    # 20 gives 0.81 (above the range), 50 gives 0.05 (below): integers 21..49
    run, seen = _runner(lambda d: 1.0 if d < 20 else (0.81 if d == 20 else (0.05 if d >= 50 else 0.85 - 0.02 * (d - 20))))
    d, ok, _ = DP.choose_delta(run)
    assert (d, ok) == (23, True)          # 0.85 - 0.06 = 0.79
    assert seen == [1, 2, 5, 10, 20, 50, 21, 22, 23]


def test_rule_truncation_disqualifies():
    run, _ = _runner(lambda d: 0.5, lambda d: 0.02 if d < 10 else 0.0)
    d, ok, _ = DP.choose_delta(run)
    assert (d, ok) == (10, True)


def test_rule_no_delta_qualifies():
    run, seen = _runner(lambda d: 0.08)
    d, ok, tried = DP.choose_delta(run)
    assert not ok and d == 1 and seen == [1]     # already below the range at the smallest offset
    run, seen = _runner(lambda d: 0.97)
    d, ok, _ = DP.choose_delta(run)
    assert not ok and seen == list(DP.LIST) and d == 1


def _c3():
    with open(os.path.join(W.CONFIG_DIR, "c3.json")) as fh:
        return json.load(fh)


def test_frozen_c3_config_follows_the_rule():
    cfg = _c3()
    rec = {r["delta"]: (r["p_hat"], r["truncated"]) for r in cfg["pilot"]}
    d, ok, _ = DP.choose_delta(lambda d: rec[d])
    assert (d, ok) == (cfg["delta"], cfg["qualifies"]) == (W.c3_delta(), True)
    assert cfg["formula"] == W.c3_formula()


@pytest.mark.parametrize("d", [20, 21])
def test_frozen_c3_pilot_values_reproduce(d):
    """The oracle gives the recorded pilot estimates on both sides of the
    chosen offset (d = 20 above the range, d = 21 inside it)."""
    cfg = _c3()
    rec = {r["delta"]: (r["p_hat"], r["truncated"]) for r in cfg["pilot"]}
    net = W.c3_network()
    ev, vd, rs = oracle.trajectories(net, W.nested_until_formula(net, d), 0, DP.N_PILOT, seed=DP.SEED,
                                     max_events=DP.CAP)
    assert (float(vd.mean()), float((rs == oracle.R_CAP).mean())) == rec[d]


def test_frozen_c4_configs_follow_the_rule():
    with open(os.path.join(W.CONFIG_DIR, "c4_networks.json")) as fh:
        doc = json.load(fh)
    nets = W.c4_random_networks()
    assert len(doc["networks"]) == len(nets) == 64
    for net, r in zip(nets, doc["networks"]):
        assert r["network"] == net.label
        rec = {t["delta"]: (t["p_hat"], t["truncated"]) for t in r["pilot"]}
        d, ok, _ = DP.choose_delta(lambda d: rec[d])
        assert (d, ok) == (r["delta"], r["qualifies"])
    # re-run the pilot of the two smallest networks with the oracle
    small = sorted(range(64), key=lambda q: nets[q].S)[:2]
    for q in small:
        rec = {t["delta"]: (t["p_hat"], t["truncated"]) for t in doc["networks"][q]["pilot"]}
        for d, (p, tr) in rec.items():
            ev, vd, rs = oracle.trajectories(nets[q], W.nested_until_formula(nets[q], d), 0, DP.N_PILOT,
                                             seed=DP.SEED, max_events=DP.CAP)
            assert (float(vd.mean()), float((rs == oracle.R_CAP).mean())) == (p, tr)
