"""Seeded synthetic workloads: reaction networks, formulas and parameter sweeps.

This module only builds inputs.  It holds no part of the method's arithmetic
(no SSA, no monitor, no Wilson rule) and is the one module that both the GPU
library's callers and the CPU oracle's tests read.

Networks are mass-action reaction networks in the form of Sec. 2.2: each
reaction j has a rate constant c_j, at most two reactant species (an equal
pair is a homodimer), and a net state-change vector v_j with at most four
non-zero entries.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Network:
    names: list
    x0: np.ndarray          # int32 [S]
    rate: np.ndarray        # float64 [M]
    reactants: np.ndarray   # int32 [M, 2], -1 = none
    chg_idx: np.ndarray     # int32 [M, 4], -1 = none
    chg_val: np.ndarray     # int32 [M, 4]
    label: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def S(self):
        return int(self.x0.shape[0])

    @property
    def M(self):
        return int(self.rate.shape[0])

    def with_rates(self, rate):
        return Network(self.names, self.x0.copy(), np.asarray(rate, np.float64).copy(),
                       self.reactants.copy(), self.chg_idx.copy(), self.chg_val.copy(),
                       self.label, dict(self.meta))


def from_reactions(names, x0, reactions, label=""):
    """Build a Network from a list of (reactants, products, rate) where
    reactants/products are lists of species names (repeats allowed)."""
    idx = {n: k for k, n in enumerate(names)}
    M = len(reactions)
    rate = np.zeros(M, np.float64)
    reac = -np.ones((M, 2), np.int32)
    ci = -np.ones((M, 4), np.int32)
    cv = np.zeros((M, 4), np.int32)
    for j, (rs, ps, c) in enumerate(reactions):
        if len(rs) > 2:
            raise ValueError("reaction order > 2")
        for q, s in enumerate(rs):
            reac[j, q] = idx[s]
        delta = {}
        for s in rs:
            delta[idx[s]] = delta.get(idx[s], 0) - 1
        for s in ps:
            delta[idx[s]] = delta.get(idx[s], 0) + 1
        entries = [(s, v) for s, v in sorted(delta.items()) if v != 0]
        if len(entries) > 4:
            raise ValueError("more than four species change in one reaction")
        for q, (s, v) in enumerate(entries):
            ci[j, q] = s
            cv[j, q] = v
        rate[j] = c
    return Network(list(names), np.asarray(x0, np.int32), rate, reac, ci, cv, label)


# ---------------------------------------------------------------------------
# Small networks with known behaviour
# ---------------------------------------------------------------------------
def immigration_death(k_in=10.0, mu=0.1, x0=0):
    """0 -> X at rate k_in, X -> 0 at rate mu * X."""
    return from_reactions(["X"], [x0], [([], ["X"], k_in), (["X"], [], mu)], "immigration-death")


def isomerization(c1=1.0, c2=0.5, n0=50):
    """A -> B at c1 * A, B -> A at c2 * B, all molecules start in A."""
    return from_reactions(["A", "B"], [n0, 0], [(["A"], ["B"], c1), (["B"], ["A"], c2)],
                          "isomerization")


def dimerization(c=0.01, n0=40):
    """A + A -> B (homodimer propensity c * A (A - 1) / 2)."""
    return from_reactions(["A", "B"], [n0, 0], [(["A", "A"], ["B"], c)], "dimerization")


MM_RATES = (0.01, 0.1, 0.1)   # k1, k-1, k2


def michaelis_menten(k1=0.01, km1=0.1, k2=0.1, e0=100, s0=1000):
    """E + S -> ES (k1), ES -> E + S (k-1), ES -> E + P (k2)."""
    return from_reactions(
        ["E", "S", "ES", "P"], [e0, s0, 0, 0],
        [(["E", "S"], ["ES"], k1), (["ES"], ["E", "S"], km1), (["ES"], ["E", "P"], k2)],
        "michaelis-menten")


# ---------------------------------------------------------------------------
# Configurations
# ---------------------------------------------------------------------------
C1_FORMULA = "F[0,100](X>=120)"
C2_FORMULA = "(P<500) U[0,60] (S<=200) & G[0,60](E>=10)"
# Companion for the sweep/surrogate: the C2 formula is FALSE on every path
# (E + ES = 100 and S + ES + P = 1000 force S > 200 while P < 500), so the
# sweep is also run with a formula whose probability crosses 0.5 in the box.
MM_COMPANION_FORMULA = "F[0,60](P>=575)"


def random_network(n_species, n_reactions, seed, frac_unimolecular=0.5, x0_max=1000,
                   log10_rate=(-3.0, 1.0)):
    """Seeded random mass-action network.

    Reaction kinds: a shuffled mix of unimolecular and bimolecular reactions;
    reactants uniform over species (bimolecular with replacement, so
    homodimers occur); 0, 1 or 2 products, uniform over species; rate
    constants log-uniform over log10_rate; initial counts uniform over
    0..x0_max."""
    rng = np.random.default_rng(seed)
    S, M = int(n_species), int(n_reactions)
    n_uni = int(round(M * frac_unimolecular))
    kinds = np.array([1] * n_uni + [2] * (M - n_uni))
    rng.shuffle(kinds)
    names = [f"X{k}" for k in range(S)]
    reactions = []
    for j in range(M):
        rs = [int(s) for s in rng.integers(0, S, size=int(kinds[j]))]
        n_prod = int(rng.integers(0, 3))
        ps = [int(s) for s in rng.integers(0, S, size=n_prod)]
        c = float(10.0 ** rng.uniform(*log10_rate))
        reactions.append(([names[s] for s in rs], [names[s] for s in ps], c))
    x0 = rng.integers(0, x0_max + 1, size=S).astype(np.int32)
    net = from_reactions(names, x0, reactions, f"random-S{S}-M{M}-seed{seed}")
    net.meta["seed"] = seed
    return net


def nested_until_formula(net, delta, species=(0, 1, 2, 3), T=100.0):
    """(Xa >= xa0 - d) U[0,T] ((Xb <= xb0 + d) U[0,T] (Xc >= xc0 + d & Xd <= xd0 - d))."""
    a, b, c, d = species
    x0 = net.x0
    n = net.names
    th = (int(x0[a]) - delta, int(x0[b]) + delta, int(x0[c]) + delta, int(x0[d]) - delta)
    return (f"({n[a]} >= {th[0]}) U[0,{T:g}] (({n[b]} <= {th[1]}) U[0,{T:g}] "
            f"({n[c]} >= {th[2]} & {n[d]} <= {th[3]}))")


C3_SEED = 1
C3_CAP = 100000
# The offsets d of the random-network formulas are fixed once by an oracle
# pilot (tests/golden/delta_pilot.py) and frozen in these files.
CONFIG_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "configs")


def _config(name):
    with open(os.path.join(CONFIG_DIR, name)) as fh:
        return json.load(fh)


def c3_network():
    return random_network(64, 256, C3_SEED)


def c3_delta():
    return int(_config("c3.json")["delta"])


def c3_formula(net=None, delta=None):
    """The C3 formula over X0..X3 with the frozen offset."""
    net = net or c3_network()
    return nested_until_formula(net, c3_delta() if delta is None else delta)


def c4_random_networks(n_random=64, seed=5, s_min=8, s_max=128):
    """Random networks of uneven size: S log-uniform in [s_min, s_max], M = 4 S."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n_random):
        S = int(round(10.0 ** rng.uniform(math.log10(s_min), math.log10(s_max))))
        out.append(random_network(S, 4 * S, seed * 1000 + q))
    return out


def c4_deltas():
    """Per-network (delta, qualifies) of the 64 random networks, in order."""
    return [(int(r["delta"]), bool(r["qualifies"])) for r in _config("c4_networks.json")["networks"]]


def c4_networks():
    """The 64 random networks with their formulas (frozen offsets)."""
    nets = c4_random_networks()
    deltas = c4_deltas()
    assert len(deltas) == len(nets)
    return [(net, nested_until_formula(net, d)) for net, (d, _) in zip(nets, deltas)]


def c4_jobs():
    """The batched sweep: 512 Michaelis-Menten rate sets under the C2 formula
    and the 64 random networks under their nested-until formulas, each an
    iterative 95% +-0.01 Wilson job of seed 1 with its own model id (the
    networks with the 10^5-event cap).  Returns [(network, formula text,
    parameter dict), ...] in launch order."""
    out = []
    for k, rr in enumerate(mm_sweep(512, seed=4)):
        out.append((michaelis_menten(*rr), C2_FORMULA,
                    dict(confidence=0.95, half_width=0.01, seed=1, model_id=k)))
    for k, (net, text) in enumerate(c4_networks()):
        out.append((net, text, dict(confidence=0.95, half_width=0.01, seed=1, model_id=512 + k,
                                    max_events=C3_CAP)))
    return out


def mm_sweep(n_sets=512, seed=4, decades=1.0):
    """Rate sets log-uniform within +-decades around the Michaelis-Menten centre."""
    rng = np.random.default_rng(seed)
    base = np.log10(np.asarray(MM_RATES))
    logs = base[None, :] + rng.uniform(-decades, decades, size=(n_sets, 3))
    return 10.0 ** logs


def surrogate_queries(n=1_000_000, seed=6, decades=1.0):
    """Log10 rate points, uniform in the sweep box."""
    rng = np.random.default_rng(seed)
    base = np.log10(np.asarray(MM_RATES))
    return (base[None, :] + rng.uniform(-decades, decades, size=(n, 3))).astype(np.float32)
