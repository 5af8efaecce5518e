"""GPU path (through the C ABI) against the CPU oracle.

Per-trajectory results (events, verdict, reason) must be bit-identical for the
same Philox streams; estimates (p_hat, n, successes, events, batches and the
Wilson interval) must be identical for the same trajectory indices.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import wilson
from paper_0912_2551_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_0912_2551_amd import binding as B
    c = B.Context(0)
    c.set_watchdog(120)
    yield c
    c.close()


def _B():
    from paper_0912_2551_amd import binding as B
    return B


def death_only():
    return W.from_reactions(["X"], [30], [(["X"], [], 1.0)], "death")


TRAJ_CASES = [
    ("c1", W.immigration_death, W.C1_FORMULA, {}, 4096),
    ("c2", W.michaelis_menten, W.C2_FORMULA, {}, 20000),
    ("mm-companion", W.michaelis_menten, W.MM_COMPANION_FORMULA, {}, 1500),
    ("iso-until", W.isomerization, "(B<=30) U[0,1.5] (A<=20)", {}, 5000),
    ("iso-globally", W.isomerization, "G[0,1](A>=22)", {}, 5000),
    ("next-or", W.isomerization, "X[0,0.05](B>=1) | F[1,2](A<=15)", {}, 3000),
    ("nested", W.immigration_death, "(X<=60) U[0,20] ((X>=20) U[0,3] (X>=70))", {}, 3000),
    ("nested-fin", W.immigration_death, "(X<=80) U[0,30] F[0,4](X>=75)", {}, 2000),
    ("nested-lo", W.isomerization, "(A<=60) U[1.5,2] ((A>=16) U[0,0.5] (A>=22))", {}, 3000),
    ("nested-F", W.isomerization, "F[1.5,2.5]((A>=15) U[0,0.4] (A>=20))", {}, 3000),
    ("nested-fin-lo", W.immigration_death, "(X<=95) U[10,30] F[0,2](X>=92)", {}, 2000),
    ("next-until", W.isomerization, "X[0,0.05]((A>=38) U[0,0.25] (B>=12))", {}, 3000),
    ("next-G", W.isomerization, "X[0,0.05](G[0,0.8](A>=30))", {}, 3000),
    ("next-F-lo", W.immigration_death, "X[0,0.15](F[2,4](X>=40))", {}, 2000),
    ("next-two", W.dimerization, "X[0,0.5](G[0,3](A>=20)) | X[0,0.2](F[0,1](B>=5))", {}, 3000),
    ("until-G", W.isomerization, "(A>=15) U[0.5,3] G[0,0.5](A<=20)", {}, 3000),
    ("until-and-G", W.isomerization, "(B<=40) U[0,2] ((A<=25) & G[0,0.3](A>=20))", {}, 3000),
    ("until-G-and", W.immigration_death, "(X<=120) U[5,40] (G[0,3](X>=95) & X>=96)", {}, 2000),
    ("until-G-absorb", death_only, "(X>=0) U[0,100] G[0,5](X<=3)", {}, 777),
    ("lower-bounds", W.immigration_death, "F[5,10](X>=60) & G[2,8](X<=90)", {}, 3000),
    ("not-or", W.immigration_death, "!(F[0,3](X>=25) | G[0,2](X<=18))", {}, 3000),
    ("arith", W.isomerization, "F[0,2](A*A <= sqrt(B*400) + 3)", {}, 3000),
    ("pow", W.isomerization, "F[0,2](pow(A,3) <= pow(B/7,2) * 200 + pow(A,1) + pow(B/50,11))", {}, 3000),
    ("linear", W.michaelis_menten, "F[0,1](2*ES + E >= 3*P - S + 1100)", {}, 2000),
    ("prop-only", W.michaelis_menten, "S >= 1000 & E = 100", {}, 129),
    ("dimer", W.dimerization, "F[0,5](A<=10)", {}, 3000),
    ("absorb-F", death_only, "F[0,100](X>=40)", {}, 777),
    ("absorb-G", death_only, "G[0,100](X>=0) & F[0,200](X<=0)", {}, 777),
    ("cap", W.immigration_death, W.C1_FORMULA, {"max_events": 500}, 2000),
    ("tmax", W.immigration_death, "F(X>=1000)", {"t_max": 5.0}, 2000),
    # response monitors: G I (p | F[0,d] q) and F I (p & G[0,d] q)
    ("resp", W.immigration_death, "G[10,40]((F[0,1](X<=90)) | X<=105)", {}, 2000),
    ("resp-dual", W.immigration_death, "F[5,30]((X>=95) & G[0,2](X>=90))", {}, 2000),
    ("resp-dual-bare", W.immigration_death, "F[0,30](G[0,3](X>=95))", {}, 2000),
    ("resp-two", W.isomerization, "G[0,2](A>=30 | F[0,0.3](B<=20)) | F[0,3](G[0,0.5](A<=18))", {}, 3000),
    ("resp-iso", W.isomerization, "F[0.5,3]((A>=25) & G[0,0.3](A>=22))", {}, 3000),
    ("resp-dimer", W.dimerization, "G[0,5](A>=30 | F[0,1](B>=8))", {}, 3000),
    ("resp-absorb", death_only, "G[0,100](X>=10 | F[0,2](X<=0))", {}, 777),
    ("resp-tmax", W.immigration_death, "G[5,inf](X<=130 | F[0,1](X<=120))", {"t_max": 30.0}, 1000),
]


# formulas with arithmetic (RPN) predicates always run on the generic kernel
GENERIC_ONLY = {"arith", "pow"}


@pytest.mark.parametrize("mode", ["generic", "specialized"])
@pytest.mark.parametrize("name,make,text,kw,count", TRAJ_CASES, ids=[c[0] for c in TRAJ_CASES])
def test_trajectory_parity(ctx, name, make, text, kw, count, mode):
    B = _B()
    net = make()
    n = ctx.network(net)
    f = ctx.formula(n, text)
    if mode == "generic":
        ctx.set_specialization(B.SPECIALIZE_OFF)
    elif name in GENERIC_ONLY:
        pytest.skip("arithmetic predicates are not specialised")
    else:
        ctx.set_specialization(B.SPECIALIZE_REQUIRED)
    try:
        for first, seed in ((0, 1), (123457, 99)):
            p = B.params(seed=seed, model_id=3, **kw)
            print(f"case {name} mode {mode} first {first} seed {seed}", flush=True)
            ev, vd, rs = ctx.trajectories(n, f, p, first, count)
            expect = B.KERNEL_SPECIALIZED if mode == "specialized" else (
                B.KERNEL_GENERIC_SMALL if net.M <= 4 else B.KERNEL_GENERIC)
            assert ctx.last_kernel() == expect
            oev, ovd, ors = oracle.trajectories(net, oracle.parse(text, net), first, count, seed=seed,
                                                model_id=3, **kw)
            assert np.array_equal(rs, ors), (name, np.nonzero(rs != ors)[0][:5])
            assert np.array_equal(vd, ovd), (name, np.nonzero(vd != ovd)[0][:5])
            assert np.array_equal(ev, oev), (name, np.nonzero(ev != oev)[0][:5])
    finally:
        ctx.set_specialization(B.SPECIALIZE_AUTO)


def _wide_mode(ctx, B, mode):
    """Run on the generic kernel or on the wide specialised kernel (counts in
    LDS, constant reactant indices); both must equal the oracle."""
    ctx.set_specialization(B.SPECIALIZE_OFF if mode == "generic" else B.SPECIALIZE_REQUIRED)


WIDE_MODES = pytest.mark.parametrize("mode", ["generic", "specialized"])


C3_PARITY_N = 2048
_c3_oracle = {}


def _c3_expected(net, text):
    """Oracle (events, verdict, reason) of C3's first trajectories (seed 1,
    the 10^5-event cap), computed once for both kernel kinds."""
    if text not in _c3_oracle:
        _c3_oracle[text] = oracle.trajectories(net, oracle.parse(text, net), 0, C3_PARITY_N, seed=1,
                                               max_events=W.C3_CAP)
    return _c3_oracle[text]


@WIDE_MODES
def test_c3_random_network_parity(ctx, mode):
    """C3 as configured (64 species, 256 channels, the nested until over
    X0..X3 with the pilot's offset): the first 2048 trajectories are
    bit-identical to the oracle's, and both verdicts occur."""
    B = _B()
    net = W.c3_network()
    text = W.c3_formula(net)
    n = ctx.network(net)
    f = ctx.formula(n, text)
    p = B.params(seed=1, max_events=W.C3_CAP)
    _wide_mode(ctx, B, mode)
    try:
        print(f"case c3 mode {mode} trajectories {C3_PARITY_N}", flush=True)
        ev, vd, rs = ctx.trajectories(n, f, p, 0, C3_PARITY_N)
        assert ctx.last_kernel() == (B.KERNEL_GENERIC if mode == "generic" else B.KERNEL_SPECIALIZED)
    finally:
        ctx.set_specialization(B.SPECIALIZE_AUTO)
    oev, ovd, ors = _c3_expected(net, text)
    assert np.array_equal(rs, ors), np.nonzero(rs != ors)[0][:5]
    assert np.array_equal(vd, ovd), np.nonzero(vd != ovd)[0][:5]
    assert np.array_equal(ev, oev), np.nonzero(ev != oev)[0][:5]
    assert 0.2 * C3_PARITY_N <= int(vd.sum()) <= 0.8 * C3_PARITY_N


@WIDE_MODES
def test_large_network_parity(ctx, mode):
    B = _B()
    net = W.random_network(128, 512, seed=7)
    text = W.nested_until_formula(net, 15)
    n = ctx.network(net)
    f = ctx.formula(n, text)
    p = B.params(seed=5, max_events=20000)
    _wide_mode(ctx, B, mode)
    try:
        ev, vd, rs = ctx.trajectories(n, f, p, 0, 70)
        assert ctx.last_kernel() == (B.KERNEL_GENERIC if mode == "generic" else B.KERNEL_SPECIALIZED)
    finally:
        ctx.set_specialization(B.SPECIALIZE_AUTO)
    oev, ovd, ors = oracle.trajectories(net, oracle.parse(text, net), 0, 70, seed=5, max_events=20000)
    assert np.array_equal(ev, oev) and np.array_equal(vd, ovd) and np.array_equal(rs, ors)


# speculative: every index up to the capacity runs in one launch and Fig. 2 is
# applied to the recorded outcomes; batched: the persistent kernel's batch
# protocol.  Both must give the oracle's iterative estimate exactly.
SPECULATE = pytest.mark.parametrize("speculate", [True, False], ids=["speculative", "batched"])


@SPECULATE
@pytest.mark.parametrize("kw", [{}, {"conservative": True}, {"paper_rounding": True}],
                         ids=["iterative", "conservative", "paper-rounding"])
def test_c1_wilson_estimate(ctx, kw, speculate):
    B = _B()
    net = W.immigration_death()
    n = ctx.network(net)
    f = ctx.formula(n, W.C1_FORMULA)
    r = ctx.estimate(n, f, B.params(confidence=0.95, half_width=0.01, seed=1, speculate=speculate, **kw))
    o = oracle.estimate(net, W.C1_FORMULA, confidence=0.95, eps=0.01, seed=1,
                        conservative=kw.get("conservative", False), literal=kw.get("paper_rounding", False))
    assert (r["n"], r["successes"], r["events"], r["batches"]) == (o["n"], o["successes"], o["events"], len(o["bounds"]))
    assert (r["p_hat"], r["lo"], r["hi"]) == (o["p_hat"], o["lo"], o["hi"])
    exact = 0.5073337972305221
    assert r["lo"] - 0.01 <= exact <= r["hi"] + 0.01


def test_estimate_independent_of_launch_shape(ctx):
    B = _B()
    net = W.immigration_death()
    n = ctx.network(net)
    f = ctx.formula(n, W.C1_FORMULA)
    ref = None
    for w in (1, 4, 16):
        ctx.set_waves_per_cu(w)
        r = ctx.estimate(n, f, B.params(seed=7))
        key = (r["n"], r["successes"], r["events"], r["batches"])
        ref = ref or key
        assert key == ref
    ctx.set_waves_per_cu(0)


def test_c2_full_size_fixed(ctx):
    """Configuration 2 at its full size: 10^6 trajectories."""
    B = _B()
    net = W.michaelis_menten()
    n = ctx.network(net)
    f = ctx.formula(n, W.C2_FORMULA)
    r = ctx.estimate(n, f, B.params(fixed_n=10**6, seed=1, confidence=0.999))
    o = oracle.estimate(net, W.C2_FORMULA, fixed_n=10**6, seed=1, confidence=0.999)
    assert (r["n"], r["successes"], r["events"]) == (o["n"], o["successes"], o["events"])
    assert r["p_hat"] == 0.0 and r["lo"] == 0.0 and abs(r["hi"] - 1.0827e-5) < 1e-8


def test_c2_full_size_sampled_trajectories(ctx):
    """Configuration 2 at its full size in the launch bench.py times (the
    autotuned configuration): 10^6 trajectories recorded on the device, 3000
    of them, sampled, equal the oracle's trajectory for that index."""
    B = _B()
    net = W.michaelis_menten()
    n = ctx.network(net)
    f = ctx.formula(n, W.C2_FORMULA)
    p = B.params(fixed_n=10**6, seed=1)
    ctx.autotune(n, f, p)
    ev, vd, rs = ctx.trajectories(n, f, p, 0, 10**6)
    text = oracle.parse(W.C2_FORMULA, net)
    rng = np.random.default_rng(11)
    for i in rng.choice(10**6, size=3000, replace=False):
        oev, ovd, ors = oracle.trajectories(net, text, int(i), 1, seed=1, model_id=0)
        assert (ev[i], vd[i], rs[i]) == (oev[0], ovd[0], ors[0]), i


@SPECULATE
def test_batch_matches_single_jobs(ctx, speculate):
    B = _B()
    rates = W.mm_sweep(6, seed=11)
    jobs, singles = [], []
    keep = []
    for k, rr in enumerate(rates):
        net = W.michaelis_menten(*rr)
        nh = ctx.network(net)
        fh = ctx.formula(nh, W.MM_COMPANION_FORMULA)
        keep.append((nh, fh))
        p = B.params(seed=1, model_id=k, half_width=0.05, speculate=speculate)
        jobs.append((nh, fh, p))
        singles.append((net, W.MM_COMPANION_FORMULA, k))
    for q, net in enumerate(W.c4_random_networks(2, seed=12)):
        text = W.nested_until_formula(net, 20)
        nh = ctx.network(net)
        fh = ctx.formula(nh, text)
        keep.append((nh, fh))
        p = B.params(seed=1, model_id=100 + q, half_width=0.1, max_events=20000, speculate=speculate)
        jobs.append((nh, fh, p))
        singles.append((net, text, 100 + q))
    res = ctx.estimate_batch(jobs)
    for (net, text, mid), r, (_, _, p) in zip(singles, res, jobs):
        o = oracle.estimate(net, text, eps=p.half_width, seed=1, model_id=mid, max_events=p.max_events)
        assert (r["n"], r["successes"], r["events"], r["batches"]) == \
            (o["n"], o["successes"], o["events"], len(o["bounds"])), (mid, r, o)


@pytest.mark.parametrize("waves_per_cu", [1, 16, 32])
def test_fixed_batch_matches_oracle(ctx, waves_per_cu):
    """Fixed-size jobs of many sizes in one launch.  A launch of fixed-size jobs
    whose grid fits on the device starts each wave on a static share of its
    home job's first indices: sizes below, at and above one share (64) and
    above all shares together must still give the oracle's counts exactly,
    whatever the number of waves."""
    B = _B()
    sizes = [1, 63, 64, 65, 1000, 5000, 70000]
    keep, jobs, refs = [], [], []
    net = W.michaelis_menten()
    nh = ctx.network(net)
    fh = ctx.formula(nh, W.C2_FORMULA)
    keep.append((nh, fh))
    for k, m in enumerate(sizes):
        jobs.append((nh, fh, B.params(fixed_n=m, seed=5, model_id=k)))
        refs.append((net, W.C2_FORMULA, m, k))
    small = W.immigration_death()
    nh2 = ctx.network(small)
    fh2 = ctx.formula(nh2, W.C1_FORMULA)
    keep.append((nh2, fh2))
    for k, m in enumerate([100, 3000]):
        jobs.append((nh2, fh2, B.params(fixed_n=m, seed=5, model_id=50 + k)))
        refs.append((small, W.C1_FORMULA, m, 50 + k))
    ctx.set_waves_per_cu(waves_per_cu)
    try:
        same = ctx.estimate_batch(jobs[:len(sizes)])      # one structure: specialised kernel
        mixed = ctx.estimate_batch(jobs)                   # two structures: generic kernel
    finally:
        ctx.set_waves_per_cu(0)
    for res, n_jobs in ((same, len(sizes)), (mixed, len(jobs))):
        for r, (net_k, text, m, mid) in zip(res, refs[:n_jobs]):
            o = oracle.estimate(net_k, text, fixed_n=m, seed=5, model_id=mid)
            assert (r["n"], r["successes"], r["events"]) == (o["n"], o["successes"], o["events"]), (m, mid)


@pytest.mark.parametrize("kind", ["generic", "specialized"])
def test_many_more_fixed_jobs_than_waves(ctx, kind):
    """A fixed-size launch of 20000 jobs of 64 trajectories on 256 waves (one
    per CU): most jobs lie far from every wave's home, and each must still be
    run in full (a wave scans every job before it leaves); sampled jobs give
    the oracle's counts."""
    B = _B()
    net = W.isomerization()
    text = "G[0,1](A>=22)"
    nh = ctx.network(net)
    fh = ctx.formula(nh, text)
    jobs = [(nh, fh, B.params(fixed_n=64, seed=7, model_id=k)) for k in range(20000)]
    ctx.set_waves_per_cu(1)
    ctx.set_specialization(B.SPECIALIZE_OFF if kind == "generic" else B.SPECIALIZE_REQUIRED)
    try:
        print(f"case many fixed jobs {kind}", flush=True)
        res = ctx.estimate_batch(jobs)
    finally:
        ctx.set_waves_per_cu(0)
        ctx.set_specialization(B.SPECIALIZE_AUTO)
    assert all(r["n"] == 64 for r in res)
    rng = np.random.default_rng(3)
    for k in rng.choice(20000, size=40, replace=False):
        o = oracle.estimate(net, text, fixed_n=64, seed=7, model_id=int(k))
        r = res[int(k)]
        assert (r["successes"], r["events"]) == (o["successes"], o["events"]), k


def test_many_fixed_jobs_beside_iterative_ones(ctx):
    """Four iterative Wilson jobs and 5000 fixed-size jobs of 64 trajectories
    in one launch on 256 waves: while an iterative job is open, waves only
    take jobs near their homes; once none is, they take any job with indices
    left, each resuming its scan past the jobs it found exhausted.  Every
    fixed job runs in full, and the iterative estimates and sampled fixed
    jobs give the oracle's results."""
    B = _B()
    net = W.isomerization()
    text = "G[0,1](A>=22)"
    nh = ctx.network(net)
    fh = ctx.formula(nh, text)
    jobs = [(nh, fh, B.params(seed=8, model_id=k, half_width=0.05)) for k in range(4)]
    jobs += [(nh, fh, B.params(fixed_n=64, seed=8, model_id=4 + k)) for k in range(5000)]
    ctx.set_waves_per_cu(1)
    try:
        print("case iterative and many fixed jobs", flush=True)
        res = ctx.estimate_batch(jobs)
    finally:
        ctx.set_waves_per_cu(0)
    assert all(r["n"] == 64 for r in res[4:])
    for k in range(4):
        o = oracle.estimate(net, text, eps=0.05, seed=8, model_id=k)
        r = res[k]
        assert (r["n"], r["successes"], r["events"], r["batches"]) == \
            (o["n"], o["successes"], o["events"], len(o["bounds"])), (k, r, o)
    rng = np.random.default_rng(4)
    for k in rng.choice(5000, size=20, replace=False):
        o = oracle.estimate(net, text, fixed_n=64, seed=8, model_id=4 + int(k))
        r = res[4 + int(k)]
        assert (r["successes"], r["events"]) == (o["successes"], o["events"]), k


@SPECULATE
def test_fig3_bernoulli_sources(ctx, speculate):
    """Fig. 3's setting (99%, +-0.025) on Bernoulli sources of known p: the
    death of one molecule (rate 1) before T = -ln(1 - p).  The device's
    iterative sample sizes equal the oracle's, and at p = 0 and p = 1 the
    reduction against the conservative size is the paper's "up to 88%"."""
    B = _B()
    net = W.from_reactions(["X"], [1], [(["X"], [], 1.0)], "death of one molecule")
    nh = ctx.network(net)
    cons = B.wilson_sample(0.5, 0.025, B.z_value(0.99))
    keep, jobs, refs = [], [], []
    for q, p in enumerate((0.0, 0.3, 1.0)):
        T = 50.0 if p == 1.0 else -math.log1p(-p)
        text = f"F[0,{T!r}](X<=0)"
        fh = ctx.formula(nh, text)
        keep.append(fh)
        for r in range(3):
            jobs.append((nh, fh, B.params(confidence=0.99, half_width=0.025, seed=1000 + r, model_id=q,
                                          speculate=speculate)))
            refs.append((text, 1000 + r, q, p))
    res = ctx.estimate_batch(jobs)
    for r, (text, seed, q, p) in zip(res, refs):
        o = oracle.estimate(net, text, confidence=0.99, eps=0.025, seed=seed, model_id=q)
        assert (r["n"], r["successes"], r["batches"]) == (o["n"], o["successes"], len(o["bounds"]))
        if p in (0.0, 1.0):
            assert 0.88 <= 1.0 - r["n"] / cons < 0.89


def test_device_stopping_rule_matches_host(ctx):
    rng = np.random.default_rng(0)
    z = wilson.z_value(0.95)
    ns, ys = [], []
    for n in range(1, 1201):
        ns.extend([n] * (n + 1))
        ys.extend(range(n + 1))
    big = rng.integers(1, 10**6, size=20000)
    ns.extend(big.tolist())
    ys.extend((rng.random(20000) * big).astype(np.int64).tolist())
    for literal in (False, True):
        out = ctx.wilson_next_device(ys, ns, 0.01, z, paper_rounding=literal)
        exp = [wilson.wilson_sample(wilson.rounded_estimate(y / n, 0.01, literal), 0.01, z)
               for y, n in zip(ys, ns)]
        assert np.array_equal(out, np.asarray(exp, dtype=np.uint64))


@pytest.mark.parametrize("make,T", [(W.immigration_death, 7.5), (W.michaelis_menten, 0.3),
                                    (W.dimerization, 2.0)])
def test_sample_state_parity(ctx, make, T):
    B = _B()
    net = make()
    n = ctx.network(net)
    got = ctx.sample_state(n, B.params(seed=4, model_id=1), T, 1000, 3000)
    exp = oracle.sample_state(net, T, 1000, 3000, seed=4, model_id=1)
    assert np.array_equal(got, exp)


def test_errors_and_edges(ctx):
    B = _B()
    net = W.immigration_death()
    n = ctx.network(net)
    with pytest.raises(B.SmcError) as e:
        ctx.formula(n, "F[0,1](Y>1)")
    assert e.value.code == B.SMC_E_PARSE
    with pytest.raises(B.SmcError) as e:           # more than 16 predicates
        ctx.formula(n, " | ".join(f"F[0,1](X>={i})" for i in range(17)))
    assert e.value.code == B.SMC_E_UNSUPPORTED
    with pytest.raises(B.SmcError) as e:           # a trace program of more than 32 nodes
        ctx.formula(n, "F[0,1](" + " & ".join(f"G[0,{i + 1}](X>=1)" for i in range(7)) + ")")
    assert e.value.code == B.SMC_E_UNSUPPORTED
    # more species than one wave's LDS holds: refused on the host, before any launch
    big = W.from_reactions([f"S{i}" for i in range(300)], [5] + [0] * 299, [(["S0"], ["S1"], 1.0)], "wide")
    nb = ctx.network(big)
    fb = ctx.formula(nb, "F[0,1](S1>=1)")
    with pytest.raises(B.SmcError) as e:
        ctx.estimate(nb, fb, B.params(fixed_n=64))
    assert e.value.code == B.SMC_E_INVALID
    with pytest.raises(B.SmcError) as e:
        ctx.formula(n, "F[0,1](pow(X,0.5)>1)")
    assert e.value.code == B.SMC_E_UNSUPPORTED
    f = ctx.formula(n, "F(X>=5)")
    assert math.isinf(f.horizon)
    with pytest.raises(B.SmcError) as e:
        ctx.estimate(n, f, B.params())
    assert e.value.code == B.SMC_E_INVALID
    f2 = ctx.formula(n, W.C1_FORMULA)
    assert f2.horizon == 100.0
    with pytest.raises(B.SmcError):
        ctx.estimate(n, f2, B.params(half_width=0.0))
    bad = W.immigration_death()
    bad.chg_val[1, 0] = -2
    with pytest.raises(B.SmcError):
        ctx.network(bad)
    ev, vd, rs = ctx.trajectories(n, f2, B.params(), 0, 0)
    assert ev.size == 0
    r = ctx.estimate(n, f2, B.params(fixed_n=1))
    o = oracle.estimate(net, W.C1_FORMULA, fixed_n=1)
    assert (r["n"], r["successes"], r["events"]) == (o["n"], o["successes"], o["events"])


def test_specialized_kernel_selection_and_estimates(ctx):
    """One specialised kernel serves a rate sweep over one structure (a batch of
    Michaelis-Menten rate sets); mixed structures use the generic kernel; the
    estimates are identical either way."""
    B = _B()
    rates = W.mm_sweep(48, seed=11)
    keep, jobs = [], []
    for k, rr in enumerate(rates):
        nh = ctx.network(W.michaelis_menten(*rr))
        fh = ctx.formula(nh, W.MM_COMPANION_FORMULA)
        keep.append((nh, fh))
        jobs.append((nh, fh, B.params(half_width=0.05, seed=3, model_id=k)))
    out = {}
    for mode in (B.SPECIALIZE_OFF, B.SPECIALIZE_AUTO):
        ctx.set_specialization(mode)
        out[mode] = ctx.estimate_batch(jobs)
        assert ctx.last_kernel() == (B.KERNEL_SPECIALIZED if mode == B.SPECIALIZE_AUTO else B.KERNEL_GENERIC_SMALL)
    keys = ("n", "successes", "events", "batches", "p_hat", "lo", "hi")
    assert [tuple(r[k] for k in keys) for r in out[B.SPECIALIZE_OFF]] == \
           [tuple(r[k] for k in keys) for r in out[B.SPECIALIZE_AUTO]]
    # a different structure in the same launch: generic kernel
    c1 = ctx.network(W.immigration_death())
    f1 = ctx.formula(c1, W.C1_FORMULA)
    mixed = jobs[:4] + [(c1, f1, B.params(half_width=0.05, seed=3, model_id=99))]
    r_mixed = ctx.estimate_batch(mixed)
    assert ctx.last_kernel() == B.KERNEL_GENERIC_SMALL
    assert [tuple(r[k] for k in keys) for r in r_mixed[:4]] == \
           [tuple(r[k] for k in keys) for r in out[B.SPECIALIZE_AUTO][:4]]
    ctx.set_specialization(B.SPECIALIZE_REQUIRED)
    with pytest.raises(B.SmcError):
        ctx.estimate_batch(mixed)
    ctx.set_specialization(B.SPECIALIZE_AUTO)


def test_autotune_keeps_results(ctx):
    """The autotuner only changes the launch configuration: estimates before
    and after tuning are identical, and a second call reuses the cached
    choice."""
    B = _B()
    net = W.michaelis_menten()
    n = ctx.network(net)
    f = ctx.formula(n, W.C2_FORMULA)
    p = B.params(fixed_n=50000, seed=3)
    before = ctx.estimate(n, f, p)
    t = ctx.autotune(n, f, p, pilot_n=1 << 14)
    assert t["candidates"] >= 5 and t["events_per_s"] > 0
    assert t["waves_per_cu"] in (4, 8, 16, 24, 28, 32)
    after = ctx.estimate(n, f, p)
    keys = ("n", "successes", "events", "p_hat", "lo", "hi")
    assert tuple(before[k] for k in keys) == tuple(after[k] for k in keys)
    t2 = ctx.autotune(n, f, p, pilot_n=1 << 14)
    assert t2 == t
    # iterative estimate under the tuned configuration matches the oracle
    c1 = W.immigration_death()
    n1 = ctx.network(c1)
    f1 = ctx.formula(n1, W.C1_FORMULA)
    r = ctx.estimate(n1, f1, B.params(confidence=0.95, half_width=0.01, seed=1))
    o = oracle.estimate(c1, W.C1_FORMULA, confidence=0.95, eps=0.01, seed=1)
    assert (r["n"], r["successes"], r["events"]) == (o["n"], o["successes"], o["events"])
    ctx.set_waves_per_cu(0)
    ctx.set_kernel_occupancy(0)
    ctx.set_specialization(B.SPECIALIZE_AUTO)


@SPECULATE
def test_mixed_batch_matches_oracle(ctx, speculate):
    """A launch of models of different structure and size (Michaelis-Menten
    rate sets and small random networks), each with its own Fig. 2 rule:
    every job's n, successes, events and truncations equal the oracle's
    iterative estimate on the same streams."""
    B = _B()
    models = []
    for k, rr in enumerate(W.mm_sweep(6, seed=31)):
        models.append((W.michaelis_menten(*rr), W.MM_COMPANION_FORMULA, 0))
    for q in range(3):
        rn = W.random_network(8 + 4 * q, 4 * (8 + 4 * q), seed=77 + q)
        models.append((rn, W.nested_until_formula(rn, 20), 3000))
    keep, jobs = [], []
    for k, (net, text, cap) in enumerate(models):
        nh = ctx.network(net)
        fh = ctx.formula(nh, text)
        keep.append((nh, fh))
        jobs.append((nh, fh, B.params(confidence=0.95, half_width=0.05, seed=5, model_id=k, max_events=cap,
                                      speculate=speculate)))
    res = ctx.estimate_batch(jobs)
    assert ctx.last_kernel() == B.KERNEL_GENERIC
    for k, ((net, text, cap), r) in enumerate(zip(models, res)):
        o = oracle.estimate(net, text, confidence=0.95, eps=0.05, seed=5, model_id=k, max_events=cap)
        got = (r["n"], r["successes"], r["events"], r["truncated"], r["batches"])
        want = (o["n"], o["successes"], o["events"], o["truncated"], len(o["bounds"]))
        assert got == want, (k, got, want)
        assert (r["lo"], r["hi"]) == (o["lo"], o["hi"])


def test_watchdog_and_cancel_stop_cleanly(ctx):
    """A tiny watchdog stops a long launch with SMC_E_TIMEOUT (the kernel sees
    the host's stop word and exits), a cancel from another thread gives
    SMC_E_CANCELLED, and the context stays usable afterwards."""
    import threading
    B = _B()
    net = W.c3_network()
    nh = ctx.network(net)
    fh = ctx.formula(nh, W.c3_formula(net))
    long_run = B.params(fixed_n=32768, seed=1, max_events=W.C3_CAP)
    ctx.set_watchdog(0.05)
    try:
        with pytest.raises(B.SmcError) as e:
            ctx.estimate(nh, fh, long_run)
        assert e.value.code == -7            # SMC_E_TIMEOUT
    finally:
        ctx.set_watchdog(120)
    timer = threading.Timer(0.1, ctx.cancel)
    timer.start()
    try:
        with pytest.raises(B.SmcError) as e:
            ctx.estimate(nh, fh, long_run)
        assert e.value.code == -6            # SMC_E_CANCELLED
    finally:
        timer.cancel()
    small = W.immigration_death()
    n1 = ctx.network(small)
    f1 = ctx.formula(n1, W.C1_FORMULA)
    r = ctx.estimate(n1, f1, B.params(fixed_n=4096, seed=1))
    o = oracle.estimate(small, W.C1_FORMULA, fixed_n=4096, seed=1)
    assert (r["n"], r["successes"], r["events"]) == (o["n"], o["successes"], o["events"])


# ---------------------------------------------------------------------------
# The batched sweep at its full configuration
# ---------------------------------------------------------------------------
def _c4_expected():
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    with open(os.path.join(here, "c4_expected.json")) as fh:
        doc = json.load(fh)
    arrays = np.load(os.path.join(here, "c4_trajectories.npz"))
    return doc, arrays


@pytest.fixture(scope="module")
def c4_run(ctx):
    """One launch of all 576 jobs, as the benchmark runs them."""
    B = _B()
    keep, jobs = [], []
    for net, text, kw in W.c4_jobs():
        nh = ctx.network(net)
        fh = ctx.formula(nh, text)
        keep.append((nh, fh))
        jobs.append((nh, fh, B.params(**kw)))
    print("c4: 576 jobs in one launch", flush=True)
    res = ctx.estimate_batch(jobs)
    return res, keep


def test_c4_every_job_matches_oracle(c4_run):
    """All 576 jobs of the sweep (512 Michaelis-Menten rate sets at +-0.01 and
    64 random networks): n, successes, events, truncations, batches and the
    Wilson interval equal the oracle's Fig. 2 estimates (stored by
    tests/golden/c4_expected.py)."""
    res, _ = c4_run
    doc, _ = _c4_expected()
    exp = doc["jobs"]
    assert len(exp) == len(res) == 576
    keys = ("n", "successes", "events", "truncated", "batches", "p_hat", "lo", "hi")
    bad = [(e["job"], {k: (r[k], e[k]) for k in keys if r[k] != e[k]}) for r, e in zip(res, exp)
           if any(r[k] != e[k] for k in keys)]
    assert not bad, bad[:5]
    assert all(r["status"] == 0 for r in res)


@WIDE_MODES
def test_c4_network_trajectories_match_oracle(ctx, mode):
    """Per-trajectory parity on eight of the sweep's random networks (8 to 128
    species), indices 0..1023 with each job's own stream, on the generic and
    the wide specialised kernel."""
    B = _B()
    doc, arrays = _c4_expected()
    jobs = W.c4_jobs()
    count = doc["per_trajectory_count"]
    for q in doc["per_trajectory_networks"]:
        net, text, kw = jobs[512 + q]
        nh = ctx.network(net)
        fh = ctx.formula(nh, text)
        p = B.params(**kw)
        _wide_mode(ctx, B, mode)
        try:
            print(f"case c4 network {q} ({net.label}) mode {mode}", flush=True)
            ev, vd, rs = ctx.trajectories(nh, fh, p, 0, count)
        finally:
            ctx.set_specialization(B.SPECIALIZE_AUTO)
        vr = (vd | (rs << 1)).astype(np.uint8)
        assert np.array_equal(vr, arrays[f"vr_{q}"]), (q, np.nonzero(vr != arrays[f"vr_{q}"])[0][:5])
        assert np.array_equal(ev, arrays[f"events_{q}"]), (q, np.nonzero(ev != arrays[f"events_{q}"])[0][:5])


# ---------------------------------------------------------------------------
# Several lanes per trajectory (generic kernels): the same results as one lane
# ---------------------------------------------------------------------------
_group_oracle = {}


def _group_case(name):
    if name == "c3":
        net = W.c3_network()
        return net, W.c3_formula(net), 1, W.C3_CAP, 1024
    S, seed, d, cap, count = {"s8": (8, 41, 5, 20000, 2000), "s20": (20, 42, 10, 20000, 2000),
                              "s128": (128, 7, 15, 20000, 140)}[name]
    net = W.random_network(S, 4 * S, seed=seed)
    return net, W.nested_until_formula(net, d), seed, cap, count


@pytest.mark.parametrize("lanes", [2, 4, 8, 16])
@pytest.mark.parametrize("name", ["s8", "s20", "c3", "s128"])
def test_lane_group_trajectory_parity(ctx, name, lanes):
    """Per-trajectory (events, verdict, reason) with 2..16 lanes per
    trajectory equal the oracle's (the canonical sequential prefix is kept)."""
    B = _B()
    net, text, seed, cap, count = _group_case(name)
    n = ctx.network(net)
    f = ctx.formula(n, text)
    model = 0 if name == "c3" else 2       # the C3 expectation is model 0's
    p = B.params(seed=seed, model_id=model, max_events=cap, lanes=lanes)
    print(f"case lanes {lanes} network {name} trajectories {count}", flush=True)
    ev, vd, rs = ctx.trajectories(n, f, p, 0, count)
    assert ctx.last_kernel() == B.KERNEL_GENERIC_GROUPED
    if name == "c3":
        oev, ovd, ors = (a[:count] for a in _c3_expected(net, text))
    else:
        if name not in _group_oracle:
            _group_oracle[name] = oracle.trajectories(net, oracle.parse(text, net), 0, count, seed=seed, model_id=2,
                                                      max_events=cap)
        oev, ovd, ors = _group_oracle[name]
    assert np.array_equal(rs, ors), np.nonzero(rs != ors)[0][:5]
    assert np.array_equal(vd, ovd), np.nonzero(vd != ovd)[0][:5]
    assert np.array_equal(ev, oev), np.nonzero(ev != oev)[0][:5]


@pytest.mark.parametrize("lanes", [4, 16])
def test_lane_groups_in_the_batched_sweep(ctx, lanes):
    """The whole batched sweep with its random networks on lane groups (the
    Michaelis-Menten jobs keep one lane) gives the oracle's estimates for all
    576 jobs."""
    B = _B()
    doc, _ = _c4_expected()
    keep, jobs = [], []
    for net, text, kw in W.c4_jobs():
        nh = ctx.network(net)
        fh = ctx.formula(nh, text)
        keep.append((nh, fh))
        jobs.append((nh, fh, B.params(lanes=lanes, **kw)))
    print(f"c4 with {lanes} lanes per network trajectory", flush=True)
    res = ctx.estimate_batch(jobs)
    assert ctx.last_kernel() == B.KERNEL_GENERIC_GROUPED
    keys = ("n", "successes", "events", "truncated", "batches", "p_hat", "lo", "hi")
    bad = [(e["job"], {k: (r[k], e[k]) for k in keys if r[k] != e[k]}) for r, e in zip(res, doc["jobs"])
           if any(r[k] != e[k] for k in keys)]
    assert not bad, bad[:5]


def test_lane_group_settings(ctx):
    B = _B()
    with pytest.raises(B.SmcError):
        ctx.set_lanes_per_trajectory(3)
    net = W.immigration_death()
    n = ctx.network(net)
    f = ctx.formula(n, W.C1_FORMULA)
    with pytest.raises(B.SmcError):
        ctx.estimate(n, f, B.params(fixed_n=64, lanes=5))
    # networks of at most four channels always run one lane per trajectory
    ctx.set_lanes_per_trajectory(8)
    try:
        r = ctx.estimate(n, f, B.params(fixed_n=4096, seed=1))
        assert ctx.last_kernel() in (B.KERNEL_SPECIALIZED, B.KERNEL_GENERIC_SMALL)
    finally:
        ctx.set_lanes_per_trajectory(0)
    o = oracle.estimate(net, W.C1_FORMULA, fixed_n=4096, seed=1)
    assert (r["n"], r["successes"], r["events"]) == (o["n"], o["successes"], o["events"])


# ---------------------------------------------------------------------------
# Tree-ordered sums over a lane group (SMC_TREE_SUMS): the statistical contract
# ---------------------------------------------------------------------------
def _mismatch_bound(count):
    # a draw lands within a few ulps of a re-associated boundary with
    # probability of order M 2^-50 per event: in these runs, practically never
    return max(1, count // 1000)


@pytest.mark.parametrize("lanes", [2, 4, 8, 16])
@pytest.mark.parametrize("name", ["s8", "s20", "c3", "s128"])
def test_tree_sums_trajectory_agreement(ctx, name, lanes):
    """With tree-ordered sums, per-trajectory (events, verdict, reason) equal
    the oracle's on the same random numbers, apart from at most one trajectory
    in a thousand (a draw within ulps of a boundary)."""
    B = _B()
    net, text, seed, cap, count = _group_case(name)
    n = ctx.network(net)
    f = ctx.formula(n, text)
    model = 0 if name == "c3" else 2
    p = B.params(seed=seed, model_id=model, max_events=cap, lanes=lanes, tree_sums=True)
    print(f"case tree lanes {lanes} network {name} trajectories {count}", flush=True)
    ev, vd, rs = ctx.trajectories(n, f, p, 0, count)
    assert ctx.last_kernel() == B.KERNEL_GENERIC_TREE
    if name == "c3":
        oev, ovd, ors = (a[:count] for a in _c3_expected(net, text))
    else:
        if name not in _group_oracle:
            _group_oracle[name] = oracle.trajectories(net, oracle.parse(text, net), 0, count, seed=seed, model_id=2,
                                                      max_events=cap)
        oev, ovd, ors = _group_oracle[name]
    differ = (ev != oev) | (vd != ovd) | (rs != ors)
    print(f"  trajectories that differ from the oracle: {int(differ.sum())} of {count}", flush=True)
    assert int(differ.sum()) <= _mismatch_bound(count), np.nonzero(differ)[0][:5]


_TREE_STAT_JOBS = (537, 553, 575)   # batched-sweep networks of 356, 292 and 188 channels


@pytest.mark.parametrize("job", _TREE_STAT_JOBS)
def test_tree_sums_distribution(ctx, job):
    """Independent random numbers: the satisfaction probability and the mean
    event count of 400000 tree-summed trajectories agree with 20000 oracle
    trajectories of another seed (two-sample tests at the 99.9% level)."""
    B = _B()
    net, text, kw = W.c4_jobs()[job]
    nh = ctx.network(net)
    fh = ctx.formula(nh, text)
    n_gpu, n_or = 400000, 20000
    p = B.params(seed=9001, model_id=kw["model_id"], max_events=kw["max_events"], lanes=8, tree_sums=True)
    print(f"case tree distribution job {job} ({net.label})", flush=True)
    ev, vd, _ = ctx.trajectories(nh, fh, p, 0, n_gpu)
    assert ctx.last_kernel() == B.KERNEL_GENERIC_TREE
    oev, ovd, _ = oracle.trajectories(net, oracle.parse(text, net), 0, n_or, seed=77, model_id=kw["model_id"],
                                      max_events=kw["max_events"])
    z = 3.2905   # two-sided 99.9%
    p1, p2 = vd.mean(), ovd.mean()
    pool = (vd.sum() + ovd.sum()) / (n_gpu + n_or)
    se = math.sqrt(pool * (1 - pool) * (1 / n_gpu + 1 / n_or))
    assert abs(p1 - p2) <= z * se, (p1, p2, se)
    e1, e2 = ev.astype(np.float64), oev.astype(np.float64)
    se_e = math.sqrt(e1.var(ddof=1) / n_gpu + e2.var(ddof=1) / n_or)
    assert abs(e1.mean() - e2.mean()) <= z * se_e, (e1.mean(), e2.mean(), se_e)


def test_tree_sums_in_the_batched_sweep(ctx):
    """The batched sweep with its random networks on 16-lane groups with tree
    sums: every job's estimate equals the oracle's, apart from at most two jobs,
    whose estimates then lie within the oracle's interval."""
    B = _B()
    doc, _ = _c4_expected()
    keep, jobs = [], []
    for net, text, kw in W.c4_jobs():
        nh = ctx.network(net)
        fh = ctx.formula(nh, text)
        keep.append((nh, fh))
        jobs.append((nh, fh, B.params(lanes=16, tree_sums=True, **kw)))
    print("c4 with 16 lanes per network trajectory, tree sums", flush=True)
    res = ctx.estimate_batch(jobs)
    assert ctx.last_kernel() == B.KERNEL_GENERIC_TREE
    keys = ("n", "successes", "events", "truncated", "batches", "p_hat", "lo", "hi")
    bad = [(e["job"], r, e) for r, e in zip(res, doc["jobs"]) if any(r[k] != e[k] for k in keys)]
    print(f"  jobs that differ from the oracle: {len(bad)}", flush=True)
    assert len(bad) <= 2, [b[0] for b in bad]
    for _, r, e in bad:
        assert e["lo"] <= r["p_hat"] <= e["hi"], (r, e)


def test_tree_sums_must_agree_within_a_call(ctx):
    B = _B()
    net = W.random_network(20, 80, seed=42)
    text = W.nested_until_formula(net, 10)
    n = ctx.network(net)
    f = ctx.formula(n, text)
    a = B.params(fixed_n=256, lanes=4, tree_sums=True, max_events=20000)
    b = B.params(fixed_n=256, lanes=4, max_events=20000)
    with pytest.raises(B.SmcError):
        ctx.estimate_batch([(n, f, a), (n, f, b)])
    # one lane per trajectory: the flag has no effect, results are the exact ones
    r1 = ctx.estimate(n, f, B.params(fixed_n=512, lanes=1, tree_sums=True, max_events=20000))
    r0 = ctx.estimate(n, f, B.params(fixed_n=512, lanes=1, max_events=20000))
    assert (r1["n"], r1["successes"], r1["events"]) == (r0["n"], r0["successes"], r0["events"])


def test_autotune_batch_keeps_the_estimates(ctx):
    """smc_autotune_batch on the batched sweep picks lanes per trajectory and
    waves per CU from pilots; the sweep then runs under that choice and gives
    the oracle's estimates for all 576 jobs; a second call returns the
    recorded choice without pilots."""
    B = _B()
    doc, _ = _c4_expected()
    keep, jobs = [], []
    for net, text, kw in W.c4_jobs():
        nh = ctx.network(net)
        fh = ctx.formula(nh, text)
        keep.append((nh, fh))
        jobs.append((nh, fh, B.params(**kw)))
    print("autotune the batched sweep", flush=True)
    tune = ctx.autotune_batch(jobs, pilot_widen=2.0)
    print(f"  {tune}", flush=True)
    assert tune["lanes"] in (1, 2, 4, 8, 16) and tune["waves_per_cu"] in (8, 16, 32)
    # the widest sweep network needs 8 lanes: requests of 2 and 4 run as 8 and are not timed
    assert 3 <= tune["candidates"] <= 5 and 0.0 < tune["seconds"] <= tune["default_seconds"]
    assert tune["lanes"] in (1, 8, 16)
    assert ctx.autotune_batch(jobs, pilot_widen=2.0) == tune
    res = ctx.estimate_batch(jobs)
    expect = B.KERNEL_GENERIC if tune["lanes"] == 1 else B.KERNEL_GENERIC_GROUPED
    assert ctx.last_kernel() == expect
    keys = ("n", "successes", "events", "truncated", "batches", "p_hat", "lo", "hi")
    bad = [(e["job"], {k: (r[k], e[k]) for k in keys if r[k] != e[k]}) for r, e in zip(res, doc["jobs"])
           if any(r[k] != e[k] for k in keys)]
    assert not bad, bad[:5]
    # jobs that fix their own lanes keep them (the same signature: the tuned
    # launch shape applies, the lanes do not)
    if tune["lanes"] > 1:
        jobs1 = [(nh, fh, B.params(**dict(kw, lanes=1))) for (nh, fh), (_, _, kw) in zip(keep, W.c4_jobs())]
        res1 = ctx.estimate_batch(jobs1)
        assert ctx.last_kernel() == B.KERNEL_GENERIC
        assert [(r["n"], r["successes"]) for r in res1] == [(e["n"], e["successes"]) for e in doc["jobs"]]


# ---------------------------------------------------------------------------
# Trace programs: formulas outside the compact monitors, decided on the
# recorded states; per-trajectory results must equal the oracle's
# ---------------------------------------------------------------------------
TRACE_CASES = [
    ("window-not-at-0", W.immigration_death, "F[0,10](G[1,2](X>=65))", {"max_events": 5000}),
    ("resp-lower", W.immigration_death, "G[0,10](X<=60 | F[1,2](X>=70))", {"max_events": 5000}),
    ("X-over-X", W.isomerization, "X[0,0.1](X[0,0.1](A<=48))", {"max_events": 5000}),
    ("temporal-left", W.immigration_death, "(F[0,1](X>=5)) U[0,5] (X>=30)", {"max_events": 5000}),
    ("three-levels", W.immigration_death, "F[0,3](F[0,2](F[0,1](X>=40)))", {"max_events": 5000}),
    ("three-registers", W.isomerization,
     "G[0,1](F[0,0.5](A>=28)) & G[0,1](F[0,0.5](B>=12)) & G[0,1](F[0,1](A<=45))", {"max_events": 5000}),
    ("tmax", W.immigration_death, "F(G[1,2](X>=95))", {"max_events": 5000, "t_max": 30.0}),
    ("cap", W.immigration_death, "G[5,100](F[1,5](X>=90))", {"max_events": 150}),
    ("absorb", death_only, "F[0,100](G[1,5](X<=3))", {"max_events": 5000}),
    ("six-preds", W.isomerization, "(A>=1 & B<=45 & A+B>=2 & A>=10 & B<=40 & A<=50) U[0,2] (A<=18)",
     {"max_events": 5000}),
    # long trajectories (hundreds to thousands of states, decided late): many
    # tests that leave the formula open before the deciding one
    ("long-nested", W.michaelis_menten, "F[0,60]((S<=300) & F[1,5](P>=600))", {"max_events": 5000}),
    ("next-in-window", W.immigration_death, "F[5,60](X[0,0.2](X>=115) & G[0,1](X>=105))",
     {"max_events": 20000}),
    ("temporal-both", W.immigration_death, "(G[0,2](X<=118)) U[1,50] (F[0,1](X>=116))", {"max_events": 20000}),
    ("long-G", W.immigration_death, "G[10,60](F[1,3](X>=85))", {"max_events": 20000}),
]


@pytest.mark.parametrize("name,make,text,kw", TRACE_CASES, ids=[c[0] for c in TRACE_CASES])
def test_trace_program_parity(ctx, name, make, text, kw):
    B = _B()
    net = make()
    n = ctx.network(net)
    f = ctx.formula(n, text)
    for first, seed in ((0, 1), (123457, 99)):
        p = B.params(seed=seed, model_id=3, **kw)
        print(f"case trace {name} first {first} seed {seed}", flush=True)
        ev, vd, rs = ctx.trajectories(n, f, p, first, 2000)
        assert ctx.last_kernel() == B.KERNEL_GENERIC_TRACE
        oev, ovd, ors = oracle.trajectories(net, oracle.parse(text, net), first, 2000, seed=seed, model_id=3, **kw)
        assert np.array_equal(rs, ors), (name, np.nonzero(rs != ors)[0][:5])
        assert np.array_equal(vd, ovd), (name, np.nonzero(vd != ovd)[0][:5])
        assert np.array_equal(ev, oev), (name, np.nonzero(ev != oev)[0][:5])


def test_random_formulas_parity(ctx):
    """Seeded random nested formulas over X with bounded windows (every
    operator; tests/formula_gen.py), whatever the library compiles them to (a
    compact monitor or a trace program), per trajectory against the oracle:
    24 formulas, 600 trajectories each."""
    import random
    from formula_gen import random_formula
    B = _B()
    net = W.immigration_death()
    n = ctx.network(net)
    r = random.Random(31)
    kernels, done, tried = set(), 0, 0
    while done < 24:
        text = random_formula(r)
        tried += 1
        assert tried < 200
        try:
            f = ctx.formula(n, text)
        except B.SmcError as e:   # beyond the trace programs' node or predicate limits
            assert e.code == B.SMC_E_UNSUPPORTED, (text, e.code)
            continue
        print(f"case random formula {done}: {text}", flush=True)
        kw = {"max_events": 5000}
        ev, vd, rs = ctx.trajectories(n, f, B.params(seed=3, model_id=done, **kw), 0, 600)
        kernels.add(ctx.last_kernel())
        oev, ovd, ors = oracle.trajectories(net, oracle.parse(text, net), 0, 600, seed=3, model_id=done, **kw)
        assert np.array_equal(rs, ors), (text, np.nonzero(rs != ors)[0][:5])
        assert np.array_equal(vd, ovd), (text, np.nonzero(vd != ovd)[0][:5])
        assert np.array_equal(ev, oev), (text, np.nonzero(ev != oev)[0][:5])
        done += 1
    assert B.KERNEL_GENERIC_TRACE in kernels and len(kernels) > 1, kernels


def test_random_networks_and_formulas_parity(ctx):
    """Seeded random networks (2 to 12 species, S to 4 S reactions: uni- and
    bimolecular, homodimers, 0 to 2 products) under seeded random formulas over
    their species, per trajectory against the oracle on the default kernel
    (specialised where supported), the generic kernel and 4-lane groups."""
    import random
    from formula_gen import random_formula
    B = _B()
    r = random.Random(77)
    kw = {"max_events": 3000}
    for q in range(8):
        S = r.randint(2, 12)
        net = W.random_network(S, r.randint(S, 4 * S), seed=900 + q)
        nh = ctx.network(net)
        for rep in range(2):
            text = random_formula(r, names=net.names, lo=-40, hi=40,
                                  around={nm: int(v) for nm, v in zip(net.names, net.x0)})
            try:
                fh = ctx.formula(nh, text)
            except B.SmcError as e:   # beyond the trace programs' limits
                assert e.code == B.SMC_E_UNSUPPORTED, (text, e.code)
                continue
            mid = 10 * q + rep
            oev, ovd, ors = oracle.trajectories(net, oracle.parse(text, net), 0, 128, seed=4, model_id=mid, **kw)
            for mode in ("default", "generic", "lanes4"):
                print(f"case random network {net.label} formula {text} mode {mode}", flush=True)
                if mode == "generic":
                    ctx.set_specialization(B.SPECIALIZE_OFF)
                try:
                    p = B.params(seed=4, model_id=mid, lanes=4 if mode == "lanes4" else 0, **kw)
                    ev, vd, rs = ctx.trajectories(nh, fh, p, 0, 128)
                finally:
                    ctx.set_specialization(B.SPECIALIZE_AUTO)
                assert np.array_equal(rs, ors), (net.label, text, mode, np.nonzero(rs != ors)[0][:5])
                assert np.array_equal(vd, ovd), (net.label, text, mode, np.nonzero(vd != ovd)[0][:5])
                assert np.array_equal(ev, oev), (net.label, text, mode, np.nonzero(ev != oev)[0][:5])


def test_trace_programs_in_a_batch(ctx):
    """Trace programs and compact monitors in one iterative launch: every
    job's estimate equals the oracle's."""
    B = _B()
    keep, jobs, singles = [], [], []
    for q, (name, make, text, kw) in enumerate(TRACE_CASES[:6] + [("compact", W.immigration_death,
                                                                   W.C1_FORMULA, {"max_events": 5000})]):
        net = make()
        nh = ctx.network(net)
        fh = ctx.formula(nh, text)
        keep.append((nh, fh))
        jobs.append((nh, fh, B.params(seed=1, model_id=40 + q, half_width=0.05, **kw)))
        singles.append((net, text, 40 + q, kw))
    print("trace programs in a batch", flush=True)
    res = ctx.estimate_batch(jobs)
    assert ctx.last_kernel() == B.KERNEL_GENERIC_TRACE
    for (net, text, mid, kw), r in zip(singles, res):
        o = oracle.estimate(net, text, eps=0.05, seed=1, model_id=mid, **kw)
        assert (r["n"], r["successes"], r["events"], r["batches"]) == \
            (o["n"], o["successes"], o["events"], len(o["bounds"])), (mid, r, o)


def test_trace_program_limits(ctx):
    B = _B()
    net = W.immigration_death()
    n = ctx.network(net)
    f = ctx.formula(n, "F[0,3](F[0,2](F[0,1](X>=40)))")
    with pytest.raises(B.SmcError) as e:           # states are recorded up to the cap: one is needed
        ctx.estimate(n, f, B.params(fixed_n=64))
    assert e.value.code == B.SMC_E_INVALID
    with pytest.raises(B.SmcError) as e:
        ctx.estimate(n, f, B.params(fixed_n=64, max_events=(1 << 20) + 1))
    assert e.value.code == B.SMC_E_INVALID
    with pytest.raises(B.SmcError) as e:           # no record areas without allocation
        ctx.estimate_batch_noalloc([(n, f, B.params(fixed_n=64, max_events=100))])
    assert e.value.code == B.SMC_E_UNSUPPORTED
    # lanes and specialisation requests fall back to the trace-capable kernel
    r = ctx.estimate(n, f, B.params(fixed_n=4096, seed=2, max_events=5000, lanes=8))
    assert ctx.last_kernel() == B.KERNEL_GENERIC_TRACE
    o = oracle.estimate(net, "F[0,3](F[0,2](F[0,1](X>=40)))", fixed_n=4096, seed=2, max_events=5000)
    assert (r["n"], r["successes"], r["events"]) == (o["n"], o["successes"], o["events"])
