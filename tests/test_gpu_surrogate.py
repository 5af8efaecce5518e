"""GPU surrogate (BF16 MFMA MLP) against the FP64 oracle, and its gain.

Tolerances: the GPU accumulates in FP32 where the oracle uses FP64 (relative
error ~ K * 2^-24 for K <= 512 terms), and an FP32 activation lying within a
few FP32 ulps of a bfloat16 rounding boundary can round to the neighbouring
bfloat16 value (one element off by 2^-8 relative).  Gradients are compared
element by element on problems whose forward activations are exact (see
_dyadic_problem), each element against its own bound with the possible
rounding flips counted (_gradient_tolerance); on random Glorot weights, where
flips also reach the forward pass, losses agree to 1e-5 relative and each
gradient block to 1e-3 in relative Euclidean norm.
For the forward pass one such flip of a layer-2 unit k moves the logit by
|W3_k h2_k| 2^-8; with trained weights (|W3_k h2_k| up to ~0.1) that is up to
~4e-4 in the logit and ~1e-4 in p, so a trained network is held to 1e-3 at
the worst point and 1e-4 at all but 1 % of the points.
"""
import numpy as np
import pytest
from scipy.spatial import Delaunay

from oracle import mlp
from paper_0912_2551_amd import workloads as W

pytestmark = pytest.mark.gpu

BLOCKS = [("W1", 0, 768), ("b1", 768, 1024), ("W2", 1024, 1024 + 65536), ("b2", 66560, 66816),
          ("W3", 66816, 67072), ("b3", 67072, 67073)]


@pytest.fixture(scope="module")
def ctx():
    from paper_0912_2551_amd import binding as B
    c = B.Context(0)
    c.set_watchdog(120)
    yield c
    c.close()


def _sample(rng, n):
    x = (np.log10(np.asarray(W.MM_RATES))[None, :] + rng.uniform(-1, 1, size=(n, 3))).astype(np.float32)
    y = rng.uniform(0, 1, size=n).astype(np.float32)
    w = rng.integers(100, 10000, size=n).astype(np.float32)
    return x, y, w


U32 = 2.0 ** -24          # unit roundoff of FP32


def _bf16_spacing(v):
    """Spacing of the bfloat16 grid at |v| (8 significant bits)."""
    m, e = np.frexp(np.abs(np.asarray(v, dtype=np.float64)))
    return np.ldexp(1.0, e - 8)


def _dyadic_problem(rng, n):
    """A batch and weights on which every forward activation the GPU rounds
    to bfloat16 is computed exactly in FP32 as well as in FP64: inputs in
    {-2..2} with mean 0 and standard deviation 1 per coordinate (so the
    standardisation is exact), W1 in quarters, W2 and W3 in 1/256 steps,
    biases on coarse grids.  Then pre1 has at most 8 significant bits (h1 is
    exact in bfloat16), and the 256-term sums of pre2 are exact in FP32, so
    h2 rounds identically on both sides.  What remains inexact is the
    sigmoid, dz and everything after it."""
    cols = []
    for _ in range(3):
        k = n // 16
        col = np.array([-2] * k + [-1] * (4 * k) + [0] * (6 * k) + [1] * (4 * k) + [2] * k, dtype=np.float64)
        assert col.size == n and col.mean() == 0.0 and np.mean(col * col) == 1.0
        cols.append(rng.permutation(col))
    x = np.stack(cols, axis=1).astype(np.float32)
    H = mlp.H
    W1 = rng.integers(-8, 9, size=(H, 3)) / 4.0
    b1 = rng.integers(-16, 17, size=H) / 16.0
    W2 = rng.integers(-32, 33, size=(H, H)) / 256.0
    b2 = rng.integers(-1024, 1025, size=H) / 4096.0
    W3 = rng.integers(-16, 17, size=H) / 256.0
    b3 = rng.integers(-16, 17) / 16.0
    params = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3, [b3], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])
    y = rng.uniform(0, 1, size=n).astype(np.float32)
    w = rng.integers(100, 10000, size=n).astype(np.float32)
    return x, y, w, params


def _gradient_tolerance(params, x, y, w):
    """Per-element bound on |GPU gradient - oracle gradient| for a dyadic
    problem: FP32 accumulation (a K-term sum of products is off by at most
    (K + 1) u sum |terms|), the FP32 logit, sigmoid and dz, and, counted
    explicitly, the layer-2 errors d2 whose bfloat16 rounding can go either
    way (FP64 value within the FP32 error of a rounding midpoint): each such
    flip moves d2b by one bfloat16 spacing."""
    W1, b1, W2, b2, W3, b3, mu, sigma = mlp.unpack(params)
    f = mlp.forward(params, x.astype(np.float64))
    y = y.astype(np.float64)
    w = w.astype(np.float64)
    n = x.shape[0]
    wsum = w.sum()
    xb, h1, h2, p, z = f["xb"], f["h1"], f["h2"], f["p"], f["z"]
    m1 = f["pre1"] > 0.0
    m2 = f["pre2"] > 0.0
    zerr = 257 * U32 * (np.abs(h2) @ np.abs(W3) + abs(b3))
    perr = p * (1 - p) * zerr + 8 * U32
    dz = w * (p - y) / wsum
    dzerr = w / wsum * (perr + 4 * U32 * (np.abs(p) + np.abs(y))) + 4 * U32 * np.abs(dz)
    d2 = (dz[:, None] * W3[None, :]) * m2
    d2err = (dzerr[:, None] * np.abs(W3)[None, :]) * m2 + U32 * np.abs(d2)
    d2b = mlp.bf16(d2)
    # distance of d2 to the nearest midpoint between bfloat16 neighbours
    sp = _bf16_spacing(d2)
    lo_edge = np.floor(d2 / sp) * sp
    to_mid = np.abs(d2 - (lo_edge + 0.5 * sp))
    flip = (to_mid <= d2err) & (d2 != 0.0)
    dflip = np.where(flip, sp, 0.0)
    a = np.abs
    t_W3 = a(h2).T @ dzerr + (n + 1) * U32 * (a(h2).T @ a(dz))
    t_b3 = dzerr.sum() + (n + 1) * U32 * a(dz).sum()
    t_b2 = d2err.sum(axis=0) + (n + 1) * U32 * a(d2).sum(axis=0)
    t_W2 = dflip.T @ a(h1) + (n + 1) * U32 * (a(d2b).T @ a(h1))
    dh1err = dflip @ a(W2) + 257 * U32 * (a(d2b) @ a(W2))
    d1 = (d2b @ W2) * m1
    t_W1 = (dh1err * m1).T @ a(xb) + (n + 1) * U32 * (a(d1).T @ a(xb))
    t_b1 = (dh1err * m1).sum(axis=0) + (n + 1) * U32 * a(d1).sum(axis=0)
    tol = mlp.pack_grads(t_W1, t_b1, t_W2, t_b2, t_W3, t_b3)
    return 2.0 * tol, int(flip.sum())


@pytest.mark.parametrize("n", [512, 96])
def test_gradients_match_oracle_elementwise(ctx, n):
    """Every gradient element within its own bound (see _gradient_tolerance)
    of the FP64 oracle's on the same bfloat16 operands; the flips of d2's
    rounding are counted, not hidden in a norm."""
    from paper_0912_2551_amd import binding as B
    rng = np.random.default_rng(100 + n)
    x, y, w, params = _dyadic_problem(rng, n)
    s = B.Surrogate(ctx)
    s.set_params(params.astype(np.float32))
    assert np.array_equal(s.get_params().astype(np.float64), params)
    loss, g = s.gradients(x, y, w)
    oloss, og = mlp.loss_and_grads(params, x.astype(np.float64), y.astype(np.float64), w.astype(np.float64))
    tol, flips = _gradient_tolerance(params, x, y, w)
    err = np.abs(g.astype(np.float64) - og)
    bad = np.nonzero(err > tol)[0]
    print(f"n={n}: d2 rounding flips possible at {flips} elements; max err/tol {np.max(err / np.maximum(tol, 1e-300)):.3f}")
    assert bad.size == 0, [(int(i), float(g[i]), float(og[i]), float(tol[i])) for i in bad[:8]]
    assert abs(loss - oloss) <= 1e-5 * abs(oloss)
    # the bound is tight enough to matter: far below the gradient's own size
    assert np.median(tol / np.maximum(np.abs(og), 1e-30)) < 1e-2


def test_adam_step_matches_oracle(ctx):
    """One GPU Adam step (FP32) against the oracle's FP64 step (Kingma and Ba,
    Algorithm 1) from the oracle's gradient.  The step is lr g / (|g| + eps)
    at t = 1; elements whose gradient is within its error bound of zero can
    take either sign and are counted, not compared."""
    from paper_0912_2551_amd import binding as B
    rng = np.random.default_rng(7)
    x, y, w, params = _dyadic_problem(rng, 512)
    s = B.Surrogate(ctx)
    s.set_params(params.astype(np.float32))
    lr = 1e-3
    s.train(x, y, w, steps=1, lr=lr)
    got = s.get_params().astype(np.float64)
    # training sets the standardisation from x: mean 0, deviation 1 here
    assert np.array_equal(got[mlp.N_WEIGHTS:], params[mlp.N_WEIGHTS:])
    _, og = mlp.loss_and_grads(params, x.astype(np.float64), y.astype(np.float64), w.astype(np.float64))
    tol, _ = _gradient_tolerance(params, x, y, w)
    exp, _, _ = mlp.adam_step(params[:mlp.N_WEIGHTS], og, np.zeros(mlp.N_WEIGHTS), np.zeros(mlp.N_WEIGHTS), 1, lr)
    eps = 1e-8
    sure = np.abs(og) > tol
    # step sensitivity to g: lr eps / (|g| + eps)^2; the step itself passes
    # through about eight FP32 roundings (moments, bias corrections, square
    # root, eps, divide, lr), and w - step through one more
    step_tol = (lr * eps / (np.abs(og) + eps) ** 2 * tol + 12 * U32 * lr
                + 2 * U32 * np.abs(params[:mlp.N_WEIGHTS]))
    d = np.abs(got[:mlp.N_WEIGHTS] - exp)
    assert np.all(d[sure] <= step_tol[sure]), np.nonzero(d[sure] > step_tol[sure])[0][:8]
    # unsure elements still move by at most lr
    assert np.all(np.abs(got[:mlp.N_WEIGHTS] - params[:mlp.N_WEIGHTS])[~sure] <= lr * (1 + 1e-6) + 4 * U32)
    assert sure.mean() > 0.8


@pytest.mark.parametrize("n", [512, 77])
def test_gradients_match_oracle(ctx, n):
    from paper_0912_2551_amd import binding as B
    rng = np.random.default_rng(n)
    x, y, w = _sample(rng, n)
    params = mlp.init_params(11, mu=tuple(np.log10(W.MM_RATES)), sigma=(0.57, 0.57, 0.57))
    s = B.Surrogate(ctx)
    s.set_params(params.astype(np.float32))
    loss, g = s.gradients(x, y, w)
    oloss, og = mlp.loss_and_grads(params, x.astype(np.float64), y.astype(np.float64), w.astype(np.float64))
    assert abs(loss - oloss) <= 1e-5 * abs(oloss)
    for name, a, b in BLOCKS:
        ref = og[a:b]
        err = np.linalg.norm(g[a:b] - ref) / max(np.linalg.norm(ref), 1e-30)
        assert err <= 1e-3, (name, err)


def test_query_matches_oracle_forward(ctx):
    from paper_0912_2551_amd import binding as B
    rng = np.random.default_rng(5)
    params = mlp.init_params(12, mu=tuple(np.log10(W.MM_RATES)), sigma=(0.57, 0.57, 0.57))
    s = B.Surrogate(ctx)
    s.set_params(params.astype(np.float32))
    # 5000 points take the per-tile kernel; from 32768 on the persistent one
    # that stages W2 in LDS (where the device has the LDS for it): exactly
    # 1024 full tiles, one point more (a tile of one), and a ragged 50000
    for count in (5000, 32768, 32769, 50000):
        x = W.surrogate_queries(count, seed=5)
        p, use = s.query(x)
        ref = mlp.forward(params, x.astype(np.float64))["p"]
        dp = np.abs(p - ref)
        assert dp.max() <= 1e-3 and np.mean(dp > 1e-4) <= 0.01, (count, dp.max())
        assert np.median(dp) <= 1e-6
        assert not use.any()            # no training hull yet: never confident


def test_training_fits_and_gate(ctx):
    from paper_0912_2551_amd import binding as B
    rng = np.random.default_rng(9)
    x = (np.log10(np.asarray(W.MM_RATES))[None, :] + rng.uniform(-1, 1, size=(512, 3))).astype(np.float32)
    c = x - np.log10(np.asarray(W.MM_RATES))
    y = (1.0 / (1.0 + np.exp(-(3 * c[:, 2] - 1.5 * c[:, 0])))).astype(np.float32)
    w = np.full(512, 1000.0, dtype=np.float32)
    s = B.Surrogate(ctx, seed=3)
    losses = s.train(x, y, w, steps=600, lr=2e-3)
    ent = float(np.mean(-(y * np.log(y) + (1 - y) * np.log(1 - y))))
    assert losses[-1] < losses[0]
    assert losses[-1] - ent < 0.1 * (losses[0] - ent)      # most of the excess loss is gone
    params = s.get_params().astype(np.float64)
    q = W.surrogate_queries(40000, seed=10)
    p, use = s.query(q)
    ref = mlp.forward(params, q.astype(np.float64))["p"]
    dp = np.abs(p - ref)
    assert dp.max() <= 1e-3
    assert np.mean(dp > 1e-4) <= 0.01
    inside = Delaunay(x.astype(np.float64)).find_simplex(q.astype(np.float64)) >= 0
    expect = inside & (np.abs(ref - 0.5) >= 0.05)
    borderline = np.abs(np.abs(ref - 0.5) - 0.05) <= dp + 1e-6
    hull = s.hull().astype(np.float64)
    margin_in = np.min(hull[:, 3][None, :] - q.astype(np.float64) @ hull[:, :3].T, axis=1)
    borderline |= np.abs(margin_in) < 1e-5
    assert np.array_equal(use[~borderline], expect[~borderline])
    assert 0.2 < use.mean() < 0.95


def test_confirm_rule(ctx):
    """smc_surrogate_confirm: an answer stands only if every trial fell on its
    side; refused points stay refused; host and device arrays agree."""
    import torch
    from paper_0912_2551_amd import binding as B
    s = B.Surrogate(ctx, seed=1)
    p = np.array([0.01, 0.01, 0.99, 0.99, 0.3, 0.7, 0.01, 0.99, 0.5], dtype=np.float32)
    gate = np.array([1, 1, 1, 1, 1, 1, 0, 0, 1], dtype=bool)
    succ = np.array([0, 1, 64, 63, 0, 64, 5, 0, 64], dtype=np.uint64)
    trials = np.array([64, 64, 64, 64, 64, 64, 64, 64, 64], dtype=np.uint64)
    want = np.array([1, 0, 1, 0, 1, 1, 0, 0, 1], dtype=bool)
    assert np.array_equal(s.confirm(p, gate, succ, trials), want)
    # no trials: nothing stands
    assert not s.confirm(p, gate, succ * 0, trials * 0).any()
    with pytest.raises(B.SmcError):
        s.confirm(p, gate, trials + 1, trials)
    dp = torch.tensor(p, device="cuda")
    du = torch.tensor(gate.astype(np.uint8), device="cuda")
    ds = torch.tensor(succ.astype(np.int64), device="cuda")
    dt = torch.tensor(trials.astype(np.int64), device="cuda")
    s.confirm_device(dp, ds, dt, len(p), du)
    assert np.array_equal(du.cpu().numpy().astype(bool), want)


def test_surrogate_gain_over_plain_smc(ctx):
    """Rate sweep of the Michaelis-Menten model under the companion formula
    (p runs from ~0 to ~1 across the box): after training, the gate is
    calibrated on held-out plain-SMC estimates (no held-out answer more than
    eps outside its interval), and each answer is confirmed by 64 plain-SMC
    trajectories.  On fresh query points the surrogate answers a large share, the largest distance of an answer outside the point's own
    plain-SMC Wilson interval stays within 2 eps, and the SMC work left over
    is a fraction of what plain SMC spends on the same queries."""
    from paper_0912_2551_amd import binding as B
    eps, n_train, n_cal, n_query, margin = 0.03, 384, 1024, 512, 0.05
    text = W.MM_COMPANION_FORMULA
    keep = []

    def run(rate_sets, seed):
        jobs = []
        for k, rr in enumerate(rate_sets):
            nh = ctx.network(W.michaelis_menten(*rr))
            fh = ctx.formula(nh, text)
            keep.append((nh, fh))
            jobs.append((nh, fh, B.params(half_width=eps, seed=seed, model_id=k)))
        return ctx.estimate_batch(jobs)

    train = W.mm_sweep(n_train, seed=21)
    res = run(train, 1)
    x = np.log10(train).astype(np.float32)
    y = np.array([r["p_hat"] for r in res], dtype=np.float32)
    w = np.array([r["n"] for r in res], dtype=np.float32)
    s = B.Surrogate(ctx, seed=4)
    losses = s.train(x, y, w, steps=2000, lr=2e-3)
    assert losses[-1] < losses[0]
    xc = W.surrogate_queries(n_cal, seed=23)
    cal = run(10.0 ** xc.astype(np.float64), 3)
    m, share = s.calibrate(xc, [r["lo"] for r in cal], [r["hi"] for r in cal], threshold=0.5, bound=eps,
                           min_margin=margin)
    assert margin <= m <= 0.5 and share > 0.3
    q = W.surrogate_queries(n_query, seed=22)
    p, gate = s.query(q, threshold=0.5, margin=margin)
    assert np.all(np.abs(p[gate] - 0.5) >= m)
    # 64 confirming trajectories per answered point, on a seed of their own
    ans = np.nonzero(gate)[0]
    probes = []
    for i in ans:
        nh = ctx.network(W.michaelis_menten(*(10.0 ** q[i].astype(np.float64))))
        fh = ctx.formula(nh, text)
        keep.append((nh, fh))
        probes.append((nh, fh, B.params(fixed_n=64, seed=5, model_id=int(i))))
    pr = ctx.estimate_batch(probes)
    succ = np.zeros(n_query, dtype=np.uint64)
    trials = np.zeros(n_query, dtype=np.uint64)
    succ[ans] = [r["successes"] for r in pr]
    trials[ans] = [r["n"] for r in pr]
    use = s.confirm(p, gate, succ, trials, threshold=0.5)
    assert not np.any(use & ~gate)
    plain = run(10.0 ** q.astype(np.float64), 2)
    plain_events = sum(r["events"] for r in plain)
    fallback_events = sum(r["events"] for r, u in zip(plain, use) if not u) + sum(r["events"] for r in pr)
    err = np.array([max(r["lo"] - pi, pi - r["hi"], 0.0) for r, pi, u in zip(plain, p, use) if u])
    print(f"margin={m:.3f} gate={gate.mean():.3f} use={use.mean():.3f} within={np.mean(err == 0):.3f} "
          f"max_err={err.max():.4f} work={fallback_events / plain_events:.3f}")
    assert use.mean() > 0.3
    assert err.max() <= 2 * eps
    assert fallback_events < 0.8 * plain_events
    # a query at another threshold than the calibrated one is refused
    _, use2 = s.query(q, threshold=0.3, margin=margin)
    assert not use2.any()
