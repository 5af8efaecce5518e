"""Pins for the oracle's surrogate MLP and for the library's hull routine.

- the exact (unquantised) backward pass against central finite differences of
  the FP64 loss: catches a dropped term, a wrong sign or a transposed operand;
- bfloat16 rounding against the definition (8 significant bits, ties to even)
  and against torch's float32 -> bfloat16 conversion;
- the library's host convex hull (no GPU needed) against scipy's Delaunay
  point location;
- the Adam step: its first step and any step under a constant gradient in
  closed form, and two steps worked out by hand.
"""
import numpy as np
import pytest
import torch
from scipy.spatial import Delaunay

from oracle import mlp


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2**-8, 1.0 + 2**-7, 1.0 + 3 * 2**-8, -3.14159, 1e-3, 0.0, 255.5, 257.0])
    r = mlp.bf16(v)
    assert r[0] == 1.0
    assert r[1] == 1.0                    # tie -> even
    assert r[2] == 1.0 + 2**-7
    assert r[3] == 1.0 + 2**-6            # tie -> even (upwards)
    assert r[6] == 0.0
    assert r[8] == 256.0                  # 257 needs 9 bits: tie -> even
    rng = np.random.default_rng(0)
    x = rng.normal(size=20000).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x.astype(np.float64)), ref)


def test_exact_gradients_against_finite_differences():
    rng = np.random.default_rng(1)
    params = mlp.init_params(3, mu=(-1.0, 0.0, 1.0), sigma=(0.5, 1.0, 2.0))
    x = rng.normal(size=(40, 3))
    y = rng.uniform(0, 1, size=40)
    w = rng.uniform(0.5, 2.0, size=40)
    loss, g = mlp.loss_and_grads(params, x, y, w, quantize=False)
    idx = list(rng.choice(mlp.N_WEIGHTS, size=60, replace=False)) + [mlp.N_WEIGHTS - 1, 0, 768, 1024]
    for i in idx:
        h = 1e-6
        pp = params.copy(); pp[i] += h
        pm = params.copy(); pm[i] -= h
        fd = (mlp.loss_and_grads(pp, x, y, w, False)[0] - mlp.loss_and_grads(pm, x, y, w, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-4 * abs(fd), (i, fd, g[i])


def test_library_hull_matches_scipy():
    from paper_0912_2551_amd import binding as B
    rng = np.random.default_rng(2)
    for n in (10, 100, 512):
        pts = rng.uniform(-1, 1, size=(n, 3)).astype(np.float32)
        planes = B.convex_hull(pts)
        assert planes.shape[0] >= 4
        q = rng.uniform(-1.2, 1.2, size=(20000, 3)).astype(np.float32)
        inside = (q.astype(np.float64) @ planes[:, :3].T.astype(np.float64) <= planes[:, 3] + 1e-6).all(axis=1)
        ref = Delaunay(pts.astype(np.float64)).find_simplex(q.astype(np.float64)) >= 0
        assert (inside != ref).sum() <= 2
        # every training point lies inside its own hull
        assert (pts.astype(np.float64) @ planes[:, :3].T <= planes[:, 3] + 1e-5).all()
    flat = np.zeros((20, 3), dtype=np.float32)
    flat[:, :2] = rng.uniform(size=(20, 2))
    assert B.convex_hull(flat).shape[0] == 0


def test_adam_first_step_and_constant_gradient():
    """From zero moments the bias corrections make the first step
    lr g / (|g| + eps) whatever beta1 and beta2 are; under a constant gradient
    the corrected moments stay g and g^2, so every step is that size."""
    g = np.array([3.0, -0.5, 1e-3, 0.0, -2e-9])
    w0 = np.array([1.0, 2.0, -1.0, 0.5, 0.0])
    lr, eps = 1e-2, 1e-8
    for b1, b2 in ((0.9, 0.999), (0.5, 0.75), (0.0, 0.0)):
        w, m, v = w0.copy(), np.zeros(5), np.zeros(5)
        for t in range(1, 8):
            w, m, v = mlp.adam_step(w, g, m, v, t, lr, b1, b2, eps)
            expect = w0 - t * lr * g / (np.abs(g) + eps)
            assert np.allclose(w, expect, rtol=1e-12, atol=1e-15), (b1, b2, t)


def test_adam_two_steps_by_hand():
    """g1 = 1, g2 = -3, beta1 = 1/2, beta2 = 3/4, eps = 0, lr = 1:
    step 1 moves by -1; then m2 = 1/4 - 3/2 = -5/4, m_hat = (-5/4)/(3/4) = -5/3,
    v2 = 3/16 + 9/4 = 39/16, v_hat = (39/16)/(7/16) = 39/7, so step 2 moves by
    (5/3) / sqrt(39/7)."""
    w, m, v = mlp.adam_step([0.0], [1.0], [0.0], [0.0], 1, 1.0, 0.5, 0.75, 0.0)
    assert w[0] == -1.0 and m[0] == 0.5 and v[0] == 0.25
    w, m, v = mlp.adam_step(w, [-3.0], m, v, 2, 1.0, 0.5, 0.75, 0.0)
    assert m[0] == -1.25 and v[0] == 2.4375
    assert abs(w[0] - (-1.0 + (5.0 / 3.0) / np.sqrt(39.0 / 7.0))) <= 1e-15
