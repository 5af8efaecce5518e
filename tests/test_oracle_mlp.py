"""Pins for the oracle's surrogate MLP and for the library's hull routine.

- the exact (unquantised) backward pass against central finite differences of
  the FP64 loss: catches a dropped term, a wrong sign or a transposed operand;
- bfloat16 rounding against the definition (8 significant bits, ties to even)
  and against torch's float32 -> bfloat16 conversion;
- the library's host convex hull (no GPU needed) against scipy's Delaunay
  point location.
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
