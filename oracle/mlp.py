"""FP64 reference of the surrogate MLP (test infrastructure only).

TEST INFRASTRUCTURE ONLY.

Network 3 -> 256 -> 256 -> 1 with ReLU hidden units and a sigmoid output on
standardised log10 rate constants; loss = sum_i w_i BCE(p_i, y_i) / sum_i w_i
with soft targets y_i (estimated probabilities) and weights w_i (sample sizes).

With quantize=True the values that the GPU feeds to its matrix units are
rounded to bfloat16 (round to nearest, ties to even) at the same points:
the standardised inputs, the three weight matrices, both hidden activations
and the layer-2 error; everything else is exact FP64.  The gradient is then
the one the GPU computes (rounding treated as the identity in the backward
pass).  With quantize=False it is the exact gradient of the FP64 network,
which the tests check against finite differences.

Training uses Adam (Kingma and Ba, "Adam: a method for stochastic
optimization", ICLR 2015, Algorithm 1): adam_step below, in FP64.

Parameter vector layout: W1[256*3] (unit-major), b1[256], W2[256*256]
(output-major), b2[256], W3[256], b3, mu[3], sigma[3].
"""
from __future__ import annotations

import numpy as np

H = 256
N_WEIGHTS = H * 3 + H + H * H + H + H + 1


def bf16(v):
    """Round to the nearest bfloat16 value (8 significant bits), ties to even."""
    v = np.asarray(v, dtype=np.float64)
    m, e = np.frexp(v)                    # v = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * 3].reshape(H, 3); o += H * 3
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H]; o += H
    b3 = p[o]; o += 1
    mu = p[o:o + 3]; sigma = p[o + 3:o + 6]
    return W1, b1, W2, b2, W3, b3, mu, sigma


def pack_grads(dW1, db1, dW2, db2, dW3, db3):
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3, [db3]])


def forward(params, x, quantize=True):
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3, mu, sigma = unpack(params)
    xb = q((np.asarray(x, dtype=np.float64) - mu) / sigma)
    pre1 = xb @ q(W1).T + b1
    h1 = q(np.maximum(pre1, 0.0))
    pre2 = h1 @ q(W2).T + b2
    h2 = q(np.maximum(pre2, 0.0))
    z = h2 @ q(W3) + b3
    p = 1.0 / (1.0 + np.exp(-z))
    return dict(xb=xb, pre1=pre1, h1=h1, pre2=pre2, h2=h2, z=z, p=p)


def loss_and_grads(params, x, y, w=None, quantize=True):
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3, mu, sigma = unpack(params)
    y = np.asarray(y, dtype=np.float64)
    w = np.ones_like(y) if w is None else np.asarray(w, dtype=np.float64)
    f = forward(params, x, quantize)
    z, p = f["z"], f["p"]
    wsum = w.sum()
    # binary cross-entropy with logits
    ell = np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))
    loss = float((w * ell).sum() / wsum)
    dz = w * (p - y) / wsum
    dW3 = f["h2"].T @ dz
    db3 = dz.sum()
    d2 = (dz[:, None] * q(W3)[None, :]) * (f["pre2"] > 0.0)
    d2b = q(d2)
    dW2 = d2b.T @ f["h1"]
    db2 = d2.sum(axis=0)
    dh1 = d2b @ q(W2)
    d1 = dh1 * (f["pre1"] > 0.0)
    dW1 = d1.T @ f["xb"]
    db1 = d1.sum(axis=0)
    return loss, pack_grads(dW1, db1, dW2, db2, dW3, db3)


def init_params(seed, mu=(0.0, 0.0, 0.0), sigma=(1.0, 1.0, 1.0)):
    """Seeded Glorot-uniform weights (numpy generator), small random biases."""
    rng = np.random.default_rng(seed)

    def glorot(shape, fan_in, fan_out):
        a = np.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-a, a, size=shape)

    W1 = glorot((H, 3), 3, H)
    W2 = glorot((H, H), H, H)
    W3 = glorot((H,), H, 1)
    b1 = rng.uniform(-0.1, 0.1, H)
    b2 = rng.uniform(-0.1, 0.1, H)
    b3 = rng.uniform(-0.1, 0.1)
    p = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3, [b3], mu, sigma])
    return p.astype(np.float32).astype(np.float64)


def adam_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015, Algorithm 1) at step t >= 1:
    biased moment estimates m <- beta1 m + (1 - beta1) g and
    v <- beta2 v + (1 - beta2) g^2, their bias-corrected values
    m / (1 - beta1^t) and v / (1 - beta2^t), then
    w <- w - lr m_hat / (sqrt(v_hat) + eps).  Returns (w, m, v), FP64."""
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * (g * g)
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return w - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
