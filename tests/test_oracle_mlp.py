"""Pins for the oracle's learned scorer (O7) and dominance counts (O8).

* The float64 gradient against central finite differences (pure float64 mode).
* A hand-computed forward value, including the bfloat16 round-to-nearest-even
  points (a halfway case that rounds to even, one that rounds up).
* Monotonicity of g for non-negative weights on random comparable pairs.
* Adam's first step in closed form (-lr * g / (|g| + eps)) and the projection
  of weights (not biases) onto w >= 0.
* Dominance counts (Def. 2) on a chain (closed form) and, for uniform data, the
  expected count M * prod(1 - t_k), the dominance-region volume of Section 4.1.
"""
import numpy as np

import datagen


def _params(d, h, seed, nonneg=True):
    rng = np.random.default_rng(seed)
    n = h * d + h + h * h + h + h + 1
    P = rng.normal(0, 0.3, n)
    if nonneg:
        W1, rest = P[:h * d], None
        P[:h * d] = np.abs(P[:h * d])
        o = h * d + h
        P[o:o + h * h] = np.abs(P[o:o + h * h])
        o += h * h + h
        P[o:o + h] = np.abs(P[o:o + h])
    return P


def test_nparams(orc):
    assert orc.mlp_nparams(6, 64) == 4673


def test_gradient_finite_differences(orc):
    d, h = 4, 8
    P = _params(d, h, 1, nonneg=False)
    x = datagen.uniform(37, d, 2)
    y = np.random.default_rng(3).normal(0, 1, 37)
    loss, g = orc.mlp_loss_grad(P, d, h, x, y, round_mode=0)
    eps = 1e-4
    fd = np.zeros_like(P)
    for q in range(P.size):
        Pp, Pm = P.copy(), P.copy()
        Pp[q] += eps
        Pm[q] -= eps
        fd[q] = (orc.mlp_loss_grad(Pp, d, h, x, y, 0)[0] - orc.mlp_loss_grad(Pm, d, h, x, y, 0)[0]) / (2 * eps)
    assert np.max(np.abs(fd - g)) / np.max(np.abs(g)) < 1e-6
    # the loss itself is the mean squared error of the forward pass
    gx = orc.mlp_forward(P, d, h, x, round_mode=0)
    assert abs(loss - np.mean((gx - y) ** 2)) < 1e-12


def test_forward_hand_computed_bf16(orc):
    """d = 1, h = 2. W1 = [1, 1], b1 = [1/256, 3/512]: z1 = x + b1.
    At x = 1: 1 + 2^-8 is halfway between bf16 neighbours 1 and 1 + 2^-7 -> rounds to
    even (1.0); 1 + 3*2^-9 rounds up to 1 + 2^-7. W2 = I, b2 = 0, w3 = [1, 1], b3 = 0.5."""
    P = np.array([1.0, 1.0, 1 / 256, 3 / 512, 1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 1.0, 1.0, 0.5])
    x = np.array([[1.0]], np.float32)
    assert orc.mlp_forward(P, 1, 2, x, round_mode=0)[0] == (1 + 1 / 256) + (1 + 3 / 512) + 0.5
    assert orc.mlp_forward(P, 1, 2, x, round_mode=1)[0] == 1.0 + (1 + 1 / 128) + 0.5
    # ReLU: x = 0 with negative biases gives b3
    P2 = P.copy()
    P2[2:4] = -1.0
    assert orc.mlp_forward(P2, 1, 2, np.array([[0.0]], np.float32), round_mode=1)[0] == 0.5


def test_monotone_for_nonneg_weights(orc):
    d, h = 6, 16
    P = _params(d, h, 7)
    P[h * d:h * d + h] -= 1.0   # biases may be anything
    x = datagen.uniform(2000, d, 8)
    y = np.minimum(1, x + np.random.default_rng(9).random(x.shape).astype(np.float32) * 0.1)
    for rm in (0, 1):
        gx = orc.mlp_forward(P, d, h, x, rm)
        gy = orc.mlp_forward(P, d, h, y.astype(np.float32), rm)
        assert (gx <= gy + 1e-12).all()


def test_adam_first_step_closed_form(orc):
    d, h = 2, 3
    n = orc.mlp_nparams(d, h)
    P = np.full(n, 0.5)
    grad = np.linspace(-1, 1, n)
    m, v = np.zeros(n), np.zeros(n)
    lr, eps = 0.01, 1e-8
    orc.mlp_adam(P, m, v, grad, d, h, lr, 1, eps=eps)
    want = 0.5 - lr * grad / (np.abs(grad) + eps)
    # projection: weight entries clipped at 0 (none here: 0.5 - 0.01 > 0)
    assert np.allclose(P, want, rtol=0, atol=1e-15)
    # a large step pushes weights negative -> clipped; biases stay negative
    P = np.full(n, 0.001)
    m, v = np.zeros(n), np.zeros(n)
    orc.mlp_adam(P, m, v, np.ones(n), d, h, 0.1, 1)
    W1 = slice(0, h * d)
    b1 = slice(h * d, h * d + h)
    W2 = slice(h * d + h, h * d + h + h * h)
    b2 = slice(h * d + h + h * h, h * d + 2 * h + h * h)
    w3 = slice(h * d + 2 * h + h * h, h * d + 3 * h + h * h)
    assert (P[W1] == 0).all() and (P[W2] == 0).all() and (P[w3] == 0).all()
    assert (P[b1] < 0).all() and (P[b2] < 0).all() and P[-1] < 0


def test_domcount_chain_and_duplicates(orc):
    v = np.arange(20, dtype=np.float32)
    x = np.stack([v, v])
    sample = np.arange(20, dtype=np.uint32)
    dc = orc.domcount(x, sample)
    assert dc.tolist() == list(range(19, -1, -1))
    # a duplicate is not dominated by its copy
    x2 = np.array([[0.5, 0.5, 0.7], [0.5, 0.5, 0.2]], np.float32)
    assert orc.domcount(x2, np.arange(3, dtype=np.uint32)).tolist() == [0, 0, 0]


def test_domcount_region_volume(orc):
    """E[dc(t)] = M * prod_k (1 - t_k) for a uniform sample (Section 4.1, V(DR(t)))."""
    x = datagen.uniform(40_000, 3, 12)
    rng = np.random.default_rng(2)
    sample = rng.choice(x.shape[1], 20_000, replace=False).astype(np.uint32)
    which = np.arange(200)
    dc = orc.domcount(x, sample, which)
    vol = np.prod(1 - x[:, which].astype(np.float64), axis=0)
    m = sample.size
    sd = np.sqrt(m * vol * (1 - vol)) + 1
    z = (dc - m * vol) / sd
    assert np.abs(z).max() < 5
    assert abs(z.mean()) < 1.5   # the 200 counts share one sample, so they are correlated
