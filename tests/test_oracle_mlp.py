"""Pins of the warm-start network's FP64 oracle (CPU).

- every gradient agrees with a central finite difference of the loss
  (step 1e-6, relative error 1e-6) on a small network;
- Adam's first step moves every weight by exactly -lr * sign(g) (up to eps),
  the closed form of the published update at step 1;
- bfloat16 rounding keeps the 8 significant bits and rounds ties to even.
"""
import numpy as np
import pytest

from oracle import mlp as omlp


def _params(rng, dims):
    ps = []
    for k in range(3):
        ps.append(rng.uniform(-0.5, 0.5, (dims[k], dims[k + 1])))
        ps.append(rng.uniform(-0.1, 0.1, dims[k + 1]))
    return ps


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_match_finite_differences(seed):
    rng = np.random.default_rng(seed)
    dims = [12, 9, 7, 11]
    ps = _params(rng, dims)
    theta = rng.uniform(-1, 1, (5, 12))
    target = rng.uniform(-1, 1, (5, 11))
    L, gs = omlp.loss_and_grads(theta, target, ps)
    h = 1e-6
    for k, (p, g) in enumerate(zip(ps, gs)):
        for idx in [tuple(rng.integers(0, s) for s in p.shape) for _ in range(6)]:
            q = [x.copy() for x in ps]
            q[k][idx] += h
            Lp, _ = omlp.loss_and_grads(theta, target, q)
            q[k][idx] -= 2 * h
            Lm, _ = omlp.loss_and_grads(theta, target, q)
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-6 * max(1e-3, abs(g[idx])) + 1e-9, (k, idx)


def test_relu_gates_the_gradient():
    """A hidden unit that is off for every sample gets no gradient into its
    incoming weights."""
    rng = np.random.default_rng(3)
    ps = _params(rng, [12, 4, 4, 3])
    ps[1][2] = -100.0                      # unit 2 of the first layer never fires
    theta = rng.uniform(-1, 1, (6, 12))
    _, gs = omlp.loss_and_grads(theta, rng.uniform(-1, 1, (6, 3)), ps)
    assert np.all(gs[0][:, 2] == 0.0) and gs[1][2] == 0.0


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    w = rng.uniform(-1, 1, 50)
    g = rng.uniform(-1, 1, 50)
    w1, m1, v1 = omlp.adam(w, np.zeros(50), np.zeros(50), g, 1, lr=1e-3)
    assert np.allclose(w1, w - 1e-3 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -3.14159, 0.0], np.float32)
    r = omlp.bf16_round(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: to even (1); 1 + 3 * 2^-8 -> 1 + 2^-6
    assert list(r[:4]) == [1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6]
    assert abs(r[4] - (-3.140625)) < 1e-12 and r[5] == 0.0


def test_store_rounding_identity_and_effect():
    """store=None and store=identity agree exactly; bfloat16 storage moves
    the gradients by a few per cent at most on a random network."""
    rng = np.random.default_rng(7)
    ps = _params(rng, [12, 16, 16, 20])
    theta, target = rng.uniform(-1, 1, (8, 12)), rng.uniform(-1, 1, (8, 20))
    L0, g0 = omlp.loss_and_grads(theta, target, ps)
    L1, g1 = omlp.loss_and_grads(theta, target, ps, store=lambda a: np.asarray(a, np.float64))
    assert L0 == L1 and all(np.array_equal(a, b) for a, b in zip(g0, g1))
    L2, g2 = omlp.loss_and_grads(theta, target, ps, store=omlp.bf16_round)
    assert abs(L2 - L0) <= 1e-2 * L0
    for a, b in zip(g2, g0):
        assert np.linalg.norm(a - b) <= 0.1 * np.linalg.norm(b)
