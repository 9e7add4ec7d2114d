"""Pins of the oracle's training step on cached features: gradients against central finite
differences of the loss, Adam's first step in closed form, and the loss falling on a problem
whose exact solution exists.  CPU only."""
import numpy as np

from oracle import train
from paper_2607_10280_amd import inputs


def problem(seed, nb=5, m=4, out=7):
    rng = np.random.Generator(np.random.PCG64(seed))
    pauli = rng.uniform(-1, 1, size=(nb, m, 15))
    a, b, d, w, bias = inputs.readout_params(m, out, seed + 1, w_std=0.3)
    bias = rng.uniform(-0.1, 0.1, size=out)
    target = rng.uniform(-1, 1, size=(nb, out))
    return pauli, [a, b, d, w, bias], target


def test_gradients_match_finite_differences():
    pauli, params, target = problem(1)
    _, *grads = train.gradients(pauli, *params, target)
    h = 1e-6
    for pi, (p, g) in enumerate(zip(params, grads)):
        flat = p.reshape(-1)
        for k in range(0, flat.size, max(1, flat.size // 7)):
            old = flat[k]
            flat[k] = old + h
            lp = train.loss(pauli, *params, target)
            flat[k] = old - h
            lm = train.loss(pauli, *params, target)
            flat[k] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g.reshape(-1)[k]) <= 1e-7 * max(1.0, abs(fd)), (pi, k, fd, g.reshape(-1)[k])


def test_adam_first_step_closed_form():
    # from zero moments, m_hat = g and v_hat = g^2 after one step: p -= lr g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p, m, v = train.adam(np.ones(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    np.testing.assert_allclose(p, 1.0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_loss_falls_on_a_solvable_problem():
    pauli, params, _ = problem(2)
    _, _, target = train.forward(pauli, *problem(3)[1][:3], params[3], params[4])  # reachable
    state = [(np.zeros_like(p), np.zeros_like(p)) for p in params]
    first = None
    for step in range(1, 201):
        lval, params, state = train.train_step(pauli, tuple(params), state, target, step, 0.01, 0.01)
        first = lval if first is None else first
    assert lval < 0.05 * first
