"""Pins of the learned proposal's training step in the oracle (oracle/mlp.py):
Adam (Kingma & Ba, ICLR 2015, Algorithm 1: beta1 = 0.9, beta2 = 0.999,
eps = 1e-8) and the cosine learning-rate decay.

The three-step, two-parameter case below was worked out by hand from the
recurrences m_t = 0.9 m_{t-1} + 0.1 g_t, v_t = 0.999 v_{t-1} + 0.001 g_t^2,
m_hat = m_t / (1 - 0.9^t), v_hat = v_t / (1 - 0.999^t),
theta -= lr m_hat / (sqrt(v_hat) + 1e-8), at lr = 0.1:

parameter a, gradients 1, -1, 1 (so v_hat = 1 at every step):
  t = 1: m = 0.1, m_hat = 1                      theta = -0.1 / (1 + 1e-8)
  t = 2: m = -0.01, m_hat = -0.01 / 0.19 = -1/19  theta = -0.0947368411578948
  t = 3: m = 0.091, m_hat = 0.091 / 0.271         theta = -0.1283161766154594
parameter b, gradients 2, 0, 1:
  t = 1: m = 0.2, v = 0.004, m_hat = 2, v_hat = 4          theta = -0.0999999995
  t = 2: m = 0.18, v = 0.003996, m_hat = 18/19,
         v_hat = 0.003996 / 0.001999 = 1.9989994997...      theta = -0.1670058244397331
  t = 3: m = 0.262, v = 0.004992004, m_hat = 0.262 / 0.271,
         v_hat = 0.004992004 / 0.002997001 = 1.6656664445... theta = -0.2419155107912991
A dropped bias correction, a swapped beta, eps inside the square root or a
wrong sign each moves these numbers far beyond the tolerance.
"""
import numpy as np
import pytest

import su2_inputs
from oracle import cdf, mlp

HAND = {
    1: (-0.09999999900000002, -0.0999999995),
    2: (-0.0947368411578948, -0.1670058244397331),
    3: (-0.1283161766154594, -0.2419155107912991),
}


def test_adam_hand_computed_two_parameters_three_steps():
    theta = np.zeros(2)
    m = np.zeros(2)
    v = np.zeros(2)
    grads = [(1.0, 2.0), (-1.0, 0.0), (1.0, 1.0)]
    for t, g in enumerate(grads, start=1):
        theta, m, v = mlp.adam_step(theta, np.array(g), m, v, t, 0.1)
        np.testing.assert_allclose(theta, HAND[t], rtol=0, atol=1e-13)


def test_adam_constant_gradient_moves_by_the_learning_rate():
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2, so every step moves theta by lr g / (|g| + eps); g = 0 never moves."""
    g = np.array([3.0, -0.25, 0.0, 1e-3])
    theta, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    total = np.zeros(4)
    for t in range(1, 8):
        lr = mlp.cosine_lr(t, 7, 0.01, 0.001)
        theta, m, v = mlp.adam_step(theta, g, m, v, t, lr)
        total -= lr * g / (np.abs(g) + mlp.ADAM_EPS)
        np.testing.assert_allclose(theta, total, rtol=1e-12, atol=0)
    assert theta[2] == 0.0


def test_cosine_schedule_end_points():
    lr0, lr_min, T = 3e-3, 1e-5, 10
    assert mlp.cosine_lr(1, T, lr0, lr_min) == pytest.approx(lr0, rel=1e-15)
    assert mlp.cosine_lr(T // 2 + 1, T, lr0, lr_min) == pytest.approx(0.5 * (lr0 + lr_min), rel=1e-15)
    assert mlp.cosine_lr(T + 1, T, lr0, lr_min) == pytest.approx(lr_min, rel=1e-15)
    assert mlp.cosine_lr(T + 7, T, lr0, lr_min) == pytest.approx(lr_min, rel=1e-15)
    lrs = [mlp.cosine_lr(t, T, lr0, lr_min) for t in range(1, T + 2)]
    assert np.all(np.diff(lrs) < 0)


def test_training_steps_lower_the_loss():
    """A few oracle training steps on integrated targets lower the loss, and a
    zero learning rate leaves the parameters as they were."""
    alphas = su2_inputs.alpha_grid(128)
    target = cdf.log_widths(np.array([cdf.knots(a) for a in alphas]))
    theta0 = su2_inputs.mlp_init(1).astype(np.float64)
    theta, hist = mlp.train(theta0, alphas, target, 40, 3e-3, 1e-5)
    assert hist[-1] < 0.7 * hist[0]
    same, _ = mlp.train(theta0, alphas, target, 3, 0.0, 0.0)
    np.testing.assert_array_equal(same, theta0)
