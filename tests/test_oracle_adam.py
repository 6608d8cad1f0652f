"""Pins of the oracle's Adam step (Kingma and Ba 2015, Algorithm 1), CPU only.

Properties of the algorithm, not of its code: the bias corrections make the
first step, and every step under a constant gradient, move each weight by
lr g / (|g| + eps) (a sign step of size ~lr); the update is invariant to a
positive scaling of the gradient when eps is negligible; a zero gradient
leaves the weights alone; and a gradient that flips sign after a steady run
moves the weight back only by the decayed first moment.  A dropped or wrong
bias correction, a swapped b1/b2 or a wrong sign fails one of them.
"""
import numpy as np

import oracle as O


def test_first_step_is_a_sign_step():
    rng = np.random.default_rng(3)
    w0 = rng.standard_normal(200)
    g = rng.standard_normal(200) * np.logspace(-3, 3, 200)
    opt = O.Adam(w0, lr=0.01)
    w1 = opt.step(g)
    assert np.allclose(w1 - w0, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_constant_gradient_gives_constant_steps():
    """With g fixed, m_hat = g and v_hat = g^2 at every step t (the bias
    corrections exactly undo the zero start)."""
    g = np.array([0.7, -2.5, 1e-3, -4e2])
    w0 = np.zeros(4)
    opt = O.Adam(w0, lr=0.05)
    prev = w0.copy()
    for t in range(1, 30):
        w = opt.step(g).copy()
        assert np.allclose(w - prev, -0.05 * g / (np.abs(g) + 1e-8), rtol=1e-10, atol=1e-14), t
        prev = w


def test_scale_invariance_and_zero_gradient():
    rng = np.random.default_rng(4)
    w0 = rng.standard_normal(50)
    gs = [rng.standard_normal(50) for _ in range(6)]
    a = O.Adam(w0, lr=1e-3, eps=0.0)
    b = O.Adam(w0, lr=1e-3, eps=0.0)
    for g in gs:
        wa = a.step(g)
        wb = b.step(1e4 * g)
    assert np.allclose(wa, wb, rtol=1e-12, atol=1e-15)
    c = O.Adam(w0, lr=1e-3)
    assert np.array_equal(c.step(np.zeros(50)), w0)


def test_sign_flip_after_steady_run():
    """After t steps of g = +1 and one step of g = -1, m = b1^(t+1) - ... :
    m_{t+1} = b1 (1 - b1^t) - (1 - b1) and v_{t+1} = 1 - b2^(t+1) (|g| = 1
    throughout), so v_hat = 1 and the last step is -lr m_hat / (1 + eps)."""
    t, b1, b2, lr = 5, 0.9, 0.999, 0.1
    opt = O.Adam(np.zeros(1), lr=lr, b1=b1, b2=b2)
    for _ in range(t):
        w_before = opt.step(np.ones(1)).copy()
    w = opt.step(-np.ones(1))
    m = b1 * (1.0 - b1 ** t) - (1.0 - b1)
    m_hat = m / (1.0 - b1 ** (t + 1))
    assert np.isclose(w[0] - w_before[0], -lr * m_hat / (1.0 + 1e-8), rtol=1e-12)
    assert m_hat > 0   # the weight keeps moving down: momentum outlasts one reversed gradient
