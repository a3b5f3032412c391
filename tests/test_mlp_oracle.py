"""Pins the float64 MLP reference: hand-computed outputs, finite differences
of the loss for every parameter block, and Adam's closed-form first step."""
import numpy as np

from oracle import mlp_oracle as M


def test_layout_size():
    assert M.NPARAMS == 4 * 64 + 64 + 64 * 64 + 64 + 64 + 1


def test_forward_hand_computed():
    # W1 copies x0 into hidden unit 0 and -x1 into unit 1; W2 passes unit 0
    # to unit 5 and unit 1 to unit 6 (after adding b2); W3 weights them 2, 3.
    d = {n: np.zeros(s) for n, s in M.SIZES}
    d["W1"][0, 0] = 1.0
    d["W1"][1, 1] = -1.0
    d["b1"][2] = 0.5  # unit 2 is 0.5 for every input, unused downstream
    d["W2"][5, 0] = 1.0
    d["W2"][6, 1] = 1.0
    d["b2"][6] = -0.25
    d["W3"][5] = 2.0
    d["W3"][6] = 3.0
    d["b3"][0] = 0.125
    p = M.pack(d)
    x = np.array([[1.0, -2.0, 7.0, 9.0], [-3.0, 0.5, 0.0, 0.0], [0.25, -0.1, 1.0, 1.0]])
    # row 0: h1 = (1, 2, .5) -> z2_5 = 1, z2_6 = 2 - .25 -> y = 2 + 3*1.75 + .125
    # row 1: h1 = (0, 0, .5) -> z2_6 = -.25 -> relu 0 -> y = .125
    # row 2: h1 = (.25, .1) -> z2_6 = -.15 -> y = 2*.25 + .125
    want = [2 + 3 * 1.75 + 0.125, 0.125, 0.5 + 0.125]
    assert np.allclose(M.forward(p, x), want, rtol=0, atol=1e-15)


def test_gradient_matches_finite_differences():
    r = np.random.default_rng(5)
    p = M.init_params(3) + r.normal(0, 0.05, M.NPARAMS)
    x = r.normal(0, 1, (37, 4))
    t = r.normal(0, 1, 37)
    L, g = M.loss_and_grad(p, x, t)
    assert abs(L - M.loss(p, x, t)) < 1e-12
    h = 1e-6
    # every bias, and a sample of every weight block
    idx = list(range(0, 256, 7)) + list(range(256, 320)) + list(range(320, 320 + 4096, 61)) \
        + list(range(4416, 4480)) + list(range(4480, 4544)) + [4544]
    for i in idx:
        e = np.zeros(M.NPARAMS)
        e[i] = h
        fd = (M.loss(p + e, x, t) - M.loss(p - e, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_zero_loss_at_the_target():
    r = np.random.default_rng(1)
    p = M.init_params(1)
    x = r.normal(0, 1, (11, 4))
    L, g = M.loss_and_grad(p, x, M.forward(p, x))
    assert L == 0.0 and np.all(g == 0.0)


def test_adam_first_step_closed_form():
    # after one step m_hat = g and v_hat = g^2, so the update is lr*g/(|g|+eps)
    r = np.random.default_rng(2)
    p = r.normal(0, 1, M.NPARAMS)
    g = r.normal(0, 1, M.NPARAMS)
    lr = 1e-3
    p1, m, v = M.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_gradient_magnitude_bounds_and_equals_the_gradient_when_nothing_cancels():
    r = np.random.default_rng(6)
    p = M.init_params(2) + r.normal(0, 0.05, M.NPARAMS)
    x = r.normal(0, 1, (50, 4))
    t = r.normal(0, 1, 50)
    _, g = M.loss_and_grad(p, x, t)
    ga = M.grad_magnitude(p, x, t)
    assert np.all(ga >= np.abs(g) - 1e-12)
    # positive weights and inputs, targets <= 0: every term of every sum has
    # the same sign, so the magnitude is the gradient itself
    pp = np.abs(p)
    xp = np.abs(x)
    tn = -np.abs(t)
    _, g2 = M.loss_and_grad(pp, xp, tn)
    assert np.allclose(M.grad_magnitude(pp, xp, tn), g2, rtol=1e-12, atol=0)
    # margins: ReLU pre-activations relative to their terms, in [0, 1]
    m = M.relu_margin(p, x)
    assert m.shape == (50,) and np.all((m >= 0) & (m <= 1 + 1e-12))
