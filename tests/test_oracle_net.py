"""Pins of the FP64 network reference (no GPU): central finite differences on
every parameter group and on the input, the zero-padding boundary, a unit
impulse through one tap, and the Adam update against its closed form."""
import numpy as np
import pytest

from oracle import net


def _rand_params(rng, scale=0.3):
    return [(rng.standard_normal((27, co, ci)) * scale, rng.standard_normal(co) * 0.1) for ci, co in net.LAYERS]


def test_param_count():
    assert net.n_params() == 8241


def test_unit_impulse_tap_layout():
    """A single weight at tap (dz,dy,dx) = (0,0,+1) copies in[x+1] to out[x] (zero at the right edge)."""
    x = np.zeros((1, 3, 3, 4, 1))
    x[0, 1, 1, :, 0] = [1, 2, 3, 4]
    w = np.zeros((27, 1, 1))
    t = net.TAPS.index((0, 0, 1))
    w[t, 0, 0] = 1.0
    y = net.conv_fwd(x, w, np.zeros(1))
    np.testing.assert_array_equal(y[0, 1, 1, :, 0], [2, 3, 4, 0])
    assert y[0, 0].sum() == 0 and y[0, 2].sum() == 0


def test_finite_differences():
    rng = np.random.default_rng(0)
    params = _rand_params(rng)
    x = rng.standard_normal((2, 4, 3, 5, 2))
    target = rng.standard_normal((2, 4, 3, 5, 1))
    mask = (rng.random((2, 4, 3, 5, 1)) > 0.2).astype(float)
    loss, grads = net.loss_and_grads(params, x, target, mask)
    theta = net.pack(params)
    g = net.pack(grads)
    eps = 1e-6
    idx = rng.choice(theta.size, 60, replace=False)
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += eps
        tm[k] -= eps
        lp, _ = net.loss_and_grads(net.unpack(tp), x, target, mask)
        lm, _ = net.loss_and_grads(net.unpack(tm), x, target, mask)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (k, fd, g[k])


def test_input_gradient_finite_differences():
    """conv_bwd_data is the adjoint of conv_fwd: <conv(x), y> = <x, conv^T(y)>."""
    rng = np.random.default_rng(1)
    w = rng.standard_normal((27, 3, 2))
    x = rng.standard_normal((1, 4, 5, 3, 2))
    y = rng.standard_normal((1, 4, 5, 3, 3))
    lhs = (net.conv_fwd(x, w, np.zeros(3)) * y).sum()
    rhs = (x * net.conv_bwd_data(y, w)).sum()
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_adam_first_step_closed_form():
    """Step 1 with bias correction moves each weight by -lr * sign(g) (up to eps)."""
    g = np.array([0.5, -2.0, 1e-3])
    th, m, v = net.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(th, -0.01 * np.sign(g), rtol=1e-4)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.14159, 1e-30])
    r = net.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0            # tie rounds to even
    assert r[2] == 1.0 + 2 ** -7  # above the tie rounds up
    assert abs(r[3] + 3.140625) < 1e-12
