"""Pins of the FP64 network reference (oracle.conv_ref) against things other
than itself: scipy's 2-D correlation, identities of the layers, adjoint
relations, central finite differences of whole losses, and the closed form
of Adam's first step."""
import numpy as np
import pytest
from scipy import signal

from oracle import conv_ref as cr


def _fd_grad(f, x, h=1e-6, idx=None):
    """Central differences of scalar f at the entries idx of x."""
    g = np.zeros(len(idx))
    for t, i in enumerate(idx):
        xp = x.copy()
        xm = x.copy()
        xp.flat[i] += h
        xm.flat[i] -= h
        g[t] = (f(xp) - f(xm)) / (2 * h)
    return g


@pytest.mark.parametrize("k", [1, 3, 5])
def test_conv2d_matches_scipy_correlate(k):
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, 1, 9, 7))
    w = rng.standard_normal((1, 1, k, k))
    y = cr.conv2d(x, w, np.zeros(1))
    ref = signal.correlate2d(x[0, 0], w[0, 0], mode="same", boundary="fill", fillvalue=0.0)
    assert np.allclose(y[0, 0], ref, rtol=0, atol=1e-13)


def test_conv2d_channels_sum_of_correlations():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 6, 5))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = cr.conv2d(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(signal.correlate2d(x[n, c], w[o, c], mode="same") for c in range(3))
            assert np.allclose(y[n, o], ref, rtol=0, atol=1e-12)


def test_conv2d_delta_filter_is_identity():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 4, 5, 6))
    w = np.zeros((4, 4, 3, 3))
    for c in range(4):
        w[c, c, 1, 1] = 1.0
    assert np.array_equal(cr.conv2d(x, w, np.zeros(4)), x)


def test_conv2d_backward_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 5, 4))
    w = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    gy = rng.standard_normal((2, 2, 5, 4))
    gx, gw, gb = cr.conv2d_backward(x, w, gy)
    loss = lambda xx, ww, bb: float(np.sum(cr.conv2d(xx, ww, bb) * gy))
    ix = rng.choice(x.size, 12, replace=False)
    iw = rng.choice(w.size, 12, replace=False)
    assert np.allclose(_fd_grad(lambda v: loss(v, w, b), x, idx=ix), gx.flat[ix], rtol=1e-7, atol=1e-8)
    assert np.allclose(_fd_grad(lambda v: loss(x, v, b), w, idx=iw), gw.flat[iw], rtol=1e-7, atol=1e-8)
    assert np.allclose(_fd_grad(lambda v: loss(x, w, v), b, idx=range(2)), gb, rtol=1e-7, atol=1e-8)


def test_pool_and_upsample_are_adjoint_pairs():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((2, 3, 4, 6))
    big = rng.standard_normal((2, 3, 8, 12))
    # <up(a), big> = <a, up^T(big)>,  <pool(big), a> = <big, pool^T(a)>
    assert np.isclose(np.sum(cr.upsample2(a) * big), np.sum(a * cr.upsample2_backward(big)), rtol=1e-13)
    assert np.isclose(np.sum(cr.avgpool2(big) * a), np.sum(big * cr.avgpool2_backward(a)), rtol=1e-13)
    # pooling a constant-by-block image recovers the blocks
    assert np.allclose(cr.avgpool2(cr.upsample2(a)), a, rtol=0, atol=1e-15)


def test_relu_backward_masks_by_output():
    y = np.array([[-1.0, 0.0, 2.0]])
    g = np.array([[5.0, 6.0, 7.0]])
    assert np.array_equal(cr.relu_backward(cr.relu(y), g), np.array([[0.0, 0.0, 7.0]]))


def test_mse_gradient():
    rng = np.random.default_rng(5)
    p = rng.standard_normal((2, 3, 4, 4))
    t = rng.standard_normal((2, 3, 4, 4))
    loss, g = cr.mse(p, t)
    assert np.isclose(loss, np.mean((p - t) ** 2))
    idx = rng.choice(p.size, 10, replace=False)
    assert np.allclose(_fd_grad(lambda v: cr.mse(v, t)[0], p, idx=idx), g.flat[idx], rtol=1e-6, atol=1e-10)


def test_unet_gradient_finite_differences():
    """Whole-network loss gradient against central differences, every layer
    kind on the path (convolutions, ReLU, pooling, upsampling, skips)."""
    rng = np.random.default_rng(6)
    layers = cr.unet_layers(3, 2, 2)
    npar = cr.param_count(layers)
    params = 0.3 * rng.standard_normal(npar)
    # positive biases keep most ReLUs away from their kink at this scale
    o = 0
    for ci, co, k, _ in layers:
        o += co * ci * k * k
        params[o:o + co] = np.abs(params[o:o + co]) + 0.1
        o += co
    x = rng.standard_normal((2, 3, 8, 8))
    t = rng.standard_normal((2, 2, 8, 8))
    loss, g = cr.unet_loss_grad(params, x, t, layers)
    idx = rng.choice(npar, 40, replace=False)
    fd = _fd_grad(lambda v: cr.unet_loss_grad(v, x, t, layers)[0], params, h=1e-6, idx=idx)
    assert np.allclose(fd, g[idx], rtol=1e-5, atol=1e-9), np.max(np.abs(fd - g[idx]))


def test_unet_parameter_count_and_shapes():
    layers = cr.unet_layers(17, 8, 32)
    # 4928 + 9248 + 18496 + 36928 + 73856 + 3 * 147584 + 295040 + 147584 + 110656 + 36928 + 27680 + 9248 + 264
    assert cr.param_count(layers) == 1213608
    y, _ = cr.unet_forward(np.zeros(cr.param_count(cr.unet_layers(3, 2, 2))), np.ones((1, 3, 16, 16)),
                           cr.unet_layers(3, 2, 2))
    assert y.shape == (1, 2, 16, 16)


def test_adam_first_step_closed_form():
    """At t = 1 the bias-corrected moments are g and g^2, so the step is
    lr * g / (|g| + eps)."""
    rng = np.random.default_rng(7)
    p = rng.standard_normal(20)
    g = rng.standard_normal(20)
    p1, m, v = cr.adam_step(p, g, np.zeros(20), np.zeros(20), 1, 1e-3)
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
