"""FP64 reference of the learned initial guess network (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of :mod:`oracle`: the GPU library
never imports it and shares no code with it.  The learned start is not part
of the paper; it is the project's addition for supplying the initial guess
X0 of the block solve (Sec. III-A solves A X = B from a starting block).

Plain numpy in float64: the definitions of 2-D cross-correlation with zero
"same" padding, ReLU, 2 x 2 average pooling, nearest 2x upsampling, the
mean squared error, their adjoints (backward passes), an encoder-decoder
composed of them, and the Adam update of Kingma and Ba (2015).  numpy's
tensordot is the only library primitive used (one channel contraction per
filter tap).  Pinned in ``tests/test_oracle_conv.py`` by finite differences,
scipy's correlate2d and adjoint identities.

Tensor layout: activations (N, C, H, W); filters (Cout, Cin, K, K); biases
(Cout,).  The network's flat parameter order is, for each convolution in
the order listed by :func:`unet_layers`: filter (Cout, Cin, K, K) row-major,
then bias (Cout,).
"""
from __future__ import annotations

import numpy as np


# ------------------------------------------------------------------ layers

def conv2d(x, w, b):
    """y[n,o,i,j] = b[o] + sum_{c,p,q} w[o,c,p,q] x[n,c,i+p-r,j+q-r], r = K//2,
    x taken as zero outside the image."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n, c, h, wd = x.shape
    co, ci, k, k2 = w.shape
    assert ci == c and k == k2 and k % 2 == 1
    r = k // 2
    xp = np.zeros((n, c, h + 2 * r, wd + 2 * r))
    xp[:, :, r:r + h, r:r + wd] = x
    y = np.zeros((n, co, h, wd))
    for p in range(k):
        for q in range(k):
            patch = xp[:, :, p:p + h, q:q + wd]                      # (n, c, h, w)
            y += np.tensordot(w[:, :, p, q], patch, axes=([1], [1])).transpose(1, 0, 2, 3)
    return y + np.asarray(b, dtype=np.float64)[None, :, None, None]


def conv2d_backward(x, w, gy):
    """Adjoint of conv2d with respect to x, w and b for the output
    gradient gy.  Returns (gx, gw, gb)."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    gy = np.asarray(gy, dtype=np.float64)
    n, c, h, wd = x.shape
    co, ci, k, _ = w.shape
    r = k // 2
    xp = np.zeros((n, c, h + 2 * r, wd + 2 * r))
    xp[:, :, r:r + h, r:r + wd] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for p in range(k):
        for q in range(k):
            patch = xp[:, :, p:p + h, q:q + wd]
            # dL/dw[o,c,p,q] = sum_{n,i,j} gy[n,o,i,j] x[n,c,i+p-r,j+q-r]
            gw[:, :, p, q] = np.tensordot(gy, patch, axes=([0, 2, 3], [0, 2, 3]))
            # dL/dx[n,c,i+p-r,j+q-r] += sum_o gy[n,o,i,j] w[o,c,p,q]
            gxp[:, :, p:p + h, q:q + wd] += np.tensordot(gy, w[:, :, p, q], axes=([1], [0])).transpose(0, 3, 1, 2)
    gx = gxp[:, :, r:r + h, r:r + wd].copy()
    gb = gy.sum(axis=(0, 2, 3))
    return gx, gw, gb


def relu(x):
    return np.maximum(x, 0.0)


def relu_backward(y, gy):
    """Gradient through ReLU given its output y."""
    return np.where(y > 0.0, gy, 0.0)


def avgpool2(x):
    n, c, h, w = x.shape
    return x.reshape(n, c, h // 2, 2, w // 2, 2).mean(axis=(3, 5))


def avgpool2_backward(gy):
    return np.repeat(np.repeat(gy, 2, axis=2), 2, axis=3) / 4.0


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=2), 2, axis=3)


def upsample2_backward(gy):
    n, c, h, w = gy.shape
    return gy.reshape(n, c, h // 2, 2, w // 2, 2).sum(axis=(3, 5))


def mse(pred, target):
    """Mean squared error over every element, and its gradient."""
    d = np.asarray(pred, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) at step t >= 1 with bias
    correction.  Returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------ network

def unet_layers(cin, cout, base):
    """Convolutions of the 4-level encoder-decoder as (cin, cout, k, relu).

    Levels at H, H/2, H/4 (two 3x3 convolutions each, encoder), a two-
    convolution bottleneck at H/8, and three decoder levels that each
    upsample, concatenate [upsampled, encoder skip] along channels and apply
    two 3x3 convolutions; a final 1x1 convolution without ReLU."""
    w1, w2, w3, w4 = base, 2 * base, 4 * base, 4 * base
    return [
        (cin, w1, 3, True), (w1, w1, 3, True),
        (w1, w2, 3, True), (w2, w2, 3, True),
        (w2, w3, 3, True), (w3, w3, 3, True),
        (w3, w4, 3, True), (w4, w4, 3, True),
        (w4 + w3, w3, 3, True), (w3, w3, 3, True),
        (w3 + w2, w2, 3, True), (w2, w2, 3, True),
        (w2 + w1, w1, 3, True), (w1, w1, 3, True),
        (w1, cout, 1, False),
    ]


def unpack(params, layers):
    """Flat parameter vector -> list of (filter, bias)."""
    out, o = [], 0
    for ci, co, k, _ in layers:
        nw = co * ci * k * k
        out.append((params[o:o + nw].reshape(co, ci, k, k), params[o + nw:o + nw + co]))
        o += nw + co
    assert o == params.size
    return out


def param_count(layers):
    return sum(co * ci * k * k + co for ci, co, k, _ in layers)


def unet_forward(params, x, layers, round_input=None):
    """Forward pass; returns (output, cache of every layer's input and output).
    round_input, if given, maps each convolution's input (after pooling,
    upsampling and concatenation) to the values the convolution multiplies:
    the inference variant that feeds the matrix cores BF16 passes a rounding
    to BF16 here."""
    wb = unpack(np.asarray(params, dtype=np.float64), layers)
    cache = []

    def conv(idx, a):
        w, b = wb[idx]
        y = conv2d(a if round_input is None else round_input(a), w, b)
        if layers[idx][3]:
            y = relu(y)
        cache.append((idx, a, y))
        return y

    a = conv(1, conv(0, x))
    s1 = a
    a = conv(3, conv(2, avgpool2(a)))
    s2 = a
    a = conv(5, conv(4, avgpool2(a)))
    s3 = a
    a = conv(7, conv(6, avgpool2(a)))
    a = conv(9, conv(8, np.concatenate([upsample2(a), s3], axis=1)))
    a = conv(11, conv(10, np.concatenate([upsample2(a), s2], axis=1)))
    a = conv(13, conv(12, np.concatenate([upsample2(a), s1], axis=1)))
    y = conv(14, a)
    return y, cache


def unet_backward(params, cache, gy, layers):
    """Gradient of a scalar loss with respect to the flat parameters, given
    dL/d(output) = gy and the forward cache.  Returns (grad params, grad x)."""
    wb = unpack(np.asarray(params, dtype=np.float64), layers)
    by_idx = {idx: (a, y) for idx, a, y in cache}
    grads = [None] * len(layers)

    def conv_back(idx, g):
        a, y = by_idx[idx]
        if layers[idx][3]:
            g = relu_backward(y, g)
        gx, gw, gb = conv2d_backward(a, wb[idx][0], g)
        grads[idx] = (gw, gb)
        return gx

    w1, w2, w3 = layers[1][1], layers[3][1], layers[5][1]
    g = conv_back(14, gy)
    g = conv_back(12, conv_back(13, g))                 # input: [up(dec2), s1]
    g_up, g_s1 = g[:, :layers[12][0] - w1], g[:, layers[12][0] - w1:]
    g = conv_back(10, conv_back(11, upsample2_backward(g_up)))
    g_up, g_s2 = g[:, :layers[10][0] - w2], g[:, layers[10][0] - w2:]
    g = conv_back(8, conv_back(9, upsample2_backward(g_up)))
    g_up, g_s3 = g[:, :layers[8][0] - w3], g[:, layers[8][0] - w3:]
    g = conv_back(6, conv_back(7, upsample2_backward(g_up)))
    g = avgpool2_backward(g) + g_s3
    g = conv_back(4, conv_back(5, g))
    g = avgpool2_backward(g) + g_s2
    g = conv_back(2, conv_back(3, g))
    g = avgpool2_backward(g) + g_s1
    gx = conv_back(0, conv_back(1, g))
    flat = np.concatenate([np.concatenate([gw.reshape(-1), gb]) for gw, gb in grads])
    return flat, gx


def unet_loss_grad(params, x, target, layers):
    """MSE loss of the network output against target, and its gradient."""
    y, cache = unet_forward(params, x, layers)
    loss, gy = mse(y, target)
    g, _ = unet_backward(params, cache, gy, layers)
    return loss, g
