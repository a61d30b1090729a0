"""Parity of the learned-start network kernels against the FP64 reference
(oracle.conv_ref), through the C ABI.

Tolerances are forward-error bounds of FP32 accumulation: an output summing
k products is within gamma_k |w| |x| of the exact sum of the same (BF16
rounded) weights and inputs, gamma_k ~ k 2^-24.  The network as a whole is
compared by relative Frobenius error (ReLU kinks make single entries
discontinuous)."""
import numpy as np
import pytest
import torch

from oracle import conv_ref as cr
from paper_2510_23221_amd import capi, synth
from tests.gpu_util import rel_fro

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _bf16(w):
    return torch.as_tensor(w, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def _np(t):
    return t.detach().to(torch.float64).cpu().numpy()


@pytest.mark.parametrize("mode,K,relu", [(0, 3, True), (0, 1, False), (1, 3, True), (2, 3, True), (2, 1, False)])
@pytest.mark.parametrize("H,W", [(20, 36), (8, 8)])
def test_conv_forward_matches_oracle(dev, mode, K, relu, H, W):
    rng = np.random.default_rng(100 + mode * 10 + K)
    N, Ca, Cb, Co = 2, 5, (3 if mode == 2 else 0), 37  # Co spans two channel tiles, ragged
    if mode == 0:
        A = rng.standard_normal((N, Ca, H, W))
        xin = A
    elif mode == 1:
        A = rng.standard_normal((N, Ca, 2 * H, 2 * W))
        xin = cr.avgpool2(A)
    else:
        A = rng.standard_normal((N, Ca, H // 2, W // 2))
    B = rng.standard_normal((N, Cb, H, W)) if mode == 2 else None
    if mode == 2:
        xin = np.concatenate([cr.upsample2(A), B], axis=1)
    w = _bf16(rng.standard_normal((Co, Ca + Cb, K, K)))
    b = rng.standard_normal(Co).astype(np.float32).astype(np.float64)
    A32 = A.astype(np.float32).astype(np.float64)
    if mode == 0:
        xin = A32
    elif mode == 1:
        xin = cr.avgpool2(A32)
    else:
        xin = np.concatenate([cr.upsample2(A32), B.astype(np.float32).astype(np.float64)], axis=1)
    y = capi.nn_conv2d(_dev(A), capi.to_bf16_bits(_dev(w)), _dev(b), B=None if B is None else _dev(B), mode=mode,
                       relu=relu)
    ref = cr.conv2d(xin, w, b)
    if relu:
        ref = cr.relu(ref)
    bound = (Ca + Cb) * K * K * 2 * U32 * cr.conv2d(np.abs(xin), np.abs(w), np.abs(b)) + 1e-30
    if mode == 1:  # the 2 x 2 average is rounded in FP32 (two additions and a scaling)
        bound += 4 * U32 * cr.conv2d(cr.avgpool2(np.abs(A32)), np.abs(w), np.zeros(Co))
    assert (np.abs(_np(y) - ref) <= bound).all(), np.max(np.abs(_np(y) - ref) / bound)


@pytest.mark.parametrize("K", [3, 1])
def test_conv_input_gradient_matches_oracle(dev, K):
    rng = np.random.default_rng(200 + K)
    N, Ci, Co, H, W = 2, 11, 9, 24, 40
    x = rng.standard_normal((N, Ci, H, W))
    w = _bf16(rng.standard_normal((Co, Ci, K, K)))
    g = rng.standard_normal((N, Co, H, W)).astype(np.float32).astype(np.float64)
    gx = capi.nn_conv2d(_dev(g), capi.to_bf16_bits(_dev(w)), transposed=True, out_channels=Ci)
    ref, _, _ = cr.conv2d_backward(x, w, g)
    # the adjoint of |w| applied to |g| sums the absolute values of the same products
    bound = Co * K * K * 2 * U32 * cr.conv2d_backward(x, np.abs(w), np.abs(g))[0] + 1e-30
    assert (np.abs(_np(gx) - ref) <= bound).all()


@pytest.mark.parametrize("mode,K", [(0, 3), (1, 3), (2, 3), (0, 1)])
def test_conv_filter_gradient_matches_oracle(dev, mode, K):
    rng = np.random.default_rng(300 + mode + K)
    N, Ca, Co, H, W = 3, 6, 10, 16, 40
    Cb = 4 if mode == 2 else 0
    if mode == 0:
        A = rng.standard_normal((N, Ca, H, W)).astype(np.float32).astype(np.float64)
        xin = A
    elif mode == 1:
        A = rng.standard_normal((N, Ca, 2 * H, 2 * W)).astype(np.float32).astype(np.float64)
        xin = cr.avgpool2(A)
    else:
        A = rng.standard_normal((N, Ca, H // 2, W // 2)).astype(np.float32).astype(np.float64)
    B = rng.standard_normal((N, Cb, H, W)).astype(np.float32).astype(np.float64) if mode == 2 else None
    if mode == 2:
        xin = np.concatenate([cr.upsample2(A), B], axis=1)
    g = rng.standard_normal((N, Co, H, W)).astype(np.float32).astype(np.float64)
    gw, gb = capi.nn_conv2d_wgrad(_dev(A), _dev(g), K, B=None if B is None else _dev(B), mode=mode)
    _, gw_ref, gb_ref = cr.conv2d_backward(xin, np.zeros((Co, Ca + Cb, K, K)), g)
    npix = N * H * W
    _, gw_abs, gb_abs = cr.conv2d_backward(np.abs(xin), np.zeros((Co, Ca + Cb, K, K)), np.abs(g))
    assert (np.abs(_np(gw) - gw_ref) <= (npix + 8) * U32 * gw_abs + 1e-12).all()
    assert (np.abs(_np(gb) - gb_ref) <= (npix + 8) * U32 * gb_abs + 1e-12).all()


def _tiny_net(rng, cin=3, cout=2, base=4):
    layers = cr.unet_layers(cin, cout, base)
    p = np.zeros(cr.param_count(layers))
    o = 0
    for ci, co, k, _ in layers:
        nw = co * ci * k * k
        p[o:o + nw] = rng.standard_normal(nw) * np.sqrt(2.0 / (ci * k * k))
        p[o + nw:o + nw + co] = 0.05 * rng.standard_normal(co)
        o += nw + co
    # what the GPU computes with: BF16 filters, FP32 biases
    q = np.empty_like(p)
    o = 0
    for ci, co, k, _ in layers:
        nw = co * ci * k * k
        q[o:o + nw] = _bf16(p[o:o + nw])
        q[o + nw:o + nw + co] = p[o + nw:o + nw + co].astype(np.float32)
        o += nw + co
    return layers, p, q


def test_unet_forward_and_gradient_match_oracle(dev):
    rng = np.random.default_rng(400)
    layers, p, q = _tiny_net(rng)
    net = capi.UNet(3, 2, 4, 16, 24, 3)
    assert net.nparams == p.size
    net.set_params(torch.as_tensor(p, dtype=torch.float32, device="cuda"))
    x = rng.standard_normal((3, 3, 16, 24)).astype(np.float32).astype(np.float64)
    t = rng.standard_normal((3, 2, 16, 24)).astype(np.float32).astype(np.float64)
    y = net.forward(_dev(x))
    y_ref, _ = cr.unet_forward(q, x, layers)
    assert rel_fro(_np(y), y_ref) <= 1e-5
    loss = net.gradient(_dev(x), _dev(t))
    loss_ref, g_ref = cr.unet_loss_grad(q, x, t, layers)
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref
    assert rel_fro(_np(net.grads), g_ref) <= 1e-3


def test_unet_infer_matches_oracle(dev):
    """The inference forward (convolutions on the BF16 matrix cores): against
    the oracle network with every convolution input rounded to BF16 it
    differs only by FP32 accumulation and the order of the sums; against the
    unrounded network by the fifteen input roundings (2^-9 each, 15 * 2^-9 <
    3e-2).  Ragged tiles in every direction: 24 x 40 pixels, 3..16
    channels."""
    rng = np.random.default_rng(410)
    layers, p, q = _tiny_net(rng)
    net = capi.UNet(3, 2, 4, 24, 40, 3)
    net.set_params(torch.as_tensor(p, dtype=torch.float32, device="cuda"))
    x = rng.standard_normal((3, 3, 24, 40)).astype(np.float32).astype(np.float64)
    y = _np(net.infer(_dev(x)))
    y_rounded, _ = cr.unet_forward(q, x, layers, round_input=_bf16)
    y_ref, _ = cr.unet_forward(q, x, layers)
    assert rel_fro(y, y_rounded) <= 1e-3, rel_fro(y, y_rounded)
    assert rel_fro(y, y_ref) <= 3e-2, rel_fro(y, y_ref)
    assert rel_fro(y_rounded, y_ref) > 0.0  # the rounding is there to be matched


def test_adam_step_matches_oracle(dev):
    rng = np.random.default_rng(500)
    layers, p, q = _tiny_net(rng)
    net = capi.UNet(3, 2, 4, 16, 16, 2)
    net.set_params(torch.as_tensor(p, dtype=torch.float32, device="cuda"))
    x = _dev(rng.standard_normal((2, 3, 16, 16)))
    t = _dev(rng.standard_normal((2, 2, 16, 16)))
    p32 = p.astype(np.float32).astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for step in (1, 2):
        net.gradient(x, t, want_loss=False)
        g = _np(net.grads)
        net.adam_step(1e-3)
        p32, m, v = cr.adam_step(p32, g, m, v, step, 1e-3)
        assert np.allclose(_np(net.params), p32, rtol=1e-5, atol=1e-7)
        p32 = _np(net.params)


def test_unet_training_reduces_loss(dev):
    """A few hundred Adam steps on one batch drive the loss well down (the
    kernels train the network, not only differentiate it)."""
    rng = np.random.default_rng(600)
    layers, p, q = _tiny_net(rng, cin=2, cout=1, base=8)
    net = capi.UNet(2, 1, 8, 32, 32, 4)
    net.set_params(torch.as_tensor(p, dtype=torch.float32, device="cuda"))
    x = rng.standard_normal((4, 2, 32, 32))
    # a smooth linear map of the input as the target
    t = cr.conv2d(cr.conv2d(x, np.full((1, 2, 3, 3), 0.1), np.zeros(1)), np.full((1, 1, 3, 3), 0.2), np.zeros(1))
    xd, td = _dev(x), _dev(t)
    first = net.gradient(xd, td)
    for _ in range(300):
        net.gradient(xd, td, want_loss=False)
        net.adam_step(2e-3)
    last = net.gradient(xd, td)
    assert last < 0.05 * first, (first, last)


def test_lstart_pack_and_unpack(dev):
    rng = np.random.default_rng(700)
    nx, ny, nz, m = 8, 16, 3, 5
    n = nx * ny * nz
    F = rng.standard_normal((m, n))
    F[2] = 0.0
    k = rng.uniform(1.0, 400.0, n)
    x, scale = capi.lstart_pack((nx, ny, nz), torch.as_tensor(F, device="cuda"), torch.as_tensor(k, device="cuda"),
                                2.0, 1.5, 0.25)
    xs, sc = _np(x), scale.cpu().numpy()
    assert np.allclose(sc, np.linalg.norm(F, axis=1) / np.sqrt(n), rtol=1e-14)
    for j in range(m):
        fj = F[j] / sc[j] if sc[j] > 0 else np.zeros(n)
        assert np.allclose(xs[j, :nz].reshape(-1), fj, rtol=1e-6, atol=1e-7)
        assert np.allclose(xs[j, nz:2 * nz].reshape(-1), (np.log(k) - 2.0) / 1.5, rtol=1e-5, atol=1e-5)
        assert np.all(xs[j, 2 * nz] == np.float32(0.25))
    T = rng.standard_normal((m, n))
    t = capi.lstart_pack_target(torch.as_tensor(T, device="cuda"), scale, 3.0)
    X0 = capi.lstart_unpack(t.reshape(m, nz, ny, nx), scale, 3.0)
    back = np.where(sc[:, None] > 0, T, 0.0)
    assert np.allclose(_np(X0), back, rtol=1e-6, atol=1e-12)


def test_jacobi_smooth_matches_oracle(dev):
    import oracle
    rng = np.random.default_rng(800)
    chip = synth.chip_stack(rng, 24, 16, 5)
    A = oracle.assemble_chip(chip)
    G = capi.HeatOperator.from_chip(chip, dev)
    B = rng.standard_normal((3, A.n))
    X = rng.standard_normal((3, A.n))
    diag = np.array([A.val[A.rowptr[i]:A.rowptr[i + 1]][A.col[A.rowptr[i]:A.rowptr[i + 1]] == i][0] for i in range(A.n)])
    ref = X.copy()
    for _ in range(3):  # odd count: the result comes back from the work block
        ref = ref + 0.6 * (B - oracle.apply_many(A, ref)) / diag
    Xd = torch.as_tensor(X, device=dev)
    capi.jacobi_smooth(G, torch.as_tensor(B, device=dev), Xd, 3, 0.6)
    assert rel_fro(_np(Xd), ref) <= 1e-13


@pytest.mark.parametrize("compute", [capi.F64, capi.F32])
def test_learned_start_cuts_block_iterations(dev, compute):
    """Train the network on pairs the pipeline generates for a few chips and
    start the block solve of unseen chips from its (smoothed) prediction:
    fewer block iterations than the zero start with the same smoothing, at
    the same FP64 residual target."""
    from paper_2510_23221_amd import lstart
    w = synth.workload(4, grid=(32, 32, 4), nchips=6, m=256, s=8)
    data = lstart.generate_pairs(w.chips, w.B, w.C, 1e-10, compute=capi.F64)
    norm = lstart.fit_normalizer(data)
    net = lstart.make_net(w.chips[0], base=8, max_batch=16, seed=0)
    log = lstart.train(net, data, norm, steps=2000, batch=16, lr=2e-3, seed=1, log_every=500)
    assert log[-1][1] < 0.05 * log[0][1], log
    chips, Bs = synth.learned_start_test_chips(4, (32, 32, 4), 8)
    recs = lstart.evaluate(net, norm, chips, Bs, 1e-8, compute=compute, smooth=20)
    zero = sum(r["zero_smooth_iters"] for r in recs)
    learned = sum(r["learned_iters"] for r in recs)
    assert all(r["learned_res"] <= 1e-8 and r["zero_smooth_res"] <= 1e-8 for r in recs)
    assert all(r["rejected"] == 0 for r in recs)
    assert learned < zero, [(r["zero_iters"], r["zero_smooth_iters"], r["learned_iters"]) for r in recs]


def test_grouped_prediction_matches_per_chip(dev):
    """Learned starts of several chips from one network pass equal the
    per-chip predictions (the network treats every image on its own)."""
    from paper_2510_23221_amd import lstart
    w = synth.workload(4, grid=(32, 32, 4), nchips=2, m=16, s=8)
    data = lstart.generate_pairs(w.chips, w.B, w.C, 1e-10, compute=capi.F64)
    norm = lstart.fit_normalizer(data)
    net = lstart.make_net(w.chips[0], base=8, max_batch=8, seed=0)
    big = lstart.make_net(w.chips[0], base=8, max_batch=24, seed=5)
    big.set_params(net.params)
    chips, Bs = synth.learned_start_test_chips(3, (32, 32, 4), 8)
    Gs = [capi.HeatOperator.from_chip(c, dev) for c in chips]
    ks = [torch.as_tensor(c.k, device=dev) for c in chips]
    Bds = [torch.as_tensor(B, device=dev) for B in Bs]
    grouped = lstart.predict_x0_group(big, norm, chips, ks, Bds, Gs, smooth=5)
    for chip, k, B, G, X0 in zip(chips, ks, Bds, Gs, grouped):
        ref = lstart.predict_x0(net, norm, chip, k, B, G, smooth=5)
        scale = float(ref.abs().max())
        assert scale > 0
        assert float((X0 - ref).abs().max()) <= 1e-6 * scale
