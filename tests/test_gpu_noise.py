"""The noise and weight normalisation of Eq. (5) on the GPU against the CPU
oracle (oracle/noise.py), through the C ABI.  Uniform noise is bit-exact
(the same integer lattice and one FP64 product on both sides); Gaussian
noise within 1e-13 of its amplitude (the library's and numpy's log and cos
differ by an ulp or two); the noisy combination within the combination's
rounding bound plus the noise's own rounding; normalised weights within an
ulp-level bound of the oracle's quotients, with identical flags."""
import numpy as np
import pytest
import torch

import oracle
from oracle import noise as onz
from paper_2510_23221_amd import capi
from tests.gpu_util import to_np
from tests.test_gpu_parity import U64

pytestmark = pytest.mark.gpu


def _noise(kind, amp, seed, off=0):
    return capi.Noise(kind, amp, seed, off)


@pytest.mark.parametrize("n,m,off", [(4096 + 37, 9, 0), (1000, 5, 123456789012), (257, 1, 3)])
def test_uniform_noise_bit_exact(dev, n, m, off):
    E = to_np(capi.noise_fill(n, m, _noise(capi.NOISE_UNIFORM, 0.01, 2024, off), device=dev))
    E_ref = onz.noise(n, m, 1, 0.01, 2024, off)
    assert np.array_equal(E, E_ref)


def test_gaussian_noise_matches_oracle(dev):
    n, m = 3001, 7
    E = to_np(capi.noise_fill(n, m, _noise(capi.NOISE_GAUSSIAN, 0.002, 77, 10), device=dev))
    E_ref = onz.noise(n, m, 2, 0.002, 77, 10)
    assert np.abs(E - E_ref).max() <= 1e-13 * 0.002


@pytest.mark.parametrize("kind", [capi.NOISE_NONE, capi.NOISE_UNIFORM, capi.NOISE_GAUSSIAN])
def test_combine_noisy_and_pairs(dev, kind):
    rng = np.random.default_rng(80 + kind)
    s, m, n = 16, 150, 2048 + 19
    X = rng.standard_normal((s, n))
    C = rng.standard_normal((m, s))
    nzd = _noise(kind, 0.01, 5, 40)
    T = to_np(capi.combine_noisy(torch.as_tensor(X, device=dev), torch.as_tensor(C, device=dev), nzd))
    E_ref = onz.noise(n, m, kind, 0.01, 5, 40)
    T_ref = oracle.gemm(X, C) + E_ref
    bound = (s + 2) * U64 * (np.abs(C) @ np.abs(X) + np.abs(E_ref)) + 1e-13 * 0.01
    assert (np.abs(T - T_ref) <= bound * 1.01).all()


def test_normalize_weights_matches_oracle(dev):
    rng = np.random.default_rng(90)
    mu = rng.standard_normal((500, 32))
    mu[17] = 0.0
    mu[40] = 1e-7 * rng.standard_normal(32)
    thr = 1e-3 * np.sqrt(32)
    Cg = torch.as_tensor(mu.copy(), device=dev)
    flags = to_np(capi.normalize_weights(Cg, thr)).astype(np.int32)
    alpha_ref, flags_ref = onz.normalize_weights(mu, thr)
    assert np.array_equal(flags, flags_ref)
    alpha = to_np(Cg)
    # sums in the same order, one quotient each: within 2 ulp of |alpha|
    assert (np.abs(alpha - alpha_ref) <= 2 * U64 * np.abs(alpha_ref) + 1e-300).all()
