"""Pins of the oracle's noise and weight normalisation (Eq. (5), Sec. III-B)
against facts independent of its code: the published known-answer vectors
of Philox4x32-10 (tests/golden), the exact lattice and the moments of the
uniform and Gaussian maps, the independence of a field's noise from how the
fields are split, and the closed form sum(alpha) = 1 of the normalised
weights."""
import os

import numpy as np
import pytest

from oracle import noise as nz

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([int(w, 16) for w in line.split()])
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for r in rows:
        out = nz.philox4x32_10(*r[:4], *r[4:6])
        assert [int(v) for v in out] == r[6:10]


def test_uniform_lattice_range_and_moments():
    a = 2.0 ** -6  # a power of two keeps E / a exact
    E = nz.noise(4000, 50, 1, a, seed=12345)
    assert E.shape == (50, 4000)
    assert (np.abs(E) < a).all()
    k = (E / a + 1.0) * 2.0 ** 52  # (2u + 1): an odd integer
    assert np.array_equal(k, np.round(k)) and (np.mod(k, 2) == 1).all()
    x = E.ravel() / a
    assert abs(x.mean()) < 5 * np.sqrt(1 / 3 / x.size)
    assert abs(x.var() - 1 / 3) < 0.01


def test_gaussian_moments():
    E = nz.noise(5000, 40, 2, 0.5, seed=7)
    x = E.ravel() / 0.5
    assert abs(x.mean()) < 5 / np.sqrt(x.size)
    assert abs(x.var() - 1.0) < 0.02
    assert abs(np.mean(x ** 4) - 3.0) < 0.1


def test_field_offset_and_seed():
    full = nz.noise(300, 12, 1, 1.0, seed=99)
    part = nz.noise(300, 5, 1, 1.0, seed=99, field_offset=7)
    assert np.array_equal(full[7:], part)
    other = nz.noise(300, 12, 1, 1.0, seed=100)
    assert not np.array_equal(full, other)
    assert np.array_equal(nz.noise(10, 3, 0, 1.0, seed=1), np.zeros((3, 10)))


def test_normalize_weights_closed_form():
    rng = np.random.default_rng(3)
    mu = rng.standard_normal((200, 16))
    mu[5] = 0.0
    mu[9, :] = 1e-6 * rng.standard_normal(16)
    alpha, flags = nz.normalize_weights(mu, 1e-3 * np.sqrt(16))
    assert flags[5] == 1 and flags[9] == 1
    ok = flags == 0
    assert np.allclose(alpha[ok].sum(axis=1), 1.0, rtol=0, atol=1e-12)
    assert np.array_equal(alpha[~ok], mu[~ok])
