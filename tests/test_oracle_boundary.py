"""Pins of the oracle's boundary source (nonhomogeneous Dirichlet / Robin
data by lifting, Sec. II-A) against closed forms and invariants:

* one temperature U on every non-adiabatic face: g = U (A 1), since a
  constant field carries no interior flux;
* a rod with Dirichlet temperatures T1, T2 at its ends and no source: the
  finite-volume solution is exactly linear, x_i = T1 + (T2 - T1)(i + 1/2)/n
  (the boundary half-cell is the same distance as the face);
* Robin ambient U at one end of an otherwise adiabatic rod, no source: the
  solution is U everywhere;
* Mixed faces at different temperatures, no source: the solution lies
  between the smallest and the largest face temperature (maximum principle).
"""
import numpy as np

import oracle
from paper_2510_23221_amd import synth

D0, AD, RB = synth.BC_DIRICHLET0, synth.BC_ADIABATIC, synth.BC_ROBIN


def test_uniform_temperature_is_a_times_ones():
    rng = np.random.default_rng(1)
    nx, ny, nz = 6, 5, 4
    k = rng.uniform(1.0, 300.0, size=nx * ny * nz)
    bc, h = [D0, RB, AD, D0, RB, RB], [0, 5e3, 0, 0, 2e4, 1e3]
    A = oracle.assemble(nx, ny, nz, 1e-3, 2e-3, 0.5e-3, k, bc, h)
    g = oracle.boundary_source(nx, ny, nz, 1e-3, 2e-3, 0.5e-3, k, bc, h, [50.0] * 6)
    ref = 50.0 * oracle.spmv(A, np.ones(A.n))
    assert np.allclose(g, ref, rtol=1e-13, atol=1e-9 * np.abs(ref).max())


def test_rod_linear_profile_between_dirichlet_ends():
    n = 40
    k = np.full(n, 3.7)
    bc, h = [D0, D0, AD, AD, AD, AD], [0] * 6
    A = oracle.assemble(n, 1, 1, 0.02, 1.0, 1.0, k, bc, h)
    g = oracle.boundary_source(n, 1, 1, 0.02, 1.0, 1.0, k, bc, h, [20.0, 80.0, 0, 0, 0, 0])
    x = np.linalg.solve(A.to_dense(), g)
    ref = 20.0 + 60.0 * (np.arange(n) + 0.5) / n
    assert np.allclose(x, ref, rtol=1e-12, atol=0)


def test_robin_end_gives_ambient_everywhere():
    n = 25
    k = np.linspace(1.0, 9.0, n)
    bc, h = [AD, RB, AD, AD, AD, AD], [0, 400.0, 0, 0, 0, 0]
    A = oracle.assemble(n, 1, 1, 0.05, 1.0, 1.0, k, bc, h)
    g = oracle.boundary_source(n, 1, 1, 0.05, 1.0, 1.0, k, bc, h, [0, 33.0, 0, 0, 0, 0])
    x = np.linalg.solve(A.to_dense(), g)
    assert np.allclose(x, 33.0, rtol=1e-12, atol=0)


def test_mixed_faces_maximum_principle():
    rng = np.random.default_rng(2)
    nx, ny, nz = 7, 6, 3
    k = rng.uniform(1.0, 150.0, size=nx * ny * nz)
    bc, h = [D0, D0, D0, D0, RB, RB], [0, 0, 0, 0, 3e4, 3e4]
    uf = [50.0, 50.0, 50.0, 50.0, 25.0, 25.0]
    A = oracle.assemble(nx, ny, nz, 1e-3, 1e-3, 0.3e-3, k, bc, h)
    g = oracle.boundary_source(nx, ny, nz, 1e-3, 1e-3, 0.3e-3, k, bc, h, uf)
    x = np.linalg.solve(A.to_dense(), g)
    assert x.min() >= 25.0 - 1e-9 and x.max() <= 50.0 + 1e-9
    assert x.max() - x.min() > 1.0
