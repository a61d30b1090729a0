"""Pins of the oracle's CG, product and combination routines against
mathematics independent of their code:

* dense direct solves (LAPACK through numpy) on tiny grids;
* finite termination: a right-hand side made of p eigenmodes with distinct
  eigenvalues is solved exactly by CG in p steps, with the closed-form
  solution sum_i c_i / lambda_i v_i;
* the A-norm error bound of CG quoted in the paper's error analysis
  (Sec. IV-B): ||e_m||_A <= 2 ((sqrt(kappa) - 1) / (sqrt(kappa) + 1))^m ||e_0||_A;
* the combination T = X C (Sec. III-B, Eq. (5)) against numpy's matmul and
  against unit weights, and the operator action F = A T (Sec. III-C) against a
  dense product.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2510_23221_amd import synth

D0, AD, RB = synth.BC_DIRICHLET0, synth.BC_ADIABATIC, synth.BC_ROBIN


def _tiny_chip(seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = 5, 4, 3
    k = rng.uniform(1.0, 400.0, size=nx * ny * nz)
    return oracle.assemble(nx, ny, nz, 1e-3, 1e-3, 0.3e-3, k, [AD, D0, AD, AD, AD, RB],
                           [0, 0, 0, 0, 0, 2e4])


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_cg_matches_dense_solve(seed):
    A = _tiny_chip(seed)
    D = A.to_dense()
    rng = np.random.default_rng(100 + seed)
    b = rng.standard_normal(A.n)
    x_ref = np.linalg.solve(D, b)
    x, it, rr = oracle.cg(A, b, 1e-14)
    assert rr < 1e-13
    assert np.linalg.norm(x - x_ref) <= 1e-10 * np.linalg.norm(x_ref)


def test_cg_finite_termination_on_eigenmodes():
    nx, ny, nz = 16, 12, 1
    lx, ly = 1.0, 0.6
    kval = 2.0
    A = oracle.assemble(nx, ny, nz, lx, ly, 1.0, np.full(nx * ny, kval), [D0, D0, D0, D0, AD, AD], [0] * 6)
    ix = np.arange(nx) + 0.5
    iy = np.arange(ny) + 0.5
    modes = [(1, 1), (2, 3), (5, 1), (7, 9)]
    coef = [1.0, -0.5, 2.0, 0.25]
    b = np.zeros(nx * ny)
    x_exact = np.zeros(nx * ny)
    for (p, q), c in zip(modes, coef):
        v = np.outer(np.sin(q * math.pi * iy / ny), np.sin(p * math.pi * ix / nx)).reshape(-1)
        lam = kval * (4 * nx ** 2 / lx ** 2 * math.sin(p * math.pi / (2 * nx)) ** 2
                      + 4 * ny ** 2 / ly ** 2 * math.sin(q * math.pi / (2 * ny)) ** 2)
        b += c * v
        x_exact += c / lam * v
    x, it, rr = oracle.cg(A, b, 1e-13)
    assert it <= len(modes) + 1
    assert np.linalg.norm(x - x_exact) <= 1e-11 * np.linalg.norm(x_exact)
    # a single mode needs exactly one step
    x1, it1, _ = oracle.cg(A, np.outer(np.sin(math.pi * iy / ny), np.sin(math.pi * ix / nx)).reshape(-1), 1e-13)
    assert it1 == 1


def test_cg_error_bound_a_norm():
    A = _tiny_chip(5)
    D = A.to_dense()
    ev = np.linalg.eigvalsh(D)
    kappa = ev.max() / ev.min()
    rho = (math.sqrt(kappa) - 1) / (math.sqrt(kappa) + 1)
    rng = np.random.default_rng(9)
    b = rng.standard_normal(A.n)
    x_star = np.linalg.solve(D, b)

    def anorm(e):
        return math.sqrt(e @ D @ e)

    e0 = anorm(x_star)  # x0 = 0
    for m in range(1, 40):
        xm, it, _ = oracle.cg(A, b, 0.0, maxit=m)
        assert it == m
        assert anorm(xm - x_star) <= 2 * rho ** m * e0 * (1 + 1e-9) + 1e-14 * e0


def test_cg_zero_rhs_and_many_columns():
    A = _tiny_chip(1)
    rng = np.random.default_rng(4)
    B = rng.standard_normal((5, A.n))
    B[2] = 0.0
    X, iters, rr = oracle.cg_many(A, B, 1e-13, nthreads=2)
    assert iters[2] == 0 and np.all(X[2] == 0.0)
    for j in (0, 1, 3, 4):
        xj, itj, _ = oracle.cg(A, B[j], 1e-13)
        assert itj == iters[j]
        assert np.array_equal(xj, X[j])
    D = A.to_dense()
    assert np.linalg.norm(D @ X.T - B.T) <= 1e-12 * np.linalg.norm(B)


def test_gemm_against_numpy_and_unit_weights():
    rng = np.random.default_rng(11)
    s, n, m = 7, 301, 53
    X = rng.standard_normal((s, n))
    C = rng.standard_normal((m, s))
    T = oracle.gemm(X, C, nthreads=3)
    T_np = C @ X  # (M, s) @ (s, N): column f of T is sum_k C[k, f] X[:, k]
    assert np.abs(T - T_np).max() <= 1e-13 * np.abs(T_np).max()
    E = np.eye(s)
    assert np.array_equal(oracle.gemm(X, E), X)
    # Eq. (5) with alpha = mu / sum(mu): combining identical basis fields
    # reproduces that field
    mu = rng.standard_normal((4, s))
    alpha = mu / mu.sum(axis=1, keepdims=True)
    same = np.tile(X[:1], (s, 1))
    assert np.allclose(oracle.gemm(same, alpha), np.tile(X[:1], (4, 1)), rtol=1e-12, atol=1e-12 * np.abs(X).max())


def test_apply_many_against_dense():
    A = _tiny_chip(2)
    D = A.to_dense()
    rng = np.random.default_rng(12)
    T = rng.standard_normal((9, A.n))
    F = oracle.apply_many(A, T, nthreads=2)
    assert np.abs(F - T @ D.T).max() <= 1e-13 * np.abs(D).max() * np.abs(T).max() * 7


def test_pair_consistency_invariant():
    """A (X c) = B c up to the solve residual (Sec. III-B / III-C)."""
    A = _tiny_chip(3)
    rng = np.random.default_rng(13)
    B = rng.standard_normal((4, A.n))
    X, iters, rr = oracle.cg_many(A, B, 1e-12)
    C = rng.standard_normal((6, 4))
    F = oracle.apply_many(A, oracle.gemm(X, C))
    Bc = C @ B
    rel = np.linalg.norm(F - Bc, axis=1) / np.linalg.norm(Bc, axis=1)
    bound = np.abs(C) @ (rr * np.linalg.norm(B, axis=1)) / np.linalg.norm(Bc, axis=1)
    assert (rel <= bound * (1 + 1e-6) + 1e-14).all()


def test_generators_deterministic():
    w1 = synth.workload(0, m=10)
    w2 = synth.workload(0, m=10)
    assert np.array_equal(w1.chips[0].k, w2.chips[0].k)
    assert np.array_equal(w1.B[0], w2.B[0]) and np.array_equal(w1.C[0], w2.C[0])
    w3 = synth.workload(1, m=3, s=4, grid=(16, 16, 8))
    assert w3.B[0].shape == (4, 16 * 16 * 8) and w3.C[0].shape == (3, 4)
    assert (w3.chips[0].k > 0).all()
