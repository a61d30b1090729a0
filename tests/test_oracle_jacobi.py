"""Pins of the oracle's Jacobi preconditioning (the optional diagonal
preconditioner of the solves; the paper leaves the preconditioner unstated)
against mathematics independent of its code:

* S A S has a unit diagonal, is symmetric, and its eigenvalues are the
  generalised eigenvalues of (A, diag(A)) (LAPACK through scipy);
* preconditioned CG with M = diag(A) produces after k steps exactly S times
  the k-th iterate of plain CG on S A S y = S b (the textbook equivalence of
  split and left preconditioning), cross-checked against the C oracle's CG;
* with M = A (a diagonal A) PCG stops after one step with the exact
  solution; with M = I it is the C oracle's plain CG;
* PCG reaches the dense solution, and needs fewer iterations than plain CG on
  a high-contrast stack.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2510_23221_amd import synth

D0, AD, RB = synth.BC_DIRICHLET0, synth.BC_ADIABATIC, synth.BC_ROBIN


def _tiny_chip(seed, nx=5, ny=4, nz=3):
    rng = np.random.default_rng(seed)
    k = rng.uniform(1.0, 400.0, size=nx * ny * nz)
    return oracle.assemble(nx, ny, nz, 1e-3, 1e-3, 0.3e-3, k, [AD, D0, AD, AD, AD, RB],
                           [0, 0, 0, 0, 0, 2e4])


@pytest.mark.parametrize("seed", [0, 1])
def test_scaling_unit_diagonal_symmetric_and_spectrum(seed):
    A = _tiny_chip(seed)
    sc, Ah = oracle.jacobi_scaling(A)
    D = A.to_dense()
    H = Ah.to_dense()
    # a few ulp: d s^2 and a_ij s_i s_j are rounded products
    assert np.allclose(np.diag(H), 1.0, rtol=0, atol=1e-15)
    assert np.abs(H - H.T).max() <= 1e-15 * np.abs(H).max()
    # S is diag(A)^(-1/2) and S A S is its two-sided product with A
    assert np.allclose(sc, 1.0 / np.sqrt(np.diag(D)), rtol=1e-15, atol=0)
    assert np.allclose(H, (sc[:, None] * D) * sc[None, :], rtol=1e-14, atol=0)
    # eig(S A S) = eig(A, diag(A))
    lam_h = np.linalg.eigvalsh(H)
    lam_g = scipy.linalg.eigh(D, np.diag(np.diag(D)), eigvals_only=True)
    assert np.allclose(np.sort(lam_h), np.sort(lam_g), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("k", [1, 3, 7])
def test_pcg_iterates_equal_scaled_cg(k):
    A = _tiny_chip(2)
    sc, Ah = oracle.jacobi_scaling(A)
    rng = np.random.default_rng(7)
    b = rng.standard_normal(A.n)
    x_pcg, it, _ = oracle.pcg(A, b, 0.0, maxit=k, minv=sc * sc)
    y, it2, _ = oracle.pcg(Ah, sc * b, 0.0, maxit=k)
    assert it == it2 == k
    assert np.allclose(x_pcg, sc * y, rtol=1e-10, atol=1e-12 * np.abs(x_pcg).max())


def test_pcg_plain_matches_c_oracle_and_diagonal_one_step():
    A = _tiny_chip(3)
    rng = np.random.default_rng(8)
    b = rng.standard_normal(A.n)
    x1, it1, r1 = oracle.pcg(A, b, 1e-12)
    x2, it2, r2 = oracle.cg(A, b, 1e-12)
    assert abs(it1 - it2) <= 1
    assert np.allclose(x1, x2, rtol=1e-9, atol=1e-12 * np.abs(x2).max())
    # a diagonal operator preconditioned by itself: one step, exact
    n = 12
    d = rng.uniform(1.0, 50.0, size=n)
    Dm = oracle.CSR(n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), d.copy())
    x, it, res = oracle.pcg(Dm, b[:n], 1e-14, minv=1.0 / d)
    assert it == 1 and np.allclose(x, b[:n] / d, rtol=1e-15, atol=0)


def test_pcg_solution_and_iteration_gain_on_stack():
    rng = np.random.default_rng(5)
    chip = synth.chip_stack(rng, 16, 16, 6)
    A = oracle.assemble_chip(chip)
    sc, _ = oracle.jacobi_scaling(A)
    b = rng.standard_normal(A.n)
    x_ref = np.linalg.solve(A.to_dense(), b)
    x, it_p, res = oracle.pcg(A, b, 1e-12, minv=sc * sc)
    _, it_c, _ = oracle.pcg(A, b, 1e-12)
    assert res <= 1e-12 * 1.01
    assert np.linalg.norm(x - x_ref) <= 1e-8 * np.linalg.norm(x_ref)
    assert it_p < it_c


def test_c_pcg_matches_dense_solve_and_numpy_pcg():
    """The C Jacobi-PCG (the timed CPU baseline): LAPACK's solution on a
    high-contrast stack, the iteration count of the numpy PCG above (same
    recurrences and stopping rule), one exact step on a diagonal operator,
    and the same results from the -O3 -march=native build."""
    rng = np.random.default_rng(6)
    chip = synth.chip_stack(rng, 12, 10, 5)
    A = oracle.assemble_chip(chip)
    B = rng.standard_normal((3, A.n))
    X, iters, rel = oracle.pcg_many(A, B, 1e-12)
    Xd = np.linalg.solve(A.to_dense(), B.T).T
    assert np.linalg.norm(X - Xd) <= 1e-8 * np.linalg.norm(Xd)
    assert (rel <= 1e-12 * 1.01).all()
    sc, _ = oracle.jacobi_scaling(A)
    for j in range(3):
        _, it_np, _ = oracle.pcg(A, B[j], 1e-12, minv=sc * sc)
        assert abs(int(iters[j]) - it_np) <= 1
    n = 12
    d = rng.uniform(1.0, 50.0, size=n)
    Dm = oracle.CSR(n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), d.copy())
    x1, it1, _ = oracle.pcg_many(Dm, B[:1, :n], 1e-14)
    assert it1[0] == 1 and np.allclose(x1[0], B[0, :n] / d, rtol=1e-15, atol=0)
    oracle.select_build(native=True)
    try:
        Xn, itn, _ = oracle.pcg_many(A, B, 1e-12)
        Xc, itc, _ = oracle.cg_many(A, B, 1e-12)
    finally:
        oracle.select_build(native=False)
    Xp, itp, _ = oracle.cg_many(A, B, 1e-12)
    assert np.abs(itn - iters).max() <= 1 and np.abs(itc - itp).max() <= 1
    assert np.linalg.norm(Xn - X) <= 1e-9 * np.linalg.norm(X)
