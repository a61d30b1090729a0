"""Nonhomogeneous boundary data by lifting (Sec. II-A; the paper's Dirichlet
50 C, Robin ambient and Mixed scenarios of Sec. V-A) on the GPU against the
oracle: the boundary source g, and the whole pipeline -- basis solutions of
A X = Q + g, normalised weights (sum one), fields T = X alpha, powers
F = A T - g -- which must reproduce the combined power maps Q alpha and keep
the boundary data (with Q = 0 every field is the lifted solution itself)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_23221_amd import capi
from tests.gpu_util import to_np
from tests.test_gpu_parity import U64, _chip

pytestmark = pytest.mark.gpu


def _faces(chip, rng):
    return [float(rng.uniform(20.0, 60.0)) for _ in range(6)]


@pytest.mark.parametrize("kind", ["2d", "ragged", "stack", "line"])
def test_boundary_source_matches_oracle(dev, kind):
    chip = _chip(kind)
    G = capi.HeatOperator.from_chip(chip, dev)
    uf = _faces(chip, np.random.default_rng(3))
    g = to_np(capi.boundary_source(G, uf))
    ref = oracle.boundary_source(chip.nx, chip.ny, chip.nz, chip.lx, chip.ly, chip.lz, chip.k, chip.bc, chip.h, uf)
    assert np.allclose(g, ref, rtol=8 * U64, atol=0)


@pytest.mark.parametrize("kind,precond", [("ragged", 0), ("stack", capi.PRECOND_JACOBI)])
def test_lifted_pipeline_keeps_boundary_data(dev, kind, precond):
    chip = _chip(kind)
    A = oracle.assemble_chip(chip)
    G = capi.HeatOperator.from_chip(chip, dev, precond=precond)
    rng = np.random.default_rng(5)
    uf = _faces(chip, rng)
    g = capi.boundary_source(G, uf)
    s, m, tol = 8, 40, 1e-10
    Q = rng.standard_normal((s, A.n)) * 1e3
    B = torch.as_tensor(Q, device=dev) + g[None, :]
    X, info = capi.block_krylov_solve(G, B, tol)
    mu = torch.as_tensor(rng.standard_normal((m, s)), device=dev)
    flags = to_np(capi.normalize_weights(mu, 1e-3 * np.sqrt(s)))
    ok = flags == 0
    T = capi.combine(X, mu)
    F = capi.apply_operator(G, T)
    capi.add_column(F, g, -1.0)
    F, T, alpha = to_np(F), to_np(T), to_np(mu)
    P = alpha @ Q  # the fields' power maps
    rel = np.linalg.norm(F[ok] - P[ok], axis=1) / np.linalg.norm(P[ok], axis=1)
    # the solve meets tol per column of B: |alpha| weighted sums of that residual
    bound = tol * (np.abs(alpha[ok]) @ np.linalg.norm(to_np(B), axis=1)) / np.linalg.norm(P[ok], axis=1)
    assert (rel <= 1.01 * bound + 1e-12).all(), (rel.max(), bound.min())
    # pure boundary lifting: every basis solution is x = A^-1 g, and so is every field
    B0 = g[None, :].repeat(s, 1).contiguous()
    X0, _ = capi.block_krylov_solve(G, B0, tol)
    T0 = to_np(capi.combine(X0, torch.as_tensor(alpha, device=dev)))
    x = np.linalg.solve(A.to_dense(), to_np(g)) if A.n <= 4096 else oracle.cg(A, to_np(g), 1e-13)[0]
    assert np.abs(T0[ok] - x[None, :]).max() <= 1e-7 * np.abs(x).max()
