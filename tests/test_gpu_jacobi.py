"""Jacobi (diagonal) preconditioning on the GPU against the CPU oracle,
through the C ABI: the scaled operator S A S, the block solve on the scaled
system inside the FP64 correction loop, preconditioned per-sample CG, and a
batch that mixes preconditioned and plain chips.

Tolerances: scaled coefficients within 4 ulp of the oracle's products; block
solve as in the parity suite (true FP64 residual <= tol per column, solution
within 1e-8 of per-column CG to 1e-13 in FP64); per-sample PCG within two
iterations per column of the oracle's PCG (same stopping rule).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_23221_amd import capi, synth
from tests.gpu_util import abs_csr, rel_fro, to_np
from tests.test_gpu_parity import U64, _chip, _solve_check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def jops(dev):
    out = {}
    for kind in ("2d", "ragged", "stack", "line"):
        chip = _chip(kind)
        A = oracle.assemble_chip(chip)
        G = capi.HeatOperator.from_chip(chip, dev, precond=capi.PRECOND_JACOBI)
        out[kind] = (chip, A, G)
    return out


@pytest.mark.parametrize("kind", ["2d", "ragged", "stack", "line"])
def test_scaled_operator_matches_oracle(jops, kind):
    chip, A, G = jops[kind]
    assert G.precond == capi.PRECOND_JACOBI
    (diag, wx, wy, wz), scale = G.scaled_coefficients()
    diag, wx, wy, wz, scale = (to_np(t) for t in (diag, wx, wy, wz, scale))
    sc, Ah = oracle.jacobi_scaling(A)
    assert np.allclose(scale, sc, rtol=4 * U64, atol=0)
    D = np.zeros(A.n)
    nbr = {}
    for r in range(A.n):
        for p in range(Ah.rowptr[r], Ah.rowptr[r + 1]):
            c = Ah.col[p]
            if c == r:
                D[r] = Ah.val[p]
            else:
                nbr[(r, c)] = -Ah.val[p]
    assert np.allclose(diag, D, rtol=8 * U64, atol=0)
    nx, ny = chip.nx, chip.ny
    for arr, off in ((wx, 1), (wy, nx), (wz, nx * ny)):
        for r in range(0, A.n, max(1, A.n // 997)):
            expect = nbr.get((r, r + off), 0.0)
            assert abs(arr[r] - expect) <= 8 * U64 * abs(expect), (r, off)


@pytest.mark.parametrize("kind,compute", [("2d", capi.F64), ("ragged", capi.F64), ("stack", capi.F64),
                                          ("2d", capi.F32), ("stack", capi.F32), ("ragged", capi.F32)])
def test_block_solve_jacobi(jops, dev, kind, compute):
    chip, A, G = jops[kind]
    rng = np.random.default_rng(60)
    B = rng.standard_normal((16, A.n))
    tol = 1e-10 if compute == capi.F64 else 1e-8
    X, info, _ = _solve_check(A, G, B, tol, compute, dev, xerr=(1e-8 if compute == capi.F64 else None))
    assert info["status"] == capi.OK


def test_jacobi_cuts_block_iterations_on_stack(jops, dev):
    """High-contrast stack (conductivities over two decades): the diagonal
    scaling reduces the block iterations to the same tolerance."""
    chip, A, Gj = jops["stack"]
    G = capi.HeatOperator.from_chip(chip, dev)
    rng = np.random.default_rng(61)
    B = torch.as_tensor(rng.standard_normal((16, A.n)), device=dev)
    _, info_p = capi.block_krylov_solve(Gj, B, 1e-10)
    _, info_n = capi.block_krylov_solve(G, B, 1e-10)
    assert info_p["max_rel_res"] <= 1e-10 and info_n["max_rel_res"] <= 1e-10
    assert info_p["iters"] < info_n["iters"], (info_p, info_n)


@pytest.mark.parametrize("kind", ["2d", "ragged", "stack"])
def test_per_sample_pcg_matches_oracle(jops, dev, kind):
    chip, A, G = jops[kind]
    rng = np.random.default_rng(62)
    B = rng.standard_normal((6, A.n))
    B[2] = 0.0
    tol = 1e-10
    X, iters, info = capi.cg_solve(G, torch.as_tensor(B, device=dev), tol)
    X = to_np(X)
    sc, _ = oracle.jacobi_scaling(A)
    it_ref = np.array([oracle.pcg(A, b, tol, minv=sc * sc)[1] for b in B])
    assert np.abs(iters - it_ref).max() <= 2, (iters, it_ref)
    assert iters[2] == 0 and np.abs(X[2]).max() == 0.0
    R = B - oracle.apply_many(A, X)
    bn = np.linalg.norm(B, axis=1)
    rel = np.linalg.norm(R, axis=1) / np.where(bn > 0, bn, 1)
    floor = 8 * U64 * np.linalg.norm(oracle.apply_many(abs_csr(A), np.abs(X)) + np.abs(B), axis=1) \
        / np.where(bn > 0, bn, 1)
    assert (rel <= 10 * tol + floor).all(), rel.max()
    X13, _, _ = oracle.cg_many(A, B, 1e-13)
    assert rel_fro(X, X13) <= 1e-6


def test_batch_mixes_jacobi_and_plain_chips(dev):
    rng = np.random.default_rng(63)
    chips = [_chip("2d"), synth.chip_stack(rng, 32, 24, 5), _chip("ragged"), synth.chip_stack(rng, 48, 48, 4)]
    As = [oracle.assemble_chip(c) for c in chips]
    Gs = [capi.HeatOperator.from_chip(c, dev, precond=(capi.PRECOND_JACOBI if i % 2 == 0 else 0))
          for i, c in enumerate(chips)]
    s = 8
    Bs = [rng.standard_normal((s, A.n)) for A in As]
    for compute, tol in ((capi.F64, 1e-10), (capi.F32, 1e-8)):
        plan = capi.BatchPlan(Gs, s, compute)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            Xs, infos = plan.solve([torch.as_tensor(B, device=dev) for B in Bs], tol, stream=stream)
        torch.cuda.synchronize()
        for k, (A, B, X, info) in enumerate(zip(As, Bs, Xs, infos)):
            X = to_np(X)
            rel = np.linalg.norm(B - oracle.apply_many(A, X), axis=1) / np.linalg.norm(B, axis=1)
            assert info["status"] == capi.OK, (k, info)
            assert rel.max() <= tol * 1.0001 + 1e-15, (k, compute, rel.max())
