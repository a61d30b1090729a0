"""The no-allocation block solve (library-held scratch) against the solve
with a caller workspace, through the C ABI: two calls in a row, the second
with a smaller input, each compared with the existing entry point on the
same inputs, to the solve's own bar (bit-for-bit: same kernels, same order;
and the oracle's residual), and a request larger than the scratch
rejected."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_23221_amd import capi, synth
from tests.gpu_util import abs_csr, to_np

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def _check_against_workspace_solve(dev, chip, B, tol, compute):
    A = oracle.assemble_chip(chip)
    G = capi.HeatOperator.from_chip(chip, dev, precond=capi.PRECOND_JACOBI)
    Bg = torch.as_tensor(B, device=dev)
    X_ref, info_ref = capi.block_krylov_solve(G, Bg, tol, compute=compute)
    X_na, info_na = capi.block_krylov_solve_noalloc(G, Bg, tol, compute=compute)
    torch.cuda.synchronize()
    assert info_na["status"] == capi.OK and info_na["iters"] == info_ref["iters"], (info_na, info_ref)
    assert torch.equal(X_na, X_ref)
    X = to_np(X_na)
    R = B - oracle.apply_many(A, X)
    bn = np.linalg.norm(B, axis=1)
    rel = np.linalg.norm(R, axis=1) / bn
    floor = 8 * U64 * np.linalg.norm(oracle.apply_many(abs_csr(A), np.abs(X)) + np.abs(B), axis=1) / bn
    assert (rel <= tol * 1.0001 + floor).all()


def test_noalloc_solve_two_calls_second_smaller(dev):
    rng = np.random.default_rng(404)
    big = synth.chip_stack(rng, 96, 80, 6)
    small = synth.chip_2d(rng, 40)
    _check_against_workspace_solve(dev, big, synth.power_blocky(rng, big, 24), 1e-8, capi.F32)
    _check_against_workspace_solve(dev, small, rng.standard_normal((5, small.n)), 1e-10, capi.F64)


def test_noalloc_solve_rejects_oversized(dev):
    rng = np.random.default_rng(405)
    chip = synth.chip_stack(rng, 256, 256, 16)
    G = capi.HeatOperator.from_chip(chip, dev)
    assert capi.workspace_bytes(G, 64, capi.F64) > capi.NOALLOC_SCRATCH_BYTES
    B = torch.zeros((64, chip.n), dtype=torch.float64, device=dev)
    with pytest.raises(capi.BlockoaError) as e:
        capi.block_krylov_solve_noalloc(G, B, 1e-8, compute=capi.F64)
    assert e.value.status == capi.EINVAL and "scratch" in str(e.value)
