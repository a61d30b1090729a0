"""Pins of the oracle's operator assembly and CSR product against facts fixed by
the mathematics of the discretised heat equation (paper Sec. II-A, Eq. (1),
boundary models of Sec. II-A) -- not against the oracle's own formulas.

* constant-k eigenmodes: sine modes for Dirichlet-0 faces, cosine modes for
  adiabatic faces, quarter-wave modes for one Dirichlet and one adiabatic face,
  with closed-form eigenvalues 4 k / d^2 sin^2(theta / 2);
* layered stacks: exact series-resistance temperature profile for any layer
  conductivities with a convective (Robin) face, along each axis;
* SPD and symmetry (dense eigen-decomposition, tiny grids);
* conservation: with every face adiabatic a uniform field carries no flux.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2510_23221_amd import synth

D0, AD, RB = synth.BC_DIRICHLET0, synth.BC_ADIABATIC, synth.BC_ROBIN


def _mode_1d(kind_lo, kind_hi, n, p):
    """1-D eigenvector and eigenvalue factor sin^2(theta/2) of the cell-centred
    second difference with the given end conditions (p is the mode number)."""
    i = np.arange(n) + 0.5
    if kind_lo == D0 and kind_hi == D0:
        th = p * math.pi / n  # p = 1..n
        v = np.sin(th * i)
    elif kind_lo == AD and kind_hi == AD:
        th = p * math.pi / n  # p = 0..n-1
        v = np.cos(th * i)
    elif kind_lo == D0 and kind_hi == AD:
        th = (p - 0.5) * math.pi / n  # p = 1..n
        v = np.sin(th * i)
    elif kind_lo == AD and kind_hi == D0:
        th = (p - 0.5) * math.pi / n
        v = np.cos(th * i)
    else:
        raise ValueError
    return v, math.sin(th / 2.0) ** 2


def _modes(kinds, n):
    lo, hi = kinds
    if lo == AD and hi == AD:
        return range(0, n)
    return range(1, n + 1)


@pytest.mark.parametrize("bc", [
    (D0, D0, D0, D0, D0, D0),
    (D0, D0, AD, AD, AD, AD),
    (AD, AD, D0, D0, AD, AD),
    (AD, AD, AD, AD, D0, D0),
    (D0, AD, AD, D0, D0, AD),
    (AD, D0, D0, AD, AD, D0),
])
def test_constant_k_eigenmodes(bc):
    nx, ny, nz = 5, 4, 3
    lx, ly, lz = 1.3, 0.7, 0.25
    kval = 3.7
    A = oracle.assemble(nx, ny, nz, lx, ly, lz, np.full(nx * ny * nz, kval), bc, [0.0] * 6)
    d = (lx / nx, ly / ny, lz / nz)
    n3 = (nx, ny, nz)
    checked = 0
    for px in _modes(bc[0:2], nx):
        for py in _modes(bc[2:4], ny):
            for pz in _modes(bc[4:6], nz):
                vx, sx = _mode_1d(bc[0], bc[1], nx, px)
                vy, sy = _mode_1d(bc[2], bc[3], ny, py)
                vz, sz = _mode_1d(bc[4], bc[5], nz, pz)
                v = np.einsum("l,j,i->lji", vz, vy, vx).reshape(-1)
                lam = kval * sum(4.0 / d[a] ** 2 * s for a, s in enumerate((sx, sy, sz)))
                Av = oracle.spmv(A, v)
                err = np.linalg.norm(Av - lam * v) / (abs(lam) * np.linalg.norm(v) + 1e-300)
                if lam == 0.0:
                    assert np.linalg.norm(Av) < 1e-12 * kval
                else:
                    assert err < 1e-12, (px, py, pz, err)
                checked += 1
    assert checked == nx * ny * nz


def _layered_profile(kl, q, d, h):
    """Exact temperature rise of a 1-D stack of cells with conductivity kl[l],
    uniform source q[l] (W/m^3), an adiabatic face at l = 0 and a convective
    face (coefficient h) past the last cell.  Heat made at or below cell l
    leaves upward through the face above it (flux d * sum q), and each face
    adds the series resistance of two half cells; the outer face adds the
    half-cell plus film resistance."""
    n = len(kl)
    phi = d * np.cumsum(q)  # W/m^2 through the face above cell l
    T = np.zeros(n)
    T[n - 1] = phi[n - 1] * (1.0 / h + d / (2.0 * kl[n - 1]))
    for l in range(n - 2, -1, -1):
        T[l] = T[l + 1] + phi[l] * (d / (2.0 * kl[l]) + d / (2.0 * kl[l + 1]))
    return T


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_layered_stack_robin_closed_form(axis):
    rng = np.random.default_rng(7 + axis)
    n_layers = 9
    other = (3, 2)
    L = 0.51e-3
    # paper's materials (Sec. V-A): silicon 150, copper 413, TIM 40 W/mK
    kl = rng.choice([150.0, 413.0, 40.0], size=n_layers) * rng.uniform(0.8, 1.2, size=n_layers)
    q = rng.uniform(0.0, 4.0e10, size=n_layers)
    h = 3.0e4
    dims = [other[0], other[1]]
    dims.insert(axis, n_layers)
    nx, ny, nz = dims
    lens = [2e-3, 1e-3]
    lens.insert(axis, L)
    bc = [AD] * 6
    bc[2 * axis + 1] = RB
    hh = [0.0] * 6
    hh[2 * axis + 1] = h
    shape_zyx = (nz, ny, nx)
    k3 = np.empty(shape_zyx)
    q3 = np.empty(shape_zyx)
    sl = [None, None, None]
    for l in range(n_layers):
        idx = [slice(None)] * 3
        idx[2 - axis] = l
        k3[tuple(idx)] = kl[l]
        q3[tuple(idx)] = q[l]
    A = oracle.assemble(nx, ny, nz, *lens, k3.reshape(-1), bc, hh)
    T1 = _layered_profile(kl, q, L / n_layers, h)
    T3 = np.empty(shape_zyx)
    for l in range(n_layers):
        idx = [slice(None)] * 3
        idx[2 - axis] = l
        T3[tuple(idx)] = T1[l]
    # the exact profile satisfies A T = q cell by cell
    r = oracle.spmv(A, T3.reshape(-1)) - q3.reshape(-1)
    assert np.linalg.norm(r) <= 1e-11 * np.linalg.norm(q3)
    # and the oracle's CG reproduces it
    x, it, rr = oracle.cg(A, q3.reshape(-1), 1e-14)
    assert np.linalg.norm(x - T3.reshape(-1)) <= 1e-9 * np.linalg.norm(T3)


def test_dirichlet_ghost_half_cell():
    """A single cell with one Dirichlet-0 face and one Robin face along x, the
    rest adiabatic: steady state of a source q is the series network
    ground --(d/2k)-- cell --(d/2k + 1/h)-- ambient in parallel."""
    k, d, h, q = 12.0, 0.3, 5.0, 7.0
    A = oracle.assemble(1, 1, 1, d, 1.0, 1.0, [k], [D0, RB, AD, AD, AD, AD], [0, h, 0, 0, 0, 0])
    g_left = 1.0 / (d / (2 * k))  # conductance per unit area
    g_right = 1.0 / (d / (2 * k) + 1.0 / h)
    T = q * d / (g_left + g_right)
    assert abs(oracle.spmv(A, np.array([T]))[0] - q) < 1e-12 * q


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_symmetric_positive_definite(seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = 4, 3, 3
    k = rng.uniform(1.0, 400.0, size=nx * ny * nz)
    bc = list(rng.choice([D0, AD, RB], size=6))
    if all(b == AD for b in bc):
        bc[5] = RB
    h = rng.uniform(1e2, 1e4, size=6)
    A = oracle.assemble(nx, ny, nz, 1e-3, 2e-3, 0.5e-3, k, bc, h).to_dense()
    assert np.allclose(A, A.T, rtol=0, atol=1e-12 * np.abs(A).max())
    assert np.linalg.eigvalsh(A).min() > 0.0
    # off-diagonals are non-positive and the matrix is diagonally dominant
    off = A - np.diag(np.diag(A))
    assert (off <= 0).all()
    assert (np.diag(A) + 1e-9 * np.abs(A).max() >= -off.sum(axis=1)).all()


def test_all_adiabatic_conserves():
    rng = np.random.default_rng(3)
    nx, ny, nz = 6, 5, 4
    k = rng.uniform(1.0, 400.0, size=nx * ny * nz)
    A = oracle.assemble(nx, ny, nz, 1.0, 1.0, 1.0, k, [AD] * 6, [0.0] * 6)
    r = oracle.spmv(A, np.ones(nx * ny * nz))
    assert np.abs(r).max() <= 1e-12 * np.abs(A.val).max()


def test_csr_structure():
    nx, ny, nz = 4, 3, 2
    A = oracle.assemble(nx, ny, nz, 1, 1, 1, np.ones(24), [D0] * 6, [0] * 6)
    # 7-point pattern: each row holds itself plus its in-grid neighbours
    for a in range(24):
        cols = A.col[A.rowptr[a]:A.rowptr[a + 1]]
        i, j, l = a % nx, (a // nx) % ny, a // (nx * ny)
        expect = {a}
        for di, dj, dl in [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]:
            ii, jj, ll = i + di, j + dj, l + dl
            if 0 <= ii < nx and 0 <= jj < ny and 0 <= ll < nz:
                expect.add(ii + nx * (jj + ny * ll))
        assert set(cols.tolist()) == expect
        assert list(cols) == sorted(cols)


def test_2d_is_five_point():
    rng = np.random.default_rng(0)
    chip = synth.chip_2d(rng, 8)
    A = oracle.assemble_chip(chip)
    counts = np.diff(A.rowptr)
    assert counts.max() == 5 and counts.min() == 3
