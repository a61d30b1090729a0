"""CPU oracle for the block Krylov + operator action path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product path never imports this
package.  It shares no code with the GPU library; both sides only share the
seeded input generators.

Everything here is plain FP64:

* :func:`assemble` -- the cell-centred finite-volume heat operator as CSR
  (paper Sec. II-A, Eq. (1) and its boundary models; divergence-form reading
  so that A is SPD, matching the "sparse symmetric matrices" of Sec. V-A).
* :func:`cg_many` -- unpreconditioned CG from x0 = 0, one right-hand side at a
  time (the direct solution method of Sec. II-D; CG baseline of Sec. V-A).
  The method's block solve reaches X = A^-1 B, which is what this computes.
* :func:`boundary_source` -- the right-hand-side source g of nonhomogeneous
  boundary data (A x = q + g), face by face from the discretisation.
* :func:`jacobi_scaling`, :func:`pcg` -- the diagonal (Jacobi) preconditioner:
  S = diag(A)^(-1/2) and the symmetrically scaled S A S, and preconditioned
  CG with M = diag(A) (the paper leaves the preconditioner unstated; these
  define the optional Jacobi mode of the solves).
* :func:`pcg_many` -- the same in C, one column per thread (the timed CPU
  baseline with the GPU path's preconditioner).
* :func:`gemm` -- T = X C by plain loops (Sec. III-B, Eq. (5), raw weights).
* :func:`apply_many` -- F = A T by CSR products (Sec. III-C, Eq. (6)).
* :mod:`oracle.conv_ref` -- FP64 convolution encoder-decoder forward and
  backward for the learned initial guess.

Parity pins live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_NATIVE = os.path.join(_HERE, "liboracle_native.so")
_lib = None
_native = False
_native_fresh = False  # the native build is recompiled once per process, for the host it runs on


def build(force: bool = False, native: bool = False) -> str:
    """Compile the C oracle with gcc.  The default build uses portable flags
    (the tests may run on another host); ``native=True`` builds the copy the
    CPU baseline times, with -O3 -march=native for the host it runs on (the
    same source, compiled for speed, not changed)."""
    lib = _LIB_NATIVE if native else _LIB
    flags = ["-O3", "-march=native"] if native else ["-O2"]
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *flags, "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, lib)
    return lib


def select_build(native: bool) -> None:
    """Route later oracle calls to the native (-O3 -march=native) or the
    portable build; the native one is compiled on first use."""
    global _lib, _native
    if native != _native:
        _lib = None
        _native = native


def _load():
    global _lib, _native_fresh
    if _lib is None:
        path = build(force=_native and not _native_fresh, native=_native)
        _native_fresh = _native_fresh or _native
        lib = ctypes.CDLL(path)
        i64, i32, dbl, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        lib.orc_nnz_bound.restype = i64
        lib.orc_nnz_bound.argtypes = [i32, i32, i32]
        lib.orc_assemble_csr.restype = i64
        lib.orc_assemble_csr.argtypes = [i32, i32, i32, dbl, dbl, dbl, vp, vp, vp, vp, vp, vp]
        lib.orc_spmv.restype = None
        lib.orc_spmv.argtypes = [i64, vp, vp, vp, vp, vp]
        lib.orc_cg.restype = i32
        lib.orc_cg.argtypes = [i64, vp, vp, vp, vp, vp, dbl, i32, vp, vp]
        lib.orc_cg_many.restype = None
        lib.orc_cg_many.argtypes = [i64, vp, vp, vp, i32, vp, i64, vp, i64, dbl, i32, vp, vp, i32]
        lib.orc_pcg_many.restype = None
        lib.orc_pcg_many.argtypes = [i64, vp, vp, vp, i32, vp, i64, vp, i64, dbl, i32, vp, vp, i32]
        lib.orc_gemm.restype = None
        lib.orc_gemm.argtypes = [i64, i32, i64, vp, i64, vp, i64, vp, i64, i32]
        lib.orc_apply_many.restype = None
        lib.orc_apply_many.argtypes = [i64, vp, vp, vp, i64, vp, i64, vp, i64, i32]
        lib.orc_max_threads.restype = i32
        lib.orc_max_threads.argtypes = []
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class CSR:
    n: int
    rowptr: np.ndarray  # int64 (n+1)
    col: np.ndarray  # int32 (nnz)
    val: np.ndarray  # float64 (nnz)

    def to_dense(self) -> np.ndarray:
        """Dense copy (tiny grids only)."""
        D = np.zeros((self.n, self.n))
        for r in range(self.n):
            for p in range(self.rowptr[r], self.rowptr[r + 1]):
                D[r, self.col[p]] += self.val[p]
        return D


def assemble(nx, ny, nz, lx, ly, lz, k, bc, h) -> CSR:
    lib = _load()
    n = nx * ny * nz
    k = np.ascontiguousarray(k, dtype=np.float64).reshape(-1)
    assert k.size == n
    bc_a = np.ascontiguousarray(bc, dtype=np.int32)
    h_a = np.ascontiguousarray(h, dtype=np.float64)
    cap = lib.orc_nnz_bound(nx, ny, nz)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(cap, dtype=np.int32)
    val = np.zeros(cap, dtype=np.float64)
    nnz = lib.orc_assemble_csr(nx, ny, nz, lx, ly, lz, _p(k), _p(bc_a), _p(h_a), _p(rowptr), _p(col), _p(val))
    if nnz < 0:
        raise ValueError("bad grid")
    return CSR(n, rowptr, col[:nnz].copy(), val[:nnz].copy())


def assemble_chip(chip) -> CSR:
    return assemble(chip.nx, chip.ny, chip.nz, chip.lx, chip.ly, chip.lz, chip.k, chip.bc, chip.h)


def spmv(A: CSR, x: np.ndarray) -> np.ndarray:
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.n)
    lib.orc_spmv(A.n, _p(A.rowptr), _p(A.col), _p(A.val), _p(x), _p(y))
    return y


def cg(A: CSR, b: np.ndarray, tol: float, maxit: int = 100000):
    """One CG solve from x0 = 0.  Returns (x, iterations, true relative residual)."""
    lib = _load()
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty(A.n)
    rr = np.zeros(1)
    scratch = np.empty(3 * A.n)
    it = lib.orc_cg(A.n, _p(A.rowptr), _p(A.col), _p(A.val), _p(b), _p(x), tol, maxit, _p(rr), _p(scratch))
    return x, int(it), float(rr[0])


def cg_many(A: CSR, B: np.ndarray, tol: float, maxit: int = 100000, nthreads: int = 0):
    """Independent CG per row of B (shape (s, N)).  Returns (X, iters, relres)."""
    lib = _load()
    B = np.ascontiguousarray(B, dtype=np.float64)
    s = B.shape[0]
    X = np.empty_like(B)
    iters = np.zeros(s, dtype=np.int32)
    relres = np.zeros(s)
    lib.orc_cg_many(A.n, _p(A.rowptr), _p(A.col), _p(A.val), s, _p(B), A.n, _p(X), A.n, tol, maxit,
                    _p(iters), _p(relres), nthreads)
    return X, iters, relres


def pcg_many(A: CSR, B: np.ndarray, tol: float, maxit: int = 100000, nthreads: int = 0):
    """Jacobi-preconditioned CG (M = diag(A)) per row of B (shape (s, N)),
    the stopping rule of :func:`pcg`.  Returns (X, iters, relres)."""
    lib = _load()
    B = np.ascontiguousarray(B, dtype=np.float64)
    s = B.shape[0]
    X = np.empty_like(B)
    iters = np.zeros(s, dtype=np.int32)
    relres = np.zeros(s)
    lib.orc_pcg_many(A.n, _p(A.rowptr), _p(A.col), _p(A.val), s, _p(B), A.n, _p(X), A.n, tol, maxit,
                     _p(iters), _p(relres), nthreads)
    return X, iters, relres


def diagonal(A: CSR) -> np.ndarray:
    """The diagonal entries of A."""
    d = np.zeros(A.n)
    for r in range(A.n):
        for p in range(A.rowptr[r], A.rowptr[r + 1]):
            if A.col[p] == r:
                d[r] += A.val[p]
    return d


def jacobi_scaling(A: CSR):
    """Symmetric diagonal scaling: S = diag(A)^(-1/2) and S A S as CSR, entry
    (i, j) = a_ij s_i s_j.  Returns (S as a vector, S A S)."""
    sc = 1.0 / np.sqrt(diagonal(A))
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    val = A.val * sc[rows] * sc[A.col]
    return sc, CSR(A.n, A.rowptr.copy(), A.col.copy(), val)


def pcg(A: CSR, b: np.ndarray, tol: float, maxit: int = 100000, minv: np.ndarray = None):
    """Preconditioned CG from x0 = 0 with M^-1 = diag(minv) (plain CG when
    minv is None): z = M^-1 r, rho = r^T z, alpha = rho / p^T A p,
    x += alpha p, r -= alpha A p, beta = rho' / rho, p = z' + beta p; stops
    when ||r|| <= tol ||b|| (the unpreconditioned residual) or after maxit
    iterations.  Returns (x, iterations, true relative residual)."""
    b = np.asarray(b, dtype=np.float64)
    w = np.ones(A.n) if minv is None else np.asarray(minv, dtype=np.float64)
    x = np.zeros(A.n)
    r = b.copy()
    z = w * r
    p = z.copy()
    rho = r @ z
    bn = np.linalg.norm(b)
    it = 0
    while np.linalg.norm(r) > tol * bn and it < maxit:
        q = spmv(A, p)
        alpha = rho / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = w * r
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
        it += 1
    res = np.linalg.norm(b - spmv(A, x)) / bn if bn > 0 else 0.0
    return x, it, res


def boundary_source(nx, ny, nz, lx, ly, lz, k, bc, h, u_face) -> np.ndarray:
    """g (N,): the right-hand-side source of nonhomogeneous boundary data
    (Sec. II-A; Dirichlet value or Robin ambient u_face per face, -x, +x, -y,
    +y, -z, +z).  A boundary face of cell a with weight w (the Dirichlet or
    Robin weight of the assembly) contributes the flux w (x_a - u_face), so
    A x = q + g with g_a = sum of w u_face over the cell's boundary faces."""
    k = np.asarray(k, dtype=np.float64).reshape(nz, ny, nx)
    d = (lx / nx, ly / ny, lz / nz)
    g = np.zeros((nz, ny, nx))

    def weight(kind, ka, dd, hh):
        if kind == 0:  # Dirichlet
            return 2.0 * ka / (dd * dd)
        if kind == 2:  # Robin
            return 1.0 / (dd * (dd / (2.0 * ka) + 1.0 / hh))
        return np.zeros_like(ka)

    # face f = 2 axis + side; axis 0 = x (last index), 1 = y, 2 = z (first)
    for f in range(6):
        ax, side = divmod(f, 2)
        sl = [slice(None)] * 3
        sl[2 - ax] = -1 if side else 0
        sl = tuple(sl)
        g[sl] += weight(bc[f], k[sl], d[ax], h[f]) * u_face[f]
    return g.reshape(-1)


def gemm(X: np.ndarray, C: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """T = X C with X (s, N) and C (M, s) in the column-major convention;
    returns T as (M, N)."""
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    C = np.ascontiguousarray(C, dtype=np.float64)
    s, n = X.shape
    m = C.shape[0]
    assert C.shape[1] == s
    T = np.empty((m, n))
    lib.orc_gemm(n, s, m, _p(X), n, _p(C), s, _p(T), n, nthreads)
    return T


def apply_many(A: CSR, T: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """F = A T for T of shape (M, N); returns (M, N)."""
    lib = _load()
    T = np.ascontiguousarray(T, dtype=np.float64)
    m = T.shape[0]
    F = np.empty_like(T)
    lib.orc_apply_many(A.n, _p(A.rowptr), _p(A.col), _p(A.val), m, _p(T), A.n, _p(F), A.n, nthreads)
    return F


def max_threads() -> int:
    return int(_load().orc_max_threads())
