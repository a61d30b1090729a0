"""Thin Python binding of the C ABI in ``include/blockoa.h``.

Argument marshalling only: every step of the path runs in the gfx950 kernels
of ``libblockoa.so``; torch provides device memory and the current stream.
There is no CPU fallback -- if the library is missing this module raises.

Array convention: a block of ``k`` fields over ``N`` cells is a torch tensor
of shape ``(k, N)`` whose rows are contiguous, i.e. a column-major ``N x k``
matrix with leading dimension ``tensor.stride(0)``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libblockoa.so")

OK, EINVAL, ENOTSPD, ENOCONV, EBREAKDOWN, EHIP, ENOMEM, ENOTIMPL = range(8)
F64, F32, BF16 = 0, 1, 2
PRECOND_NONE, PRECOND_JACOBI = 0, 1
NOISE_NONE, NOISE_UNIFORM, NOISE_GAUSSIAN = 0, 1, 2


class Noise(ctypes.Structure):
    """The noise term of Eq. (5): kind, amplitude (half-width or standard
    deviation), generator seed and the global index of the call's field 0."""
    _fields_ = [("kind", ctypes.c_int), ("amplitude", ctypes.c_double), ("seed", ctypes.c_ulonglong),
                ("field_offset", ctypes.c_ulonglong)]
BC_DIRICHLET0, BC_ADIABATIC, BC_ROBIN = 0, 1, 2
STATUS_NAMES = {0: "BKO_OK", 1: "BKO_EINVAL", 2: "BKO_ENOTSPD", 3: "BKO_ENOCONV",
                4: "BKO_EBREAKDOWN", 5: "BKO_EHIP", 6: "BKO_ENOMEM", 7: "BKO_ENOTIMPL"}
TORCH_DTYPE = {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16}
DTYPE_CODE = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}
DTYPE_NAME = {"f64": F64, "f32": F32, "bf16": BF16}

#: every symbol include/blockoa.h declares
EXPORTED = ("bko_version", "bko_last_error", "bko_operator_bytes", "bko_assemble_heat_operator",
            "bko_operator_dims", "bko_destroy_operator", "bko_block_krylov_workspace_bytes",
            "bko_block_krylov_solve", "bko_combine", "bko_apply_operator", "bko_residual",
            "bko_timing_enable", "bko_timing_query", "bko_timing_reset", "bko_cg_workspace_bytes",
            "bko_cg_solve", "bko_batch_plan_create", "bko_batch_plan_destroy", "bko_batch_workspace_bytes",
            "bko_batch_tune", "bko_batch_solve", "bko_nn_conv2d", "bko_nn_wgrad_work_floats",
            "bko_nn_conv2d_wgrad", "bko_unet_create", "bko_unet_destroy", "bko_unet_sizes", "bko_unet_set_params",
            "bko_unet_forward", "bko_unet_infer", "bko_unet_gradient", "bko_unet_adam_step", "bko_lstart_pack",
            "bko_lstart_pack_target", "bko_lstart_unpack", "bko_jacobi_smooth", "bko_operator_set_precond",
            "bko_operator_get_precond", "bko_timing_set_stride", "bko_combine_apply_workspace_bytes",
            "bko_combine_apply", "bko_combine_noisy", "bko_noise_fill", "bko_normalize_weights",
            "bko_boundary_source", "bko_add_column", "bko_apply_operator_tiling",
            "bko_copy", "bko_block_krylov_solve_noalloc", "bko_batch_run", "bko_batch_output_tuning")


class BlockoaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("refinements", ctypes.c_int), ("deflated", ctypes.c_int),
                ("status", ctypes.c_int), ("max_rel_res", ctypes.c_double), ("x0_rejected", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libblockoa.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2510_23221_amd.build` "
                          "(there is no fallback path)")
    lib = ctypes.CDLL(path)
    vp, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    sig = {
        "bko_version": (ctypes.c_char_p, []),
        "bko_last_error": (ctypes.c_char_p, []),
        "bko_operator_bytes": (i32, [i32, i32, i32, ctypes.POINTER(sz)]),
        "bko_assemble_heat_operator": (i32, [i32, i32, i32, dbl, dbl, dbl, vp, vp, vp, vp, sz, vp,
                                             ctypes.POINTER(vp)]),
        "bko_operator_dims": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "bko_destroy_operator": (i32, [vp]),
        "bko_block_krylov_workspace_bytes": (i32, [vp, i32, i32, ctypes.POINTER(sz)]),
        "bko_block_krylov_solve": (i32, [vp, i32, vp, i32, vp, i32, vp, i32, i32, dbl, i32, vp, sz,
                                         ctypes.POINTER(SolveInfo), vp]),
        "bko_combine": (i32, [i32, i32, i32, vp, i32, i32, vp, i32, i32, vp, i32, i32, i32, vp]),
        "bko_apply_operator": (i32, [vp, i32, vp, i32, i32, vp, i32, i32, i32, vp]),
        "bko_residual": (i32, [vp, i32, vp, i32, vp, i32, vp, i32, vp]),
        "bko_timing_enable": (i32, [i32]),
        "bko_timing_query": (i32, [i32, ctypes.POINTER(i32), ctypes.POINTER(dbl)]),
        "bko_timing_reset": (i32, []),
        "bko_cg_workspace_bytes": (i32, [vp, i32, ctypes.POINTER(sz)]),
        "bko_batch_plan_create": (i32, [i32, ctypes.POINTER(vp), i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                        ctypes.POINTER(vp)]),
        "bko_batch_run": (i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(i32), ctypes.POINTER(vp), ctypes.POINTER(i32),
                                ctypes.POINTER(vp), ctypes.POINTER(i32), ctypes.POINTER(vp), ctypes.POINTER(i32),
                                ctypes.POINTER(vp), ctypes.POINTER(i32), dbl, i32, vp, sz, ctypes.POINTER(SolveInfo),
                                vp]),
        "bko_batch_output_tuning": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_int64)]),
        "bko_batch_plan_destroy": (i32, [vp]),
        "bko_nn_conv2d": (i32, [vp, i32, vp, i32, i32, i32, i32, i32, i32, i32, vp, i32, vp, vp, i32, vp]),
        "bko_nn_wgrad_work_floats": (sz, [i32, i32, i32, i32, i32, i32]),
        "bko_nn_conv2d_wgrad": (i32, [vp, i32, vp, i32, i32, vp, i32, i32, i32, i32, i32, vp, vp, vp, vp]),
        "bko_unet_create": (i32, [i32, i32, i32, i32, i32, i32, ctypes.POINTER(vp)]),
        "bko_unet_destroy": (i32, [vp]),
        "bko_unet_sizes": (i32, [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(sz), ctypes.POINTER(sz)]),
        "bko_unet_set_params": (i32, [vp, vp, vp, vp]),
        "bko_unet_forward": (i32, [vp, vp, vp, vp, i32, vp, vp]),
        "bko_unet_infer": (i32, [vp, vp, vp, vp, i32, vp, vp]),
        "bko_unet_gradient": (i32, [vp, vp, vp, vp, vp, i32, ctypes.POINTER(ctypes.c_float), vp]),
        "bko_unet_adam_step": (i32, [vp, vp, ctypes.c_float, vp]),
        "bko_lstart_pack": (i32, [i32, i32, i32, vp, i32, i32, vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                  vp, vp, vp]),
        "bko_lstart_pack_target": (i32, [i32, vp, i32, i32, vp, dbl, vp, vp]),
        "bko_lstart_unpack": (i32, [i32, vp, i32, vp, dbl, vp, i32, vp]),
        "bko_jacobi_smooth": (i32, [vp, i32, vp, i32, vp, i32, vp, i32, i32, dbl, vp]),
        "bko_batch_workspace_bytes": (i32, [vp, ctypes.POINTER(sz)]),
        "bko_batch_tune": (i32, [vp, vp, sz, ctypes.POINTER(i32), vp]),
        "bko_batch_solve": (i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(i32), ctypes.POINTER(vp),
                                  ctypes.POINTER(i32), ctypes.POINTER(vp), ctypes.POINTER(i32), dbl, i32, vp, sz,
                                  ctypes.POINTER(SolveInfo), vp]),
        "bko_cg_solve": (i32, [vp, i32, vp, i32, vp, i32, dbl, i32, vp, sz, ctypes.POINTER(i32),
                               ctypes.POINTER(SolveInfo), vp]),
        "bko_operator_set_precond": (i32, [vp, i32]),
        "bko_operator_get_precond": (i32, [vp, ctypes.POINTER(i32)]),
        "bko_timing_set_stride": (i32, [i32]),
        "bko_combine_apply_workspace_bytes": (i32, [vp, i32, ctypes.POINTER(sz)]),
        "bko_combine_apply": (i32, [vp, i32, i32, vp, i32, vp, i32, vp, i32, vp, i32, vp, sz, vp]),
        "bko_combine_noisy": (i32, [i32, i32, i32, vp, i32, vp, i32, vp, i32, ctypes.POINTER(Noise), vp]),
        "bko_noise_fill": (i32, [i32, i32, vp, i32, ctypes.POINTER(Noise), vp]),
        "bko_normalize_weights": (i32, [i32, i32, vp, i32, dbl, vp, vp]),
        "bko_boundary_source": (i32, [vp, vp, ctypes.POINTER(dbl), vp, vp]),
        "bko_add_column": (i32, [i32, i32, vp, i32, vp, dbl, vp]),
        "bko_apply_operator_tiling": (i32, [vp, i32, vp, i32, i32, vp, i32, i32, i32, ctypes.POINTER(i32)]),
        "bko_copy": (i32, [vp, vp, sz, vp]),
        "bko_block_krylov_solve_noalloc": (i32, [vp, i32, vp, i32, vp, i32, vp, i32, i32, dbl, i32,
                                                 ctypes.POINTER(SolveInfo), vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != OK:
        raise BlockoaError(status, load_library().bko_last_error().decode())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _block(t: torch.Tensor, name: str):
    """(k, N) tensor -> (pointer, ld, dtype code).  Rows must be contiguous."""
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a (k, N) tensor with contiguous rows")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    ld = t.stride(0) if t.shape[0] > 1 else max(t.stride(0), t.shape[1])
    return _ptr(t), ld, DTYPE_CODE[t.dtype]


def version() -> str:
    return load_library().bko_version().decode()


def operator_bytes(nx: int, ny: int, nz: int) -> int:
    out = ctypes.c_size_t()
    _check(load_library().bko_operator_bytes(nx, ny, nz, ctypes.byref(out)))
    return out.value


class HeatOperator:
    """Discretised steady heat operator A of one chip (device-resident).

    Owns the device buffers (conductivity and coefficient storage) through
    torch; the C handle holds host metadata only."""

    def __init__(self, nx: int, ny: int, nz: int, lx: float, ly: float, lz: float,
                 k: torch.Tensor, bc: Sequence[int], h: Sequence[float], stream=None):
        lib = load_library()
        self.dims = (nx, ny, nz)
        self.n = nx * ny * nz
        self.k = k.to(dtype=torch.float64).contiguous()
        if not self.k.is_cuda:
            raise ValueError("k must live on the GPU")
        nbytes = operator_bytes(nx, ny, nz)
        self.coeff = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.k.device)
        off = (-self.coeff.data_ptr()) % 256
        self._coeff_ptr = self.coeff.data_ptr() + off
        bc_a = (ctypes.c_int * 6)(*[int(b) for b in bc])
        h_a = (ctypes.c_double * 6)(*[float(x) for x in h])
        handle = ctypes.c_void_p()
        _check(lib.bko_assemble_heat_operator(nx, ny, nz, lx, ly, lz, _ptr(self.k), bc_a, h_a,
                                              ctypes.c_void_p(self._coeff_ptr), nbytes, _stream(stream),
                                              ctypes.byref(handle)))
        self.handle = handle

    @classmethod
    def from_chip(cls, chip, device="cuda", stream=None, precond: int = 0) -> "HeatOperator":
        k = torch.as_tensor(chip.k, dtype=torch.float64, device=device)
        op = cls(chip.nx, chip.ny, chip.nz, chip.lx, chip.ly, chip.lz, k, chip.bc, chip.h, stream)
        if precond:
            op.precond = precond
        return op

    @property
    def precond(self) -> int:
        """PRECOND_NONE or PRECOND_JACOBI: the preconditioner of every solve on this operator."""
        out = ctypes.c_int()
        _check(load_library().bko_operator_get_precond(self.handle, ctypes.byref(out)))
        return out.value

    @precond.setter
    def precond(self, kind: int):
        _check(load_library().bko_operator_set_precond(self.handle, int(kind)))

    def _arrays(self, first: int, count: int, esize: int):
        n = self.n
        base = self._coeff_ptr - self.coeff.data_ptr()
        sizes = [8] * 4 + [4] * 4 + [8] * 4 + [4] * 4 + [8]
        off = 0
        for k in range(first):
            off = (off + sizes[k] * n + 255) // 256 * 256
        out = []
        for k in range(first, first + count):
            assert sizes[k] == esize
            t = self.coeff[base + off: base + off + esize * n].view(torch.float64 if esize == 8 else torch.float32)
            out.append(t)
            off = (off + esize * n + 255) // 256 * 256
        return out

    def coefficients(self):
        """(diag, wx, wy, wz) FP64 views of the coefficient storage (for tests)."""
        return tuple(self._arrays(0, 4, 8))

    def scaled_coefficients(self):
        """(diag, wx, wy, wz) FP64 views of the Jacobi-scaled operator S A S and
        the scale S = diag(A)^(-1/2) (for tests)."""
        return tuple(self._arrays(8, 4, 8)), self._arrays(16, 1, 8)[0]

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load_library().bko_destroy_operator(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_bytes(A: HeatOperator, s: int, compute: int = F64) -> int:
    out = ctypes.c_size_t()
    _check(load_library().bko_block_krylov_workspace_bytes(A.handle, s, compute, ctypes.byref(out)))
    return out.value


def _aligned_workspace(nbytes: int, device) -> tuple:
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


def block_krylov_solve(A: HeatOperator, B: torch.Tensor, tol: float, compute: int = F64,
                       max_iter: int = 100000, X0: Optional[torch.Tensor] = None,
                       X: Optional[torch.Tensor] = None, work=None, stream=None, check: bool = True):
    """Solve A X = B (B: (s, N) FP64 on the GPU).  Returns (X, info dict).

    ``check=False`` returns non-converged results instead of raising."""
    s = B.shape[0]
    bp, ldb, bt = _block(B, "B")
    if bt != F64:
        raise ValueError("B must be float64")
    if X is None:
        X = torch.empty_like(B)
    xp, ldx, _ = _block(X, "X")
    x0p, ldx0 = (ctypes.c_void_p(0), 0)
    if X0 is not None:
        x0p, ldx0, x0t = _block(X0, "X0")
        if x0t != F64:
            raise ValueError("X0 must be float64")
    nbytes = workspace_bytes(A, s, compute)
    if work is None:
        buf, wptr = _aligned_workspace(nbytes, B.device)
    else:
        buf, wptr = work, work.data_ptr()
    info = SolveInfo()
    st = load_library().bko_block_krylov_solve(A.handle, s, bp, ldb, xp, ldx, x0p, ldx0, compute, tol,
                                               max_iter, ctypes.c_void_p(wptr), nbytes, ctypes.byref(info),
                                               _stream(stream))
    if check and st != OK:
        _check(st)
    d = info.as_dict()
    d["status_name"] = STATUS_NAMES.get(st, str(st))
    return X, d


#: device scratch bytes of block_krylov_solve_noalloc (include/blockoa.h)
NOALLOC_SCRATCH_BYTES = 128 << 20


def block_krylov_solve_noalloc(A: HeatOperator, B: torch.Tensor, tol: float, compute: int = F64,
                               max_iter: int = 100000, X0: Optional[torch.Tensor] = None,
                               X: Optional[torch.Tensor] = None, stream=None, check: bool = True):
    """block_krylov_solve on the library's own scratch memory (no workspace
    argument; the C entry point allocates nothing).  Returns (X, info)."""
    s = B.shape[0]
    bp, ldb, bt = _block(B, "B")
    if bt != F64:
        raise ValueError("B must be float64")
    if X is None:
        X = torch.empty_like(B)
    xp, ldx, _ = _block(X, "X")
    x0p, ldx0 = (ctypes.c_void_p(0), 0)
    if X0 is not None:
        x0p, ldx0, x0t = _block(X0, "X0")
        if x0t != F64:
            raise ValueError("X0 must be float64")
    info = SolveInfo()
    st = load_library().bko_block_krylov_solve_noalloc(A.handle, s, bp, ldb, xp, ldx, x0p, ldx0, compute, tol,
                                                       max_iter, ctypes.byref(info), _stream(stream))
    if check and st != OK:
        _check(st)
    d = info.as_dict()
    d["status_name"] = STATUS_NAMES.get(st, str(st))
    return X, d


class BatchPlan:
    """A batch of chips solved together (one s for all): grouped launches
    over every chip, graph-captured iteration chunks on a non-null stream,
    per-chip workgroup counts chosen by the autotuner.  With per-chip field
    counts ``m`` the plan also runs the outputs (``run``): one grouped
    combination and one grouped operator action over all chips, in the
    dtypes ``comb_compute`` (arithmetic of T = X C), ``t_dtype`` and
    ``f_dtype`` (storage of T and F)."""

    def __init__(self, ops: Sequence[HeatOperator], s: int, compute: int = F64, m: Optional[Sequence[int]] = None,
                 comb_compute: int = F64, t_dtype=torch.float64, f_dtype=torch.float64):
        lib = load_library()
        self.ops = list(ops)
        self.s = s
        self.compute = compute
        self.m = None if m is None else [int(v) for v in m]
        self.t_dtype, self.f_dtype = t_dtype, f_dtype
        arr = (ctypes.c_void_p * len(self.ops))(*[o.handle.value for o in self.ops])
        marr = None if self.m is None else (ctypes.c_int * len(self.ops))(*self.m)
        dt = (ctypes.c_int * 4)(compute, comb_compute, DTYPE_CODE[t_dtype], DTYPE_CODE[f_dtype])
        h = ctypes.c_void_p()
        _check(lib.bko_batch_plan_create(len(self.ops), arr, s, marr, dt, ctypes.byref(h)))
        self.handle = h
        self._work = None

    def workspace_bytes(self) -> int:
        out = ctypes.c_size_t()
        _check(load_library().bko_batch_workspace_bytes(self.handle, ctypes.byref(out)))
        return out.value

    def _workspace(self, device):
        nbytes = self.workspace_bytes()
        if self._work is None or self._work[2] < nbytes:
            buf, ptr = _aligned_workspace(nbytes, device)
            self._work = (buf, ptr, nbytes)
        return self._work[1], self._work[2]

    def tune(self, device="cuda", stream=None) -> int:
        """Run the autotuner; returns the chosen row tiles per workgroup."""
        ptr, nbytes = self._workspace(device)
        tpw = ctypes.c_int()
        _check(load_library().bko_batch_tune(self.handle, ctypes.c_void_p(ptr), nbytes, ctypes.byref(tpw),
                                             _stream(stream)))
        return tpw.value

    def solve(self, Bs: Sequence[torch.Tensor], tol: float, max_iter: int = 100000, X0s=None, Xs=None,
              stream=None, check: bool = True):
        """Bs: one (s, N_c) FP64 tensor per chip.  Returns (Xs, list of info dicts)."""
        nc = len(self.ops)
        if len(Bs) != nc:
            raise ValueError("one right-hand-side block per chip")
        if Xs is None:
            Xs = [torch.empty_like(b) for b in Bs]
        bp, lb, xp, lx = [], [], [], []
        for b, x in zip(Bs, Xs):
            p, ld, t = _block(b, "B")
            if t != F64:
                raise ValueError("B must be float64")
            bp.append(p.value)
            lb.append(ld)
            p, ld, _ = _block(x, "X")
            xp.append(p.value)
            lx.append(ld)
        VP, I32 = ctypes.c_void_p * nc, ctypes.c_int * nc
        x0a, lx0a = None, None
        if X0s is not None:
            x0p, lx0 = [], []
            for x0 in X0s:
                if x0 is None:
                    x0p.append(None)
                    lx0.append(0)
                else:
                    p, ld, _ = _block(x0, "X0")
                    x0p.append(p.value)
                    lx0.append(ld)
            x0a, lx0a = VP(*x0p), I32(*lx0)
        ptr, nbytes = self._workspace(Bs[0].device)
        infos = (SolveInfo * nc)()
        st = load_library().bko_batch_solve(self.handle, VP(*bp), I32(*lb), VP(*xp), I32(*lx), x0a, lx0a, tol,
                                            max_iter, ctypes.c_void_p(ptr), nbytes, infos, _stream(stream))
        if check and st != OK:
            _check(st)
        out = []
        for i in infos:
            d = i.as_dict()
            d["status_name"] = STATUS_NAMES.get(d["status"], str(d["status"]))
            out.append(d)
        return Xs, out

    def run(self, Bs: Sequence[torch.Tensor], Cs: Sequence[torch.Tensor], tol: float, Xs=None, Ts=None, Fs=None,
            max_iter: int = 100000, stream=None, check: bool = True):
        """The whole path for every chip: Bs (s, N_c) FP64, Cs (M_c, s) FP64
        (row j holds field j's weights); returns (Xs, Ts, Fs, infos) with
        T, F of shape (M_c, N_c)."""
        nc = len(self.ops)
        if self.m is None:
            raise ValueError("the plan was created without field counts")
        if len(Bs) != nc or len(Cs) != nc:
            raise ValueError("one right-hand-side block and one weight block per chip")
        dev = Bs[0].device
        if Xs is None:
            Xs = [torch.empty_like(b) for b in Bs]
        if Ts is None:
            Ts = [torch.empty((mc, o.n), dtype=self.t_dtype, device=dev) for mc, o in zip(self.m, self.ops)]
        if Fs is None:
            Fs = [torch.empty((mc, o.n), dtype=self.f_dtype, device=dev) for mc, o in zip(self.m, self.ops)]
        cols = {k: ([], []) for k in "BXCTF"}
        for k, arrs, name in (("B", Bs, "B"), ("X", Xs, "X"), ("T", Ts, "T"), ("F", Fs, "F")):
            for t in arrs:
                if t.shape[0] == 0:
                    cols[k][0].append(None)
                    cols[k][1].append(t.shape[1])
                    continue
                p, ld, _ = _block(t, name)
                cols[k][0].append(p.value)
                cols[k][1].append(ld)
        for c, mc in zip(Cs, self.m):
            if mc == 0:  # no fields: C is not read
                cols["C"][0].append(None)
                cols["C"][1].append(self.s)
                continue
            if c.dtype != torch.float64 or c.dim() != 2 or tuple(c.shape) != (mc, self.s) or c.stride(1) != 1 \
                    or not c.is_cuda:
                raise ValueError("C must be an (M_c, s) float64 GPU tensor with contiguous rows")
            cols["C"][0].append(c.data_ptr())
            cols["C"][1].append(max(c.stride(0), self.s))
        VP, I32 = ctypes.c_void_p * nc, ctypes.c_int * nc
        arg = {k: (VP(*v[0]), I32(*v[1])) for k, v in cols.items()}
        ptr, nbytes = self._workspace(dev)
        infos = (SolveInfo * nc)()
        st = load_library().bko_batch_run(self.handle, *arg["B"], *arg["X"], *arg["C"], *arg["T"], *arg["F"], tol,
                                          max_iter, ctypes.c_void_p(ptr), nbytes, infos, _stream(stream))
        if check and st != OK:
            _check(st)
        out = []
        for i in infos:
            d = i.as_dict()
            d["status_name"] = STATUS_NAMES.get(d["status"], str(d["status"]))
            out.append(d)
        return Xs, Ts, Fs, out

    def output_tuning(self):
        """(tile height cap, fields per workgroup) chosen on the first run
        (-1, -1 before it)."""
        ty, fpw = ctypes.c_int(), ctypes.c_int64()
        _check(load_library().bko_batch_output_tuning(self.handle, ctypes.byref(ty), ctypes.byref(fpw)))
        return ty.value, fpw.value

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load_library().bko_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _f32(t, name):
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 tensor on the GPU")
    return _ptr(t)


def nn_conv2d(A, w_bf16, bias=None, B=None, mode=0, relu=False, transposed=False, out_channels=None):
    """One convolution of the learned-start network (see include/blockoa.h).
    A: (N, Ca, h, w) with (h, w) = (H, W), (2H, 2W) or (H/2, W/2) for modes 0,
    1, 2; B: (N, Cb, H, W) for mode 2.  w_bf16: int16 tensor of BF16 bits."""
    N, Ca = A.shape[0], A.shape[1]
    if mode == 0:
        H, W = A.shape[2], A.shape[3]
    elif mode == 1:
        H, W = A.shape[2] // 2, A.shape[3] // 2
    else:
        H, W = B.shape[2], B.shape[3]
    Cb = 0 if B is None else B.shape[1]
    K = w_bf16.shape[-1]
    Co = out_channels if out_channels is not None else (w_bf16.shape[1] if transposed else w_bf16.shape[0])
    out = torch.empty((N, Co, H, W), dtype=torch.float32, device=A.device)
    _check(load_library().bko_nn_conv2d(_f32(A, "A"), Ca, None if B is None else _f32(B, "B"), Cb, mode, N, H, W, Co,
                                        K, _ptr(w_bf16), int(transposed), None if bias is None else _f32(bias, "bias"),
                                        _ptr(out), int(relu), _stream()))
    return out


def nn_conv2d_wgrad(A, g, K, B=None, mode=0):
    """Filter and bias gradients of nn_conv2d for output gradient g (N, Co, H, W)."""
    N, Co, H, W = g.shape
    Ca = A.shape[1]
    Cb = 0 if B is None else B.shape[1]
    lib = load_library()
    nw = lib.bko_nn_wgrad_work_floats(N, H, W, Ca + Cb, Co, K)
    work = torch.empty(max(nw, 1), dtype=torch.float32, device=A.device)
    gw = torch.empty((Co, Ca + Cb, K, K), dtype=torch.float32, device=A.device)
    gb = torch.empty(Co, dtype=torch.float32, device=A.device)
    _check(lib.bko_nn_conv2d_wgrad(_f32(A, "A"), Ca, None if B is None else _f32(B, "B"), Cb, mode, _f32(g, "g"), N, H,
                                   W, Co, K, _ptr(work), _ptr(gw), _ptr(gb), _stream()))
    return gw, gb


def to_bf16_bits(t: torch.Tensor) -> torch.Tensor:
    """float32 tensor -> int16 tensor of its BF16 bits (round to nearest even)."""
    return t.to(torch.bfloat16).view(torch.int16)


class UNet:
    """The learned-start encoder-decoder (layer table in include/blockoa.h);
    parameters, gradients and Adam state live in one device buffer."""

    def __init__(self, cin: int, cout: int, base: int, height: int, width: int, max_batch: int, device="cuda"):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.bko_unet_create(cin, cout, base, height, width, max_batch, ctypes.byref(h)))
        self.handle = h
        self.cin, self.cout, self.base, self.height, self.width, self.max_batch = cin, cout, base, height, width, max_batch
        npar, sb, wb = ctypes.c_int64(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib.bko_unet_sizes(h, ctypes.byref(npar), ctypes.byref(sb), ctypes.byref(wb)))
        self.nparams = npar.value
        self._state, self._state_ptr = _aligned_workspace(sb.value, device)
        self._work, self._work_ptr = _aligned_workspace(wb.value, device)

    def _view(self, k):
        off = self._state_ptr - self._state.data_ptr()
        return self._state[off + 4 * k * self.nparams: off + 4 * (k + 1) * self.nparams].view(torch.float32)

    @property
    def params(self) -> torch.Tensor:
        return self._view(0)

    @property
    def grads(self) -> torch.Tensor:
        return self._view(1)

    def set_params(self, p: torch.Tensor):
        p = p.to(device=self._state.device, dtype=torch.float32).contiguous()
        if p.numel() != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters")
        _check(load_library().bko_unet_set_params(self.handle, ctypes.c_void_p(self._state_ptr), _ptr(p), _stream()))
        torch.cuda.current_stream().synchronize()

    def forward(self, x: torch.Tensor, y: Optional[torch.Tensor] = None) -> torch.Tensor:
        n = x.shape[0]
        if y is None:
            y = torch.empty((n, self.cout, self.height, self.width), dtype=torch.float32, device=x.device)
        _check(load_library().bko_unet_forward(self.handle, ctypes.c_void_p(self._state_ptr),
                                               ctypes.c_void_p(self._work_ptr), _f32(x, "x"), n, _f32(y, "y"),
                                               _stream()))
        return y

    def infer(self, x: torch.Tensor, y: Optional[torch.Tensor] = None) -> torch.Tensor:
        """The forward pass with the convolutions on the BF16 matrix cores."""
        n = x.shape[0]
        if y is None:
            y = torch.empty((n, self.cout, self.height, self.width), dtype=torch.float32, device=x.device)
        _check(load_library().bko_unet_infer(self.handle, ctypes.c_void_p(self._state_ptr),
                                             ctypes.c_void_p(self._work_ptr), _f32(x, "x"), n, _f32(y, "y"),
                                             _stream()))
        return y

    def gradient(self, x: torch.Tensor, target: torch.Tensor, want_loss: bool = True):
        loss = ctypes.c_float()
        _check(load_library().bko_unet_gradient(self.handle, ctypes.c_void_p(self._state_ptr),
                                                ctypes.c_void_p(self._work_ptr), _f32(x, "x"), _f32(target, "target"),
                                                x.shape[0], ctypes.byref(loss) if want_loss else None, _stream()))
        return loss.value if want_loss else None

    def adam_step(self, lr: float):
        _check(load_library().bko_unet_adam_step(self.handle, ctypes.c_void_p(self._state_ptr), lr, _stream()))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load_library().bko_unet_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lstart_pack(chip_dims, F: torch.Tensor, k_cell: torch.Tensor, kmu: float, ksig: float, hval: float,
                x: Optional[torch.Tensor] = None, scale: Optional[torch.Tensor] = None):
    """Network input of the fields F ((m, N) FP64, one field per row) of one
    chip.  Returns (x (m, 2 nz + 1, ny, nx) float32, scale (m,) float64);
    x and scale may be given (contiguous, e.g. slices of the input of a
    batch that spans several chips)."""
    nx, ny, nz = chip_dims
    m = F.shape[0]
    fp, ldf, ft = _block(F, "F")
    if ft != F64:
        raise ValueError("F must be float64")
    if x is None:
        x = torch.empty((m, 2 * nz + 1, ny, nx), dtype=torch.float32, device=F.device)
    elif x.shape != (m, 2 * nz + 1, ny, nx) or x.dtype != torch.float32 or not x.is_contiguous():
        raise ValueError("x must be a contiguous float32 (m, 2 nz + 1, ny, nx) tensor")
    if scale is None:
        scale = torch.empty(m, dtype=torch.float64, device=F.device)
    elif scale.shape != (m,) or scale.dtype != torch.float64 or not scale.is_contiguous():
        raise ValueError("scale must be a contiguous float64 (m,) tensor")
    k = k_cell.to(dtype=torch.float64).contiguous()
    _check(load_library().bko_lstart_pack(nx, ny, nz, fp, ldf, m, _ptr(k), kmu, ksig, hval, _ptr(scale), _ptr(x),
                                          _stream()))
    return x, scale


def lstart_pack_target(T: torch.Tensor, scale: torch.Tensor, gain: float) -> torch.Tensor:
    m, n = T.shape
    tp, ldt, tt = _block(T, "T")
    t = torch.empty((m, n), dtype=torch.float32, device=T.device)
    _check(load_library().bko_lstart_pack_target(n, tp, ldt, m, _ptr(scale), gain, _ptr(t), _stream()))
    return t


def jacobi_smooth(A: HeatOperator, B: torch.Tensor, X: torch.Tensor, sweeps: int, omega: float = 0.6,
                  stream=None) -> torch.Tensor:
    """In-place damped Jacobi sweeps on X ((m, N) FP64) for right-hand sides B."""
    m = B.shape[0]
    bp, ldb, _ = _block(B, "B")
    xp, ldx, _ = _block(X, "X")
    work = torch.empty_like(X)
    _check(load_library().bko_jacobi_smooth(A.handle, m, bp, ldb, xp, ldx, _ptr(work), X.shape[1], sweeps, omega,
                                            _stream(stream)))
    return X


def lstart_unpack(y: torch.Tensor, scale: torch.Tensor, gain: float, X0: Optional[torch.Tensor] = None):
    m = y.shape[0]
    n = y[0].numel()
    if X0 is None:
        X0 = torch.empty((m, n), dtype=torch.float64, device=y.device)
    xp, ldx, _ = _block(X0, "X0")
    _check(load_library().bko_lstart_unpack(n, _f32(y, "y"), m, _ptr(scale), gain, xp, ldx, _stream()))
    return X0


def cg_workspace_bytes(A: HeatOperator, m: int) -> int:
    out = ctypes.c_size_t()
    _check(load_library().bko_cg_workspace_bytes(A.handle, m, ctypes.byref(out)))
    return out.value


def cg_solve(A: HeatOperator, B: torch.Tensor, tol: float, max_iter: int = 100000,
             X: Optional[torch.Tensor] = None, stream=None, check: bool = True):
    """Per-sample CG baseline: an independent FP64 CG for every row of B
    ((m, N) FP64 on the GPU).  Returns (X, per-column iteration counts as a
    numpy array, info dict)."""
    import numpy as np

    m = B.shape[0]
    bp, ldb, bt = _block(B, "B")
    if bt != F64:
        raise ValueError("B must be float64")
    if X is None:
        X = torch.empty_like(B)
    xp, ldx, _ = _block(X, "X")
    nbytes = cg_workspace_bytes(A, m)
    buf, wptr = _aligned_workspace(nbytes, B.device)
    iters = (ctypes.c_int * m)()
    info = SolveInfo()
    st = load_library().bko_cg_solve(A.handle, m, bp, ldb, xp, ldx, tol, max_iter, ctypes.c_void_p(wptr), nbytes,
                                     iters, ctypes.byref(info), _stream(stream))
    if check and st != OK:
        _check(st)
    d = info.as_dict()
    d["status_name"] = STATUS_NAMES.get(st, str(st))
    return X, np.array(iters[:], dtype=np.int64), d


def combine(X: torch.Tensor, C: torch.Tensor, out_dtype=torch.float64, compute: int = F64,
            T: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """T = X C with X (s, N) and C (M, s); returns T (M, N)."""
    s, n = X.shape
    m = C.shape[0]
    if C.shape[1] != s:
        raise ValueError("C must be (M, s)")
    if T is None:
        T = torch.empty((m, n), dtype=out_dtype, device=X.device)
    xp, ldx, xt = _block(X, "X")
    if C.stride(1) != 1:
        raise ValueError("C must have contiguous rows")
    cp, ldc, ct = _ptr(C), C.stride(0) if m > 1 else s, DTYPE_CODE[C.dtype]
    tp, ldt, tt = _block(T, "T")
    _check(load_library().bko_combine(n, s, m, xp, ldx, xt, cp, ldc, ct, tp, ldt, tt, compute, _stream(stream)))
    return T


def boundary_source(A: HeatOperator, u_face: Sequence[float], stream=None) -> torch.Tensor:
    """g (N,) FP64: the right-hand-side source of nonhomogeneous boundary data
    (face temperatures in the order -x, +x, -y, +y, -z, +z), A x = q + g."""
    g = torch.empty(A.n, dtype=torch.float64, device=A.k.device)
    uf = (ctypes.c_double * 6)(*[float(v) for v in u_face])
    _check(load_library().bko_boundary_source(A.handle, _ptr(A.k), uf, _ptr(g), _stream(stream)))
    return g


def add_column(F: torch.Tensor, g: torch.Tensor, alpha: float = 1.0, stream=None) -> torch.Tensor:
    """F[j, :] += alpha g for every row j of F ((M, N) FP64), in place."""
    m, n = F.shape
    fp, ldf, _ = _block(F, "F")
    _check(load_library().bko_add_column(n, m, fp, ldf, _ptr(g), float(alpha), _stream(stream)))
    return F


def combine_noisy(X: torch.Tensor, C: torch.Tensor, noise: Optional[Noise] = None, T: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    """T = X C + E in FP64 (X (s, N), C (M, s)); E the counter-based noise."""
    s, n = X.shape
    m = C.shape[0]
    if C.shape[1] != s or C.dtype != torch.float64 or X.dtype != torch.float64:
        raise ValueError("X (s, N) and C (M, s) must be FP64")
    if T is None:
        T = torch.empty((m, n), dtype=torch.float64, device=X.device)
    xp, ldx, _ = _block(X, "X")
    if C.stride(1) != 1:
        raise ValueError("C must have contiguous rows")
    tp, ldt, _ = _block(T, "T")
    nz = ctypes.byref(noise) if noise is not None else None
    _check(load_library().bko_combine_noisy(n, s, m, xp, ldx, _ptr(C), C.stride(0) if m > 1 else s, tp, ldt, nz,
                                            _stream(stream)))
    return T


def noise_fill(n: int, m: int, noise: Noise, device="cuda", stream=None) -> torch.Tensor:
    """The noise alone: E (M, N) FP64."""
    E = torch.empty((m, n), dtype=torch.float64, device=device)
    ep, lde, _ = _block(E, "E")
    _check(load_library().bko_noise_fill(n, m, ep, lde, ctypes.byref(noise), _stream(stream)))
    return E


def normalize_weights(C: torch.Tensor, min_abs_sum: float, stream=None) -> torch.Tensor:
    """alpha = mu / sum(mu) per field, in place on C (M, s) FP64; returns the
    per-field flags (1: |sum| < min_abs_sum, left unnormalised)."""
    m, s = C.shape
    if C.dtype != torch.float64 or C.stride(1) != 1:
        raise ValueError("C must be FP64 with contiguous rows")
    flags = torch.empty(m, dtype=torch.int32, device=C.device)
    _check(load_library().bko_normalize_weights(s, m, _ptr(C), C.stride(0) if m > 1 else s, float(min_abs_sum),
                                                _ptr(flags), _stream(stream)))
    return flags


def combine_apply(A: HeatOperator, X: torch.Tensor, C: torch.Tensor, T: Optional[torch.Tensor] = None,
                  F: Optional[torch.Tensor] = None, work: Optional[torch.Tensor] = None, stream=None):
    """T = X C and F = A T = (A X) C in FP64 in one pass over the fields
    (X (s, N), C (M, s)); returns (T, F), each (M, N)."""
    s, n = X.shape
    m = C.shape[0]
    if C.shape[1] != s or C.dtype != torch.float64 or X.dtype != torch.float64:
        raise ValueError("X (s, N) and C (M, s) must be FP64")
    if T is None:
        T = torch.empty((m, n), dtype=torch.float64, device=X.device)
    if F is None:
        F = torch.empty((m, n), dtype=torch.float64, device=X.device)
    lib = load_library()
    need = ctypes.c_size_t()
    _check(lib.bko_combine_apply_workspace_bytes(A.handle, s, ctypes.byref(need)))
    if work is None or work.numel() < need.value + 256:
        work = torch.empty(need.value + 256, dtype=torch.uint8, device=X.device)
    wp = work.data_ptr() + ((-work.data_ptr()) % 256)
    xp, ldx, _ = _block(X, "X")
    if C.stride(1) != 1:
        raise ValueError("C must have contiguous rows")
    tp, ldt, _ = _block(T, "T")
    fp, ldf, _ = _block(F, "F")
    _check(lib.bko_combine_apply(A.handle, s, m, xp, ldx, _ptr(C), C.stride(0) if m > 1 else s, tp, ldt, fp, ldf,
                                 ctypes.c_void_p(wp), need.value, _stream(stream)))
    return T, F


def apply_operator(A: HeatOperator, T: torch.Tensor, out_dtype=torch.float64, compute: int = F64,
                   F: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """F = A T (T: (M, N)); returns F (M, N)."""
    m = T.shape[0]
    if F is None:
        F = torch.empty((m, A.n), dtype=out_dtype, device=T.device)
    tp, ldt, tt = _block(T, "T")
    fp, ldf, ft = _block(F, "F")
    _check(load_library().bko_apply_operator(A.handle, m, tp, ldt, tt, fp, ldf, ft, compute, _stream(stream)))
    return F


def apply_operator_tiling(A: HeatOperator, T: torch.Tensor, F: torch.Tensor, compute: int = F64) -> int:
    """Rows per tile of the LDS-tiled operator-action kernel that
    apply_operator(A, T, F=F, compute=compute) runs, or 0 for the per-cell
    kernel."""
    tp, ldt, tt = _block(T, "T")
    fp, ldf, ft = _block(F, "F")
    out = ctypes.c_int()
    _check(load_library().bko_apply_operator_tiling(A.handle, T.shape[0], tp, ldt, tt, fp, ldf, ft, compute,
                                                    ctypes.byref(out)))
    return out.value


def copy(dst: torch.Tensor, src: torch.Tensor, stream=None) -> torch.Tensor:
    """dst = src by the library's 16-byte vector copy kernel (contiguous
    tensors of equal byte size)."""
    if not (dst.is_cuda and src.is_cuda and dst.is_contiguous() and src.is_contiguous()):
        raise ValueError("copy needs contiguous GPU tensors")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("copy needs tensors of equal byte size")
    _check(load_library().bko_copy(_ptr(dst), _ptr(src), nbytes, _stream(stream)))
    return dst


def residual(A: HeatOperator, B: torch.Tensor, X: torch.Tensor, R: Optional[torch.Tensor] = None,
             stream=None) -> torch.Tensor:
    """R = B - A X in FP64."""
    if R is None:
        R = torch.empty_like(B)
    bp, ldb, _ = _block(B, "B")
    xp, ldx, _ = _block(X, "X")
    rp, ldr, _ = _block(R, "R")
    _check(load_library().bko_residual(A.handle, B.shape[0], bp, ldb, xp, ldx, rp, ldr, _stream(stream)))
    return R


# ------------------------------------------------------------------ timing hooks

FAMILY = {"apply": 0, "combine": 1, "gram": 2, "update_w": 3, "factor": 4, "spmm": 5, "resid": 6, "update_dqp": 7}


def timing_stride(every: int = 1):
    """Time one launch in every `every` of each selected family."""
    _check(load_library().bko_timing_set_stride(int(every)))


def timing_enable(families=None):
    """Time the named kernel families (None: all; [] or False: none)."""
    if families is True or families is None:
        mask = (1 << len(FAMILY)) - 1
    elif families is False:
        mask = 0
    else:
        mask = 0
        for f in families:
            mask |= 1 << FAMILY[f]
    _check(load_library().bko_timing_enable(mask))


def timing_reset():
    _check(load_library().bko_timing_reset())


def timing_query(family: str):
    n = ctypes.c_int()
    ms = ctypes.c_double()
    _check(load_library().bko_timing_query(FAMILY[family], ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value
