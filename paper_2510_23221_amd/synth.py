"""Seeded synthetic workloads: chip stacks, power maps and combination weights.

This module only draws inputs.  It holds none of the method's arithmetic: no
operator coefficients, no solves, no products.  Both the HIP path and the CPU
oracle take their inputs from here, so the two sides see identical numbers.

Physical parameters follow the paper's chip model (Sec. V-A, "IC Problem
Details"): a 10 mm x 10 mm x 0.51 mm stack, 0.15 mm device layers, silicon /
copper / TIM conductivities, 156 active blocks in the core layer of which six
are high-power (3-6 W/mm^2) and the rest 0.5-1 W/mm^2, and two L2-cache regions
per cache layer at 0.02-0.04 W/mm^2.  The paper's own floorplans are not
published, so these generators stand in for them.

Array conventions
-----------------
* A grid has ``nx * ny * nz`` cells, flattened x-fastest, then y, then z
  (layer 0 is the bottom, layer ``nz - 1`` the top).
* A block of ``s`` fields over ``N`` cells is a C-ordered array of shape
  ``(s, N)``: that is column-major ``N x s`` with leading dimension ``N``,
  each column one contiguous field.
* Combination weights ``C`` (``s x M`` column-major) are a C-ordered array of
  shape ``(M, s)``.
* Boundary faces are ordered -x, +x, -y, +y, -z, +z.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

BC_DIRICHLET0 = 0
BC_ADIABATIC = 1
BC_ROBIN = 2

#: per-layer conductivity pattern of the stacked chip, top layer first (W/mK):
#: core silicon, TIM, copper-rich via/bond layer, underfill-like layer, then
#: the same four again for the cache tier.
STACK_K_TOP_DOWN = (150.0, 5.0, 400.0, 1.0, 150.0, 5.0, 400.0, 1.0)

MM = 1.0e-3  # metres per millimetre
DEVICE_LAYER_THICKNESS = 0.15 * MM  # m; areal power is spread over this depth


@dataclass
class Chip:
    """One chip: grid, geometry, conductivity per cell and boundary faces."""

    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    k: np.ndarray  # (N,) float64, x-fastest
    bc: Tuple[int, int, int, int, int, int]
    h: Tuple[float, float, float, float, float, float]
    name: str = ""

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def dims(self) -> Tuple[int, int, int]:
        return (self.nx, self.ny, self.nz)


@dataclass
class Workload:
    """A chip (or several), its right-hand sides and its combination weights."""

    name: str
    chips: List[Chip]
    B: List[np.ndarray]  # per chip, (s, N) float64
    C: List[np.ndarray]  # per chip, (M, s) float64
    tol: float
    scheme: str  # "f64" | "mixed" | "mixed_bf16"
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def s(self) -> int:
        return self.B[0].shape[0]

    @property
    def m(self) -> int:
        return self.C[0].shape[0]


# ---------------------------------------------------------------- conductivity

def k_two_rectangles(rng: np.random.Generator, nx: int, ny: int,
                     lo: float = 1.0, hi: float = 150.0, nrect: int = 2) -> np.ndarray:
    """2-D piecewise-constant conductivity: a U(lo, hi) background and
    ``nrect`` axis-aligned rectangles (inclusive integer corners drawn
    uniformly and sorted per axis; later rectangles overwrite earlier ones),
    each with its own U(lo, hi) value."""
    k = np.full((ny, nx), rng.uniform(lo, hi))
    for _ in range(nrect):
        i0, i1 = np.sort(rng.integers(0, nx, size=2))
        j0, j1 = np.sort(rng.integers(0, ny, size=2))
        k[j0:j1 + 1, i0:i1 + 1] = rng.uniform(lo, hi)
    return k.reshape(-1).astype(np.float64)


def k_layered_stack(rng: np.random.Generator, nx: int, ny: int, nz: int,
                    pattern_top_down=STACK_K_TOP_DOWN, jitter: float = 0.2) -> np.ndarray:
    """Per-layer conductivity taken cyclically from ``pattern_top_down``
    (top layer first), times an independent U(1-jitter, 1+jitter) factor per
    cell."""
    k = np.empty((nz, ny, nx))
    for l in range(nz):
        k[l] = pattern_top_down[(nz - 1 - l) % len(pattern_top_down)]
    k *= rng.uniform(1.0 - jitter, 1.0 + jitter, size=k.shape)
    return k.reshape(-1).astype(np.float64)


# ---------------------------------------------------------------- power maps

def power_gaussian_blobs(rng: np.random.Generator, chip: Chip, s: int,
                         max_blobs: int = 5) -> np.ndarray:
    """``s`` 2-D power maps, each a sum of U{1..max_blobs} Gaussian blobs with
    centre U(0,1)^2, width U(0.05, 0.2) and amplitude U(0,1), sampled at the
    cell centres of a unit square.  Returns (s, N)."""
    xc = (np.arange(chip.nx) + 0.5) / chip.nx
    yc = (np.arange(chip.ny) + 0.5) / chip.ny
    X, Y = np.meshgrid(xc, yc)  # (ny, nx)
    out = np.zeros((s, chip.nz, chip.ny, chip.nx))
    for c in range(s):
        nb = int(rng.integers(1, max_blobs + 1))
        q = np.zeros_like(X)
        for _ in range(nb):
            cx, cy = rng.uniform(0.0, 1.0, size=2)
            sig = rng.uniform(0.05, 0.2)
            amp = rng.uniform(0.0, 1.0)
            q += amp * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * sig * sig))
        out[c, :] = q  # same map on every layer (nz == 1 for the 2-D case)
    return out.reshape(s, -1)


def power_blocky(rng: np.random.Generator, chip: Chip, s: int,
                 blocks_x: int = 12, blocks_y: int = 13, n_hot: int = 6) -> np.ndarray:
    """``s`` block-structured volumetric power maps (W/m^3) for a stacked chip.

    Top layer: ``blocks_x x blocks_y`` (156) active blocks; ``n_hot`` of them
    at U(3, 6) W/mm^2 and the rest at U(0.5, 1) W/mm^2.  Second silicon layer
    (index ``nz - 5``, clamped to 0): two half-plane caches at
    U(0.02, 0.04) W/mm^2.  Areal densities are spread over a 0.15 mm device
    layer.  Returns (s, N)."""
    nx, ny, nz = chip.dims
    ib = (np.arange(nx) * blocks_x) // nx  # block column of each cell column
    jb = (np.arange(ny) * blocks_y) // ny
    cache_layer = max(nz - 5, 0)
    out = np.zeros((s, nz, ny, nx))
    to_vol = 1.0e6 / DEVICE_LAYER_THICKNESS  # W/mm^2 -> W/m^2 -> W/m^3
    for c in range(s):
        dens = rng.uniform(0.5, 1.0, size=(blocks_y, blocks_x))
        hot = rng.choice(blocks_x * blocks_y, size=n_hot, replace=False)
        dens.reshape(-1)[hot] = rng.uniform(3.0, 6.0, size=n_hot)
        out[c, nz - 1] = dens[jb][:, ib] * to_vol
        left, right = rng.uniform(0.02, 0.04, size=2)
        half = nx // 2
        out[c, cache_layer, :, :half] += left * to_vol
        out[c, cache_layer, :, half:] += right * to_vol
    return out.reshape(s, -1)


def combo_weights(rng: np.random.Generator, s: int, m: int) -> np.ndarray:
    """Combination weights C ~ N(0, 1), ``s x M`` column-major -> (M, s)."""
    return rng.standard_normal(size=(m, s))


# ---------------------------------------------------------------- chips

def chip_2d(rng: np.random.Generator, n: int = 64) -> Chip:
    """Nondimensional unit-square chip, Dirichlet-0 on all in-plane faces,
    adiabatic z faces (a 5-point operator)."""
    k = k_two_rectangles(rng, n, n)
    return Chip(n, n, 1, 1.0, 1.0, 1.0 / n, k,
                (BC_DIRICHLET0,) * 4 + (BC_ADIABATIC,) * 2, (0.0,) * 6, name=f"2d{n}")


def chip_stack(rng: np.random.Generator, nx: int, ny: int, nz: int,
               lx: float = 10 * MM, ly: float = 10 * MM, lz: float = 0.51 * MM,
               h_range=(1.0e3, 1.0e4)) -> Chip:
    """Layered stack, top face convective (Robin, h ~ U(h_range)), all other
    faces adiabatic."""
    k = k_layered_stack(rng, nx, ny, nz)
    h_top = rng.uniform(*h_range)
    bc = (BC_ADIABATIC,) * 5 + (BC_ROBIN,)
    h = (0.0,) * 5 + (h_top,)
    return Chip(nx, ny, nz, lx, ly, lz, k, bc, h, name=f"stack{nx}x{ny}x{nz}")


# ---------------------------------------------------------------- configurations

def seed_for(config_index: int, chip_index: Optional[int] = None) -> int:
    base = 1000 + config_index
    return base if chip_index is None else base * 100000 + chip_index


def workload(config_index: int, *, m: Optional[int] = None, s: Optional[int] = None,
             grid: Optional[Tuple[int, int, int]] = None, nchips: Optional[int] = None) -> Workload:
    """Build one of the five reference workloads (0-based index), optionally
    shrunk (``m``, ``s``, ``grid``, ``nchips``) for tests.

    0: 2-D 64x64, 5-point, Dirichlet-0, two-rectangle k, s=8 Gaussian-blob
       maps, FP64, tol 1e-10, M=1000.
    1: 128x128x8 stack, 7-point, Robin top, s=32 blocky maps, FP32 SpMM with
       FP64 Gram / refinement to 1e-8, M=5000, FP64 T and F.
    2: 64 stacks of uneven size (32..256 squared, 4..12 layers), s=16, M=500.
    3: 256x256x16 stack, s=64, M=20000, BF16 combine / apply.
    4: learned start: 40 training chips at 128x128x8 (500 pairs each) and
       256 unseen chips, s=16.
    """
    if config_index == 0:
        rng = np.random.default_rng(seed_for(0))
        n = grid[0] if grid else 64
        chip = chip_2d(rng, n)
        s_ = s or 8
        B = power_gaussian_blobs(rng, chip, s_)
        C = combo_weights(rng, s_, m or 1000)
        return Workload("2d-64x64-s8-f64", [chip], [B], [C], 1e-10, "f64")
    if config_index in (1, 3):
        rng = np.random.default_rng(seed_for(config_index))
        if config_index == 1:
            dims, s_d, m_d, scheme = (128, 128, 8), 32, 5000, "mixed"
        else:
            dims, s_d, m_d, scheme = (256, 256, 16), 64, 20000, "mixed_bf16"
        dims = grid or dims
        chip = chip_stack(rng, *dims)
        s_ = s or s_d
        B = power_blocky(rng, chip, s_)
        C = combo_weights(rng, s_, m or m_d)
        name = f"stack-{dims[0]}x{dims[1]}x{dims[2]}-s{s_}-m{C.shape[0]}"
        return Workload(name, [chip], [B], [C], 1e-8, scheme)
    if config_index == 2:
        nc = nchips or 64
        chips, Bs, Cs = [], [], []
        for i in range(nc):
            rng = np.random.default_rng(seed_for(2, i))
            side = int(rng.choice(np.arange(32, 257, 16)))
            nz = int(rng.integers(4, 13))
            if grid:  # test shrink: cap the grid
                side = min(side, grid[0])
                nz = min(nz, grid[2])
            chip = chip_stack(rng, side, side, nz)
            s_ = s or 16
            chips.append(chip)
            Bs.append(power_blocky(rng, chip, s_))
            Cs.append(combo_weights(rng, s_, m or 500))
        return Workload(f"batch-{nc}chips-s{Bs[0].shape[0]}-m{Cs[0].shape[0]}",
                        chips, Bs, Cs, 1e-8, "mixed")
    if config_index == 4:
        nc = nchips or 40
        chips, Bs, Cs = [], [], []
        for i in range(nc):
            rng = np.random.default_rng(seed_for(4, i))
            d = grid or (128, 128, 8)
            chip = chip_stack(rng, *d)
            s_ = s or 16
            chips.append(chip)
            Bs.append(power_blocky(rng, chip, s_))
            Cs.append(combo_weights(rng, s_, m or 500))
        return Workload("learned-start", chips, Bs, Cs, 1e-8, "mixed")
    raise ValueError(f"unknown configuration index {config_index}")


def learned_start_test_chips(n: int, grid: Tuple[int, int, int] = (128, 128, 8), s: int = 16):
    """Unseen chips for the learned start: the training generator with seeds
    disjoint from the training chips'.  Returns (chips, power maps)."""
    chips, Bs = [], []
    for i in range(n):
        rng = np.random.default_rng(seed_for(4, 50000 + i))
        chip = chip_stack(rng, *grid)
        chips.append(chip)
        Bs.append(power_blocky(rng, chip, s))
    return chips, Bs


def random_block(rng: np.random.Generator, s: int, n: int) -> np.ndarray:
    """Standard-normal (s, N) block, for probes and parity tests."""
    return rng.standard_normal(size=(s, n))
