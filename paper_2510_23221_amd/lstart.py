"""Learned initial guess for the block solve (the project's addition; the
paper's block solve of Sec. III-A starts from any initial block).

Pipeline, every numerical step in the library's kernels:

1. Training pairs come from the method itself: per training chip, a block
   solve of its s power maps (Sec. III-A), M random combinations of the
   basis solutions (Sec. III-B, Eq. (5)) and their operator action (Sec.
   III-C, Eq. (6)) give M exact (power F, temperature T) pairs.
2. A convolutional encoder-decoder (``capi.UNet``) maps the normalised power
   planes plus log-conductivity planes and the film coefficient to the
   temperature planes; it is trained with the library's forward, backward
   and Adam kernels on the MSE of T / (rms(F) gain).
3. For a new chip, the network's prediction for each basis power map,
   followed by a few damped Jacobi sweeps (the prediction's error is mostly
   high-frequency, which the sweeps damp and which dominates its residual),
   is the X0 of the block solve; columns that start worse than zero fall
   back to the zero start inside the solve, which also judges the result by
   its own FP64 residual.

Inputs are scaled by the RMS of F per sample and outputs by the same factor,
so the prediction is equivariant to the scale of the power map (T is linear
in F) and every plane the network sees is O(1) per cell.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

from . import capi, synth


@dataclass
class Normalizer:
    kmu: float
    ksig: float
    hmu: float
    hsig: float
    gain: float

    def hval(self, chip: synth.Chip) -> float:
        return float((math.log(top_h(chip) + 1.0) - self.hmu) / self.hsig)


def top_h(chip: synth.Chip) -> float:
    return float(chip.h[5]) if chip.bc[5] == synth.BC_ROBIN else 0.0


@dataclass
class ChipPairs:
    chip: synth.Chip
    G: capi.HeatOperator
    k: torch.Tensor  # (N,) float64 on the device
    F: torch.Tensor  # (M, N) float64: sources of the fields
    T: torch.Tensor  # (M, N) float64: the fields


def generate_pairs(chips: List[synth.Chip], Bs: List[np.ndarray], Cs: List[np.ndarray], tol: float,
                   device="cuda", compute=capi.F32, precond: int = capi.PRECOND_NONE) -> List[ChipPairs]:
    """BlocKOA pairs of every training chip: block solve, combination and
    operator action, all on the GPU."""
    out = []
    for chip, B, C in zip(chips, Bs, Cs):
        G = capi.HeatOperator.from_chip(chip, device, precond=precond)
        Bd = torch.as_tensor(B, device=device)
        X, _ = capi.block_krylov_solve(G, Bd, tol, compute=compute)
        T = capi.combine(X, torch.as_tensor(C, device=device))
        F = capi.apply_operator(G, T)
        out.append(ChipPairs(chip, G, torch.as_tensor(chip.k, device=device), F, T))
    return out


def fit_normalizer(data: List[ChipPairs]) -> Normalizer:
    """Input and output scales from the training set."""
    logk = np.concatenate([np.log(d.chip.k) for d in data])
    logh = np.array([math.log(top_h(d.chip) + 1.0) for d in data])
    ratios = []
    for d in data:
        nF = torch.linalg.vector_norm(d.F, dim=1)
        nT = torch.linalg.vector_norm(d.T, dim=1)
        ok = nF > 0
        ratios.append((nT[ok] / nF[ok]).cpu().numpy())
    return Normalizer(float(logk.mean()), float(logk.std() + 1e-12), float(logh.mean()), float(logh.std() + 1e-3),
                      float(np.median(np.concatenate(ratios))))


def _pack(norm: Normalizer, chip: synth.Chip, k: torch.Tensor, F: torch.Tensor):
    return capi.lstart_pack(chip.dims, F, k, norm.kmu, norm.ksig, norm.hval(chip))


def make_net(chip: synth.Chip, base: int, max_batch: int, seed: int, device="cuda") -> capi.UNet:
    """Network for chips of this grid, He-initialised filters, zero biases."""
    nx, ny, nz = chip.dims
    net = capi.UNet(2 * nz + 1, nz, base, ny, nx, max_batch, device)
    rng = np.random.default_rng(seed)
    p = np.zeros(net.nparams, dtype=np.float32)
    w1, w2, w3 = base, 2 * base, 4 * base
    cin, cout = 2 * nz + 1, nz
    spec = [(cin, w1, 3), (w1, w1, 3), (w1, w2, 3), (w2, w2, 3), (w2, w3, 3), (w3, w3, 3), (w3, w3, 3), (w3, w3, 3),
            (2 * w3, w3, 3), (w3, w3, 3), (w3 + w2, w2, 3), (w2, w2, 3), (w2 + w1, w1, 3), (w1, w1, 3), (w1, cout, 1)]
    o = 0
    for ci, co, k in spec:
        nw = co * ci * k * k
        p[o:o + nw] = rng.standard_normal(nw) * math.sqrt(2.0 / (ci * k * k))
        o += nw + co
    assert o == net.nparams
    net.set_params(torch.as_tensor(p, device=device))
    return net


def train(net: capi.UNet, data: List[ChipPairs], norm: Normalizer, steps: int, batch: int, lr: float,
          seed: int = 0, log_every: int = 0):
    """Adam on random batches (one chip per batch, fields drawn at random);
    cosine learning-rate decay.  Returns [(step, loss)] at log points."""
    rng = np.random.default_rng(seed)
    nz = data[0].chip.nz
    log = []
    for step in range(steps):
        d = data[int(rng.integers(len(data)))]
        idx = torch.as_tensor(rng.choice(d.F.shape[0], size=batch, replace=False), device=d.F.device)
        F = d.F.index_select(0, idx)
        T = d.T.index_select(0, idx)
        x, scale = _pack(norm, d.chip, d.k, F)
        t = capi.lstart_pack_target(T, scale, norm.gain).reshape(batch, nz, d.chip.ny, d.chip.nx)
        want = log_every > 0 and (step % log_every == 0 or step == steps - 1)
        loss = net.gradient(x, t, want_loss=want)
        if want:
            log.append((step, loss))
        net.adam_step(lr * 0.5 * (1.0 + math.cos(math.pi * step / max(1, steps))))
    return log


def predict_x0(net: capi.UNet, norm: Normalizer, chip: synth.Chip, k: torch.Tensor, B: torch.Tensor,
               G: Optional[capi.HeatOperator] = None, smooth: int = 0, omega: float = 0.6) -> torch.Tensor:
    """Initial block X0 (s, N) FP64 for the power maps B (s, N) of a chip,
    optionally followed by `smooth` damped Jacobi sweeps with operator G (the
    network's error is mostly high-frequency; the sweeps damp it)."""
    s = B.shape[0]
    X0 = torch.empty_like(B)
    for j0 in range(0, s, net.max_batch):
        j1 = min(s, j0 + net.max_batch)
        x, scale = _pack(norm, chip, k, B[j0:j1])
        y = net.infer(x)
        capi.lstart_unpack(y, scale, norm.gain, X0[j0:j1])
    if smooth > 0:
        capi.jacobi_smooth(G, B, X0, smooth, omega)
    return X0


def predict_x0_group(net: capi.UNet, norm: Normalizer, chips: List[synth.Chip], ks: List[torch.Tensor],
                     Bs: List[torch.Tensor], Gs: List[capi.HeatOperator], smooth: int = 0,
                     omega: float = 0.6) -> List[torch.Tensor]:
    """predict_x0 for several chips of one grid with one network pass over
    all their power maps (net.max_batch >= the total number of maps): the
    small layers then have enough images to fill the GPU."""
    nx, ny, nz = chips[0].dims
    counts = [B.shape[0] for B in Bs]
    total = sum(counts)
    if total > net.max_batch or any(c.dims != chips[0].dims for c in chips):
        raise ValueError("the chips must share a grid and their maps fit one network batch")
    dev = Bs[0].device
    x = torch.empty((total, 2 * nz + 1, ny, nx), dtype=torch.float32, device=dev)
    scale = torch.empty(total, dtype=torch.float64, device=dev)
    o = 0
    for chip, k, B, c in zip(chips, ks, Bs, counts):
        capi.lstart_pack(chip.dims, B, k, norm.kmu, norm.ksig, norm.hval(chip), x=x[o:o + c], scale=scale[o:o + c])
        o += c
    y = net.infer(x)
    out, o = [], 0
    for G, B, c in zip(Gs, Bs, counts):
        X0 = torch.empty_like(B)
        capi.lstart_unpack(y[o:o + c], scale[o:o + c], norm.gain, X0)
        if smooth > 0:
            capi.jacobi_smooth(G, B, X0, smooth, omega)
        out.append(X0)
        o += c
    return out


def evaluate(net: Optional[capi.UNet], norm: Optional[Normalizer], chips: List[synth.Chip], Bs: List[np.ndarray],
             tol: float, device="cuda", compute=capi.F32, smooth: int = 0, precond: int = capi.PRECOND_NONE,
             group: int = 1):
    """Block solves of every chip from the zero start, from the zero start
    after the same smoothing sweeps, and (if net is given) from the learned
    start, all with the given preconditioner.  With group > 1 the learned
    starts of `group` consecutive chips come from one network pass
    (predict_x0_group) and each chip is charged an equal share of its time.
    Returns per-chip records (iterations, final residuals, seconds)."""
    recs = []
    for g0 in range(0, len(chips), group):
        gchips, gB = chips[g0:g0 + group], Bs[g0:g0 + group]
        Gs = [capi.HeatOperator.from_chip(chip, device, precond=precond) for chip in gchips]
        ks = [torch.as_tensor(chip.k, device=device) for chip in gchips]
        Bds = [torch.as_tensor(B, device=device) for B in gB]
        grecs = []
        for G, Bd in zip(Gs, Bds):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info0 = capi.block_krylov_solve(G, Bd, tol, compute=compute)
            t1 = time.perf_counter()
            rec = {"zero_iters": info0["iters"], "zero_res": info0["max_rel_res"], "zero_s": t1 - t0}
            if smooth > 0:
                Z = torch.zeros_like(Bd)
                capi.jacobi_smooth(G, Bd, Z, smooth)
                _, infoz = capi.block_krylov_solve(G, Bd, tol, compute=compute, X0=Z)
                rec.update({"zero_smooth_iters": infoz["iters"], "zero_smooth_res": infoz["max_rel_res"]})
            grecs.append(rec)
        if net is not None:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if group > 1:
                X0s = predict_x0_group(net, norm, gchips, ks, Bds, Gs, smooth)
            else:
                X0s = [predict_x0(net, norm, gchips[0], ks[0], Bds[0], Gs[0], smooth)]
            torch.cuda.synchronize()
            share = (time.perf_counter() - t0) / len(gchips)
            for rec, G, Bd, X0 in zip(grecs, Gs, Bds, X0s):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                _, info1 = capi.block_krylov_solve(G, Bd, tol, compute=compute, X0=X0)
                t2 = time.perf_counter()
                rec.update({"learned_iters": info1["iters"], "learned_res": info1["max_rel_res"],
                            "infer_s": share, "learned_s": t2 - t1, "rejected": info1["x0_rejected"]})
        recs.extend(grecs)
    return recs
