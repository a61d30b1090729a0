#!/usr/bin/env python3
"""Throughput of the block Krylov + operator action path on one MI355X.

One step = the whole hot path over one synthetic chip, with inputs resident
in HBM: block solve of A X = B for s power maps (FP32 block iteration with
FP64 Gram / factorisations / refinement to relative residual 1e-8), the
combination T = X C into M fields (FP64), and the operator action F = A T
(FP64).  value = M pairs / step time.

Default workload: 128 x 128 x 8 stacked chip, 7-point stencil, s = 32,
M = 5000 (the configuration the pairs/s metric is quoted on).

Prints one JSON line.  Extra keys: ``roofline`` (the dominant kernel,
measured with HIP events around its launches on the launch stream),
``output`` / ``stencil`` (the output kernels' own rooflines), ``copy`` (the
library's 16-byte vector copy over a field-sized buffer: the achievable HBM
rate every fraction is also quoted against), ``census_*`` (one instrumented
step: per-family milliseconds and launches), ``solve`` (iterations,
refinements, residual), ``stage_errors``, ``per_sample_cg`` (the paper's
direct method on the same GPU: one FP64 CG per power map, timed on a subset
of columns and reported per pair), ``ablations`` (Table 7's modules removed
on the same GPU), ``sub_records`` (the other workloads at a few steps each:
plain FP64 BlocKOA on the same chip, the 256 x 256 x 16 stack with BF16
fields, the batch of 64 uneven chips, the learned start against the zero
start) and ``cpu_baseline`` (the CPU oracle on the host cores).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# dense matrix-core peaks of MI355X, TFLOP/s
MFMA_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}

# HBM bytes per (working) launch: rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE x 1
# (the factors that make the counters read the known bytes of the library's
# copy kernel), per (workload, kernel family, output route, block-iteration
# type).  Only kernels
# whose code has not changed since the counters were taken carry a figure
# (profiles/pmc_traffic_stack128x128x8.md, profiles/pmc_traffic_stack256x256x16.md).
TRAFFIC_BYTES = {
    ("stack-128x128x8-s32-m5000", "update_dqp", "", "f32"): 92.5e6,
    ("stack-128x128x8-s32-m5000", "update_w", "", "f32"): 55.7e6,
    ("stack-128x128x8-s32-m5000", "spmm", "", "f32"): 41.9e6,
    ("stack-128x128x8-s32-m5000", "apply", "", "f32"): 11187.2e6,
    ("stack-128x128x8-s32-m5000", "combine", "", "f32"): 5410.8e6,
    ("stack-256x256x16-s64-m20000", "update_dqp", "", "f32"): 1343.3e6,
    ("stack-256x256x16-s64-m20000", "update_w", "", "f32"): 820.3e6,
    ("stack-256x256x16-s64-m20000", "spmm", "", "f32"): 844.4e6,
    ("stack-256x256x16-s64-m20000", "apply", "", "f32"): 94964.7e6,
    ("stack-256x256x16-s64-m20000", "combine", "", "f32"): 43407.0e6,
}

# one launch in this many of the dominant block-solve kernel carries events
# in the timed region
TIMING_STRIDE = 8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=1, help="single-chip workload index (0, 1, 3)")
    ap.add_argument("--workload", choices=["single", "batched", "learned"], default="single",
                    help="single chip (default), batch of uneven chips, or learned start")
    ap.add_argument("--nchips", type=int, default=None)
    ap.add_argument("--train-epochs", type=float, default=4.0)
    ap.add_argument("--test-chips", type=int, default=256)
    ap.add_argument("--infer-chips", type=int, default=16,
                    help="unseen chips whose learned starts come from one network pass")
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cg-columns", type=int, default=512, help="columns of the per-sample CG baseline (0: skip)")
    ap.add_argument("--precond", choices=["none", "jacobi"], default="jacobi",
                    help="preconditioner of the block solve and of the per-sample CG baseline alike")
    ap.add_argument("--noise", choices=["none", "uniform", "gaussian"], default="none",
                    help="noise term of Eq. (5) added to every field (then the outputs take two passes)")
    ap.add_argument("--noise-amp", type=float, default=0.01, help="noise half-width (uniform) or std (gaussian), K")
    ap.add_argument("--outputs", choices=["two-pass", "one-pass"], default="two-pass",
                    help="FP64 fields: combination then operator action of the written T (default), or one pass "
                         "over the fields for T and F")
    ap.add_argument("--compute", choices=["auto", "f64", "f32"], default="auto",
                    help="block-iteration arithmetic (auto: the workload's scheme)")
    ap.add_argument("--no-sub-records", action="store_true",
                    help="headline workload only (skip the FP64, large-stack, batch and learned-start records)")
    ap.add_argument("--only", choices=["apply", "combine", "copy"], default=None,
                    help="run one kernel family at the workload's shape (for counter profiles)")
    return ap.parse_args()


def only_kernel(args, w, G, X, C, T, F, t_dtype, comb_compute, apply_compute):
    """Launch one kernel family `steps` times at the workload shape and print
    its event-timed average.  `copy` is the library's 16-byte vector copy of
    T into F (the calibration kernel for HBM byte counters)."""
    import torch

    from paper_2510_23221_amd import capi

    n, m = T.shape[1], T.shape[0]
    wt = T.element_size()

    def run():
        if args.only == "apply":
            capi.apply_operator(G, T, out_dtype=t_dtype, compute=apply_compute, F=F)
        elif args.only == "combine":
            capi.combine(X, C, out_dtype=t_dtype, compute=comb_compute, T=T)
        else:
            capi.copy(F, T)

    T.normal_()
    X.normal_()
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        run()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    nbytes = {"apply": n * m * 2 * wt, "combine": n * m * wt, "copy": n * m * 2 * wt}[args.only]
    print(json.dumps({"only": args.only, "avg_ms": round(ms, 4), "bytes": nbytes,
                      "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1), "shape": [m, n], "dtype": str(t_dtype)}),
          flush=True)


def copy_rate(dst, src, reps=5):
    """The library's 16-byte vector copy of a field-sized buffer, timed with
    events on the launch stream: bytes read + written per launch over the
    average launch time (the achievable HBM rate)."""
    import torch

    from paper_2510_23221_amd import capi

    for _ in range(2):
        capi.copy(dst, src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        capi.copy(dst, src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 2 * src.numel() * src.element_size()
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "bytes_per_launch": int(nbytes), "avg_us": round(ms * 1e3, 2), "kernel": "copy16 (library)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this library runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(chips and fields would shard across GPUs without communication; only the one-GPU path is built)",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        print(json.dumps(bench_batched(args, args.steps, args.warmup)), flush=True)
        return
    if args.workload == "learned":
        print(json.dumps(bench_learned(args)), flush=True)
        return
    res, w = bench_single(args, args.config, args.steps, args.warmup, headline=True)
    if res is None:
        return
    if not args.no_sub_records and args.config == 1 and args.m is None:
        sub = {}
        few = max(1, min(args.steps, 3))
        sub["fp64_blockoa"], _ = bench_single(args, 1, few, 1, compute_override="f64")
        note("fp64 BlocKOA done")
        sub["large_bf16"], _ = bench_single(args, 3, 2, 1)
        note("256x256x16 BF16 stack done")
        sub["batch"] = bench_batched(args, 2, 1)
        note("64-chip batch done")
        sub["learned"] = bench_learned(args)
        note("learned start done")
        res["sub_records"] = sub
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, "jacobi" if args.precond == "jacobi" else "none")
    print(json.dumps(res), flush=True)


def note(msg):
    """Progress on stderr (the JSON line stays the only stdout line)."""
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def bench_single(args, config, steps, warmup, headline=False, compute_override=None):
    """One chip of a single-chip workload: `warmup` untimed steps, one
    instrumented census step, then `steps` timed steps.  Returns the record
    (and the workload)."""
    import torch

    from paper_2510_23221_amd import capi, synth

    dev = torch.device("cuda:0")
    w = synth.workload(config, m=args.m if headline else None)
    chip = w.chips[0]
    s, m, n = w.s, w.m, chip.n
    mixed = w.scheme.startswith("mixed")
    ov = compute_override or (args.compute if headline else "auto")
    if ov != "auto":
        mixed = ov == "f32"
    compute = capi.F32 if mixed else capi.F64
    t_dtype = torch.bfloat16 if w.scheme == "mixed_bf16" else torch.float64
    comb_compute = capi.BF16 if w.scheme == "mixed_bf16" else capi.F64
    apply_compute = capi.F32 if w.scheme == "mixed_bf16" else capi.F64

    pc = capi.PRECOND_JACOBI if args.precond == "jacobi" else capi.PRECOND_NONE
    G = capi.HeatOperator.from_chip(chip, dev, precond=pc)
    B = torch.as_tensor(w.B[0], device=dev)
    C = torch.as_tensor(w.C[0], device=dev)
    X = torch.empty_like(B)
    T = torch.empty((m, n), dtype=t_dtype, device=dev)
    F = torch.empty((m, n), dtype=t_dtype, device=dev)
    wbytes = capi.workspace_bytes(G, s, compute)
    work = torch.empty(wbytes + 256, dtype=torch.uint8, device=dev)
    wview = work[(-work.data_ptr()) % 256:]
    if headline and args.only:
        only_kernel(args, w, G, X, C, T, F, t_dtype, comb_compute, apply_compute)
        return None, w

    infos = []
    noise_kind = {"none": capi.NOISE_NONE, "uniform": capi.NOISE_UNIFORM, "gaussian": capi.NOISE_GAUSSIAN}[args.noise]
    if not headline:
        noise_kind = capi.NOISE_NONE
    if noise_kind != capi.NOISE_NONE and t_dtype != torch.float64:
        raise SystemExit("bench.py: --noise needs FP64 fields")
    # one pass over the fields for both outputs only when asked for (FP64
    # fields, no noise); otherwise the combination, then the operator action
    # of the T actually written
    fused = t_dtype == torch.float64 and args.outputs == "one-pass" and noise_kind == capi.NOISE_NONE
    cwork = torch.empty(capi_bytes_combine_apply(capi, G, s) + 256, dtype=torch.uint8, device=dev) if fused else None
    noise = capi.Noise(noise_kind, args.noise_amp, 20251021, 0)

    def outputs():
        if fused:
            capi.combine_apply(G, X, C, T=T, F=F, work=cwork)
        elif noise_kind != capi.NOISE_NONE:
            capi.combine_noisy(X, C, noise, T=T)
            capi.apply_operator(G, T, out_dtype=t_dtype, compute=apply_compute, F=F)
        else:
            capi.combine(X, C, out_dtype=t_dtype, compute=comb_compute, T=T)
            capi.apply_operator(G, T, out_dtype=t_dtype, compute=apply_compute, F=F)

    def step():
        _, info = capi.block_krylov_solve(G, B, w.tol, compute=compute, X=X, work=wview)
        outputs()
        infos.append(info)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()

    # ---- algorithmic bytes per launch of each HBM-bound kernel family
    wv = 4 if mixed else 8                      # block-solve storage
    wcv = 4 if mixed else 8                     # coefficients used by the block solve
    wt = 2 if t_dtype == torch.bfloat16 else 8  # T and F
    wc = 4 if apply_compute == capi.F32 else 8  # coefficients used by the operator action
    ldw = -(-n // 256) * 256                    # padded rows of the block-solve workspace
    per_launch_bytes = {
        "apply": n * m * 2 * wt + n * 4 * wc,
        # one pass: T and F written, X and A X read; else T written, X read
        "combine": (2 * n * m * 8 + 2 * n * s * 8 + s * m * 8) if fused else (n * m * wt + n * s * 8 + s * m * 8),
        "spmm": n * s * 2 * wv + n * 4 * wcv,    # stencil + P^T AP Gram: P read, AP written
        "update_w": ldw * s * 3 * wv,           # W, AP read; W written
        "update_dqp": ldw * s * 5 * wv,         # D, P, W read; D, P written
        "resid": n * s * 3 * 8 + n * 4 * 8,
    }

    # census step: every kernel family timed (events around each launch)
    capi.timing_reset()
    capi.timing_enable(None)
    step()
    torch.cuda.synchronize()
    census = {f: capi.timing_query(f) for f in capi.FAMILY}
    capi.timing_enable(False)
    dom = max(per_launch_bytes, key=lambda k: census[k][1])
    out_fam = "combine" if fused else "apply"

    # timed region: only the reported kernels carry events, one launch in
    # TIMING_STRIDE of the block-solve family (the events' own cost stays
    # off the step time); the sample's mean is the family's mean
    stride = TIMING_STRIDE if dom not in ("apply", "combine") else 1
    capi.timing_reset()
    capi.timing_stride(stride)
    fams = sorted({dom, out_fam, "combine"})
    capi.timing_enable(fams)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    capi.timing_enable(False)
    capi.timing_stride(1)
    ms_per_step = (t1 - t0) * 1e3 / steps
    fam = {f: capi.timing_query(f) for f in capi.FAMILY}
    it_total = sum(i["iters"] for i in infos[-steps:])
    ref_total = sum(i["refinements"] for i in infos[-steps:])

    # launches that move their full algorithmic bytes: one spmm, update_w and
    # update_dqp per block iteration, one more update_dqp per inner solve (its
    # first QR); the rest of a convergence-check chunk exits at once
    working = {"spmm": it_total, "update_w": it_total, "update_dqp": it_total + ref_total,
               "apply": steps, "combine": steps, "resid": None}
    # the copy reference writes into a scratch buffer: T and F stay as the step left them
    copy_ref = None
    if headline:
        scratch = torch.empty_like(T)
        copy_ref = copy_rate(scratch, T)
        del scratch

    def roof(kind, strided):
        timed, tot = fam[kind]
        if timed == 0 or kind not in per_launch_bytes:
            return None
        avg_ms = tot / timed
        launches = census[kind][0] * steps  # every launch of the timed steps
        work = working.get(kind) or launches
        # achieved: the family's algorithmic bytes over its kernel time
        gbs = per_launch_bytes[kind] * work / (avg_ms * launches * 1e-3) / 1e9
        key = (w.name, kind, "one-pass" if (kind == "combine" and fused) else "", "f32" if mixed else "f64")
        out = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": TRAFFIC_BYTES.get(key), "kernel": kind,
               "launches": launches, "working_launches": work, "timed_launches": timed,
               "avg_us": round(avg_ms * 1e3, 2), "bytes_per_launch": int(per_launch_bytes[kind])}
        if copy_ref:
            out["frac_of_copy"] = round(gbs / copy_ref["achieved"], 4)
        if kind == "combine":
            # the combination's matrix-core rate against the peak of its type
            # (2 N s M flops per output field block; the one-pass form has two)
            flops = 2.0 * n * s * m * (2 if fused else 1)
            mt = "f64" if comb_compute == capi.F64 else ("f32" if comb_compute == capi.F32 else "bf16")
            tf = flops / (avg_ms * 1e-3) / 1e12
            out["mfma"] = {"dtype": mt, "tflops": round(tf, 2), "peak_tflops": MFMA_PEAK_TFLOPS[mt],
                           "frac": round(tf / MFMA_PEAK_TFLOPS[mt], 4),
                           "intensity_cap_frac": round(min(1.0, (2.0 * s / wt) / (MFMA_PEAK_TFLOPS[mt] * 1e12 /
                                                                               (HBM_PEAK_GBS * 1e9))), 4)}
        return out

    value = m / (ms_per_step * 1e-3)
    scheme = "f32+f64" if mixed else "f64"
    res = {
        "metric": "data pairs/s at rel residual <=1e-8 (BlocKOA: block solve + combine + operator action)",
        "value": round(value, 1),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": scheme if t_dtype == torch.float64 else scheme + "+bf16",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": list(chip.dims), "s": s, "M": m, "tol": w.tol,
                   "scheme": w.scheme if compute_override is None else f"{w.scheme} with {compute_override} iteration",
                   "block_iteration": "f32" if mixed else "f64",
                   "T_F_dtype": str(t_dtype).replace("torch.", ""), "precond": args.precond,
                   "outputs": "one pass (T = X C, F = (A X) C)" if fused else "two passes (T = X C, F = A T)",
                   "noise": args.noise if noise_kind == capi.NOISE_NONE else f"{args.noise} {args.noise_amp}"},
        "roofline": roof(dom, True),
        "output": roof(out_fam, False),
        "census_ms_per_step": {k: round(v[1], 4) for k, v in census.items()},
        "census_launches_per_step": {k: v[0] for k, v in census.items()},
        "solve": {"iters_per_step": it_total / steps, "refinements_per_step": ref_total / steps,
                  "max_rel_res": max(i["max_rel_res"] for i in infos[-steps:])},
    }
    if not fused:
        res["combine"] = roof("combine", False)
    if copy_ref:
        res["copy"] = copy_ref
    res["stage_errors"] = stage_errors(G, X, C, T, F)
    if fused:
        # the operator action on its own (the stencil over the M fields), for
        # the stencil's HBM rate; the step itself forms F in the one pass
        res["stencil"] = stencil_rate(G, T, F, t_dtype, apply_compute, per_launch_bytes["apply"], None)
    else:
        res["stencil"] = res["output"]
    if headline and args.cg_columns > 0:
        res["per_sample_cg"] = per_sample_cg(G, B, C, w, args.cg_columns, value)
        res["ablations"] = ablations(G, B, C, X, w, args.cg_columns, value, compute, wview, outputs,
                                     res["per_sample_cg"]["value"])
    del T, F, work
    torch.cuda.empty_cache()
    return res, w


def bench_batched(args, steps, warmup):
    """Batch of uneven chips (64 stacks, 32^2..256^2 x 4..12 layers, s = 16,
    M = 500 each): one batch run per step -- every chip's block solve with
    grouped launches and graph-captured iteration chunks on a side stream,
    then one grouped combination and one grouped operator action over all
    chips (FP64 T and F, F = A T of the T written).  value = all pairs /
    step time."""
    import torch

    from paper_2510_23221_amd import capi, synth

    dev = torch.device("cuda:0")
    w = synth.workload(2, m=args.m, nchips=args.nchips)
    pc = capi.PRECOND_JACOBI if args.precond == "jacobi" else capi.PRECOND_NONE
    Gs = [capi.HeatOperator.from_chip(c, dev, precond=pc) for c in w.chips]
    Bs = [torch.as_tensor(B, device=dev) for B in w.B]
    Cs = [torch.as_tensor(C, device=dev) for C in w.C]
    Xs = [torch.empty_like(B) for B in Bs]
    Ts = [torch.empty((w.m, G.n), dtype=torch.float64, device=dev) for G in Gs]
    Fs = [torch.empty((w.m, G.n), dtype=torch.float64, device=dev) for G in Gs]
    plan = capi.BatchPlan(Gs, w.s, capi.F32, m=[w.m] * len(Gs))
    stream = torch.cuda.Stream()
    infos = []
    with torch.cuda.stream(stream):
        tpw = plan.tune(dev, stream=stream)

        def step():
            _, _, _, inf = plan.run(Bs, Cs, w.tol, Xs=Xs, Ts=Ts, Fs=Fs, stream=stream)
            infos.append(inf)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        # census step: every kernel family timed
        capi.timing_reset()
        capi.timing_enable(None)
        step()
        torch.cuda.synchronize()
        census = {f: capi.timing_query(f) for f in capi.FAMILY}
        capi.timing_enable(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / steps
    pairs = w.m * len(w.chips)
    last = infos[-1]
    cells = sum(G.n for G in Gs)
    out_bytes = {"combine": cells * w.m * 8 + cells * w.s * 8 + len(Gs) * w.s * w.m * 8,
                 "apply": cells * w.m * 16 + cells * 4 * 8}

    def out_roof(kind):
        n_l, tot = census[kind]
        if n_l == 0:
            return None
        gbs = out_bytes[kind] / (tot / n_l * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "kernel": kind + " (grouped over all chips)",
                "avg_us": round(tot / n_l * 1e3, 2), "bytes_per_launch": int(out_bytes[kind]), "launches": n_l}

    ty, fpw = plan.output_tuning()
    res = {"metric": "data pairs/s at rel residual <=1e-8, batch of uneven chips", "value": round(pairs / (ms * 1e-3), 1),
           "unit": "pairs/s", "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": w.name, "nchips": len(w.chips), "cells_total": int(cells),
                      "s": w.s, "M_per_chip": w.m, "tol": w.tol, "scheme": "mixed", "T_F_dtype": "float64",
                      "precond": args.precond, "outputs": "grouped: one combination, then F = A T of the T written"},
           "autotuned": {"tiles_per_workgroup": tpw, "tile_rows_cap": ty, "fields_per_workgroup": fpw},
           "census_ms_per_step": {k: round(v[1], 3) for k, v in census.items()},
           "census_launches_per_step": {k: v[0] for k, v in census.items()},
           "output": out_roof("apply"), "combine": out_roof("combine"),
           "iters": {"min": min(i["iters"] for i in last), "max": max(i["iters"] for i in last),
                     "mean": sum(i["iters"] for i in last) / len(last)},
           "max_rel_res": max(i["max_rel_res"] for i in last),
           "all_ok": all(i["status"] == capi.OK for i in last)}
    plan.close()
    del Ts, Fs
    torch.cuda.empty_cache()
    return res


def bench_learned(args):
    """Learned start: generate the training pairs with BlocKOA (40 chips at
    128 x 128 x 8, 500 pairs each), train the encoder-decoder with the
    library's kernels, then solve unseen chips (s = 16) from the zero start,
    the smoothed zero start and the smoothed learned start."""
    import numpy as np
    import torch

    from paper_2510_23221_amd import capi, lstart, synth

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    w = synth.workload(4, m=args.m, nchips=args.nchips)
    pc = capi.PRECOND_JACOBI if args.precond == "jacobi" else capi.PRECOND_NONE
    data = lstart.generate_pairs(w.chips, w.B, w.C, 1e-10, compute=capi.F32, precond=pc)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    norm = lstart.fit_normalizer(data)
    batch = 16
    net = lstart.make_net(w.chips[0], base=32, max_batch=batch, seed=0)
    steps = max(1, int(args.train_epochs * len(w.chips) * w.m / batch))
    t0 = time.perf_counter()
    log = lstart.train(net, data, norm, steps=steps, batch=batch, lr=5e-4, seed=1, log_every=max(1, steps // 10))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    chips, Bs = synth.learned_start_test_chips(args.test_chips, w.chips[0].dims, w.s)
    # the trained parameters in a network sized for the maps of several
    # chips, so that their learned starts come from one inference pass
    group = max(1, args.infer_chips)
    inet = lstart.make_net(w.chips[0], base=32, max_batch=group * w.s, seed=0)
    inet.set_params(net.params)
    recs = lstart.evaluate(inet, norm, chips, Bs, w.tol, compute=capi.F32, smooth=20, precond=pc, group=group)
    z = np.array([r["zero_iters"] for r in recs])
    zs = np.array([r["zero_smooth_iters"] for r in recs])
    ln = np.array([r["learned_iters"] for r in recs])
    t_zero = sum(r["zero_s"] for r in recs)
    t_learn = sum(r["learned_s"] + r["infer_s"] for r in recs)
    res = {"metric": "block iterations and solve throughput, learned vs zero start",
           "unit": "basis solutions/s (network inference included for the learned start)",
           "value": round(len(recs) * w.s / t_learn, 2), "zero_start_value": round(len(recs) * w.s / t_zero, 2),
           "n_gpus": 1, "data": "synthetic", "dtype": "bf16 weights, f32 activations; f32+f64 solve",
           "config": {"workload": "learned-start-128x128x8", "train_chips": len(w.chips), "pairs": len(w.chips) * w.m,
                      "s": w.s, "test_chips": len(recs), "tol": w.tol, "params": net.nparams, "epochs": args.train_epochs,
                      "smoothing_sweeps": 20, "precond": args.precond, "chips_per_inference": group},
           "seconds": {"generate_pairs": round(t_gen, 2), "train": round(t_train, 2)},
           "train_loss": [(a, round(b, 6)) for a, b in log],
           "iters": {"zero": float(z.mean()), "zero_smoothed": float(zs.mean()), "learned": float(ln.mean())},
           "learned_fewer_than_zero_smoothed": int((ln < zs).sum()),
           "rejected_columns": int(sum(r["rejected"] for r in recs)),
           "max_rel_res": {"zero": max(r["zero_res"] for r in recs), "learned": max(r["learned_res"] for r in recs)}}
    return res


def capi_bytes_combine_apply(capi, G, s):
    import ctypes
    out = ctypes.c_size_t()
    capi._check(capi.load_library().bko_combine_apply_workspace_bytes(G.handle, s, ctypes.byref(out)))
    return out.value


def stage_errors(G, X, C, T, F, nsample=64):
    """Error of each output stage of the last step, on 64 evenly spaced
    fields (max over them of the relative 2-norm error):
      T: against X C formed in FP64 from the solve's X (rounding X and C to
        BF16 alone gives about 2^-8 times T_cancellation);
      F (stage-local, the pair's consistency): against A T of the T actually
        written, in FP64;
      F against the FP64 pipeline, A (X C): for low-precision fields this is
        large where A cancels (|A||T| >> |A T|), which is why pairs are judged
        stage-locally."""
    import torch

    from paper_2510_23221_amd import capi

    m = C.shape[0]
    idx = torch.linspace(0, m - 1, min(nsample, m), device=C.device).round().long().unique()
    T64 = C[idx].to(torch.float64) @ X
    Tw = T[idx].to(torch.float64)
    Fw = F[idx].to(torch.float64)
    F_stage = capi.apply_operator(G, Tw.contiguous())
    F64 = capi.apply_operator(G, T64.contiguous())

    def rel(a, b):
        return float(((a - b).norm(dim=1) / b.norm(dim=1).clamp_min(1e-300)).max())

    # cancellation in the sums: the error bound of a rounded input or product
    # scales with || |C| |X| || / || X C ||
    canc = float(((C[idx].to(torch.float64).abs() @ X.abs()).norm(dim=1) / T64.norm(dim=1).clamp_min(1e-300)).max())
    return {"fields": int(idx.numel()), "T_vs_XC": rel(Tw, T64), "T_cancellation": round(canc, 2),
            "F_vs_AT_stage": rel(Fw, F_stage), "F_vs_fp64_pipeline": rel(Fw, F64),
            "field_dtype": str(T.dtype).replace("torch.", "")}


def stencil_rate(G, T, F, t_dtype, apply_compute, nbytes, traffic, reps=5):
    """F = A T over all fields, timed alone with events on the launch stream
    (two warm-up launches, then `reps`): algorithmic bytes per launch over the
    average launch time."""
    import torch

    from paper_2510_23221_amd import capi

    for _ in range(2):
        capi.apply_operator(G, T, out_dtype=t_dtype, compute=apply_compute, F=F)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        capi.apply_operator(G, T, out_dtype=t_dtype, compute=apply_compute, F=F)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "apply", "avg_us": round(ms * 1e3, 2),
            "bytes_per_launch": int(nbytes), "launches": reps}


def per_sample_cg(G, B, C, w, cols, value):
    """The paper's direct method on the same GPU: an independent FP64 CG per
    power map (no shared Krylov space, no operator action), batched as
    columns.  The power maps are combinations b = B c of the basis maps, the
    sources of the fields the pairs carry.  pairs/s = columns / solve time."""
    import torch

    from paper_2510_23221_amd import capi

    cols = min(cols, w.m)
    Bc = (C[:cols] @ B).contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, iters, info = capi.cg_solve(G, Bc, w.tol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rate = cols / dt
    return {"value": round(rate, 2), "unit": "pairs/s", "columns": cols, "seconds": round(dt, 3),
            "mean_iters": round(float(iters.mean()), 1), "max_rel_res": info["max_rel_res"],
            "blockoa_over_cg": round(value / rate, 1)}


def ablations(G, B, C, X, w, cols, value, compute, wview, outputs, cg_rate):
    """The paper's ablation of BlocKOA's two modules (Sec. V, Table 7) on the
    same GPU and workload, as pairs/s:
      without block Krylov: the s basis solutions by per-column FP64 CG (same
        preconditioner), then the same combination and operator action;
      without operator action: every field's power map b = B c solved by the
        block solve itself, s columns at a time (timed on the first `cols`
        maps, rounded to whole blocks, and scaled linearly);
      without both: per-column CG of every power map (the per-sample CG
        baseline above)."""
    import torch

    from paper_2510_23221_amd import capi

    s, m = B.shape[0], C.shape[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Xcg, iters, _ = capi.cg_solve(G, B, w.tol)
    X.copy_(Xcg)
    outputs()
    torch.cuda.synchronize()
    t_wo_block = time.perf_counter() - t0
    nb = max(1, min(cols, m) // s)
    Bc = (C[:nb * s] @ B).contiguous()
    Xb = torch.empty_like(Bc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = 0
    for i in range(nb):
        _, info = capi.block_krylov_solve(G, Bc[i * s:(i + 1) * s], w.tol, compute=compute, X=Xb[i * s:(i + 1) * s],
                                          work=wview)
        its += info["iters"]
    torch.cuda.synchronize()
    t_wo_op = time.perf_counter() - t0
    r_block = m / t_wo_block
    r_op = nb * s / t_wo_op
    return {"unit": "pairs/s",
            "blockoa": round(value, 1),
            "wo_block_krylov": {"value": round(r_block, 1), "cg_mean_iters": round(float(iters.mean()), 1),
                                "blockoa_over": round(value / r_block, 2)},
            "wo_operator_action": {"value": round(r_op, 1), "columns": nb * s, "block_solves": nb,
                                   "mean_block_iters": round(its / nb, 1), "blockoa_over": round(value / r_op, 1)},
            "wo_all": {"value": cg_rate, "blockoa_over": round(value / cg_rate, 1)}}


def cpu_baseline(w, precond="jacobi", min_seconds=10.0, max_reps=5):
    """The CPU oracle as it stands, built -O3 -march=native on the host that
    runs it, over the whole workload (no extrapolation): per-column CG for the
    s basis solves (with the GPU path's preconditioner: Jacobi PCG, or plain
    CG), then combination and operator action of all M fields in chunks of
    500.  Repeated until min_seconds have elapsed; the median run is
    reported.  The other preconditioner's run is reported beside it."""
    import numpy as np

    import oracle

    oracle.select_build(native=True)
    chip = w.chips[0]
    A = oracle.assemble_chip(chip)
    cores = oracle.max_threads()

    def run(solver):
        t0 = time.perf_counter()
        X, iters, _ = solver(A, w.B[0], w.tol)
        t1 = time.perf_counter()
        for c0 in range(0, w.m, 500):
            T = oracle.gemm(X, w.C[0][c0:c0 + 500])
            oracle.apply_many(A, T)
        t2 = time.perf_counter()
        return t2 - t0, t1 - t0, iters

    main_solver = oracle.pcg_many if precond == "jacobi" else oracle.cg_many
    other_solver = oracle.cg_many if precond == "jacobi" else oracle.pcg_many
    runs, iters_seen, t_solve = [], None, []
    t_start = time.perf_counter()
    while len(runs) < max_reps and (time.perf_counter() - t_start < min_seconds or not runs):
        t, ts, iters_seen = run(main_solver)
        runs.append(t)
        t_solve.append(ts)
    t_other, ts_other, iters_other = run(other_solver)
    oracle.select_build(native=False)
    t = float(np.median(runs))
    return {"value": round(w.m / t, 2), "unit": "pairs/s", "cores": cores, "kind": "oracle",
            "sample": f"whole workload ({w.s} basis solves by {'Jacobi PCG' if precond == 'jacobi' else 'CG'} to "
                      f"rel res {w.tol:g}, mean {float(np.mean(iters_seen)):.0f} iterations, then combination + "
                      f"operator action of all {w.m} fields), median of {len(runs)} runs, gcc -O3 -march=native",
            "seconds_measured": round(float(sum(runs)), 2), "solve_seconds": round(float(np.median(t_solve)), 3),
            "other_preconditioner": {"solver": "CG" if precond == "jacobi" else "Jacobi PCG",
                                     "value": round(w.m / t_other, 2),
                                     "mean_iters": round(float(np.mean(iters_other)), 1),
                                     "solve_seconds": round(ts_other, 3)}}


if __name__ == "__main__":
    main()
