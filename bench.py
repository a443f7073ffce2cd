#!/usr/bin/env python3
"""Benchmark: ms per solve of the 74x74, 6-LGS, 35-layer tomographic system at
relative residual 1e-6, on one MI355X.

One step = one frame through the whole hot path: CG solve of
(Sigma_ss + Sigma_eta) zeta = s with the fused 2RBT products (FP32, with
FP64 residual replacement certifying the tolerance), preconditioned by the
block-circulant inverse of the embedding (default; --preconditioner none for
plain CG, which is also reported on the same line), followed by the LGS
projection phi = W_phi Sigma_phi_s zeta.  Kernel generation and spectra
(set-up, done once per atmosphere) are timed separately.  Inputs: 20 seeded
frames of slopes measured through von Karman layers, resident in HBM before
the timed region.

Prints one JSON line.  The roofline object is for the dominant kernel, the
persistent CG kernel: algorithmic bytes per iteration (packed FP32 slope
spectra, plus the preconditioner spectra when preconditioned, + slopes in and
out) times iterations per launch, over the launch duration measured with HIP
events on the library's stream.  The cpu_baseline object
times the FP64 oracle (CG with its step-by-step 2RBT product) on one frame.
The batch_matvec object measures the product of 64 distinct systems of the same
geometry per call (tt_matvec_batch, L = 256): the HBM-bound form of the
product, with its own roofline for the batched column kernel; batch_solve
solves one frame on each of those systems together (TT_SOLVER_BATCHED) and
reports the throughput in ms per solve.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "ms per solve at rel. residual 1e-6 (6 LGS, 74x74 SH), plain vs learned PCG"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=20)
    ap.add_argument("--pad", type=int, default=148)
    ap.add_argument("--precision", choices=["f32", "f64"], default="f32",
                    help="timed form (the FP16 / BF16 column-transform forms are reported under variants)")
    ap.add_argument("--solver", choices=["persistent", "kernels"], default="persistent")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--preconditioner", choices=["circulant", "none"], default="none",
                    help="headline solver: plain CG (the method, default) or CG with the block-circulant inverse")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true", help="skip the FP64 / kernel-solver side numbers")
    ap.add_argument("--batch", type=int, default=64,
                    help="distinct 74x74 systems in the batched-product measurement (0: skip it)")
    ap.add_argument("--batch-pad", type=int, default=256, help="FFT side L of the batched systems")
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--batch-only", action="store_true", help="run only the batched-product measurement")
    ap.add_argument("--uneven", type=int, default=64, help="uneven systems in the uneven batched measurement (0: skip)")
    ap.add_argument("--batch-solve-frames", type=int, default=0,
                    help="with --batch-only: also time the batched solves (plain and preconditioned CG) with this "
                         "many measured frames of lgs6_74x74 as right-hand sides")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner records")
    ap.add_argument("--learned-only", action="store_true", help="run only the learned-preconditioner records")
    ap.add_argument("--learned-pad-74", type=int, default=256,
                    help="padding of the 74x74 system in the batched (learned and plain) solves of the learned record")
    ap.add_argument("--learned-pad-10", type=int, default=20,
                    help="padding of the 10x10 system in the batched solves of the learned record")
    ap.add_argument("--no-multi", action="store_true", help="skip the many-frames-of-one-system records")
    ap.add_argument("--multi-pad", type=int, default=256,
                    help="padding of the 74x74 system in the many-frames records (batched solver)")
    ap.add_argument("--learned-steps", type=int, default=3000, help="optimiser steps of the learned preconditioner")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 256 MiB device buffer 3 times (reference kernel for rocprofv3 "
                         "FETCH_SIZE / WRITE_SIZE scale factors)")
    return ap.parse_args()


def traffic_record(pc):
    """HBM traffic of the persistent kernel measured with rocprofv3 counters
    (profiles/*_traffic.md), valid only while the kernel source is unchanged."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_cg_persistent_{'pcg' if pc else 'cg'}_f32_74x74_L148_traffic.md")
    src = os.path.join(ROOT, "paper_1806_07938_amd", "csrc", "persistent.hip")
    try:
        rec = {}
        for line in open(path):
            if ":" in line and line.split(":")[0] in ("traffic_bytes_per_iteration", "kernel_source_sha256"):
                k, v = line.split(":", 1)
                rec[k] = v.strip()
        if rec.get("kernel_source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
            return None
        return float(rec["traffic_bytes_per_iteration"])
    except (OSError, KeyError, ValueError):
        return None


def _oracle_cg_frame(args):
    """One frame through the oracle's FP64 CG (worker process, one BLAS thread)."""
    from threadpoolctl import threadpool_limits
    from oracle.solve import cg
    op, s, tol = args
    with threadpool_limits(1):
        t0 = time.perf_counter()
        x, it = cg(op, s, tol=tol, maxiter=20000)
        return time.perf_counter() - t0, it


def cpu_baseline(wl, frames, tol):
    """FP64 oracle as it stands (textbook CG with its step-by-step 2RBT product,
    numpy FFTs) on every host core: one frame per worker process, as many
    frames as workers, solved concurrently; ms per solve = wall time / frames."""
    import multiprocessing as mp
    from oracle.covariance import kernel_tables
    from oracle.toeplitz import ToeplitzOperator
    workers = max(1, min(16, os.cpu_count() or 1, len(frames)))
    t0 = time.perf_counter()
    op = ToeplitzOperator(wl, tables=kernel_tables(wl, workers=workers))
    setup = time.perf_counter() - t0
    jobs = [(op, frames[i].astype(np.float64), tol) for i in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_cg_frame, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    its = [it for _, it in res]
    return {
        "value": round(wall * 1e3 / workers, 1), "unit": "ms per solve", "cores": workers, "kind": "oracle",
        "sample": (f"{workers} frames of the same workload solved concurrently, one per process on {workers} host "
                   f"cores (one BLAS thread each): FP64 textbook CG to rel. residual {tol:g} "
                   f"({min(its)}-{max(its)} iterations) with the oracle's numpy 2RBT product; wall {wall:.1f} s for "
                   f"the {workers} solves, single-frame time {np.median([t for t, _ in res]):.1f} s; covariance "
                   f"tables built beforehand in {setup:.1f} s, not included"),
    }


def batch_traffic_record():
    """HBM traffic of the batched column kernel measured with rocprofv3 counters
    (profiles/k_bcolt_*_traffic.md), valid only while its source is unchanged."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_bcolt_f32_74x74_L256_x64_traffic.md")
    src = os.path.join(ROOT, "paper_1806_07938_amd", "csrc", "batch.hip")
    try:
        rec = {}
        for line in open(path):
            if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "kernel_source_sha256"):
                k, v = line.split(":", 1)
                rec[k] = v.strip()
        if rec.get("kernel_source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
            return None
        return float(rec["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def _uneven_frame(i):
    import workloads as W
    return W.turbulent_slopes(W.uneven_family(i))[0].astype(np.float32)


def batch_uneven(args):
    """args.uneven systems of workloads.uneven_family (grids 40 / 60 / 74 / 84 in
    turn, 4-8 LGS, 10-35 layers, noise 0.01-0.5 rad^2, L the power of two >= 2n):
    the batched product (with the column kernel's roofline) and one measured
    frame per system solved together by lockstep plain CG, and by lockstep CG
    preconditioned by the block-circulant inverse with its spectra stored in
    FP16."""
    import multiprocessing as mp
    import torch
    import workloads as W
    from paper_1806_07938_amd import Context, system_from
    ctxs, keep = [], []
    t0 = time.perf_counter()
    for i in range(args.uneven):
        c = Context(0)
        keep.append(system_from(c, W.uneven_family(i), target=False))
        ctxs.append(c)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    workers = max(1, min(16, os.cpu_count() or 1))
    with mp.get_context("fork").Pool(workers) as pool:
        frames = pool.map(_uneven_frame, range(args.uneven))
    grids = sorted({c.info["n"] for c in ctxs})
    label = (f"{args.uneven} uneven systems (grids {'/'.join(map(str, grids))}, 4-8 LGS, 10-35 layers, noise "
             "0.01-0.5 rad^2, r0 0.10-0.25 m, L = 128 / 256)")
    out = {"batch_tuning_uneven": tune(ctxs, 0),
           "batch_matvec_uneven": batch_matvec(args, ctxs, setup_s, label=label, split=0),
           "batch_solve_uneven": batch_solve(args, ctxs, frames, 0, label=label),
           # mixed precision on the uneven mix: the block-circulant preconditioner
           # with its spectra stored in FP16, the operator in FP32
           "batch_solve_uneven_pcg_f16": batch_solve(args, ctxs, frames, 1, precision=2, label=label)}
    for c in ctxs + keep:
        c.close()
    return out


def multi_rhs(args, ctx, frames, pc):
    """All frames of the nominal system solved together: the base context and
    len(frames) - 1 views sharing its spectra (tt_create_view), lockstep CG
    (TT_SOLVER_BATCHED), plain or preconditioned by the block-circulant inverse."""
    import torch
    from paper_1806_07938_amd import solve_batch
    from paper_1806_07938_amd.tt import SOLVER_BATCHED, TT_NOT_CONVERGED
    views = [ctx.view() for _ in range(len(frames) - 1)]
    S = [torch.tensor(f, device="cuda:0") for f in frames]
    allow = (0, TT_NOT_CONVERGED)
    solve_batch([ctx] + views, S, tol=args.tol, solver=SOLVER_BATCHED, preconditioner=pc, allow=allow)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, infos, st = solve_batch([ctx] + views, S, tol=args.tol, solver=SOLVER_BATCHED, preconditioner=pc,
                                  allow=allow)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    for v in views:
        v.close()
    it = np.array([i.iterations for i in infos], dtype=np.float64)
    return {"workload": (f"{len(frames)} frames of the 74x74 / 6 LGS system (L={ctx.info['pad_L']}) solved together on one "
                         "system and its views (shared spectra), lockstep "
                         + ("CG preconditioned by the block-circulant inverse" if pc else "plain CG")
                         + f" to rel. residual {args.tol:g}"),
            "frames": len(frames), "ms_per_batch": round(wall, 2), "ms_per_solve": round(wall / len(frames), 3),
            "iterations_mean": round(float(it.mean()), 1), "iterations_max": int(it.max()),
            "all_converged": bool(st == 0 and all(i.status == 0 and i.rel_residual <= args.tol for i in infos))}


def batch_systems(args):
    """args.batch distinct 74x74 / 6 LGS systems (seeded layer weights and r0,
    L = args.batch_pad); returns (contexts, kernel objects, set-up seconds)."""
    import torch
    import workloads as W
    from paper_1806_07938_amd import Context, system_from
    ctxs, keep = [], []
    t0 = time.perf_counter()
    for i in range(args.batch):
        wl = W.lgs6_74x74_family(i, pad_L=args.batch_pad)
        c = Context(0)
        keep.append(system_from(c, wl, target=False))
        ctxs.append(c)
    torch.cuda.synchronize()
    return ctxs, keep, time.perf_counter() - t0


def batch_solve(args, ctxs, frames, pc, precision=0, label=None):
    """TT_SOLVER_BATCHED over the same systems: one frame each (the measured
    frames of lgs6_74x74 reused in turn as right-hand sides), FP32 CG (plain,
    or preconditioned by the block-circulant inverse when pc) with the FP64
    residual replacement, to args.tol; one untimed batch (it also builds the
    preconditioner spectra, timed apart), then one timed."""
    import torch
    from paper_1806_07938_amd import solve_batch
    from paper_1806_07938_amd.tt import SOLVER_BATCHED, TT_NOT_CONVERGED
    S = [torch.tensor(frames[i % len(frames)], device="cuda:0") for i in range(len(ctxs))]
    if label:   # one right-hand side per system (frames[i] belongs to ctxs[i])
        assert len(frames) == len(ctxs)
    t0 = time.perf_counter()
    prec = precision if precision else 0
    if pc:   # preconditioner spectra, once per system (host FP64), before the untimed batch
        solve_batch(ctxs, S, tol=args.tol, max_iter=0, solver=SOLVER_BATCHED, preconditioner=pc,
                    allow=(0, TT_NOT_CONVERGED), precision=prec)
    torch.cuda.synchronize()
    pc_setup_s = time.perf_counter() - t0
    solve_batch(ctxs, S, tol=args.tol, solver=SOLVER_BATCHED, preconditioner=pc, allow=(0, TT_NOT_CONVERGED),
                precision=prec, graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, infos, st = solve_batch(ctxs, S, tol=args.tol, solver=SOLVER_BATCHED, preconditioner=pc,
                                  allow=(0, TT_NOT_CONVERGED), precision=prec, graph=True)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    it = np.array([i.iterations for i in infos], dtype=np.float64)
    return {
        "workload": ((label or f"{len(ctxs)} distinct 74x74 / 6 LGS / 35-layer systems, L={args.batch_pad}")
                     + ", one frame each, solved together (TT_SOLVER_BATCHED: "
                     + ("CG preconditioned by the block-circulant inverse" if pc else "plain CG")
                     + ({2: " (its spectra stored in FP16)", 3: " (its spectra stored in BF16)"}.get(prec, ""))
                     + f" in lockstep, chunks replayed from HIP graphs, FP32 + FP64 residual replacement) to rel. "
                     f"residual {args.tol:g}"),
        "systems": len(ctxs), "ms_per_batch": round(wall, 2), "ms_per_solve": round(wall / len(ctxs), 3),
        "preconditioner_setup_s": round(pc_setup_s, 1) if pc else None,
        "iterations_mean": round(float(it.mean()), 1), "iterations_max": int(it.max()),
        "rel_residual_max": max(i.rel_residual for i in infos),
        "all_converged": bool(st == 0 and all(i.status == 0 and i.rel_residual <= args.tol for i in infos)),
    }


def tune(ctxs, op=0):
    """tt_tune_batch on the batch: the chosen frequency split and the timing table."""
    from paper_1806_07938_amd.tt import tune_batch
    best, ms = tune_batch(ctxs, op=op)
    return {"split": best, "ms_per_call_by_split": {str(k): (round(v, 4) if v else None) for k, v in ms.items()}}


def batch_matvec(args, ctxs, setup_s, precision=0, label=None, split=2):
    """tt_matvec_batch over the systems: spectra of all of them streamed once
    per call.  Roofline of the column kernel: algorithmic bytes = the packed
    spectra of every system (FP32, or FP16 / BF16 storage plus one FP32 factor
    per frequency for precision 2 / 3), over its HIP-event duration."""
    import torch
    dev = torch.device("cuda:0")
    from paper_1806_07938_amd import matvec_batch
    rng = np.random.default_rng(1806)
    xs = [torch.tensor(rng.standard_normal(c.info["n_slopes"]).astype(np.float32), device=dev) for c in ctxs]
    ys = [torch.empty_like(x) for x in xs]
    for _ in range(3):
        matvec_batch(ctxs, xs, ys, precision=precision, split=split)
    torch.cuda.synchronize()
    phases = []
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        phases.append(matvec_batch(ctxs, xs, ys, timing=True, precision=precision, split=split)[1])
    wall_ms = (time.perf_counter() - t0) * 1e3 / args.batch_steps
    ph = np.array(phases).mean(axis=0)
    spectra = float(sum(c.info["spectra_bytes_f32"] for c in ctxs))
    if precision:
        spectra = float(sum(c.info["spectra_bytes_f32"] // 2 + 4 * c.info["pad_L"] * (c.info["pad_L"] // 2 + 1)
                            for c in ctxs))
    slopes = float(sum(2 * 4 * c.info["n_slopes"] for c in ctxs))
    col_gbs = spectra / (ph[1] * 1e-3) / 1e9
    # the recorded counters are those of the frequency split 2
    traffic = batch_traffic_record() if (args.batch == 64 and args.batch_pad == 256 and not precision and split == 2
                                         and not label) else None
    pname = {0: "FP32", 2: "FP16 (per-frequency power-of-two scale)", 3: "BF16"}[precision]
    return {
        "workload": ((label or f"{args.batch} distinct 74x74 / 6 LGS / 35-layer systems (seeded layer weights, r0 "
                      f"in [0.10, 0.25] m), L={args.batch_pad}")
                     + f", one product each per call, spectra stored in {pname}, FP32 arithmetic"),
        "systems": len(ctxs), "pad_L": args.batch_pad if not label else "per system", "steps": args.batch_steps,
        "frequency_split": split or "tuned",
        "ms_per_call_wall": round(wall_ms, 4),
        "ms_per_call_gpu": round(float(ph.sum()), 4),
        "us_per_system_product": round(float(ph.sum()) * 1e3 / len(ctxs), 3),
        "phase_ms": {"row_fwd": round(float(ph[0]), 4), "col": round(float(ph[1]), 4),
                     "row_inv": round(float(ph[2]), 4)},
        "algorithmic_bytes": {"spectra": int(spectra), "slopes_in_out": int(slopes)},
        "whole_product_gbs": round((spectra + slopes) / (ph.sum() * 1e-3) / 1e9, 1),
        "roofline": {"bound": "hbm", "achieved": round(col_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(col_gbs / HBM_PEAK_GBS, 4), "traffic": round(traffic) if traffic else None,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0, copy-calibrated)",
                     "kernel": ("k_bcolt (batched column transforms and per-frequency products, spectra slot-major, "
                                "direct loads to LDS; power-of-two L)"),
                     "avg_launch_ms": round(float(ph[1]), 4)},
        "setup_s": round(setup_s, 1),
    }


def learned_record(wl_of, family, n_systems, steps, frames, tol, label, pad_batched=None):
    """Train the learned preconditioner on n_systems systems of one geometry
    (family(i): random r0 and layer weights; 20000 (r = A e, e) pairs drawn by
    the library), then solve `frames` of the nominal system wl_of() with
    flexible CG preconditioned by it and with plain CG, both in the batched
    solver (one frame per call), and the persistent plain CG.  The batched
    solves use the same system padded to pad_batched (the power-of-two
    transforms of the batched kernels), the persistent one its own padding."""
    import torch
    from paper_1806_07938_amd import Context, Learned, system_from
    from paper_1806_07938_amd.tt import PRECOND_LEARNED, SOLVER_BATCHED, SOLVER_PERSISTENT, TT_NOT_CONVERGED, tune_batch
    ctxs, keep = [], []
    for i in range(n_systems):
        c = Context(0)
        keep.append(system_from(c, family(i), target=False))
        ctxs.append(c)
    wl = wl_of()
    net = Learned(wl.n_gs, 32, seed=1806)
    t0 = time.perf_counter()
    tinfo = net.train(ctxs, n_pairs=20000, steps=steps, batch=16, lr=3e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    for c in ctxs + keep:
        c.close()
    ctx = Context(0)
    kk = system_from(ctx, wl, target=True)
    ctxb, kkb = ctx, None
    if pad_batched and pad_batched != wl.pad_L:
        ctxb = Context(0)
        kkb = system_from(ctxb, wl_of(pad_batched), target=True)
    ctxb.set_learned(net)
    tune_batch([ctxb])
    S = [torch.tensor(f, device="cuda:0") for f in frames]
    res = {}
    allow = (0, TT_NOT_CONVERGED)
    for name, sv, pcm in (("learned_fpcg", SOLVER_BATCHED, PRECOND_LEARNED), ("batched_plain_cg", SOLVER_BATCHED, 0),
                          ("persistent_plain_cg", SOLVER_PERSISTENT, 0)):
        gr = sv == SOLVER_BATCHED
        cx = ctxb if gr else ctx
        cx.solve(S[0], tol=tol, solver=sv, preconditioner=pcm, allow=allow, graph=gr)
        torch.cuda.synchronize()
        ii = []
        t0 = time.perf_counter()
        for s in S:
            ii.append(cx.solve(s, tol=tol, solver=sv, preconditioner=pcm, allow=allow, graph=gr)[2])
        torch.cuda.synchronize()
        res[name] = {"ms_per_solve": round((time.perf_counter() - t0) * 1e3 / len(S), 3),
                     "pad_L": cx.info["pad_L"],
                     "iterations_mean": round(float(np.mean([i.iterations for i in ii])), 1),
                     "converged": all(i.status == 0 and i.rel_residual <= tol for i in ii),
                     "fallback": [int(i.fallback) for i in ii] if pcm else None}
    if kkb is not None:
        ctxb.close()
        kkb.close()
    ctx.close()
    kk.close()
    net.close()
    return {"workload": label, "training": {"systems": n_systems, "pairs": 20000, "steps": steps, "batch": 16,
                                            "objective_first": round(tinfo["objective_first"], 1),
                                            "objective_last": round(tinfo["objective_last"], 1),
                                            "device_ms": round(tinfo["ms"], 1), "wall_s": round(train_s, 2)},
            "frames": len(S), "tol": tol, **res}


def learned_records(args, W, frames):
    c1 = W.lgs3_10x10()
    return {
        "learned_74x74": learned_record(
            lambda pad=args.pad: W.lgs6_74x74(pad_L=pad), lambda i: W.lgs6_74x74_family(i, pad_L=args.pad), 8,
            args.learned_steps, frames[:3], args.tol,
            "learned preconditioner (P = K^T K, 4-layer masked CNN, 32 channels) trained on 8 systems of the "
            "74x74 / 6 LGS geometry with random r0 and layer weights, then flexible CG on 3 frames of the "
            f"nominal system to rel. residual {args.tol:g}, against plain CG",
            pad_batched=args.learned_pad_74),
        "learned_10x10": learned_record(
            lambda pad=c1.pad_L: W.lgs3_10x10(pad_L=pad), W.lgs3_10x10_family, 8, args.learned_steps,
            W.turbulent_slopes(c1, frames=5).astype(np.float32), 1e-10,
            "the same at 10x10 / 3 LGS (8 training systems with random r0 and layer weights), 5 frames of "
            "lgs3_10x10 to rel. residual 1e-10", pad_batched=args.learned_pad_10),
    }


def persistent_roofline(infos, wl, info, prec, pc, pad):
    """Roofline of the persistent solver kernel.  Algorithmic bytes per
    iteration are those of one 2RBT product (the packed slope spectra and the
    slopes in and out); with a preconditioner its spectra are reported apart
    and are not counted in frac."""
    kms = np.array([i.kernel_ms for i in infos])
    if kms.sum() <= 0:
        return None
    iters = np.array([i.iterations for i in infos], dtype=np.float64)
    launches = np.array([i.kernel_launches for i in infos], dtype=np.float64)
    from paper_1806_07938_amd.tt import PREC_F32
    elem = 4 if prec == PREC_F32 else 8
    spectra = info["spectra_bytes_f32"] if prec == PREC_F32 else info["spectra_bytes_f64"]
    bytes_iter = spectra + 2 * wl.n_slopes * elem
    C = 2 * wl.n_gs
    pc_bytes = pad * (pad // 2 + 1) * C * C * elem if pc else 0   # general Hermitian packing
    avg_launch_ms = kms.sum() / launches.sum()
    ipl = iters.sum() / launches.sum()
    achieved = bytes_iter * ipl / (avg_launch_ms * 1e-3) / 1e9
    tpi = traffic_record(pc) if (prec == PREC_F32 and pad == 148) else None
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": round(tpi * ipl) if tpi else None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0, copy-calibrated)",
            "kernel": (f"k_cg_persistent<float, true, 1, {1 if pc else 0}> (FP32 column transforms on the matrix "
                       "cores)" if prec == PREC_F32 else f"k_cg_persistent<double, true, 0, {1 if pc else 0}>"),
            "avg_launch_ms": round(avg_launch_ms, 4), "bytes_per_iteration": int(bytes_iter),
            "bytes_per_iteration_basis": "packed slope spectra + slopes in and out (one 2RBT product)",
            "preconditioner_spectra_bytes_per_iteration": int(pc_bytes) if pc else None,
            "iterations_per_launch": round(float(ipl), 1)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library solves one system on one GPU (asked for --gpus {args.gpus}); "
              "a system is not sharded across GPUs.", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    from paper_1806_07938_amd import Context, system_from
    from paper_1806_07938_amd.tt import (METHOD_CG, METHOD_MINRES, PRECOND_CIRCULANT, PRECOND_NONE, PREC_BF16,
                                         PREC_F16, PREC_F32, PREC_F64, SOLVER_KERNELS, SOLVER_PERSISTENT,
                                         TT_NOT_CONVERGED, close_all)

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        cx = torch.ones(64 * 1024 * 1024, device=dev)
        cy = torch.empty_like(cx)
        for _ in range(3):
            cy.copy_(cx)
        torch.cuda.synchronize()
        del cx, cy
    if args.batch_only:
        bctx, bkeep, bsetup = batch_systems(args)
        res = {"batch_tuning": tune(bctx, 0)}
        sp = res["batch_tuning"]["split"]
        res.update({"batch_matvec": batch_matvec(args, bctx, bsetup, split=sp),
                    "batch_matvec_f16": batch_matvec(args, bctx, bsetup, precision=2, split=sp),
                    "batch_matvec_bf16": batch_matvec(args, bctx, bsetup, precision=3, split=sp)})
        if args.batch_solve_frames > 0:
            fr = W.turbulent_slopes(W.lgs6_74x74(), frames=args.batch_solve_frames).astype(np.float32)
            res["batch_solve"] = batch_solve(args, bctx, fr, 0)
            res["batch_solve_pcg"] = batch_solve(args, bctx, fr, 1)
        torch.cuda.synchronize()
        close_all()
        print(json.dumps(res), flush=True)
        return
    wl = W.lgs6_74x74(pad_L=args.pad)
    frames = W.turbulent_slopes(wl, frames=args.frames).astype(np.float32)
    if args.learned_only:
        res = learned_records(args, W, frames)
        torch.cuda.synchronize()
        close_all()
        print(json.dumps(res), flush=True)
        return

    ctx = Context(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern = system_from(ctx, wl, target=True)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    info = ctx.info

    S = torch.tensor(frames, device=dev)
    zeta = torch.empty(wl.n_slopes, dtype=torch.float64, device=dev)
    phi = torch.empty(info["n_vphi"], dtype=torch.float32, device=dev)
    prec = PREC_F32 if args.precision == "f32" else PREC_F64
    solver = SOLVER_PERSISTENT if args.solver == "persistent" else SOLVER_KERNELS
    pc = PRECOND_CIRCULANT if (args.preconditioner == "circulant" and solver == SOLVER_PERSISTENT) else PRECOND_NONE

    def run(k, prec=prec, solver=solver, allow=(0,), pc=pc, method=METHOD_CG):
        return ctx.solve(S[k % args.frames], zeta=zeta, phi=phi, tol=args.tol, precision=prec, solver=solver,
                         allow=allow, preconditioner=pc, method=method)[2]

    t0 = time.perf_counter()
    if pc:   # the preconditioner spectra are built once per system, before the timed solves
        ctx.solve(S[0], zeta=zeta, phi=phi, tol=args.tol, precision=prec, max_iter=0, preconditioner=pc,
                  allow=(0, TT_NOT_CONVERGED))
    torch.cuda.synchronize()
    pc_setup_ms = (time.perf_counter() - t0) * 1e3

    for k in range(args.warmup):
        run(k)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        infos.append(run(k))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps

    iters = np.array([i.iterations for i in infos], dtype=np.float64)
    relres = max(i.rel_residual for i in infos)
    ok = all(i.status == 0 for i in infos) and relres <= args.tol
    roofline = persistent_roofline(infos, wl, info, prec, pc, args.pad) if solver == SOLVER_PERSISTENT else None
    method_name = "CG preconditioned by the block-circulant inverse" if pc else "plain CG"

    out = {
        "metric": METRIC, "value": round(ms_per_step, 4), "unit": "ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == PREC_F32 else "f64", "data": "synthetic",
        "config": {"workload": (f"39 m pupil, 28% obstruction, 74x74 SH (3972 valid/WFS), 6 LGS at 90 km on a 60 "
                                f"arcsec ring, 35 layers 30 m-26.5 km, r0 0.157 m, L0 25 m, sigma^2 0.1 rad^2, "
                                f"L={args.pad}, on-axis target; {method_name} to rel. residual {args.tol:g}, "
                                f"then the LGS projection"),
                   "n": wl.n, "n_gs": wl.n_gs, "n_layer": wl.n_layer, "n_slopes": wl.n_slopes, "pad_L": args.pad,
                   "solver": args.solver, "preconditioner": "circulant" if pc else "none",
                   "precision": args.precision + ("+f64 residual replacement" if prec == PREC_F32 else ""),
                   "frames": args.frames},
        "valid": bool(ok),
        "iterations_mean": round(float(iters.mean()), 1),
        "refinements_mean": round(float(np.mean([i.refinements for i in infos])), 2),
        "rel_residual_max": relres,
        "setup_ms": round(setup_ms, 1),
        "preconditioner_setup_ms": round(pc_setup_ms, 1) if pc else None,
        "roofline": roofline,
    }
    if not args.no_variants:
        side = {}
        # other forms on frames 0-2 (status and the FP64 residual reached are
        # reported per frame)
        CG, MR = METHOD_CG, METHOD_MINRES
        for name, p, sv, vpc, mth in (("f32_persistent_plain_cg", PREC_F32, SOLVER_PERSISTENT, PRECOND_NONE, CG),
                                      ("f32_persistent_circulant_pcg", PREC_F32, SOLVER_PERSISTENT, PRECOND_CIRCULANT, CG),
                                      ("f32_persistent_minres", PREC_F32, SOLVER_PERSISTENT, PRECOND_NONE, MR),
                                      ("f64_persistent_plain_cg", PREC_F64, SOLVER_PERSISTENT, PRECOND_NONE, CG),
                                      ("f64_persistent_circulant_pcg", PREC_F64, SOLVER_PERSISTENT, PRECOND_CIRCULANT, CG),
                                      ("f64_persistent_minres", PREC_F64, SOLVER_PERSISTENT, PRECOND_NONE, MR),
                                      ("f32_kernels_plain_cg", PREC_F32, SOLVER_KERNELS, PRECOND_NONE, CG)):
            if p == prec and sv == solver and vpc == pc and mth == CG:
                continue
            allow = (0, TT_NOT_CONVERGED)
            run(0, p, sv, allow, vpc, mth)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ii = [run(k, p, sv, allow, vpc, mth) for k in range(3)]
            torch.cuda.synchronize()
            side[name] = {"ms_per_solve": round((time.perf_counter() - t0) * 1e3 / 3, 3),
                          "iterations_mean": round(float(np.mean([i.iterations for i in ii])), 1),
                          "status": [int(i.status) for i in ii],
                          "rel_residual": [float(f"{i.rel_residual:.3e}") for i in ii],
                          "converged": all(i.status == 0 and i.rel_residual <= args.tol for i in ii)}
            if sv == SOLVER_PERSISTENT and mth == CG:
                side[name]["roofline"] = persistent_roofline(ii, wl, info, p, vpc, args.pad)
        # the 160-point axes of the precision configuration: the same system at
        # L = 160, plain CG (persistent) and CG preconditioned by the block-circulant
        # inverse with its spectra stored in FP16 (batched solver, one frame per call)
        from paper_1806_07938_amd.tt import SOLVER_BATCHED
        wl160 = W.lgs6_74x74(pad_L=160)
        c160 = Context(0)
        k160 = system_from(c160, wl160, target=True)
        for name, p, sv, vpc in (("f32_persistent_plain_cg_L160", PREC_F32, SOLVER_PERSISTENT, PRECOND_NONE),
                                 ("f16_spectra_batched_circulant_pcg_L160", PREC_F16, SOLVER_BATCHED,
                                  PRECOND_CIRCULANT)):
            allow = (0, TT_NOT_CONVERGED)
            c160.solve(S[0], tol=args.tol, precision=p, solver=sv, preconditioner=vpc, allow=allow)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ii = [c160.solve(S[k], tol=args.tol, precision=p, solver=sv, preconditioner=vpc, allow=allow)[2]
                  for k in range(3)]
            torch.cuda.synchronize()
            side[name] = {"ms_per_solve": round((time.perf_counter() - t0) * 1e3 / 3, 3),
                          "iterations_mean": round(float(np.mean([i.iterations for i in ii])), 1),
                          "status": [int(i.status) for i in ii],
                          "rel_residual": [float(f"{i.rel_residual:.3e}") for i in ii],
                          "converged": all(i.status == 0 and i.rel_residual <= args.tol for i in ii)}
        c160.close()
        k160.close()
        out["variants"] = side
    if not args.no_multi:
        # the same system padded to args.multi_pad: the batched kernels run their
        # power-of-two transforms at 256 (11.5 against 22.4 ms per solve at 148)
        cm, km = ctx, None
        if args.multi_pad != args.pad:
            cm = Context(0)
            km = system_from(cm, W.lgs6_74x74(pad_L=args.multi_pad), target=False)
        out["multi_rhs"] = multi_rhs(args, cm, frames, 0)
        out["multi_rhs_pcg"] = multi_rhs(args, cm, frames, 1)
        if km is not None:
            cm.close()
            km.close()
    if not args.no_learned:
        out.update(learned_records(args, W, frames))
    if args.batch > 0:
        bctx, bkeep, bsetup = batch_systems(args)
        out["batch_tuning"] = tune(bctx, 0)
        sp = out["batch_tuning"]["split"]
        out["batch_matvec"] = batch_matvec(args, bctx, bsetup, split=sp)
        out["batch_matvec_f16"] = batch_matvec(args, bctx, bsetup, precision=2, split=sp)
        out["batch_matvec_bf16"] = batch_matvec(args, bctx, bsetup, precision=3, split=sp)
        out["batch_solve"] = batch_solve(args, bctx, frames, 0)
        out["batch_solve_pcg"] = batch_solve(args, bctx, frames, 1)
        out["batch_solve_pcg_f16"] = batch_solve(args, bctx, frames, 1, precision=2)
        for c in bctx + bkeep:
            c.close()
    if args.uneven > 0:
        out.update(batch_uneven(args))
    torch.cuda.synchronize()
    close_all()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, frames, args.tol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
