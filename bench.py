"""Benchmark: persistent homology of a 256^3 volume on one MI355X.

Workload: the 256^3 float32 volume of 200 Gaussian blobs plus U[-0.05,0.05)
noise (synth.blobs3d, seed 2), diagrams in degrees 0, 1 and 2.  One step is one
cr_persistence call on the volume already resident in HBM: every stage of the
path (stencil, sort, degree 0, degree 1, degree 2, output) and the read-back of
the row count.  The metric is cells of the cubical complex per second,
N = (2*256-1)^3 = 133,432,831 cells per step.

Also reported (one JSON line):
  roofline     -- the stencil kernel (filtration + apparent pairs + survivor
                  compaction, the HBM-streaming pass) against the 8 TB/s HBM peak;
                  its duration is the mean of HIP events recorded around it on the
                  call's stream during the timed steps; "issue" gives its profiled
                  VALU instructions per launch against the single-issue ceiling,
                  "cold" the same stage with the last-level cache flushed before
                  the call (outside the timed steps);
  cpu_baseline -- the CPU oracle timed on a bounded sample of the workload;
  stages       -- mean per-stage times over the timed steps;
  batched      -- 512 2D images of sides 28..512 (half uniform noise, half
                  sigma-2 fields): images/s of one batched call replayed from a
                  HIP graph (after the autotuner picked its launch parameters),
                  of the eager batched call, and of 512 plain calls;
  fwd_bwd      -- 32 volumes of 128^3 (sigma-3 fields), loss = sum over finite
                  degree-1/2 bars with lifetime > 0.1 of lifetime^2: one batched
                  forward + backward against 32 per-volume forward + backward.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-forms]
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
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4  # G wavefront VALU instructions per second, single issue


def stencil_bytes(shape, survivors_total: int) -> int:
    """Algorithmic bytes of one stencil launch: read every pixel once (4 B),
    write each survivor's 64-bit key (8 B), write the vertex-forest link of
    every pixel (4 B) and the dual-forest link of every top cell (4 B)."""
    P = 1
    C = 1
    for n in shape:
        P *= n
        C *= n - 1
    return 4 * P + 8 * survivors_total + 4 * P + 4 * C


def sort_bytes(n_keys: int, bits: int) -> int:
    """Algorithmic bytes of the sort of the surviving cells: every 8-bit pass
    reads and writes each 64-bit key once (16 B)."""
    return 16 * n_keys * ((bits + 7) // 8)


def profiled_fields(kernel_md: str):
    """Per-launch counter values recorded in profiles/<kernel_md> (HBM bytes from
    FETCH_SIZE + WRITE_SIZE scaled by a plain copy's counts, instruction counts),
    or None when the kernel's source no longer has the digest they were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", kernel_md)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("    "):
            k, v = line.strip().split(":", 1)
            fields[k.strip()] = v.strip()
    src = os.path.join(ROOT, fields.get("source", ""))
    if not os.path.isfile(src):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != fields.get("source_sha256"):
        return None
    return fields


def profiled_traffic(kernel_md: str):
    f = profiled_fields(kernel_md)
    return int(f["traffic_bytes"]) if f and "traffic_bytes" in f else None


def issue_rate(kernel_md: str, ms: float):
    """The kernel's vector instruction issue rate (profiled VALU wavefront
    instructions per launch over the measured duration) against the chip's
    single-issue ceiling: 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64
    instruction = 614.4 G/s."""
    f = profiled_fields(kernel_md)
    if not f or "valu_insts" not in f:
        return None
    n = int(f["valu_insts"])
    achieved = n / (ms * 1e-3) / 1e9
    return {"valu_insts": n, "achieved": achieved, "peak": VALU_PEAK_GINST, "unit": "G wave-instr/s",
            "frac": achieved / VALU_PEAK_GINST}


def copy_ceiling(nbytes: int = 1 << 28, reps: int = 5) -> float:
    """GB/s (read + write) of a device-to-device copy of nbytes: the practical
    HBM ceiling the stencil is compared with."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        dst.copy_(src)
    ev[1].record()
    torch.cuda.synchronize()
    return 2 * nbytes * reps / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e9


def cpu_baseline(vol):
    import numpy as np
    import oracle
    sample = np.ascontiguousarray(vol[:128, :128, :128])
    t0 = time.perf_counter()
    d = oracle.persistence(sample, maxdim=2)
    dt = time.perf_counter() - t0
    cells = 255 ** 3
    return {"value": cells / dt, "unit": "cells/s", "cores": 1, "kind": "oracle",
            "sample": "the 128^3 corner [:128,:128,:128] of the same volume, degrees 0-2, "
                      f"{cells} cells, {len(d)} bars, {dt:.2f} s on one host core"}


def bench_batched(reps: int = 3) -> dict:
    """512 images: HIP-graph replay, eager batched call and 512 plain calls."""
    import torch
    import paper_2005_12692_amd as cr
    import synth
    imgs = synth.config("C4")
    ts = [torch.from_numpy(i).cuda() for i in imgs]
    packed, shapes, offs = cr.pack(ts)
    n = len(imgs)
    d = cr.persistence_batched(packed, shapes, offs)            # sizes the capacity and warms up
    cap = int(d.pair_offsets[-1].item())
    t = time.perf_counter()
    tuned = cr.autotune(packed, shapes, offs, capacity=cap, repeats=1)
    tune_s = time.perf_counter() - t
    print(f"batched: autotuned in {tune_s:.1f} s: {tuned}", file=sys.stderr, flush=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    prealloc = cr._empty_out(cap, n, packed.device)
    eager_s = timed(lambda: cr.persistence_batched(packed, shapes, offs, out=prealloc, check=False))
    g = cr.BatchedGraph(packed, shapes, offs, capacity=cap)
    graph_s = timed(g.launch)
    rows = int(g.result().dim.shape[0])
    g.close()
    print(f"batched: graph {graph_s * 1e3:.1f} ms, eager {eager_s * 1e3:.1f} ms", file=sys.stderr, flush=True)
    plain_s = timed(lambda: [cr.persistence(x) for x in ts])
    print(f"batched: plain loop {plain_s * 1e3:.1f} ms", file=sys.stderr, flush=True)
    return {"workload": "512 2D float32 images, sides uniform in 28..512, half U[0,1) noise, half sigma-2 "
                        "Gaussian fields (seed 3); H0+H1",
            "images": n, "pixels": int(offs[-1]), "rows": rows,
            "graph_img_per_s": n / graph_s, "eager_batched_img_per_s": n / eager_s,
            "plain_img_per_s": n / plain_s, "graph_vs_plain": plain_s / graph_s,
            "graph_ms": graph_s * 1e3, "eager_batched_ms": eager_s * 1e3, "plain_loop_ms": plain_s * 1e3,
            "tuning": tuned, "autotune_s": tune_s}


def bench_fwd_bwd(reps: int = 2) -> dict:
    """32 volumes: batched forward + backward against a per-volume loop."""
    import torch
    import paper_2005_12692_amd as cr
    import synth
    vols = synth.config("C5")
    ts = [torch.from_numpy(v).cuda() for v in vols]
    packed, shapes, offs = cr.pack(ts)

    def loss_of(birth, death, dim):
        life = death - birth
        act = (dim >= 1) & torch.isfinite(death) & (life > 0.1)
        return (life[act] ** 2).sum(), int(act.sum())

    def batched():
        x = packed.detach().requires_grad_(True)
        dim, birth, death, bp, dp, po = cr.PersistenceBatchedFn.apply(x, shapes)
        loss, nact = loss_of(birth, death, dim)
        loss.backward()
        return x.grad, nact

    def per_volume():
        grads, nact = [], 0
        for v in ts:
            x = v.detach().requires_grad_(True)
            dim, birth, death, bp, dp = cr.PersistenceFn.apply(x)
            loss, k = loss_of(birth, death, dim)
            loss.backward()
            grads.append(x.grad.reshape(-1))
            nact += k
        return torch.cat(grads), nact

    gb, nact = batched()
    gp, nact_p = per_volume()
    same = bool(torch.equal(gb, gp)) or bool(torch.allclose(gb, gp, rtol=1e-6, atol=1e-6))
    torch.cuda.synchronize()

    def timed(fn):
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    b_s = timed(batched)
    print(f"fwd_bwd: batched {b_s * 1e3:.1f} ms", file=sys.stderr, flush=True)
    p_s = timed(per_volume)
    print(f"fwd_bwd: per-volume loop {p_s * 1e3:.1f} ms", file=sys.stderr, flush=True)
    return {"workload": "32 x 128^3 float32 sigma-3 Gaussian fields (seed 4); loss = sum over finite H1/H2 "
                        "bars with lifetime > 0.1 of lifetime^2; forward + backward",
            "volumes": len(vols), "active_bars": nact, "batched_ms": b_s * 1e3, "per_volume_loop_ms": p_s * 1e3,
            "batched_vs_loop": p_s / b_s, "gradients_agree": same and nact == nact_p}


def bench_next(x, d, reps: int = 3) -> dict:
    """The widened inputs and outputs: a masked volume (+inf outside the
    inscribed ball), a long 1D signal, and the lifetime image of the 256^3
    diagram."""
    import torch
    import paper_2005_12692_amd as cr
    import synth
    n = x.shape[0]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    mask = torch.from_numpy(synth.ball_mask((n, n, n))).cuda()
    xm = torch.where(mask, x, torch.full_like(x, float("inf")))
    m_s = timed(lambda: cr.persistence(xm, maxdim=2))
    m_rows = int(cr.persistence(xm, maxdim=2).dim.shape[0])
    print(f"next: masked volume {m_s * 1e3:.1f} ms", file=sys.stderr, flush=True)
    ns = 1 << 24
    sig = torch.from_numpy(synth.random_walk(ns)).cuda()
    s_s = timed(lambda: cr.persistence(sig))
    s_rows = int(cr.persistence(sig).dim.shape[0])
    print(f"next: 1D signal {s_s * 1e3:.1f} ms", file=sys.stderr, flush=True)
    npix = x.numel()
    rows = int(d.dim.shape[0])
    l_s = timed(lambda: cr.lifetime_image(d, npix, "birth"))
    # per call: read dim, birth, death (4 B each) and the location (8 B) of
    # every row, one 4 B max per row, and clear 3 channels of 4 B per pixel
    lbytes = rows * (4 + 4 + 4 + 8 + 4) + 3 * 4 * npix
    l_ach = lbytes / l_s / 1e9
    print(f"next: lifetime image {l_s * 1e3:.2f} ms", file=sys.stderr, flush=True)
    cells = (2 * n - 1) ** 3
    return {"masked_volume": {"workload": "the same 256^3 volume, +inf outside the inscribed ball; H0+H1+H2",
                              "ms": m_s * 1e3, "cells_per_s": cells / m_s, "rows": m_rows},
            "signal_1d": {"workload": "random walk of 2^24 N(0,1) steps (seed 7); H0",
                          "ms": s_s * 1e3, "samples_per_s": ns / s_s, "rows": s_rows},
            "lifetime_image": {"workload": "3 channels of the 256^3 diagram, birth locations",
                               "ms": l_s * 1e3, "rows": rows, "algorithmic_bytes": lbytes,
                               "achieved_GBs": l_ach, "peak_GBs": HBM_PEAK_GBS, "frac": l_ach / HBM_PEAK_GBS,
                               "note": "whole entry point: clear, scatter and the one synchronising "
                                       "read-back of the argument-check flag"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched, fwd+bwd, masked, 1D and lifetime-image measurements")
    ap.add_argument("--copy-only", action="store_true",
                    help="only time a 256 MiB device copy (the reference kernel for profiler byte counts)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; --gpus must be 1 (sharding over several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_only:
        print(json.dumps({"copy_GBs": copy_ceiling(), "bytes_per_copy": 2 * (1 << 28)}), flush=True)
        return

    import paper_2005_12692_amd as cr
    import synth

    n = 256
    vol = synth.blobs3d(n, 2)
    x = torch.from_numpy(vol).cuda()
    cells = (2 * n - 1) ** 3
    for i in range(args.warmup):
        t = time.perf_counter()
        d = cr.persistence(x, maxdim=2, stage_times=True)
        print(f"warmup {i}: {1e3 * (time.perf_counter() - t):.1f} ms {cr.stage_times()}", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    stage_sum = {k: 0.0 for k in cr.STAGES}
    t0 = time.perf_counter()
    for i in range(args.steps):
        d = cr.persistence(x, maxdim=2, stage_times=True)
        for k, v in cr.stage_times().items():
            stage_sum[k] += v
        print(f"step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / args.steps
    stages = {k: v / args.steps for k, v in stage_sum.items()}
    st = cr.stats()
    surv = int(sum(st["survivors"]))
    nbytes = stencil_bytes((n, n, n), surv)
    achieved = nbytes / (stages["stencil"] * 1e-3) / 1e9
    sort_bits = 2 + 32 + (((2 * n - 1) ** 3) - 1).bit_length()
    sbytes = sort_bytes(surv, sort_bits)
    s_achieved = sbytes / (stages["sort_cells"] * 1e-3) / 1e9
    rows = int(d.dim.shape[0])
    # the same stages with the last-level cache flushed before each call (the
    # 64 MiB input would otherwise stay in the 256 MB Infinity Cache), outside
    # the timed steps: three calls, median stage times
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
    cold = {k: [] for k in cr.STAGES}
    for _ in range(3):
        flush.fill_(1.0)
        torch.cuda.synchronize()
        cr.persistence(x, maxdim=2, stage_times=True)
        for k, v in cr.stage_times().items():
            cold[k].append(v)
    del flush
    cold = {k: float(np.median(v)) for k, v in cold.items()}
    c_achieved = nbytes / (cold["stencil"] * 1e-3) / 1e9
    cs_achieved = sbytes / (cold["sort_cells"] * 1e-3) / 1e9
    line = {
        "metric": "PH cells/s (3D 256^3, degrees 0-2)",
        "value": cells / (ms * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3D 256^3 float32: 200 Gaussian blobs + U[-0.05,0.05) noise, seed 2; "
                               "H0+H1+H2, plain per-volume call",
                   "cells": cells, "pixels": n ** 3},
        "roofline": {"bound": "hbm", "kernel": "k_stencil (filtration + apparent pairs + compaction)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": profiled_traffic("k_stencil_256cube_traffic.md"),
                     "algorithmic_bytes": nbytes, "ms": stages["stencil"],
                     "issue": issue_rate("k_stencil_256cube_traffic.md", stages["stencil"]),
                     "cold": {"ms": cold["stencil"], "achieved": c_achieved, "frac": c_achieved / HBM_PEAK_GBS}},
        "roofline_sort": {"bound": "hbm", "kernel": "cell sort, %d 8-bit passes (count + scan + scatter)"
                          % ((sort_bits + 7) // 8), "achieved": s_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": s_achieved / HBM_PEAK_GBS, "traffic": profiled_traffic("k_sort_256cube_traffic.md"),
                          "algorithmic_bytes": sbytes,
                          "ms": stages["sort_cells"],
                          "cold": {"ms": cold["sort_cells"], "achieved": cs_achieved,
                                   "frac": cs_achieved / HBM_PEAK_GBS}},
        "latency_bound": {"stage": "degree 1 (boundary reduction)", "ms": stages["degree1"],
                          "share": stages["degree1"] / ms,
                          "note": "dependent-load chains of the long columns; no bandwidth roofline applies"},
        "stages_ms": stages,
        "survivors": st["survivors"],
        "rows": rows,
        "rows_per_dim": np.bincount(d.dim.cpu().numpy(), minlength=3).tolist(),
        "reduction": {"arena_entries_used": st["arena_used"], "additions": st["red_adds"],
                      "entries_merged": st["red_merged"],
                      "rounds": st["red_rounds"]},
    }
    line["copy_ceiling_GBs"] = copy_ceiling()
    if not args.no_forms:
        line["batched"] = bench_batched()
        line["fwd_bwd"] = bench_fwd_bwd()
        line["next"] = bench_next(x, d)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(vol)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
