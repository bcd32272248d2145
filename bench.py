#!/usr/bin/env python3
"""Throughput of the per-cell chemistry hot path on one MI355X.

A step is one pass of the whole path over the field: reference mapping
(Sec. 2.3 criterion), heavy-first work-queue construction from the previous
step's per-cell cost, persistent-kernel Rodas4 integration of every unmapped
cell, and the enthalpy-consistent update of mapped cells.  Consecutive steps
advance the same field, as consecutive flow time steps would.

Prints one JSON line: cells*dt/s of that path, the plain static-launch
integration of the same field for comparison, the integration kernel's
roofline position, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cells·dt/s (53-sp mech): plain vs balanced+surrogate at stated max err"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_state(field, torch):
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to("cuda").contiguous()
    n = field.n_cells
    return dict(T=dev(field.T), p=dev(field.p), Y=dev(field.Y),
                h=torch.zeros(n, dtype=torch.float64, device="cuda"),
                cost=torch.zeros(n, dtype=torch.int32, device="cuda"),
                status=torch.zeros(n, dtype=torch.uint8, device="cuda"),
                flags=torch.zeros(n, dtype=torch.uint8, device="cuda"),
                ref=torch.zeros(1, dtype=torch.int64, device="cuda"))


def run_mode(chem, mech, field, mode, steps, warmup, torch, synth):
    """Returns (ms_per_step, per-step stats of the timed steps)."""
    from paper_2011_07978_amd.chem import CHEM_SCHED_PLAIN, CHEM_SCHED_QUEUE
    S = make_state(field, torch)
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    if mode == "plain":
        chem.set_options(schedule=CHEM_SCHED_PLAIN)
    else:
        chem.set_options(schedule=CHEM_SCHED_QUEUE)

    def one_step():
        if mode == "plain":
            return chem.integrate(S["T"], S["p"], S["Y"], field.dt, h=S["h"], cost=S["cost"],
                                  status=S["status"], stats=True)
        chem.map_reference(S["T"], S["p"], S["Y"], Yf, Yo, 1e-4, 1.0, False,
                           flags=S["flags"], ref_index=S["ref"])
        return chem.integrate(S["T"], S["p"], S["Y"], field.dt, flags=S["flags"],
                              ref_index=S["ref"], h=S["h"], cost=S["cost"], status=S["status"],
                              stats=True)

    for w in range(warmup):
        st = one_step()
        log(f"{mode} warmup {w + 1}/{warmup}: {st['ms_total']:.1f} ms, "
            f"steps {st['steps_accepted']}+{st['steps_rejected']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(steps):
        st = one_step()
        stats.append(st)
        log(f"{mode} step {k + 1}/{steps}: {st['ms_total']:.1f} ms (integrate kernel "
            f"{st['ms_integrate']:.1f} ms), mapped {st['cells_mapped']}, failed {st['cells_failed']}")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return ms, stats


def cpu_baseline(mech, field, synth, warmup, steps, budget_s=20.0, threads=None):
    """The oracle, as it stands, on uniformly drawn cells of the same field and
    the same path (mapping on the full field, integration of unmapped cells,
    step sizes carried from step to step).  It advances its own sample through
    the same warm-up steps (untimed; their cost bounds the sample size), then
    times the same number of steps.  Cells are independent, so cells per second
    on a uniform sample estimate the full field's rate."""
    from oracle import Oracle
    o = Oracle(mech)
    threads = threads or min(16, os.cpu_count() or 1)
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    flags_all, ref = o.map_reference(field.T, field.Y, Yf, Yo, 1e-4)
    order = np.random.default_rng(12345).permutation(field.n_cells)
    # warm-up in batches until the budget is used: those cells are the sample
    Ts, Ys, hs, idxs = [], [], [], []
    spent, pos, batch = 0.0, 0, 512
    while spent < budget_s and pos < field.n_cells:
        idx = order[pos:pos + batch]
        pos += batch
        sub = synth.subsample(field, idx)
        fl = flags_all[idx].copy()
        T, Y, h = sub.T, sub.Y, np.zeros(idx.size)
        t1 = time.perf_counter()
        for _ in range(warmup):
            T, Y, h = o.integrate_batch(T, sub.p, Y, sub.dt, h=h, flags=fl, threads=threads,
                                        schedule=1)[:3]
        spent += time.perf_counter() - t1
        Ts.append(T); Ys.append(Y); hs.append(h); idxs.append(idx)
    idx = np.concatenate(idxs)
    T, Y, h = np.concatenate(Ts), np.concatenate(Ys, axis=1), np.concatenate(hs)
    p = field.p[idx]
    fl = flags_all[idx].copy()
    t1 = time.perf_counter()
    for _ in range(steps):
        T, Y, h = o.integrate_batch(T, p, Y, field.dt, h=h, flags=fl, threads=threads,
                                    schedule=1)[:3]
    elapsed = time.perf_counter() - t1
    return dict(value=idx.size * steps / elapsed, unit="cells·dt/s", cores=threads, kind="oracle",
                sample=f"{idx.size} uniformly drawn cells of the {field.n_cells}-cell field; "
                       f"{warmup} untimed warm-up step(s) ({spent:.1f} s) then {steps} timed "
                       f"step(s) ({elapsed:.1f} s), mapped cells skipped as on the GPU path, "
                       f"{threads} OpenMP threads, schedule(dynamic,16)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="surrogate", choices=["small", "flame", "mapped", "large",
                                                             "surrogate"])
    ap.add_argument("--cells", type=int, default=0, help="override the field size")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="CPU budget of the oracle warm-up (sizes the sample)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures the path on one GPU only (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE {world}); multi-GPU sharding is a design note, not a measured path.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2011_07978_amd import accounting, synth
    from paper_2011_07978_amd.chem import Chem

    wl = synth.WORKLOADS[args.workload]
    mech = synth.mechanism(wl["mech"])
    field = wl["field"](args.cells) if args.cells else wl["field"]()
    log(f"workload {args.workload}: {field.n_cells} cells, {mech.n_species} species, "
        f"{mech.n_reactions} reactions, dt {field.dt}")
    chem = Chem(0)
    chem.set_mechanism(mech)
    chem.reserve(field.n_cells)

    ms_bal, st_bal = run_mode(chem, mech, field, "balanced", args.steps, args.warmup, torch, synth)
    value = field.n_cells / (ms_bal / 1e3)
    plain = None
    if not args.no_plain:
        ms_pl, st_pl = run_mode(chem, mech, field, "plain", args.steps, args.warmup, torch, synth)
        plain = dict(value=field.n_cells / (ms_pl / 1e3), ms_per_step=ms_pl,
                     integrate_ms=float(np.mean([s["ms_integrate"] for s in st_pl])))

    # roofline of the dominant kernel (the integration kernel), per launch
    sc = accounting.step_cost(mech)
    fl = [sc.flops(s["steps_accepted"], s["steps_rejected"]) for s in st_bal]
    kms = [s["ms_integrate"] for s in st_bal]
    achieved = float(np.mean([f / (m * 1e-3) / 1e12 for f, m in zip(fl, kms)]))
    roof = dict(bound="alu", achieved=achieved, peak=accounting.FP64_VECTOR_PEAK_TFLOPS,
                unit="TFLOP/s", frac=achieved / accounting.FP64_VECTOR_PEAK_TFLOPS, traffic=None,
                kernel="k_integrate_queue", kernel_ms=float(np.mean(kms)),
                flops_per_launch=float(np.mean(fl)),
                steps_per_launch=float(np.mean([s["steps_accepted"] + s["steps_rejected"]
                                                for s in st_bal])),
                transcendentals_per_launch=float(np.mean(
                    [sc.transcendentals(s["steps_accepted"], s["steps_rejected"]) for s in st_bal])))

    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(mech, field, synth, args.warmup, args.steps, budget_s=args.cpu_seconds)

    out = {
        "metric": METRIC, "value": value, "unit": "cells·dt/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_bal,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {field.n_cells} cells, {mech.n_species} species / "
                               f"{mech.n_reactions} reactions, dt {field.dt} s, rtol 1e-8, atol 1e-12, "
                               "map (Z_tol 1e-4) + heavy-first queue + Rodas4 + mapped update",
                   "cells": field.n_cells, "species": mech.n_species,
                   "reactions": mech.n_reactions, "dt": field.dt, "parallelism": "single GPU"},
        "plain": plain,
        "speedup_vs_plain": (value / plain["value"]) if plain else None,
        "mapped_cells_per_step": float(np.mean([s["cells_mapped"] for s in st_bal])),
        "failed_cells": int(sum(s["cells_failed"] for s in st_bal)),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
