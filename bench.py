#!/usr/bin/env python3
"""Throughput of the per-cell chemistry hot path on one MI355X.

A step is one pass of the whole path over the field: reference mapping
(Sec. 2.3 criterion), the learned surrogate with its conservation step and
gate on the cells mapping leaves (headline mode), heavy-first work-queue
construction from the previous step's per-cell cost, persistent-kernel Rodas4
integration of every remaining cell, and the enthalpy-consistent update of
mapped cells.  Consecutive steps advance the same field, as consecutive flow
time steps would.

Prints one JSON line: cells*dt/s of that path, the plain static-launch
integration and the balanced path without the surrogate on the same field for
comparison, the surrogate's error against the CPU oracle, the integration
kernel's roofline position, and the CPU oracle timed on a bounded sample.
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
# HBM bytes per attempted Rodas4 step of k_integrate_queue<54> (FETCH_SIZE x 2
# + WRITE_SIZE, the factors from a 1 GiB copy), from the counter passes over
# the headline workload in profiles/k_integrate_queue_54__counters_surrogate_field_1M.md
# (None: not measured for the current kernel).  Beyond the cell's own state it
# is register spill traffic that leaves the caches, proportional to attempted
# steps.
TRAFFIC_BYTES_PER_ATTEMPT = 128.36


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


def run_mode(chem, mech, field, mode, steps, warmup, torch, synth, record_idx=None, gate=None,
             after_warmup=None, snapshot=False):
    """Returns (ms_per_step, per-step stats of the timed steps, record, state).
    record: host copies of T, Y and flags of record_idx after the first step
    (taken in the untimed warm-up).  after_warmup(S) runs between the warm-up
    and the timed steps (launch tuning); with snapshot, S["snapshot"] holds a
    copy of the state the timed steps start from."""
    from paper_2011_07978_amd.chem import CHEM_SCHED_PLAIN, CHEM_SCHED_QUEUE
    S = make_state(field, torch)
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    chem.set_options(schedule=CHEM_SCHED_PLAIN if mode == "plain" else CHEM_SCHED_QUEUE)

    def one_step(S):
        if mode == "plain":
            return chem.integrate(S["T"], S["p"], S["Y"], field.dt, h=S["h"], cost=S["cost"],
                                  status=S["status"], stats=True)
        chem.map_reference(S["T"], S["p"], S["Y"], Yf, Yo, 1e-4, 1.0, False,
                           flags=S["flags"], ref_index=S["ref"])
        if mode == "surrogate":
            return chem.integrate_surrogate(S["T"], S["p"], S["Y"], field.dt, S["flags"], S["ref"],
                                            gate=gate, h=S["h"], cost=S["cost"],
                                            status=S["status"], stats=True)
        return chem.integrate(S["T"], S["p"], S["Y"], field.dt, flags=S["flags"],
                              ref_index=S["ref"], h=S["h"], cost=S["cost"], status=S["status"],
                              stats=True)

    record = None
    S["warmup_ms"] = []
    for w in range(warmup):
        st = one_step(S)
        S["warmup_ms"].append(st["ms_total"])
        log(f"{mode} warmup {w + 1}/{warmup}: {st['ms_total']:.1f} ms, "
            f"steps {st['steps_accepted']}+{st['steps_rejected']}, surrogate {st['cells_surrogate']}")
        if w == 0 and record_idx is not None:
            ix = torch.as_tensor(record_idx, device="cuda")
            record = dict(T=S["T"][ix].cpu().numpy(), Y=S["Y"][:, ix].cpu().numpy(),
                          flags=S["flags"][ix].cpu().numpy())
    torch.cuda.synchronize()
    if after_warmup is not None:
        after_warmup(S)
    if snapshot:
        S["snapshot"] = {k: v.clone() for k, v in S.items() if torch.is_tensor(v)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(steps):
        st = one_step(S)
        stats.append(st)
        log(f"{mode} step {k + 1}/{steps}: {st['ms_total']:.1f} ms (integrate kernel "
            f"{st['ms_integrate']:.1f} ms, surrogate {st['ms_surrogate']:.2f} ms), mapped "
            f"{st['cells_mapped']}, surrogate {st['cells_surrogate']}, failed {st['cells_failed']}")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    S["one_step"] = one_step
    return ms, stats, record, S


def graph_replay(chem, mech, field, mode, snapshot, steps, torch, synth, gate=None):
    """The timed steps of `mode` recorded into one HIP graph (chem_graph_*) and
    replayed once from the state they started from: the same kernels without
    per-step host launches.  A context of its own on a created stream, with
    the tuned launch shape and the surrogate's parameters; its workspaces are
    warmed by one eager step on a scratch copy.  Returns ms per step."""
    from paper_2011_07978_amd.chem import CHEM_SCHED_QUEUE, Chem
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = Chem(0, stream=stream)
        g.set_mechanism(mech)
        o = chem.options()
        g.set_options(schedule=CHEM_SCHED_QUEUE, queue_chunk=o.queue_chunk, slots_per_cu=o.slots_per_cu)
        g.reserve(field.n_cells)
        if mode == "surrogate":
            g.surrogate_set_params(chem.surrogate_get_params())
        Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)

        def step(S):
            g.map_reference(S["T"], S["p"], S["Y"], Yf, Yo, 1e-4, 1.0, False, flags=S["flags"],
                            ref_index=S["ref"])
            if mode == "surrogate":
                g.integrate_surrogate(S["T"], S["p"], S["Y"], field.dt, S["flags"], S["ref"], gate=gate,
                                      h=S["h"], cost=S["cost"], status=S["status"])
            else:
                g.integrate(S["T"], S["p"], S["Y"], field.dt, flags=S["flags"], ref_index=S["ref"],
                            h=S["h"], cost=S["cost"], status=S["status"])
        scratch = {k: v.clone() for k, v in snapshot.items()}
        step(scratch)                      # warm every workspace eagerly
        stream.synchronize()
        del scratch
        G = {k: v.clone() for k, v in snapshot.items()}
        stream.synchronize()
        g.graph_begin()
        for _ in range(steps):
            step(G)
        graph = g.graph_end()
        stream.synchronize()
        t0 = time.perf_counter()
        graph.launch()
        stream.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        graph.close()
        del G
    log(f"graph replay of {steps} {mode} steps: {ms:.1f} ms per step")
    return ms


def train_surrogate(chem, mech, args, torch, accounting):
    """Solver-generated pairs and training (untimed, reported separately)."""
    from paper_2011_07978_amd import surrogate
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pairs = surrogate.generate_pairs(chem, n_cells=args.sur_cells, n_steps=args.sur_steps, seed=900,
                                     log=lambda m: log(m))
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    tr, va = surrogate.split(pairs)
    t0 = time.perf_counter()
    hist = surrogate.train(chem, tr, epochs=args.sur_epochs, batch=4096, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"surrogate: {pairs.n} pairs in {t_pairs:.1f} s, {args.sur_epochs} epochs in {t_train:.1f} s, "
        f"loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    val = surrogate.validate(chem, va, gate=dict(tau_T=args.tau_T, margin=args.margin,
                                                 max_dT=args.max_dT, T_max=args.T_max))
    fl = accounting.surrogate_train_flops_per_sample(mech.n_species) * tr.n * args.sur_epochs
    return dict(pairs=pairs.n, train_pairs=tr.n, validation_pairs=va.n, epochs=args.sur_epochs,
                seconds_pairs=t_pairs, seconds_train=t_train,
                train_samples_per_s=tr.n * args.sur_epochs / t_train,
                train_bf16_tflops=fl / t_train / 1e12, loss_history=[float(x) for x in hist],
                validation={k: v for k, v in val.items() if k != "stats"})


def first_step_error(mech, field, synth, rec, idx, threads):
    """The oracle's first step (mapping on the full field, exact integration of
    the unmapped sample cells and of the reference cell, mapped update) against
    the GPU path's first step on a stratified sample."""
    from oracle import Oracle
    o = Oracle(mech)
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    flags_full, ref = o.map_reference(field.T, field.Y, Yf, Yo, 1e-4)
    cells = list(idx)
    ref_pos = -1
    if ref >= 0:
        if ref in cells:
            ref_pos = cells.index(ref)
        else:
            cells.append(ref)
            ref_pos = len(cells) - 1
    sub = synth.subsample(field, np.asarray(cells))
    t0 = time.perf_counter()
    To, Yo_ = o.step_mapped(sub.T, sub.p, sub.Y, field.dt, flags_full[cells], ref_pos,
                            threads=threads, schedule=1)[:2]
    secs = time.perf_counter() - t0
    m = len(idx)
    dT = np.abs(rec["T"] - To[:m])
    dY = np.abs(rec["Y"] - Yo_[:, :m]).max(axis=0)
    acc = rec["flags"] == 3
    cls = field.cls[idx]
    out = dict(sample=f"{m} cells, stratified by class ({', '.join(field.class_names)}), seed 7; "
                      f"oracle {secs:.1f} s on {threads} threads",
               mean_abs_dT=float(dT.mean()), max_abs_dT=float(dT.max()), max_abs_dY=float(dY.max()),
               by_class={})
    weights = np.bincount(field.cls, minlength=len(field.class_names)) / field.n_cells
    whole = 0.0
    for c, name in enumerate(field.class_names):
        sel = cls == c
        if not sel.any():
            continue
        a = sel & acc
        out["by_class"][name] = dict(cells=int(sel.sum()), surrogate=int(a.sum()),
                                     mean_abs_dT=float(dT[sel].mean()),
                                     max_abs_dT=float(dT[sel].max()),
                                     max_abs_dY=float(dY[sel].max()),
                                     mean_abs_dT_surrogate=float(dT[a].mean()) if a.any() else None)
        whole += weights[c] * float(dT[sel].mean())
    out["field_mean_abs_dT_by_class_weights"] = whole
    a = acc
    out["surrogate_cells_mean_abs_dT"] = float(dT[a].mean()) if a.any() else None
    out["surrogate_cells_max_abs_dT"] = float(dT[a].max()) if a.any() else None
    return out


def trajectory_drift(field, S_sur, S_fp64, n_steps):
    """The two paths advanced the same field for the same steps: the state
    difference accumulates every surrogate step's error."""
    dT = (S_sur["T"] - S_fp64["T"]).abs().cpu().numpy()
    out = dict(flow_steps=n_steps, mean_abs_dT=float(dT.mean()), max_abs_dT=float(dT.max()),
               by_class={})
    for c, name in enumerate(field.class_names):
        sel = field.cls == c
        if sel.any():
            out["by_class"][name] = dict(mean_abs_dT=float(dT[sel].mean()),
                                         max_abs_dT=float(dT[sel].max()))
    return out


def steady_state_error(chem, S, torch, surrogate_step, balanced_step):
    """From the current steady state: one step with the surrogate against the
    same step by the FP64 path (mapping + Rosenbrock), on surrogate cells."""
    A = {k: (v.clone() if torch.is_tensor(v) else v) for k, v in S.items()}
    B = {k: (v.clone() if torch.is_tensor(v) else v) for k, v in S.items()}
    surrogate_step(A)
    balanced_step(B)
    torch.cuda.synchronize()
    acc = A["flags"] == 3
    n_acc = int(acc.sum())
    if n_acc == 0:
        return dict(surrogate_cells=0)
    dT = (A["T"] - B["T"]).abs()[acc]
    dY = (A["Y"] - B["Y"]).abs()[:, acc].amax(dim=0)
    return dict(surrogate_cells=n_acc, mean_abs_dT=float(dT.mean()), max_abs_dT=float(dT.max()),
                p99_abs_dT=float(torch.quantile(dT[:1 << 20].float(), 0.99)),
                max_abs_dY=float(dY.max()))


def host_cores():
    """CPU threads this process may use, capped at 16 (the CPU share of one
    GPU on the benchmark hosts)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(mech, field, synth, warmup, steps, budget_s=20.0, threads=None):
    """The oracle, as it stands, on uniformly drawn cells of the same field and
    the same path (mapping on the full field, integration of unmapped cells,
    step sizes carried from step to step).  It advances its own sample through
    the same warm-up steps (untimed; their cost bounds the sample size), then
    times the same number of steps three ways: all threads with
    schedule(dynamic, 16) (the CPU analogue of a balanced run), all threads
    with schedule(static) (unbalanced), and one thread on every threads-th
    cell of the sample.  Cells are independent, so cells per second on a
    uniform sample estimate the full field's rate."""
    from oracle import Oracle
    o = Oracle(mech)
    threads = threads or host_cores()
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
    T0, Y0, h0 = np.concatenate(Ts), np.concatenate(Ys, axis=1), np.concatenate(hs)
    p = field.p[idx]
    fl0 = flags_all[idx].copy()

    def timed(sel, nthreads, schedule):
        T, Y, h = T0[sel], Y0[:, sel], h0[sel]
        t1 = time.perf_counter()
        for _ in range(steps):
            T, Y, h = o.integrate_batch(T, p[sel], Y, field.dt, h=h, flags=fl0[sel], threads=nthreads,
                                        schedule=schedule)[:3]
        el = time.perf_counter() - t1
        return sel.size * steps / el, el

    everything = np.arange(idx.size)
    dyn, t_dyn = timed(everything, threads, 1)
    sta, t_sta = timed(everything, threads, 0)
    one_sel = everything[::threads]
    one, t_one = timed(one_sel, 1, 0)
    return dict(value=dyn, unit="cells·dt/s", cores=threads, kind="oracle",
                sample=f"{idx.size} uniformly drawn cells of the {field.n_cells}-cell field; "
                       f"{warmup} untimed warm-up step(s) ({spent:.1f} s) then {steps} timed "
                       f"step(s), mapped cells skipped as on the GPU path; value: {threads} OpenMP "
                       f"threads, schedule(dynamic,16) ({t_dyn:.1f} s)",
                static=dict(value=sta, cores=threads, schedule="static", seconds=t_sta),
                one_core=dict(value=one, cores=1, cells=int(one_sel.size), seconds=t_one),
                static_over_dynamic=sta / dyn)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="surrogate",
                    choices=["small", "flame", "flame_shuffled", "flame_hot_last", "flame_falloff",
                             "flame_plog", "mapped", "large", "surrogate", "unit", "mapping-study"],
                    help="unit: the load-balancing benchmark of Sec. 3 (layouts C1-C4); "
                         "mapping-study: mapped vs unmapped error over Z_tol and the T criterion")
    ap.add_argument("--unit-problems", type=int, default=100,
                    help="unit benchmark: problems (cells) per slot")
    ap.add_argument("--unit-reps", type=int, default=3)
    ap.add_argument("--study-steps", type=int, default=10, help="mapping study: flow steps")
    ap.add_argument("--cells", type=int, default=0, help="override the field size")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-error", action="store_true", help="skip the oracle error sample")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="CPU budget of the oracle warm-up (sizes the sample)")
    ap.add_argument("--error-per-class", type=int, default=512)
    ap.add_argument("--sur-cells", type=int, default=262144, help="cells of the pair field")
    ap.add_argument("--sur-steps", type=int, default=8, help="flow steps of the pair field")
    ap.add_argument("--sur-epochs", type=int, default=8)
    ap.add_argument("--tau-T", type=float, default=0.5)
    ap.add_argument("--margin", type=float, default=0.01, help="gate: training-box margin")
    ap.add_argument("--max-dT", type=float, default=1.0, help="gate: largest predicted |dT| (K)")
    ap.add_argument("--T-max", type=float, default=1000.0, help="gate: hottest cell offered (K)")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip replaying the timed steps from one recorded HIP graph")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip choosing queue chunk and slots per CU on the warmed-up state")
    ap.add_argument("--headline-only", action="store_true",
                    help="time the headline path alone (no comparison legs, oracle error or CPU "
                         "baseline; for profiler runs)")
    ap.add_argument("--surrogate-save", default="", help="write the trained surrogate parameters")
    ap.add_argument("--surrogate-load", default="",
                    help="load surrogate parameters instead of generating pairs and training")
    args = ap.parse_args()
    if args.headline_only:
        args.no_plain = args.no_cpu = args.no_error = args.no_graph = args.no_autotune = True
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures the path on one GPU only (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE {world}); multi-GPU sharding is a design note, not a measured path.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2011_07978_amd import accounting, synth
    from paper_2011_07978_amd.chem import Chem

    if args.workload in ("unit", "mapping-study"):
        from paper_2011_07978_amd import studies
        mech = synth.mechanism("mech53")
        chem = Chem(0)
        chem.set_mechanism(mech)
        t0 = time.perf_counter()
        if args.workload == "unit":
            res = studies.unit_benchmark(chem, torch, synth, mech, n_per_slot=args.unit_problems,
                                         reps=args.unit_reps, log=log)
            line = {"metric": "chi_su = tau_unbalanced / tau_balanced (Sec. 3 unit benchmark)",
                    "value": res["layouts"]["C1"]["chi_su"], "unit": "ratio",
                    "higher_is_better": True, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
                    "config": {"workload": f"unit benchmark: {res['slots']} slots x "
                                           f"{args.unit_problems} problems, heavy/light "
                                           "pseudo-problems, 53 species / 325 reactions",
                               "parallelism": "single GPU"},
                    "unit_benchmark": res}
        else:
            res = studies.mapping_study(chem, torch, synth, mech,
                                        n_cells=args.cells or 262144, steps=args.study_steps, log=log)
            best = [r for r in res["runs"] if r["Z_tol"] == 1e-4 and not r["use_T"]][0]
            line = {"metric": "mean |dT| of the mapped path vs unmapped (Z_tol 1e-4)",
                    "value": best["mean_abs_dT"], "unit": "K", "higher_is_better": False,
                    "n_gpus": 1, "dtype": "f64", "data": "synthetic",
                    "config": {"workload": f"mapping study: {res['cells']} cells, {res['steps']} "
                                           "flow steps, 53 species / 325 reactions",
                               "parallelism": "single GPU"},
                    "mapping_study": res}
        line["wall_s"] = time.perf_counter() - t0
        print(json.dumps(line), flush=True)
        return

    wl = synth.WORKLOADS[args.workload]
    mech = synth.mechanism(wl["mech"])
    field = wl["field"](args.cells) if args.cells else wl["field"]()
    use_sur = args.workload == "surrogate"
    log(f"workload {args.workload}: {field.n_cells} cells, {mech.n_species} species, "
        f"{mech.n_reactions} reactions, dt {field.dt}")
    chem = Chem(0)
    chem.set_mechanism(mech)
    threads = host_cores()

    sur = None
    gate = dict(tau_T=args.tau_T, y_min=-1e-10, margin=args.margin, max_dT=args.max_dT,
                T_max=args.T_max)
    if use_sur:
        if args.surrogate_load:
            chem.surrogate_load(args.surrogate_load)
            sur = dict(loaded=os.path.basename(args.surrogate_load))
            log(f"surrogate parameters loaded from {args.surrogate_load}")
        else:
            sur = train_surrogate(chem, mech, args, torch, accounting)
        if args.surrogate_save:
            chem.surrogate_save(args.surrogate_save)
    chem.reserve(field.n_cells)
    tune = None

    def autotune(S):
        """Launch shape of the queue from the warmed-up state (the timed steps'
        own starting point): chem_autotune times every configuration on copies
        of it; the fastest queue configuration is kept for every queue leg."""
        nonlocal tune
        res = chem.autotune(S["T"], S["p"], S["Y"], field.dt, flags=S["flags"], ref_index=S["ref"])
        q = min((r for r in res if r[0] == 1), key=lambda r: r[3])
        from paper_2011_07978_amd.chem import CHEM_SCHED_QUEUE
        chem.set_options(schedule=CHEM_SCHED_QUEUE, queue_chunk=q[1], slots_per_cu=q[2])
        tune = dict(chosen=dict(queue_chunk=q[1], slots_per_cu=q[2], ms=q[3]),
                    measured=[dict(schedule="plain" if r[0] == 0 else "queue", queue_chunk=r[1],
                                   slots_per_cu=r[2], ms=r[3]) for r in res])
        log(f"autotune: {res} -> chunk {q[1]} slots {q[2]}")

    rec_idx = None
    if use_sur and not args.no_error and args.warmup >= 1:
        rec_idx = synth.stratified_indices(field, args.error_per_class, seed=7)

    head_mode = "surrogate" if use_sur else "balanced"
    ms_h, st_h, rec, S_h = run_mode(chem, mech, field, head_mode, args.steps, args.warmup, torch,
                                    synth, record_idx=rec_idx, gate=gate,
                                    after_warmup=None if args.no_autotune else autotune,
                                    snapshot=not args.no_graph)
    value = field.n_cells / (ms_h / 1e3)
    graph = None
    if not args.no_graph:
        ms_g = graph_replay(chem, mech, field, head_mode, S_h["snapshot"], args.steps, torch, synth,
                            gate=gate)
        graph = dict(ms_per_step=ms_g, value=field.n_cells / (ms_g / 1e3),
                     note=f"the {args.steps} timed {head_mode} steps recorded into one HIP graph and "
                          "replayed once from the same starting state, same launch shape")
        del S_h["snapshot"]
    balanced = None
    if use_sur and not args.headline_only:
        ms_b, st_b, _, S_b = run_mode(chem, mech, field, "balanced", args.steps, args.warmup, torch,
                                      synth)
        balanced = dict(value=field.n_cells / (ms_b / 1e3), ms_per_step=ms_b,
                        integrate_ms=float(np.mean([s["ms_integrate"] for s in st_b])))
        sur["drift_vs_fp64_path"] = trajectory_drift(field, S_h, S_b, args.warmup + args.steps)
        sur["steady_state_vs_fp64_path"] = steady_state_error(chem, S_h, torch, S_h["one_step"],
                                                              S_b["one_step"])
        del S_b
    plain = None
    if not args.no_plain:
        ms_pl, st_pl, _, S_p = run_mode(chem, mech, field, "plain", args.steps, args.warmup, torch,
                                        synth)
        plain = dict(value=field.n_cells / (ms_pl / 1e3), ms_per_step=ms_pl,
                     integrate_ms=float(np.mean([s["ms_integrate"] for s in st_pl])))
        del S_p


    # roofline of the dominant kernel (the integration kernel), per launch
    sc = accounting.step_cost(mech)
    fl = [sc.flops(s["steps_accepted"], s["steps_rejected"]) for s in st_h]
    kms = [s["ms_integrate"] for s in st_h]
    achieved = float(np.mean([f / (m * 1e-3) / 1e12 for f, m in zip(fl, kms)]))
    kname = "k_big_queue" if mech.n_species + 1 > 64 else "k_integrate_queue"
    # HBM bytes per launch of the wavefront kernel, from the rocprofv3
    # FETCH_SIZE / WRITE_SIZE passes over the headline workload (scaled by the
    # same counters over a copy kernel of known size), per attempted step
    traffic = None
    plain_kinetics = getattr(mech, "falloff", None) is None and getattr(mech, "plog_count", None) is None
    if (kname == "k_integrate_queue" and mech.n_species == 53 and plain_kinetics
            and TRAFFIC_BYTES_PER_ATTEMPT is not None):
        traffic = TRAFFIC_BYTES_PER_ATTEMPT * float(np.mean([s["steps_accepted"] + s["steps_rejected"]
                                                             for s in st_h]))
    roof = dict(bound="alu", achieved=achieved, peak=accounting.FP64_VECTOR_PEAK_TFLOPS,
                unit="TFLOP/s", frac=achieved / accounting.FP64_VECTOR_PEAK_TFLOPS, traffic=traffic,
                traffic_unit="bytes per launch" if traffic else None,
                kernel=kname, kernel_ms=float(np.mean(kms)),
                flops_per_launch=float(np.mean(fl)),
                steps_per_launch=float(np.mean([s["steps_accepted"] + s["steps_rejected"]
                                                for s in st_h])),
                transcendentals_per_launch=float(np.mean(
                    [sc.transcendentals(s["steps_accepted"], s["steps_rejected"]) for s in st_h])))

    if use_sur:
        n_try = np.mean([s["cells_surrogate"] + s["cells_rejected"] for s in st_h])
        ms_s = float(np.mean([s["ms_surrogate"] for s in st_h]))
        f_inf = accounting.surrogate_flops_per_cell(mech.n_species) * n_try
        sur.update(gate=gate, cells_offered_per_step=float(n_try),
                   cells_accepted_per_step=float(np.mean([s["cells_surrogate"] for s in st_h])),
                   ms_surrogate_per_step=ms_s,
                   inference_bf16_tflops=f_inf / (ms_s * 1e-3) / 1e12 if ms_s > 0 else None,
                   inference_bf16_frac=(f_inf / (ms_s * 1e-3) / 1e12 / accounting.BF16_MFMA_PEAK_TFLOPS)
                   if ms_s > 0 else None)
        if rec is not None:
            log("oracle first-step error on a stratified sample ...")
            sur["first_step_error_vs_oracle"] = first_step_error(mech, field, synth, rec, rec_idx,
                                                                 threads)

    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(mech, field, synth, args.warmup, args.steps, budget_s=args.cpu_seconds,
                           threads=threads)

    desc = (f"{args.workload}: {field.n_cells} cells, {mech.n_species} species / "
            f"{mech.n_reactions} reactions, dt {field.dt} s, rtol 1e-8, atol 1e-12, map (Z_tol 1e-4)"
            + (" + BF16 MLP surrogate with conservation and gate (tau_T %g K, max |dT| %g K, T <= %g K)"
               % (args.tau_T, args.max_dT, args.T_max)
               if use_sur else "")
            + " + heavy-first queue + Rodas4 + mapped update"
            + f"; timed: flow steps {args.warmup + 1}-{args.warmup + args.steps} of a run from the "
              f"pristine field, after {args.warmup} untimed warm-up step(s)")
    out = {
        "metric": METRIC, "value": value, "unit": "cells·dt/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_h,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "cells": field.n_cells, "species": mech.n_species,
                   "reactions": mech.n_reactions, "dt": field.dt, "parallelism": "single GPU",
                   "timed_window": [args.warmup + 1, args.warmup + args.steps]},
        "step_ms": [s["ms_total"] for s in st_h],
        "integrate_kernel_ms": kms,
        "first_step_ms": S_h["warmup_ms"][0] if S_h["warmup_ms"] else None,
        "max_cell_steps": [s["max_cell_steps"] for s in st_h],
        "warmup_ms": S_h["warmup_ms"],
        "plain": plain,
        "balanced_without_surrogate": balanced,
        "speedup_vs_plain": (value / plain["value"]) if plain else None,
        "speedup_vs_balanced": (value / balanced["value"]) if balanced else None,
        "mapped_cells_per_step": float(np.mean([s["cells_mapped"] for s in st_h])),
        "failed_cells": int(sum(s["cells_failed"] for s in st_h)),
        "surrogate": sur,
        "graph_replay": graph,
        "autotune": tune,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
