"""Studies beyond the headline benchmark, run through the library's public calls.

- unit_benchmark: the paper's load-balancing benchmark (Sec. 3) on one GPU.
  The persistent slots play the processes; CHEM_SCHED_BLOCKS (every slot owns a
  contiguous block of cells) is the unbalanced standard model and the
  heavy-first work queue is the balanced model.  chi_su = tau_unb / tau_bal is
  compared with the largest speed-up a perfect balancer reaches.
- mapping_study: the reference-mapping error study (App. A): the mapped path
  against the unmapped one over consecutive flow steps, for several Z_tol with
  and without the temperature criterion.
"""
from __future__ import annotations

import numpy as np

RU_ERG = 8.314462618e7      # erg/(mol K)
T_FORMATION = 298.15         # K, reference temperature of the chemical enthalpy


def speedup_bound(theta: float, x: float, xi: float) -> float:
    """Largest chi_su for heavy/light cost ratio xi (Sec. 3).  The slowest
    process of the unbalanced run has heavy ratio theta (cost theta xi +
    1 - theta per problem, light cost 1); a perfect balancer gives every
    process the mean load, x theta xi + 1 - x theta.  (The printed denominator
    has 1/x - 1 in place of 1/x - theta; the two agree for C1.)"""
    return (theta * xi + 1.0 - theta) / (x * theta * xi + 1.0 - x * theta)


def _median_ms(fn, reps):
    return float(np.median([fn() for _ in range(reps)]))


def _prototypes(chem, torch, synth, mech, seed, warm_steps=2):
    """One heavy (igniting) and one light (cold) problem with step-size
    history, from the bimodal field after warm_steps flow steps."""
    from paper_2011_07978_amd.chem import CHEM_SCHED_QUEUE
    f = synth.field_bimodal(mech.name, 256, seed=seed)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to("cuda").contiguous()
    T, p, Y = dev(f.T), dev(f.p), dev(f.Y)
    h = torch.zeros(f.n_cells, dtype=torch.float64, device="cuda")
    chem.set_options(schedule=CHEM_SCHED_QUEUE)
    for _ in range(warm_steps):
        chem.integrate(T, p, Y, f.dt, h=h)
    torch.cuda.synchronize()
    Th, ph, Yh, hh = T.cpu().numpy(), p.cpu().numpy(), Y.cpu().numpy(), h.cpu().numpy()
    hot, cold = 0, f.n_cells - 1          # hot cells come first in this field
    heavy = (Th[hot], ph[hot], Yh[:, hot].copy(), hh[hot])
    light = (Th[cold], ph[cold], Yh[:, cold].copy(), hh[cold])
    return heavy, light, f.dt


def unit_benchmark(chem, torch, synth, mech, n_per_slot=100, reps=3,
                   layouts=("C1", "C2", "C3", "C4"), seed=910, log=print):
    from paper_2011_07978_amd.chem import CHEM_SCHED_BLOCKS, CHEM_SCHED_PLAIN, CHEM_SCHED_QUEUE
    heavy, light, dt = _prototypes(chem, torch, synth, mech, seed)
    chem.set_options(schedule=CHEM_SCHED_QUEUE)
    slots = chem.slots()
    out = {"slots": slots, "problems_per_slot": n_per_slot, "dt": dt, "reps": reps,
           "heavy_T0": float(heavy[0]), "light_T0": float(light[0]), "layouts": {}}
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to("cuda").contiguous()

    def blocks_ms(problem):
        """Static-partition time of a field made of one problem only."""
        f, h0, _ = synth.field_unit("C4", problem, problem, slots, n_per_slot, dt)
        chem.reserve(f.n_cells)
        p = dev(f.p)
        chem.set_options(schedule=CHEM_SCHED_BLOCKS)

        def one():
            T, Y, h = dev(f.T), dev(f.Y), dev(h0)
            return chem.integrate(T, p, Y, dt, h=h, stats=True)["ms_total"]
        one()
        return _median_ms(one, reps)

    # cost ratio in time: every slot runs n_per_slot copies of one problem
    t_all_heavy, t_all_light = blocks_ms(heavy), blocks_ms(light)
    xi_time = t_all_heavy / t_all_light
    out.update(ms_all_heavy_blocks=t_all_heavy, ms_all_light_blocks=t_all_light, xi_time=xi_time)
    log(f"unit: all-heavy {t_all_heavy:.1f} ms, all-light {t_all_light:.2f} ms -> xi (time) {xi_time:.2f}")
    for name in layouts:
        x, theta = synth.UNIT_LAYOUTS[name]
        f, h0, is_heavy = synth.field_unit(name, heavy, light, slots, n_per_slot, dt)
        n = f.n_cells
        chem.reserve(n)
        T0, p, Y0, hh0 = dev(f.T), dev(f.p), dev(f.Y), dev(h0)
        T, Y, h = T0.clone(), Y0.clone(), hh0.clone()
        cost = torch.zeros(n, dtype=torch.int32, device="cuda")

        def call(schedule, use_cost):
            T.copy_(T0); Y.copy_(Y0); h.copy_(hh0)
            chem.set_options(schedule=schedule)
            st = chem.integrate(T, p, Y, dt, h=h, cost=cost if use_cost else None, stats=True)
            return st

        call(CHEM_SCHED_QUEUE, True)          # first call: per-cell cost for the next ones
        c = cost.cpu().numpy().astype(np.float64)
        xi = float(c[is_heavy].mean() / max(c[~is_heavy].mean(), 1e-30))
        # what the paper's planner (Algorithm 1) would move between the slots,
        # on the same per-cell costs: slowest slot before and after
        from paper_2011_07978_amd.chem import plan_balance
        ops, after = plan_balance(np.full(slots, n_per_slot), c, 0.01)
        before = c.reshape(slots, n_per_slot).sum(axis=1)
        alg1 = {"operations": len(ops), "problems_moved": int(sum(o[3] for o in ops)),
                "max_load_before": float(before.max()), "max_load_after": float(after.max()),
                "mean_load": float(before.mean()),
                "chi_planned": float(before.max() / after.max())}
        t_bal = _median_ms(lambda: call(CHEM_SCHED_QUEUE, True)["ms_total"], reps)
        t_unb = _median_ms(lambda: call(CHEM_SCHED_BLOCKS, False)["ms_total"], reps)
        t_plain = _median_ms(lambda: call(CHEM_SCHED_PLAIN, False)["ms_total"], reps)
        chem.set_options(schedule=CHEM_SCHED_QUEUE)
        r = {"x": x, "theta": theta, "cells": n, "xi_attempts": xi,
             "ms_unbalanced_blocks": t_unb, "ms_balanced_queue": t_bal,
             "ms_plain_one_cell_per_workgroup": t_plain,
             "chi_su": t_unb / t_bal, "chi_su_bound": speedup_bound(theta, x, xi),
             "chi_su_bound_time": speedup_bound(theta, x, xi_time),
             "chi_plain_over_queue": t_plain / t_bal, "algorithm1_plan": alg1}
        out["layouts"][name] = r
        log(f"unit {name}: x {x} theta {theta} xi {xi:.1f}: blocks {t_unb:.1f} ms, queue {t_bal:.1f} ms, "
            f"plain {t_plain:.1f} ms -> chi_su {r['chi_su']:.2f} (bound {r['chi_su_bound']:.2f} "
            f"from attempts, {r['chi_su_bound_time']:.2f} from time); Algorithm 1 plan: "
            f"{alg1['operations']} operations, {alg1['problems_moved']} problems, "
            f"planned chi {alg1['chi_planned']:.2f}")
    return out


def chemical_enthalpy_drop(mech, Y0, Y1):
    """Per-cell heat released between two states at constant p and total h:
    sum_k h_k(298.15 K) (Y0_k - Y1_k), with h_k the NASA-7 enthalpy per unit
    mass (erg/g).  Y is species-major [N, cells]."""
    a = np.asarray(mech.nasa, dtype=np.float64)
    T = T_FORMATION
    hRT = a[:, 0] + T * (a[:, 1] / 2 + T * (a[:, 2] / 3 + T * (a[:, 3] / 4 + T * a[:, 4] / 5))) + a[:, 5] / T
    hk = hRT * RU_ERG * T / np.asarray(mech.W, dtype=np.float64)
    return hk @ (np.asarray(Y0) - np.asarray(Y1))


def mapping_study(chem, torch, synth, mech, n_cells=262144, steps=10,
                  z_tols=(1e-2, 1e-4, 1e-6), T_tol=1.0, seed=103, log=print):
    from paper_2011_07978_amd.chem import CHEM_SCHED_QUEUE
    f = synth.field_mapped(n_cells, seed=seed)
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to("cuda").contiguous()
    chem.set_options(schedule=CHEM_SCHED_QUEUE)
    chem.reserve(f.n_cells)

    def run(z_tol, use_T):
        T, p, Y = dev(f.T), dev(f.p), dev(f.Y)
        n = f.n_cells
        h = torch.zeros(n, dtype=torch.float64, device="cuda")
        cost = torch.zeros(n, dtype=torch.int32, device="cuda")
        flags = torch.zeros(n, dtype=torch.uint8, device="cuda")
        ref = torch.zeros(1, dtype=torch.int64, device="cuda")
        mapped = 0
        ms = []
        for _ in range(steps):
            if z_tol is None:
                st = chem.integrate(T, p, Y, f.dt, h=h, cost=cost, stats=True)
            else:
                chem.map_reference(T, p, Y, Yf, Yo, z_tol, T_tol=T_tol, use_T=use_T, flags=flags,
                                   ref_index=ref)
                st = chem.integrate(T, p, Y, f.dt, flags=flags, ref_index=ref, h=h, cost=cost,
                                    stats=True)
            mapped += st["cells_mapped"]
            ms.append(st["ms_total"])
        torch.cuda.synchronize()
        # mean over the steps after the first (which relaxes the synthetic field)
        ms_later = float(np.mean(ms[1:])) if len(ms) > 1 else float(ms[0])
        return T.cpu().numpy(), Y.cpu().numpy(), mapped / steps, ms_later

    T_ref, Y_ref, _, ms_ref = run(None, False)
    q_ref = chemical_enthalpy_drop(mech, f.Y, Y_ref)
    Q_ref = float(q_ref.sum())
    out = {"cells": f.n_cells, "steps": steps, "dt": f.dt, "T_tol": T_tol,
           "unmapped": {"ms_per_step_after_first": ms_ref, "heat_release_erg_per_g_sum": Q_ref}, "runs": []}
    cls = np.asarray(f.cls)
    for use_T in (False, True):
        for z in z_tols:
            T, Y, mapped, ms = run(z, use_T)
            dT = np.abs(T - T_ref)
            q = chemical_enthalpy_drop(mech, f.Y, Y)
            r = {"Z_tol": z, "use_T": use_T, "mapped_per_step": mapped,
                 "mapped_fraction": mapped / f.n_cells, "ms_per_step_after_first": ms,
                 "speedup_vs_unmapped": ms_ref / ms,
                 "mean_abs_dT": float(dT.mean()), "max_abs_dT": float(dT.max()),
                 "max_abs_dY": float(np.abs(Y - Y_ref).max()),
                 "heat_release_rel_err": float(abs(q.sum() - Q_ref) / abs(Q_ref)),
                 "by_class_mean_abs_dT": {name: float(dT[cls == i].mean())
                                          for i, name in enumerate(f.class_names)}}
            out["runs"].append(r)
            log(f"mapping Z_tol {z:g} use_T {use_T}: {mapped:.0f} mapped/step, {ms:.1f} ms/step, "
                f"mean |dT| {r['mean_abs_dT']:.2e} K, max {r['max_abs_dT']:.2e} K, "
                f"heat release rel err {r['heat_release_rel_err']:.2e}")
    return out
