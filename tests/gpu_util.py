"""Helpers shared by the GPU parity tests (test code only)."""
import sys

import numpy as np
import torch

from paper_2011_07978_amd.chem import Chem

DEV = "cuda"


def say(*a):
    """Name the case before each GPU step (flushed, so a lost box still tells)."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype).contiguous()


def host(t):
    return t.detach().cpu().numpy()


def chem_for(mech, **opts):
    c = Chem(0)
    c.set_mechanism(mech)
    if opts:
        c.set_options(**opts)
    return c


def run_integrate(c, field, dt=None, schedule=None, flags=None, ref=None, h=None, cost=None,
                  stats=True):
    """Copies the field to the device, integrates once, returns host arrays."""
    if schedule is not None:
        c.set_options(schedule=schedule)
    n = field.n_cells
    T = dev(field.T)
    p = dev(field.p)
    Y = dev(field.Y)
    hh = dev(h) if h is not None else torch.zeros(n, dtype=torch.float64, device=DEV)
    st = torch.zeros(n, dtype=torch.uint8, device=DEV)
    steps = torch.zeros(2 * n, dtype=torch.int32, device=DEV)
    cst = cost if cost is not None else torch.zeros(n, dtype=torch.int32, device=DEV)
    s = c.integrate(T, p, Y, field.dt if dt is None else dt, flags=flags, ref_index=ref, h=hh,
                    cost=cst, status=st, steps=steps, stats=stats)
    torch.cuda.synchronize()
    stp = host(steps).reshape(-1, 2)
    return dict(T=host(T), Y=host(Y), h=host(hh), status=host(st), nacc=stp[:, 0],
                nrej=stp[:, 1], stats=s, cost=cst)


def compare_to_oracle(out, ref_T, ref_Y, nacc_ref=None, nrej_ref=None, rtol_T=1e-6, atol_Y=1e-8):
    """Element-wise parity at the stated tolerance; returns a report dict."""
    dT = np.abs(out["T"] - ref_T) / np.abs(ref_T)
    dY = np.abs(out["Y"] - ref_Y)
    rep = dict(max_rel_T=float(dT.max(initial=0.0)), max_abs_Y=float(dY.max(initial=0.0)))
    if nacc_ref is not None:
        same = (out["nacc"] == nacc_ref) & (out["nrej"] == nrej_ref)
        rep["step_sequence_differs"] = int((~same).sum())
    rep["ok"] = rep["max_rel_T"] <= rtol_T and rep["max_abs_Y"] <= atol_Y
    return rep


RU_ERG = 8.314462618e7
EPS = 2.0 ** -52


def rounding_scale(o, mech, T, p, Y):
    """Per-component rounding scale of f = (dT/dt, dY_k/dt) for a log-space
    rate evaluation.  Each gross rate m_j k Pi C (forward and reverse; m_j the
    third-body concentration, or the fall-off factor G) is the exponential of
    a sum whose terms reach |ln k_f| + |ln K_c| + ~64 in size, so it carries a
    relative error of about eps times that.  Species k collects
    sum_j |nu_kj| of those errors, times W_k / rho; dT/dt collects the
    species' errors weighted by |H_k / W_k| / cp.  Returns that scale [n]."""
    N, R = mech.n_species, mech.n_reactions
    kf, kr, q, _ = o.kinetics(T, p, Y)
    rho = o.density(T, p, Y)
    C = rho * Y / mech.W
    m = np.ones(R)
    tb = mech.third_body != 0
    m[tb] = C.sum()
    for j, k, a in zip(mech.eff_reaction, mech.eff_species, mech.eff_value):
        m[j] += (a - 1.0) * C[k]
    fo = getattr(mech, "falloff", None)
    if fo is not None:
        for j in np.nonzero(fo)[0]:
            m[j] = o.falloff_factor(j, T, m[j])
    Cx = np.r_[C, 1.0]
    gross = m * (kf * Cx[mech.reactants].prod(axis=1) + kr * Cx[mech.products].prod(axis=1))
    with np.errstate(divide="ignore", invalid="ignore"):
        lsize = np.abs(np.log(kf)) + np.abs(np.log(kf) - np.log(kr))
    lsize = np.nan_to_num(lsize, nan=0.0, posinf=0.0) + 64.0
    err = np.zeros(N)
    for side in (mech.reactants, mech.products):
        for col in side.T:
            ok = col >= 0
            np.add.at(err, col[ok], (gross * lsize)[ok])
    err *= mech.W / rho * EPS
    _, hRT, _ = o.thermo(T)
    hw = np.abs(RU_ERG * T * hRT / mech.W) / o.cp(T, Y)
    return np.r_[hw @ err, err]


def check_rhs_jac(o, mech, field, f, J, label):
    """f [n, nn] and J [n, nn, nn] of the kernels against the oracle's RHS and
    complex-step Jacobian, per component: f_r within 20 of its rounding
    scale; the Jacobian's species columns scaled by their own mass fraction,
    J_rc |Y_c|, within 20 of row r's rounding scale (a derivative with
    respect to ln C_c of a gross rate is at most its order times the rate);
    and every entry within 5e-13 of its row's largest entry (the temperature
    column, and species absent from the cell, whose scaled column is zero).
    On gfx950 the worst cells reach about 2.5 of the scale and 6e-14 of the
    row, so the bounds leave a factor of about 8."""
    worst_f = worst_Jc = worst_Jr = 0.0
    for i in range(field.n_cells):
        y = np.concatenate([[field.T[i]], field.Y[:, i]])
        fo = o.rhs(field.p[i], y)
        Jo = o.jac_cs(field.p[i], y)
        sc = rounding_scale(o, mech, field.T[i], field.p[i], field.Y[:, i])
        # a species in no reaction has a zero scale: its rate must be exactly zero
        ratio = lambda d, s: np.where(s > 0, d / np.where(s > 0, s, 1.0), np.where(d > 0, np.inf, 0.0))
        worst_f = max(worst_f, float(ratio(np.abs(f[i] - fo), sc).max()))
        dJ = np.abs(J[i] - Jo)
        worst_Jc = max(worst_Jc, float(ratio(dJ[:, 1:] * np.abs(y[1:])[None, :], sc[:, None]).max()))
        rows = np.abs(Jo).max(axis=1)
        rows = np.where(rows > 0, rows, 1.0)
        worst_Jr = max(worst_Jr, float((dJ.max(axis=1) / rows).max()))
    print(f"{label}: f {worst_f:.3g} of its rounding scale; J column-scaled {worst_Jc:.3g} of it; "
          f"J row-relative {worst_Jr:.3g}", flush=True)
    assert worst_f <= 20.0, worst_f
    assert worst_Jc <= 20.0, worst_Jc
    assert worst_Jr <= 5e-13, worst_Jr
