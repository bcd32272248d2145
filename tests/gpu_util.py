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
