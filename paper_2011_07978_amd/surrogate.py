"""Training-data generation and training of the learned surrogate.

Pairs come from the Rosenbrock solver of libchem itself: a seeded field of
cold, mixing-layer and igniting cells is advanced for several flow steps; in
every step each cell draws its own dt (half at the flow step, half spread
log-uniformly over a 16x range), cells sharing a dt are integrated together,
and (state, dt, advanced state) is recorded.  Training and evaluation run in
libchem's kernels (chem_surrogate_train, chem_integrate_surrogate); this
module only moves tensors.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import synth


class Pairs:
    """Device-resident training pairs (species-major Y)."""

    def __init__(self, T0, p, Y0, dt, T1, Y1):
        self.T0, self.p, self.Y0, self.dt, self.T1, self.Y1 = T0, p, Y0, dt, T1, Y1

    @property
    def n(self):
        return int(self.T0.shape[0])

    def take(self, idx):
        idx = torch.as_tensor(idx, device=self.T0.device, dtype=torch.int64)
        return Pairs(self.T0[idx].contiguous(), self.p[idx].contiguous(),
                     self.Y0[:, idx].contiguous(), self.dt[idx].contiguous(),
                     self.T1[idx].contiguous(), self.Y1[:, idx].contiguous())


def generate_pairs(chem, n_cells=262144, n_steps=8, seed=900, log=None) -> Pairs:
    """Solver-generated pairs: n_cells x n_steps samples."""
    f = synth.surrogate_pairs_field(n_cells, seed)
    dev = torch.device("cuda")
    T = torch.as_tensor(f.T, device=dev).contiguous()
    p = torch.as_tensor(f.p, device=dev).contiguous()
    Y = torch.as_tensor(f.Y, device=dev).contiguous()
    N = Y.shape[0]
    out = {k: [] for k in ("T0", "p", "Y0", "dt", "T1", "Y1")}
    t0 = time.time()
    for s in range(n_steps):
        dt_h = synth.surrogate_dt(n_cells, seed * 1000 + s)
        dt = torch.as_tensor(dt_h, device=dev)
        T1 = T.clone()
        Y1 = Y.clone()
        for v in np.unique(dt_h):
            idx = torch.as_tensor(np.nonzero(dt_h == v)[0], device=dev)
            Tg = T[idx].contiguous()
            pg = p[idx].contiguous()
            Yg = Y[:, idx].contiguous()
            st = torch.zeros(idx.numel(), dtype=torch.uint8, device=dev)
            chem.integrate(Tg, pg, Yg, float(v), status=st)
            ok = st == 0
            T1[idx] = torch.where(ok, Tg, torch.nan)
            Y1[:, idx] = torch.where(ok[None, :], Yg, torch.nan)
        good = torch.isfinite(T1) & torch.isfinite(Y1).all(dim=0)
        for k, v in (("T0", T), ("p", p), ("Y0", Y), ("dt", dt), ("T1", T1), ("Y1", Y1)):
            out[k].append(v[..., good] if v.dim() == 2 else v[good])
        # the next step starts from the flow-step advance of every cell
        T = torch.where(good, T1, T).contiguous()
        Y = torch.where(good[None, :], Y1, Y).contiguous()
        if log:
            torch.cuda.synchronize()
            log(f"pairs: step {s + 1}/{n_steps} done ({time.time() - t0:.1f} s)")
    cat = lambda k, ax: torch.cat(out[k], dim=ax).contiguous()
    return Pairs(cat("T0", 0), cat("p", 0), cat("Y0", 1), cat("dt", 0), cat("T1", 0),
                 cat("Y1", 1))


def split(pairs: Pairs, frac_train=0.9, seed=901):
    """Seeded train / validation split."""
    perm = np.random.default_rng(seed).permutation(pairs.n)
    k = int(frac_train * pairs.n)
    return pairs.take(np.sort(perm[:k])), pairs.take(np.sort(perm[k:]))


def train(chem, pairs: Pairs, **params):
    """chem_surrogate_train on device pairs; returns the per-epoch loss."""
    return chem.surrogate_train(pairs.T0, pairs.p, pairs.Y0, pairs.dt, pairs.T1, pairs.Y1,
                                **params)


def validate(chem, pairs: Pairs, dt=1e-6, gate=None):
    """Surrogate-with-fallback on the validation pairs of step dt; returns
    the acceptance rate and the |T - T_solver| statistics of accepted cells."""
    sel = torch.nonzero(pairs.dt == dt).flatten()
    v = pairs.take(sel)
    T = v.T0.clone()
    Y = v.Y0.clone()
    flags = torch.zeros(v.n, dtype=torch.uint8, device=T.device)
    st = chem.integrate_surrogate(T, v.p, Y, dt, flags, gate=gate, stats=True)
    acc = flags == 3
    dT = (T - v.T1).abs()
    dY = (Y - v.Y1).abs().amax(dim=0)
    res = dict(n=v.n, accepted=int(acc.sum()), stats=st,
               mean_dT_accepted=float(dT[acc].mean()) if acc.any() else 0.0,
               max_dT_accepted=float(dT[acc].max()) if acc.any() else 0.0,
               max_dY_accepted=float(dY[acc].max()) if acc.any() else 0.0,
               mean_dT_all=float(dT.mean()))
    return res
