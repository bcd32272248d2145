"""Algorithmic work of the integration path, for roofline accounting.

Counts what the method must compute per unit of work, independent of how the
kernels schedule it: floating-point operations of the right-hand side, the
analytic Jacobian, LU factorisation, triangular solves and the Rodas4 stage
arithmetic (an FMA counts as 2), and transcendental calls (exp, log, pow)
separately.  Units are one attempted Rosenbrock step and one accepted step.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
HBM_PEAK_GBS = 8000.0


@dataclass
class StepCost:
    n: int
    F_rhs: int          # one f(y)
    F_jac: int          # analytic Jacobian on top of f(y) at the same point
    F_build: int        # M = I/(gamma h) - J
    F_lu: int           # LU with partial pivoting, n x n
    F_solve: int        # forward + backward substitution
    F_stage: int        # Rodas4 stage combinations, error norm
    X_rhs: int          # transcendentals per f(y): exp for each k_f, exp(g_k) and its
                        # inverse for each species (the K_c factors), ln T

    @property
    def F_attempt(self):
        """Every attempted step: factor, six solves, five new stage RHS."""
        return self.F_build + self.F_lu + 6 * self.F_solve + 5 * self.F_rhs + self.F_stage

    @property
    def F_accept(self):
        """Every accepted step additionally evaluates f and J at the new point
        (the first evaluation of each cell is counted here as well)."""
        return self.F_rhs + self.F_jac

    def flops(self, accepted, rejected):
        return (accepted + rejected) * self.F_attempt + accepted * self.F_accept

    def transcendentals(self, accepted, rejected):
        return (accepted + rejected) * (5 * self.X_rhs + 1) + accepted * self.X_rhs


def step_cost(mech) -> StepCost:
    N, R = int(mech.n_species), int(mech.n_reactions)
    n = N + 1
    slots = (np.asarray(mech.reactants) >= 0).sum(1) + (np.asarray(mech.products) >= 0).sum(1)
    tb = np.asarray(mech.third_body) != 0
    n_tb = int(tb.sum())
    eff_per = np.bincount(np.asarray(mech.eff_reaction, dtype=np.int64), minlength=R)
    n_eff = int(eff_per.sum())
    # species-reaction incidences with non-zero net stoichiometry
    nnz = 0
    for j in range(R):
        nu = {}
        for k in mech.reactants[j]:
            if k >= 0:
                nu[k] = nu.get(k, 0) - 1
        for k in mech.products[j]:
            if k >= 0:
                nu[k] = nu.get(k, 0) + 1
        nnz += sum(1 for v in nu.values() if v != 0)
    S1, S2 = int(slots.sum()), int((slots ** 2).sum())
    F_rhs = 40 * N + 18 * R + 2 * nnz + 2 * n_eff + n_tb + 6
    F_jac = (25 * R + 2 * (S1 + S2) + int((2 * slots * (1 + eff_per))[tb].sum())
             + 6 * N * N + 6 * N + 2 * n * N + 6 * n + 12 * N)
    F_lu = (n - 1) * n // 2 + (n - 1) * n * (2 * n - 1) // 3
    F_solve = 2 * n * n - n
    return StepCost(n=n, F_rhs=F_rhs, F_jac=F_jac, F_build=n * n, F_lu=F_lu, F_solve=F_solve,
                    F_stage=65 * n, X_rhs=R + 2 * N + 1)


def state_bytes(mech) -> int:
    """HBM bytes one cell's integration must move: read T, p, Y, h and write
    T, Y, h (FP64) plus status and step counters."""
    n = int(mech.n_species) + 1
    return 8 * (n + 2) + 8 * (n + 1) + 1 + 8


BF16_MFMA_PEAK_TFLOPS = 2500.0   # dense bfloat16 matrix-core peak of MI355X


def surrogate_flops_per_cell(n_species: int, hidden: int = 256, layers: int = 4) -> int:
    """Multiply-adds of one surrogate forward pass on the unpadded widths
    (N + 3 inputs, N + 1 outputs), an FMA counting 2."""
    nin, nout = n_species + 3, n_species + 1
    macs = nin * hidden + (layers - 1) * hidden * hidden + hidden * nout
    return 2 * macs


def surrogate_train_flops_per_sample(n_species: int) -> int:
    """Forward, input-gradient and weight-gradient products: 3 x forward."""
    return 3 * surrogate_flops_per_cell(n_species)
