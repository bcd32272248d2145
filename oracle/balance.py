"""Load-balancing benchmark arithmetic — TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and the benchmark's reporting may import
this module.  It holds the paper's unit-benchmark quantities (Sec. 3): the
speed-up ratio chi_su of balanced over unbalanced runs and the largest speed-up
a perfect balancer can reach for a heavy/light problem mix.
"""
from __future__ import annotations

import numpy as np

# Sec. 3, configurations C1-C4: a fraction x of the processes holds heavy
# problems at ratio theta (heavy problems / problems of that process); the
# other processes hold light problems only.  x * theta = 0.2, the fixed ratio
# of heavy problems to all problems.
UNIT_CONFIGS = {
    "C1": (0.2, 1.0),    # very unbalanced
    "C2": (0.25, 0.8),   # slightly unbalanced
    "C3": (0.5, 0.4),    # slightly balanced
    "C4": (1.0, 0.2),    # very balanced
}


def speedup_bound(theta: float, x: float, xi: float) -> float:
    """Largest chi_su for heavy/light cost ratio xi (Sec. 3, reading).

    Unbalanced time is set by a process with ratio theta: theta xi + (1 - theta)
    per problem (light cost 1).  A perfect balancer gives every process the mean
    load: heavy fraction x theta over all problems, x theta xi + (1 - x theta).
    The printed denominator has 1/x - 1 where this has 1/x - theta (the two
    agree at theta = 1, C1); as printed it would give 3 for C4 at xi = 2,
    although C4 is balanced by construction."""
    return (theta * xi + (1.0 - theta)) / (theta * x * xi + 1.0 - theta * x)


def speedup_bound_as_printed(theta: float, x: float, xi: float) -> float:
    """The expression exactly as printed in Sec. 3 (kept to document the reading)."""
    return (theta * xi + (1.0 - theta)) / ((theta * xi + (1.0 / x - 1.0)) / (1.0 / x))


def slot_loads(config: str, n_slots: int, n_per_slot: int, xi: float) -> np.ndarray:
    """Brute-force loads: per process, the sum of its problem costs (heavy xi,
    light 1) for configuration C1-C4 with whole numbers of processes and
    heavy problems."""
    x, theta = UNIT_CONFIGS[config]
    n_theta = int(round(x * n_slots))
    n_heavy = int(round(theta * n_per_slot))
    loads = np.full(n_slots, float(n_per_slot))
    loads[:n_theta] = n_heavy * xi + (n_per_slot - n_heavy)
    return loads


def ideal_speedup(loads: np.ndarray) -> float:
    """Static time (slowest process) over perfectly balanced time (mean load)."""
    return float(np.max(loads) / np.mean(loads))


def plan_balance(n_prob, t_cost, min_frac=0.01):
    """Algorithm 1 (Sec. 2.2), plain loops: the list of balancing operations
    (sender, receiver, first, count, load, planned) and the loads after they
    move their problems.

    Readings of the garbled passages: the mean load is the sum of the loads
    over the number of processes; "|L_i - mean| ~ 0" is |L_i - mean| <= 1e-12
    mean; "find N_send s.t. dL ~ sum t" takes, in the sender's list order
    from where its last emitted send stopped, the shortest prefix whose cost
    reaches dL (all remaining problems if none does); operations with
    dL < min_frac * mean are computed but not emitted."""
    n_prob = [int(v) for v in n_prob]
    n_proc = len(n_prob)
    lists, pos = [], 0
    for k in range(n_proc):
        lists.append([float(t) for t in t_cost[pos:pos + n_prob[k]]])
        pos += n_prob[k]
    loads = []
    for k in range(n_proc):
        s = 0.0
        for t in lists[k]:
            s += t
        loads.append(s)
    total = 0.0
    for v in loads:
        total += v
    mean = total / n_proc
    order = sorted(range(n_proc), key=lambda k: (loads[k], k))
    L = [loads[k] for k in order]
    after = list(loads)
    cursor = [0] * n_proc
    ops = []
    i, j = 0, n_proc - 1
    while i != j:
        dL = min(mean - L[i], L[j] - mean)
        rr, rs = order[i], order[j]
        first, cnt, sent = cursor[rs], 0, 0.0
        while first + cnt < n_prob[rs] and sent < dL:
            sent += lists[rs][first + cnt]
            cnt += 1
        if dL >= min_frac * mean and cnt > 0:
            ops.append((rs, rr, first, cnt, sent, dL))
            cursor[rs] += cnt
            after[rs] -= sent
            after[rr] += sent
        L[i] += dL
        L[j] -= dL
        if abs(L[i] - mean) <= 1e-12 * mean:
            i += 1
        else:
            j -= 1
    return ops, np.array(after)
