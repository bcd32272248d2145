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


def unit_transfers(loads):
    """Brute force of the balancing plan for integer loads whose mean is an
    integer (Algorithm 1, Sec. 2.2, by its goal: every process ends at the
    mean load, the lightest processes filled first from the heaviest).

    Moves one unit of load at a time from the current sender to the current
    receiver: receivers are the processes below the mean, lightest first
    (ties: lower index first); senders those above it, heaviest first (ties:
    higher index first, the heavy end of the same ascending order).  A
    receiver is served until it reaches the mean, a sender gives until it
    does.  Returns {(sender, receiver): units}, in the order first used."""
    loads = [int(v) for v in loads]
    n = len(loads)
    total = sum(loads)
    assert total % n == 0, "brute force needs an integer mean"
    mean = total // n
    order = sorted(range(n), key=lambda k: (loads[k], k))
    receivers = [k for k in order if loads[k] < mean]
    senders = [k for k in reversed(order) if loads[k] > mean]
    have = list(loads)
    flow = {}
    ri = si = 0
    while ri < len(receivers) and si < len(senders):
        r, s = receivers[ri], senders[si]
        have[r] += 1
        have[s] -= 1
        flow[(s, r)] = flow.get((s, r), 0) + 1
        if have[r] == mean:
            ri += 1
        if have[s] == mean:
            si += 1
    assert all(v == mean for v in have)
    return flow


def check_plan(n_prob, t_cost, ops, loads_after, min_frac=0.01, rel=1e-12):
    """Checks a balancing plan (operations (sender, receiver, first, count,
    load, planned) and the loads after them) against what the plan must
    satisfy whatever its internal steps; returns the list of violations.

      - every problem leaves its process at most once, operations of one
        sender take its problems in list order without gaps;
      - an operation's load is the cost of the problems it names, and they
        are the fewest from its first whose cost reaches the planned load
        (or every remaining problem);
      - no process both sends and receives, and nobody sends to itself;
      - planned loads are at least min_frac of the mean; the planned loads a
        receiver gets sum to at most its deficit, a sender's to at most its
        surplus;
      - load is conserved, and the loads after are the loads before moved by
        the operations."""
    n_prob = [int(v) for v in n_prob]
    t_cost = [float(v) for v in t_cost]
    starts = [0]
    for c in n_prob:
        starts.append(starts[-1] + c)
    loads = [sum(t_cost[starts[k]:starts[k + 1]]) for k in range(len(n_prob))]
    mean = sum(loads) / len(loads)
    bad = []
    nxt = {}
    moved = list(loads)
    got_planned, gave_planned = {}, {}
    for op in ops:
        s, r, first, cnt, load, planned = op
        if s == r or cnt <= 0:
            bad.append(("self or empty", op))
        if first != nxt.get(s, 0) or first + cnt > n_prob[s]:
            bad.append(("not in list order", op))
        nxt[s] = first + cnt
        costs = t_cost[starts[s] + first:starts[s] + first + cnt]
        if abs(sum(costs) - load) > rel * max(1.0, abs(load)):
            bad.append(("load is not the problems' cost", op))
        if sum(costs) < planned * (1 - rel) and first + cnt < n_prob[s]:
            bad.append(("stops short of the planned load", op))
        if cnt > 1 and sum(costs[:-1]) >= planned:
            bad.append(("not the fewest problems", op))
        if planned < min_frac * mean * (1 - rel):
            bad.append(("below the threshold", op))
        got_planned[r] = got_planned.get(r, 0.0) + planned
        gave_planned[s] = gave_planned.get(s, 0.0) + planned
        moved[s] -= load
        moved[r] += load
    if set(got_planned) & set(gave_planned):
        bad.append(("a process both sends and receives", None))
    for r, v in got_planned.items():
        if v > (mean - loads[r]) + rel * max(1.0, mean) * len(loads):
            bad.append(("receiver planned beyond its deficit", r))
    for s, v in gave_planned.items():
        if v > (loads[s] - mean) + rel * max(1.0, mean) * len(loads):
            bad.append(("sender planned beyond its surplus", s))
    if abs(sum(loads_after) - sum(loads)) > rel * max(1.0, sum(loads)) * len(loads):
        bad.append(("load not conserved", None))
    for k in range(len(loads)):
        if abs(loads_after[k] - moved[k]) > rel * max(1.0, abs(moved[k])) * len(loads):
            bad.append(("loads after do not follow the operations", k))
    return bad
