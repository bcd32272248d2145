"""Pins of the load-balancing benchmark arithmetic (Sec. 3).

The speed-up bound is pinned against brute force (slowest process over mean
load of explicit heavy/light problem lists), its closed-form limits, and the
printed expression where that one is consistent (C1)."""
import numpy as np
import pytest

from oracle import balance


@pytest.mark.parametrize("cfg", ["C1", "C2", "C3", "C4"])
@pytest.mark.parametrize("xi", [1.0, 2.0, 7.5, 40.0, 300.0])
def test_bound_equals_brute_force(cfg, xi):
    x, theta = balance.UNIT_CONFIGS[cfg]
    loads = balance.slot_loads(cfg, n_slots=20, n_per_slot=10, xi=xi)
    n_heavy = (loads.sum() - loads.size * 10) / (xi - 1.0) if xi != 1.0 else 40.0
    assert n_heavy == pytest.approx(0.2 * 20 * 10)
    assert balance.ideal_speedup(loads) == pytest.approx(balance.speedup_bound(theta, x, xi),
                                                         rel=1e-14)


def test_heavy_share_is_one_fifth_everywhere():
    for cfg, (x, theta) in balance.UNIT_CONFIGS.items():
        assert x * theta == pytest.approx(0.2, rel=1e-15), cfg


def test_balanced_configuration_cannot_speed_up():
    for xi in (1.0, 2.0, 10.0, 1e6):
        assert balance.speedup_bound(0.2, 1.0, xi) == pytest.approx(1.0, rel=1e-15)


def test_equal_costs_cannot_speed_up():
    for cfg, (x, theta) in balance.UNIT_CONFIGS.items():
        assert balance.speedup_bound(theta, x, 1.0) == pytest.approx(1.0, rel=1e-15)


def test_large_ratio_limit_is_one_over_x():
    for cfg, (x, theta) in balance.UNIT_CONFIGS.items():
        assert balance.speedup_bound(theta, x, 1e12) == pytest.approx(1.0 / x, rel=1e-9), cfg


def test_printed_expression_agrees_for_c1_and_not_for_c4():
    for xi in (2.0, 10.0, 100.0):
        assert balance.speedup_bound_as_printed(1.0, 0.2, xi) == pytest.approx(
            balance.speedup_bound(1.0, 0.2, xi), rel=1e-14)
    # as printed, the balanced configuration would gain 3x at xi = 2
    assert balance.speedup_bound_as_printed(0.2, 1.0, 2.0) == pytest.approx(3.0, rel=1e-14)


def test_product_bound_matches_oracle():
    """The benchmark's own bound (product package) against the oracle's."""
    from paper_2011_07978_amd import studies
    rng = np.random.default_rng(5)
    for _ in range(200):
        x, theta, xi = rng.uniform(0.05, 1.0), rng.uniform(0.05, 1.0), 10 ** rng.uniform(0, 4)
        assert studies.speedup_bound(theta, x, xi) == pytest.approx(
            balance.speedup_bound(theta, x, xi), rel=1e-13)


# ---------------------------------------------------------------- Algorithm 1
# The library's planner (host C++, no GPU needed) against hand-worked plans,
# the brute-force unit-by-unit plan of the oracle and the oracle's checker.
def _planner():
    from paper_2011_07978_amd import chem
    try:
        chem.load_library()
    except RuntimeError:
        pytest.skip("libchem.so not built")
    return chem.plan_balance


def test_plan_hand_worked_one_heavy_process():
    """Loads 1, 1, 1, 5 of unit problems, mean 2: the heavy process sends one
    problem to each light one, in its list order."""
    ops, after = _planner()([1, 1, 1, 5], [1.0] * 8)
    assert [(o[0], o[1], o[2], o[3]) for o in ops] == [(3, 0, 0, 1), (3, 1, 1, 1), (3, 2, 2, 1)]
    assert list(after) == [2.0, 2.0, 2.0, 2.0]


def test_plan_hand_worked_two_senders():
    """Loads 0, 0, 6, 6 (three problems of cost 2 each on the heavy ones),
    mean 3.  Worked by hand: process 0 (lightest, lowest index) is filled from
    process 3 (heaviest, highest index) with 3 units, which takes two
    problems (4 >= 3); both are then at the mean; process 1 is filled from
    process 2 the same way."""
    ops, after = _planner()([0, 0, 3, 3], [2.0] * 6)
    assert [(o[0], o[1], o[2], o[3]) for o in ops] == [(3, 0, 0, 2), (2, 1, 0, 2)]
    assert [o[5] for o in ops] == [3.0, 3.0]
    assert list(after) == [4.0, 4.0, 2.0, 2.0]


def test_plan_hand_worked_sender_split_over_receivers():
    """Loads 2, 3, 10 of unit problems, mean 5: process 2 gives 3 units to
    process 0, then 2 to process 1, continuing in its list order."""
    ops, after = _planner()([2, 3, 10], [1.0] * 15)
    assert ops == [(2, 0, 0, 3, 3.0, 3.0), (2, 1, 3, 2, 2.0, 2.0)]
    assert list(after) == [5.0, 5.0, 5.0]


def test_plan_balanced_input_moves_nothing():
    ops, after = _planner()([4, 4, 4], [1.0] * 12)
    assert ops == [] and list(after) == [4.0, 4.0, 4.0]


def test_plan_without_load_moves_nothing():
    """No problems anywhere, or only zero-cost ones: the mean load is zero,
    every process already sits at it."""
    for n_prob, t in (([0, 0, 0], []), ([2, 0, 1], [0.0, 0.0, 0.0])):
        ops, after = _planner()(n_prob, t)
        assert ops == [] and list(after) == [0.0, 0.0, 0.0]


def test_plan_small_imbalance_is_not_emitted():
    """A transfer below 1 % of the mean load is planned but not sent."""
    ops, _ = _planner()([100, 100], [1.0] * 100 + [1.0] * 99 + [1.5])
    assert ops == []


def test_unit_transfers_hand_worked():
    """The brute force itself on the plans worked above."""
    assert balance.unit_transfers([1, 1, 1, 5]) == {(3, 0): 1, (3, 1): 1, (3, 2): 1}
    assert balance.unit_transfers([0, 0, 6, 6]) == {(3, 0): 3, (2, 1): 3}
    assert balance.unit_transfers([2, 3, 10]) == {(2, 0): 3, (2, 1): 2}
    assert balance.unit_transfers([4, 4, 4]) == {}


@pytest.mark.parametrize("seed", range(12))
def test_plan_equals_unit_brute_force(seed):
    """Unit-cost problems and an integer mean: every planned transfer is a
    whole number of problems, and the library's plan moves exactly what the
    oracle's unit-by-unit brute force moves, between the same pairs, in the
    same order (min_frac 0: nothing is dropped)."""
    rng = np.random.default_rng(seed)
    n_proc = int(rng.integers(2, 30))
    n_prob = rng.integers(0, 40, n_proc)
    n_prob[-1] += (-n_prob.sum()) % n_proc          # integer mean
    ops, after = _planner()(n_prob, np.ones(int(n_prob.sum())), 0.0)
    flow = balance.unit_transfers(n_prob)
    assert [(o[0], o[1]) for o in ops] == list(flow)
    assert [o[3] for o in ops] == list(flow.values())
    assert [o[5] for o in ops] == [float(v) for v in flow.values()]
    assert np.all(after == n_prob.sum() // n_proc)
    assert balance.check_plan(n_prob, np.ones(int(n_prob.sum())), ops, after, 0.0) == []


@pytest.mark.parametrize("seed", range(8))
def test_plan_properties_random(seed):
    """Real-valued costs: the oracle's checker finds no violation, and each
    receiver ends within (sends received) problems above the mean."""
    rng = np.random.default_rng(seed)
    n_proc = int(rng.integers(2, 40))
    n_prob = rng.integers(0, 60, n_proc)
    t = rng.lognormal(0.0, 1.0, int(n_prob.sum())) * np.repeat(rng.uniform(0.2, 5.0, n_proc), n_prob)
    ops, after = _planner()(n_prob, t)
    assert balance.check_plan(n_prob, t, ops, after, 0.01) == []
    loads = np.array([t[a:b].sum() for a, b in zip(np.r_[0, np.cumsum(n_prob)[:-1]], np.cumsum(n_prob))])
    mean = loads.mean()
    for r_ in {o[1] for o in ops}:
        k = sum(1 for o in ops if o[1] == r_)
        assert after[r_] <= mean + k * t.max() + 1e-9 * mean


def test_checker_catches_broken_plans():
    """The checker is not vacuous: plans with a planted mistake fail it."""
    n_prob, t = [2, 3, 10], [1.0] * 15
    good = [(2, 0, 0, 3, 3.0, 3.0), (2, 1, 3, 2, 2.0, 2.0)]
    after = [5.0, 5.0, 5.0]
    assert balance.check_plan(n_prob, t, good, after) == []
    gap = [(2, 0, 0, 3, 3.0, 3.0), (2, 1, 4, 2, 2.0, 2.0)]
    assert balance.check_plan(n_prob, t, gap, after)
    extra = [(2, 0, 0, 4, 4.0, 3.0), (2, 1, 4, 2, 2.0, 2.0)]
    assert balance.check_plan(n_prob, t, extra, [6.0, 5.0, 4.0])
    over = [(2, 0, 0, 4, 4.0, 4.0), (2, 1, 4, 1, 1.0, 1.0)]
    assert balance.check_plan(n_prob, t, over, after)
    assert balance.check_plan(n_prob, t, good, [5.0, 5.0, 6.0])


def test_library_planner_rejects_bad_input():
    from paper_2011_07978_amd import chem
    try:
        L = chem.load_library()
    except RuntimeError:
        pytest.skip("libchem.so not built")
    import ctypes as C
    ops = (chem.BalanceOp * 4)()
    n = C.c_int64(0)
    cnt = np.array([2, 1], dtype=np.int64)
    good = np.array([1.0, 2.0, 3.0])
    P = lambda a, t: a.ctypes.data_as(C.POINTER(t))
    # no processes, negative count, negative / non-finite cost, null output
    assert L.chem_plan_balance(0, P(cnt, C.c_int64), P(good, C.c_double), 0.01, ops, 4, C.byref(n), None) != 0
    bad_cnt = np.array([2, -1], dtype=np.int64)
    assert L.chem_plan_balance(2, P(bad_cnt, C.c_int64), P(good, C.c_double), 0.01, ops, 4, C.byref(n), None) != 0
    for v in (-1.0, np.inf, np.nan):
        t = good.copy(); t[1] = v
        assert L.chem_plan_balance(2, P(cnt, C.c_int64), P(t, C.c_double), 0.01, ops, 4, C.byref(n), None) != 0
    assert L.chem_plan_balance(2, P(cnt, C.c_int64), P(good, C.c_double), 0.01, ops, 4, None, None) != 0
    # too small an output array: error, but the count of operations is reported
    heavy = np.array([1, 1, 1, 5], dtype=np.int64)
    t = np.ones(8)
    rc = L.chem_plan_balance(4, P(heavy, C.c_int64), P(t, C.c_double), 0.01, ops, 1, C.byref(n), None)
    assert rc != 0 and n.value == 3
    # no load at all: nothing to do
    zero = np.array([0, 0, 0], dtype=np.int64)
    assert L.chem_plan_balance(3, P(zero, C.c_int64), None, 0.01, ops, 4, C.byref(n), None) == 0
    assert n.value == 0
    # one process: nothing to do
    one = np.array([3], dtype=np.int64)
    assert L.chem_plan_balance(1, P(one, C.c_int64), P(good, C.c_double), 0.01, ops, 4, C.byref(n), None) == 0
    assert n.value == 0
