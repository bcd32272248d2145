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
