"""Pins of the oracle's tabulated pressure dependence (PLOG rates).

For a PLOG reaction, ln k_f is linear in ln p between two tabulated pressures
and takes the end entry outside the table.  Pinned at the tabulated pressures
(each entry's own Arrhenius form), at the geometric midpoint of two pressures
(the mean of the two ln k), outside the table, by continuity at the table
points, by reactions without a table ignoring the pressure, by a table of
identical entries reducing to the plain Arrhenius form bit for bit, and
through the whole right-hand side: central finite differences of the
complex-step Jacobian, element and mass conservation, and the invariants of
an integration at several pressures."""
import dataclasses

import numpy as np
import pytest

from oracle import Oracle
from paper_2011_07978_amd import synth

RU_J = 8.314462618
P_ATM = synth.P_ATM


@pytest.fixture(scope="module")
def pl():
    return Oracle(synth.mechanism("mech53pl"))


def _lnk(A, b, Ea, T):
    return np.log(A) + b * np.log(T) - Ea / (RU_J * T)


def _plog(mech):
    return np.nonzero(mech.plog_count > 0)[0]


def test_mechanism_has_tables_of_every_length():
    m = synth.mechanism("mech53pl")
    assert set(np.unique(m.plog_count[m.plog_count > 0])) == {2, 3, 4, 5}
    assert np.all(m.third_body[_plog(m)] == 0)


def test_tabulated_pressures_midpoints_and_ends(pl):
    mech = pl.mech
    for j in _plog(mech)[:20]:
        cnt = mech.plog_count[j]
        t = mech.plog_params[j, :cnt]
        for T in (500.0, 1300.0, 2400.0):
            lk = [_lnk(t[i, 1], t[i, 2], t[i, 3], T) for i in range(cnt)]
            for i in range(cnt):
                assert pl.ln_kf(j, T, t[i, 0]) == pytest.approx(lk[i], rel=1e-14, abs=1e-12)
            for i in range(cnt - 1):
                pm = np.sqrt(t[i, 0] * t[i + 1, 0])
                assert pl.ln_kf(j, T, pm) == pytest.approx(0.5 * (lk[i] + lk[i + 1]), rel=1e-12, abs=1e-11)
                # continuous at the upper table point of each interval
                assert pl.ln_kf(j, T, t[i + 1, 0] * (1 - 1e-13)) == pytest.approx(lk[i + 1], abs=1e-9)
            assert pl.ln_kf(j, T, t[0, 0] / 7.0) == pytest.approx(lk[0], rel=1e-14, abs=1e-12)
            assert pl.ln_kf(j, T, t[cnt - 1, 0] * 7.0) == pytest.approx(lk[-1], rel=1e-14, abs=1e-12)


def test_other_reactions_ignore_pressure(pl):
    mech = pl.mech
    for j in np.nonzero(mech.plog_count == 0)[0][:20]:
        ref = _lnk(mech.A[j], mech.b[j], mech.Ea[j], 1100.0)
        for p in (0.01 * P_ATM, P_ATM, 300 * P_ATM):
            assert pl.ln_kf(j, 1100.0, p) == pytest.approx(ref, rel=1e-14, abs=1e-12)


def test_rate_constants_follow_the_table(pl):
    f = synth.field_bimodal("mech53pl", 2000, shuffle=True)
    mech = pl.mech
    for i, p in enumerate((0.2 * P_ATM, 3 * P_ATM, 40 * P_ATM)):
        kf, kr, q, om = pl.kinetics(f.T[i], p, f.Y[:, i])
        for j in _plog(mech)[:10]:
            assert np.log(kf[j]) == pytest.approx(pl.ln_kf(j, f.T[i], p), rel=1e-13)


def test_identical_entries_reduce_to_arrhenius():
    base = synth.mechanism("mech53pl")
    prm = base.plog_params.copy()
    for j in _plog(base):
        prm[j, :, 1], prm[j, :, 2], prm[j, :, 3] = base.A[j], base.b[j], base.Ea[j]
    flat = Oracle(dataclasses.replace(base, plog_params=prm))
    plain = Oracle(dataclasses.replace(base, plog_count=None, plog_params=None))
    f = synth.field_bimodal("mech53pl", 2000, shuffle=True)
    for i in range(4):
        y = np.concatenate([[f.T[i]], f.Y[:, i]])
        for p in (0.05 * P_ATM, 2.5 * P_ATM, 500 * P_ATM):
            assert np.array_equal(flat.rhs(p, y), plain.rhs(p, y))


def test_rates_conserve_elements_and_mass(pl):
    mech = pl.mech
    f = synth.field_bimodal("mech53pl", 2000, shuffle=True)
    for i, p in enumerate((0.3 * P_ATM, P_ATM, 20 * P_ATM)):
        kf, kr, q, om = pl.kinetics(f.T[i], p, f.Y[:, i])
        scale = np.abs(q).max() * 10
        np.testing.assert_allclose(mech.composition.T.astype(float) @ om, 0.0, atol=1e-12 * scale)
        np.testing.assert_allclose(mech.W @ om, 0.0, atol=1e-12 * scale * mech.W.max())


def test_jacobian_with_plog_matches_finite_differences(pl):
    f = synth.field_bimodal("mech53pl", 2000, shuffle=True)
    rng = np.random.default_rng(6)
    for i, p in enumerate((0.4 * P_ATM, 7 * P_ATM, 150 * P_ATM)):
        y = np.concatenate([[f.T[i]], f.Y[:, i]])
        J = pl.jac(p, y)
        v = rng.standard_normal(y.size) * np.abs(y) * 1e-4
        eps = 1e-3
        fd = (pl.rhs(p, y + eps * v) - pl.rhs(p, y - eps * v)) / (2 * eps)
        Jv = J @ v
        np.testing.assert_allclose(fd, Jv, rtol=1e-4, atol=1e-6 * np.abs(Jv).max())


def test_integration_invariants_with_plog(pl):
    mech = pl.mech
    f = synth.field_bimodal("mech53pl", 4000, shuffle=True)
    sub = synth.subsample(f, np.arange(9))
    p = P_ATM * np.array([0.05, 0.3, 1.0, 2.0, 5.0, 10.0, 50.0, 100.0, 400.0])
    T, Y, h, st, na, nr = pl.integrate_batch(sub.T, p, sub.Y, sub.dt, threads=8)
    assert np.all(st == 0)
    np.testing.assert_allclose(Y.sum(0), 1.0, atol=1e-13)
    E0 = (mech.composition.T / mech.W) @ sub.Y
    E1 = (mech.composition.T / mech.W) @ Y
    np.testing.assert_allclose(E1, E0, rtol=1e-12, atol=1e-15)
