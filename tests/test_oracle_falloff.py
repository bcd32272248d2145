"""Pins of the oracle's fall-off kinetics (Lindemann and Troe forms).

The fall-off factor G multiplies the high-pressure rate constant, G = Pr/(1+Pr) F
with Pr = k0 [M] / k_inf.  Pinned against its limits (low pressure: k -> k0 [M];
high pressure: k -> k_inf), Troe's broadening F between Fcent and 1, the centre of the
Troe curve (log10 Pr = -c makes f1 = 0, so F = Fcent), the two points of half
broadening (f1 = +-1, solved by hand), Fcent = 1 reducing Troe
to Lindemann, monotonicity in [M], and through the whole
right-hand side: central finite differences of the complex-step Jacobian,
element and mass conservation, and the invariants of an integration."""
import numpy as np
import pytest

from oracle import Oracle
from paper_2011_07978_amd import synth

RU_J = 8.314462618


@pytest.fixture(scope="module")
def fo():
    return Oracle(synth.mechanism("mech53fo"))


def _kinf_k0(mech, j, T):
    kinf = mech.A[j] * T ** mech.b[j] * np.exp(-mech.Ea[j] / (RU_J * T))
    A0, b0, E0 = mech.fo_params[j, :3]
    return kinf, A0 * T ** b0 * np.exp(-E0 / (RU_J * T))


def _reactions(mech, kind):
    return np.nonzero(mech.falloff == kind)[0]


def test_lindemann_limits(fo):
    mech = fo.mech
    for j in _reactions(mech, 1)[:6]:
        for T in (400.0, 1500.0):
            kinf, k0 = _kinf_k0(mech, j, T)
            Mlo = 1e-12 * kinf / k0          # Pr = 1e-12
            assert fo.falloff_factor(j, T, Mlo) * kinf == pytest.approx(k0 * Mlo, rel=1e-10)
            Mhi = 1e12 * kinf / k0           # Pr = 1e12
            assert fo.falloff_factor(j, T, Mhi) == pytest.approx(1.0, rel=1e-10)
            M1 = kinf / k0                   # Pr = 1: G = 1/2
            assert fo.falloff_factor(j, T, M1) == pytest.approx(0.5, rel=1e-12)


def _fcent(mech, j, T):
    a, T3, T1, T2 = mech.fo_params[j, 3:]
    return (1 - a) * np.exp(-T / T3) + a * np.exp(-T / T1) + (np.exp(-T2 / T) if T2 > 0 else 0.0)


def test_troe_centre_and_limits(fo):
    mech = fo.mech
    js = _reactions(mech, 2)
    assert js.size >= 4
    for j in js[:8]:
        for T in (500.0, 1200.0, 2500.0):
            kinf, k0 = _kinf_k0(mech, j, T)
            Fc = _fcent(mech, j, T)
            c = -0.4 - 0.67 * np.log10(Fc)
            Pr = 10.0 ** (-c)                # f1 = 0 there: F = Fcent
            G = fo.falloff_factor(j, T, Pr * kinf / k0)
            assert G == pytest.approx(Pr / (1 + Pr) * Fc, rel=1e-12)
            # log10 F = log10 Fcent / (1 + f1^2): F lies between Fcent and 1
            # at every pressure
            for e in np.linspace(-6, 6, 25):
                P = 10.0 ** e
                F = fo.falloff_factor(j, T, P * kinf / k0) / (P / (1 + P))
                assert Fc * (1 - 1e-12) <= F <= 1.0 + 1e-12


def test_troe_half_broadening_points(fo):
    """Where the broadening is half its centre value (log10 F = log10 Fcent / 2)
    the Troe form has f1 = +-1, which, solved by hand for x = log10 Pr + c,
    gives x = n / (1 + d) above the centre and x = -n / (1 - d) below it
    (d = 0.14): the curve is narrower on the high-pressure side.  Both points
    are found by bisection on the oracle's fall-off factor and compared with
    these closed forms, which pins the centre c, the width n and the
    asymmetry d together."""
    mech = fo.mech
    d = 0.14
    checked = 0
    for j in _reactions(mech, 2)[:8]:
        for T in (500.0, 1200.0, 2500.0):
            kinf, k0 = _kinf_k0(mech, j, T)
            Fc = _fcent(mech, j, T)
            if not (1e-3 < Fc < 0.9):
                continue
            lFc = np.log10(Fc)
            c, n = -0.4 - 0.67 * lFc, 0.75 - 1.27 * lFc

            def phi(x):   # log10 F / log10 Fcent at log10 Pr = x - c
                P = 10.0 ** (x - c)
                F = fo.falloff_factor(j, T, P * kinf / k0) / (P / (1 + P))
                return np.log10(F) / lFc

            def half(lo, hi):   # phi(lo) > 1/2 > phi(hi), phi monotone between
                for _ in range(200):
                    mid = 0.5 * (lo + hi)
                    if phi(mid) > 0.5:
                        lo = mid
                    else:
                        hi = mid
                return 0.5 * (lo + hi)

            x_up = half(0.0, 0.99 * n / d)
            x_dn = half(0.0, -20.0)
            assert x_up == pytest.approx(n / (1 + d), rel=1e-9, abs=1e-10)
            assert x_dn == pytest.approx(-n / (1 - d), rel=1e-9, abs=1e-10)
            checked += 1
    assert checked >= 4


def test_troe_with_unit_fcent_is_lindemann():
    """a = 1, T1 huge and no T2 term: Fcent = exp(-T/T1) = 1 to rounding, so
    log10 F = 0 at every pressure and Troe's form equals Lindemann's."""
    import dataclasses
    base = synth.mechanism("mech53fo")
    prm = base.fo_params.copy()
    js = _reactions(base, 2)
    prm[js, 3] = 1.0
    prm[js, 5] = 1e300
    prm[js, 6] = 0.0
    o = Oracle(dataclasses.replace(base, fo_params=prm))
    for j in js[:8]:
        for T in (600.0, 2000.0):
            kinf, k0 = _kinf_k0(base, j, T)
            for Pr in (1e-3, 0.3, 1.0, 50.0):
                G = o.falloff_factor(j, T, Pr * kinf / k0)
                assert G == pytest.approx(Pr / (1 + Pr), rel=1e-12)


@pytest.mark.parametrize("kind", [1, 2])
def test_rate_grows_with_third_body(fo, kind):
    mech = fo.mech
    for j in _reactions(mech, kind)[:6]:
        for T in (400.0, 1800.0):
            kinf, k0 = _kinf_k0(mech, j, T)
            G = [fo.falloff_factor(j, T, 10.0 ** e * kinf / k0) for e in np.linspace(-4, 4, 33)]
            assert np.all(np.diff(G) > 0)


def test_rates_conserve_elements_and_mass(fo):
    mech = fo.mech
    f = synth.field_bimodal("mech53fo", 2000, shuffle=True)
    for i in range(6):
        kf, kr, q, om = fo.kinetics(f.T[i], f.p[i], f.Y[:, i])
        scale = np.abs(q).max() * 10
        np.testing.assert_allclose(mech.composition.T.astype(float) @ om, 0.0, atol=1e-12 * scale)
        np.testing.assert_allclose(mech.W @ om, 0.0, atol=1e-12 * scale * mech.W.max())


def test_jacobian_with_falloff_matches_finite_differences(fo):
    f = synth.field_bimodal("mech53fo", 2000, shuffle=True)
    rng = np.random.default_rng(5)
    for i in range(3):
        y = np.concatenate([[f.T[i]], f.Y[:, i]])
        J = fo.jac(f.p[i], y)            # complex step for fall-off mechanisms
        v = rng.standard_normal(y.size) * np.abs(y) * 1e-4
        eps = 1e-3
        fd = (fo.rhs(f.p[i], y + eps * v) - fo.rhs(f.p[i], y - eps * v)) / (2 * eps)
        Jv = J @ v
        np.testing.assert_allclose(fd, Jv, rtol=1e-4, atol=1e-6 * np.abs(Jv).max())


def test_integration_invariants_with_falloff(fo):
    mech = fo.mech
    f = synth.field_bimodal("mech53fo", 4000, shuffle=True)
    sub = synth.subsample(f, np.arange(10))
    T, Y, h, st, na, nr = fo.integrate_batch(sub.T, sub.p, sub.Y, sub.dt, threads=8)
    assert np.all(st == 0)
    np.testing.assert_allclose(Y.sum(0), 1.0, atol=1e-13)
    E0 = (mech.composition.T / mech.W) @ sub.Y
    E1 = (mech.composition.T / mech.W) @ Y
    np.testing.assert_allclose(E1, E0, rtol=1e-12, atol=1e-15)
