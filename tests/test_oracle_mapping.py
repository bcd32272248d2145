"""Pins of the oracle's reference mapping (paper Sec. 2.3).

The criterion Z_i < Z_tol and |T_i - T_ref| < T_tol with the first qualifying
cell as reference is checked on hand-built fields whose mixture fractions are
known by construction (Z is linear in Y, 0 for the oxidiser stream and 1 for
the fuel stream), including the degenerate cases.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_2011_07978_amd import synth


@pytest.fixture(scope="module")
def o53():
    return Oracle(synth.mechanism("mech53"))


def _mix(mech, s):
    """Cells mixing oxidiser (s = 0) and fuel (s = 1) streams; Z = s by linearity."""
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    s = np.asarray(s, float)
    return np.outer(Yo, 1.0 - s) + np.outer(Yf, s)


def test_stream_values_and_linearity(o53):
    mech = o53.mech
    w, bf, bo = o53.map_weights(synth.stream_fuel(mech), synth.stream_oxidiser(mech))
    assert bf > bo
    s = np.array([0.0, 1.0, 0.25, 0.5, 1e-3, -0.2, 1.7])
    Z = o53.mixture_fraction(_mix(mech, s), w, bf, bo)
    assert Z[0] == 0.0 and Z[1] == 1.0
    np.testing.assert_allclose(Z, s, atol=4e-16)


def test_element_definition(o53):
    """beta(Y) = sum_e c_e Z_e(Y) with c_e = (Z_e,fuel - Z_e,ox)/W_e."""
    mech = o53.mech
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    w, bf, bo = o53.map_weights(Yf, Yo)
    a = mech.composition.astype(float)
    We = mech.elem_mass

    def Ze(Y):
        return (a * We[None, :] * (Y / mech.W)[:, None]).sum(0)

    c = (Ze(Yf) - Ze(Yo)) / We
    rng = np.random.default_rng(1)
    for _ in range(5):
        Y = rng.dirichlet(np.full(mech.n_species, 0.5))
        assert abs(c @ Ze(Y) - w @ Y) <= 1e-14 * max(1.0, abs(w @ Y))


def _flags(o, mech, s, T, Z_tol, T_tol=1.0, use_T=False):
    Y = _mix(mech, s)
    return o.map_reference(np.asarray(T, float), Y, synth.stream_fuel(mech),
                           synth.stream_oxidiser(mech), Z_tol, T_tol, use_T)


def test_hand_built_fields(o53):
    mech = o53.mech
    s = [0.5, 0.0, 2e-5, 0.3, -1e-3, 5e-5, 0.9]
    T = [900, 400, 401, 700, 420, 399.5, 380]
    flags, ref = _flags(o53, mech, s, T, 1e-4)
    assert ref == 1
    assert flags.tolist() == [0, 1, 2, 0, 2, 2, 0]
    # with the temperature criterion (|T - T_ref| < 1 K, strict)
    flags, ref = _flags(o53, mech, s, T, 1e-4, T_tol=1.0, use_T=True)
    assert ref == 1
    assert flags.tolist() == [0, 1, 0, 0, 0, 2, 0]   # |401-400| = 1 is not < 1
    # no candidate at all
    flags, ref = _flags(o53, mech, [0.5, 0.2, 0.9], [900, 800, 700], 1e-4)
    assert ref == -1 and flags.tolist() == [0, 0, 0]
    # every cell a candidate: the first is the reference
    flags, ref = _flags(o53, mech, [0.0, 0.0, 1e-6, -0.5], [300, 310, 320, 330], 1e-4)
    assert ref == 0 and flags.tolist() == [1, 2, 2, 2]
    # empty field
    flags, ref = _flags(o53, mech, np.zeros(0), np.zeros(0), 1e-4)
    assert ref == -1 and flags.size == 0


def test_threshold_is_strict(o53):
    mech = o53.mech
    w, bf, bo = o53.map_weights(synth.stream_fuel(mech), synth.stream_oxidiser(mech))
    s = np.array([0.0, 3e-3, 1e-2])
    Z = o53.mixture_fraction(_mix(mech, s), w, bf, bo)
    flags, ref = _flags(o53, mech, s, [400, 400, 400], Z[1])       # Z_tol == Z_1 exactly
    assert ref == 0 and flags.tolist() == [1, 0, 0]
    flags, ref = _flags(o53, mech, s, [400, 400, 400], np.nextafter(Z[1], 1.0))
    assert flags.tolist() == [1, 2, 0]


def test_scatter_conserves_enthalpy(o53):
    mech = o53.mech
    f = synth.field_mapped(3000, seed=5)
    cold = np.nonzero(f.cls == 0)[0][:6]
    T, Y = f.T[cold].copy(), f.Y[:, cold].copy()
    flags = np.array([1, 2, 2, 2, 2, 0], np.uint8)
    rng = np.random.default_rng(2)
    dY = rng.standard_normal(mech.n_species) * 1e-6
    dY -= dY.mean()
    Yref_old = Y[:, 0].copy()
    Yref_new = Yref_old + dY
    T2, Y2 = o53.map_scatter(T, Y, flags, Yref_old, Yref_new)
    for i in range(6):
        if flags[i] != 2:
            assert T2[i] == T[i] and np.array_equal(Y2[:, i], Y[:, i])
            continue
        np.testing.assert_array_equal(Y2[:, i], Y[:, i] + (Yref_new - Yref_old))
        h0 = o53.enthalpy(T[i], Y[:, i])
        h1 = o53.enthalpy(T2[i], Y2[:, i])
        assert abs(h1 - h0) <= 1e-12 * o53.cp(T[i], Y[:, i]) * T[i]
    # zero increment leaves the cell untouched
    T3, Y3 = o53.map_scatter(T, Y, flags, Yref_old, Yref_old)
    np.testing.assert_allclose(T3, T, rtol=1e-15)


def test_failed_reference_is_not_copied(o53):
    """A mapped cell copies the reference's increment only when the
    reference's integration succeeded: with one attempted step allowed over a
    long dt the reference stops at the step limit (status 1), and the mapped
    cells keep their state with status 7; a reference with a bad input state
    (T <= 0, status 4) does the same."""
    mech = o53.mech
    f = synth.field_mapped(2000, seed=31)
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    flags, ref = o53.map_reference(f.T, f.Y, Yf, Yo, 1e-4)
    mapped = flags == 2
    assert ref >= 0 and mapped.sum() > 1000
    T, Y, _, st = o53.step_mapped(f.T, f.p, f.Y, 1e-2, flags, ref, max_steps=1)[:4]
    assert st[ref] == 1
    assert np.all(st[mapped] == 7)
    assert np.array_equal(T[mapped], f.T[mapped]) and np.array_equal(Y[:, mapped], f.Y[:, mapped])
    # the same field with a normal step maps every candidate (status 5)
    T, Y, _, st = o53.step_mapped(f.T, f.p, f.Y, 1e-6, flags, ref)[:4]
    assert st[ref] == 0 and np.all(st[mapped] == 5)
    assert not np.array_equal(Y[:, mapped], f.Y[:, mapped])
    # a reference with a bad input state
    Tb = f.T.copy()
    Tb[ref] = -1.0
    T, Y, _, st = o53.step_mapped(Tb, f.p, f.Y, 1e-6, flags, ref)[:4]
    assert st[ref] == 4 and np.all(st[mapped] == 7)
    assert np.array_equal(Y[:, mapped], f.Y[:, mapped])
