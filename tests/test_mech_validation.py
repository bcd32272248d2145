"""Mechanism validation of the boundary (chem_validate_mechanism, the check
chem_set_mechanism runs before it uploads anything): the rejections the
mechanism description promises, on the host, without a GPU."""
import copy

import numpy as np
import pytest

from paper_2011_07978_amd import chem, synth

OK, BAD_ARG, BAD_MECH = 0, -1, -7


@pytest.fixture(scope="module")
def base():
    return synth.mechanism("mech53")


def broken(m, **kw):
    b = copy.deepcopy(m)
    for k, v in kw.items():
        setattr(b, k, v)
    return b


def check(m, code, words):
    rc, why = chem.validate_mechanism(m)
    assert rc == code, (rc, why)
    for w in words:
        assert w in why, why


@pytest.mark.parametrize("name", ["small", "mech53", "mech53fo", "mech53pl", "mech130"])
def test_generated_mechanisms_pass(name):
    rc, why = chem.validate_mechanism(synth.mechanism(name))
    assert rc == OK and why == ""


def test_element_unbalanced_reaction(base):
    j = 17
    prod = base.products.copy()
    # swap one product for a species of different composition
    k = int(prod[j, 0])
    other = next(q for q in range(base.n_species)
                 if not np.array_equal(base.composition[q], base.composition[k]))
    prod[j, 0] = other
    check(broken(base, products=prod), BAD_MECH, ["reaction 17", "unbalanced"])


def test_molar_mass_inconsistent_with_composition(base):
    W = base.W.copy()
    W[5] *= 1.0 + 1e-6
    check(broken(base, W=W), BAD_MECH, ["species 5", "W inconsistent"])
    W = base.W.copy()
    W[2] = -W[2]
    check(broken(base, W=W), BAD_MECH, ["species 2"])


def test_negative_heat_capacity(base):
    nasa = base.nasa.copy()
    # cp/R = a1 + a2 T + ...: a large negative a2 makes cp negative at high T
    nasa[3, 1] = -1e-2
    check(broken(base, nasa=nasa), BAD_MECH, ["species 3", "cp <= 0"])
    nasa = base.nasa.copy()
    nasa[4, 0] = -10.0
    check(broken(base, nasa=nasa), BAD_MECH, ["species 4", "cp <= 0 at 200 K"])


def test_size_limits(base):
    check(broken(base, n_species=161), BAD_MECH, ["N=161"])
    check(broken(base, n_reactions=4097), BAD_MECH, ["R=4097"])
    check(broken(base, n_species=0), BAD_MECH, ["N=0"])
    check(broken(base, n_elements=17), BAD_MECH, ["E=17"])


def test_rate_parameters_and_indices(base):
    A = base.A.copy()
    A[9] = 0.0
    check(broken(base, A=A), BAD_MECH, ["reaction 9", "rate parameters"])
    Ea = base.Ea.copy()
    Ea[10] = np.nan
    check(broken(base, Ea=Ea), BAD_MECH, ["reaction 10"])
    rea = base.reactants.copy()
    rea[3, 0] = base.n_species
    check(broken(base, reactants=rea), BAD_MECH, ["reaction 3", "bad reactant"])
    rea = base.reactants.copy()
    rea[4, :] = -1
    check(broken(base, reactants=rea), BAD_MECH, ["reaction 4", "empty side"])


def test_efficiency_rules(base):
    plain = int(np.nonzero(base.third_body == 0)[0][0])
    er = base.eff_reaction.copy()
    er[0] = plain
    check(broken(base, eff_reaction=er), BAD_MECH, ["efficiency 0"])
    # a species listed twice for one reaction
    er = np.concatenate([base.eff_reaction, base.eff_reaction[:1]]).astype(np.int32)
    es = np.concatenate([base.eff_species, base.eff_species[:1]]).astype(np.int32)
    ev = np.concatenate([base.eff_value, base.eff_value[:1]])
    check(broken(base, eff_reaction=er, eff_species=es, eff_value=ev), BAD_MECH, ["duplicate"])


def test_falloff_and_plog_rules():
    fo = synth.mechanism("mech53fo")
    plain = int(np.nonzero(fo.third_body == 0)[0][0])
    t = fo.falloff.copy()
    t[plain] = 2
    check(broken(fo, falloff=t), BAD_MECH, [f"reaction {plain}", "fall-off"])
    pl = synth.mechanism("mech53pl")
    j = int(np.nonzero(pl.plog_count)[0][0])
    P = pl.plog_params.copy()
    P[j, 1, 0] = P[j, 0, 0]            # pressures not strictly increasing
    check(broken(pl, plog_params=P), BAD_MECH, [f"reaction {j}", "PLOG"])
    c = pl.plog_count.copy()
    c[j] = 9
    check(broken(pl, plog_count=c), BAD_MECH, [f"reaction {j}", "PLOG"])
