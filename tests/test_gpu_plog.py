"""Tabulated pressure dependence (PLOG) on both integrators: 53 species
(one-wavefront kernel) and 64 species (workgroup kernel), with PLOG tables on a
fifth of the reactions without a third body and fall-off on half of the
third-body reactions.  The cells sit at pressures from 0.05 to 400 atm, below,
inside and above the tables (0.1 to 100 atm).  RHS and analytic Jacobian
against the oracle's complex-step Jacobian, a flow step against the oracle
under the three launch schedules (bit-identical to each other), and invalid
tables refused by chem_set_mechanism."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle  # noqa: E402
from paper_2011_07978_amd import synth  # noqa: E402
from paper_2011_07978_amd.chem import (CHEM_SCHED_BLOCKS, CHEM_SCHED_PLAIN,  # noqa: E402
                                       CHEM_SCHED_QUEUE)

pytestmark = pytest.mark.gpu

MECHS = ["mech53pl", "mech64pl"]
P_SET = synth.P_ATM * np.array([0.05, 0.1, 0.3, 1.0, 3.0, 10.0, 30.0, 100.0, 400.0])


def _cells(name, n_hot, n_cold, seed, hot_max=None):
    """Hot and cold cells of the bimodal field at pressures from P_SET (hot
    cells up to hot_max: a hot cell far above the field's own pressure may
    leave the solver's step-size range on both sides alike)."""
    f = synth.field_bimodal(name, 1000, seed=21)
    idx = np.concatenate([np.arange(n_hot), 1000 - 1 - np.arange(n_cold)])
    sub = synth.subsample(f, idx)
    rng = np.random.default_rng(seed)
    hot = P_SET if hot_max is None else P_SET[P_SET <= hot_max]
    p = np.concatenate([rng.permutation(np.resize(hot, n_hot)),
                        rng.permutation(np.resize(P_SET, n_cold))])
    return dataclasses.replace(sub, p=p)


@pytest.mark.parametrize("name", MECHS)
def test_rhs_and_jacobian_with_plog(name):
    from tests.gpu_util import chem_for, dev, host, say
    mech = synth.mechanism(name)
    f = _cells(name, 12, 15, 1)
    o = Oracle(mech)
    c = chem_for(mech)
    n, nn = f.n_cells, mech.n_species + 1
    say("plog rhs_jac", name, n)
    fd = torch.zeros(n * nn, dtype=torch.float64, device="cuda")
    J = torch.zeros(n * nn * nn, dtype=torch.float64, device="cuda")
    c.eval_rhs_jac(dev(f.T), dev(f.p), dev(f.Y), fd, J)
    torch.cuda.synchronize()
    fd = host(fd).reshape(n, nn)
    J = host(J).reshape(n, nn, nn)
    from tests.gpu_util import check_rhs_jac
    check_rhs_jac(o, mech, f, fd, J, "plog " + name)


@pytest.mark.parametrize("name", MECHS)
def test_flow_step_with_plog(name):
    from tests.gpu_util import chem_for, compare_to_oracle, run_integrate, say
    mech = synth.mechanism(name)
    f = _cells(name, 10, 18, 2, hot_max=10 * synth.P_ATM)
    o = Oracle(mech)
    ref = o.integrate_batch(f.T, f.p, f.Y, f.dt, threads=16, schedule=1)
    assert np.all(ref[3] == 0)
    c = chem_for(mech)
    outs = []
    for sched in (CHEM_SCHED_QUEUE, CHEM_SCHED_PLAIN, CHEM_SCHED_BLOCKS):
        say("plog integrate", name, f.n_cells, "schedule", sched)
        out = run_integrate(c, f, schedule=sched)
        assert np.all(out["status"] == 0)
        rep = compare_to_oracle(out, ref[0], ref[1], ref[4], ref[5])
        print(name, sched, rep, out["stats"])
        assert rep["ok"], rep
        assert rep["step_sequence_differs"] <= 2
        outs.append(out)
    for other in outs[1:]:
        assert np.array_equal(outs[0]["T"], other["T"]) and np.array_equal(outs[0]["Y"], other["Y"])


def test_bad_plog_tables_are_rejected():
    from paper_2011_07978_amd.chem import Chem, ChemError
    from tests.gpu_util import say
    base = synth.mechanism("mech53pl")
    j = int(np.nonzero(base.plog_count >= 3)[0][0])
    j_tb = int(np.nonzero(base.third_body == 1)[0][0])
    cases = []
    for cnt in (1, 9):                                            # too few / too many entries
        t = base.plog_count.copy(); t[j] = cnt
        cases.append(dataclasses.replace(base, plog_count=t))
    t = base.plog_count.copy(); t[j_tb] = 2                        # on a third-body reaction
    prm = base.plog_params.copy(); prm[j_tb, :2] = base.plog_params[j, :2]
    cases.append(dataclasses.replace(base, plog_count=t, plog_params=prm))
    for (i, col, v) in ((1, 0, None), (0, 0, 0.0), (0, 1, -1.0), (2, 3, np.nan)):
        prm = base.plog_params.copy()
        prm[j, i, col] = prm[j, i - 1, 0] if v is None else v     # pressures not increasing, p <= 0, A <= 0, NaN
        cases.append(dataclasses.replace(base, plog_params=prm))
    cases.append(dataclasses.replace(base, plog_params=None))      # table missing
    for i, m in enumerate(cases):
        say("bad PLOG case", i)
        c = Chem(0)
        with pytest.raises(ChemError):
            c.set_mechanism(m)
    Chem(0).set_mechanism(base)                                    # the valid one loads
