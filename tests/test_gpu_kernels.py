"""Kernel-level parity of the HIP path with the CPU oracle: rates/RHS, the
analytic Jacobian and one fixed-size Rodas4 step."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle  # noqa: E402
from paper_2011_07978_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _fields():
    return [("small", synth.field_small(300)),
            ("mech53", synth.subsample(synth.field_mapped(30000, seed=11),
                                       np.arange(0, 30000, 97)))]


@pytest.mark.parametrize("name,field", _fields())
def test_rhs_and_jacobian_match_oracle(name, field):
    """Per component, against the rounding scale of the log-space rate
    evaluation (tests.gpu_util.check_rhs_jac)."""
    from tests.gpu_util import check_rhs_jac, chem_for, dev, host, say
    mech = synth.mechanism(name)
    o = Oracle(mech)
    c = chem_for(mech)
    n, nn = field.n_cells, mech.n_species + 1
    say("rhs_jac", name, n)
    f = torch.zeros(n * nn, dtype=torch.float64, device="cuda")
    J = torch.zeros(n * nn * nn, dtype=torch.float64, device="cuda")
    c.eval_rhs_jac(dev(field.T), dev(field.p), dev(field.Y), f, J)
    torch.cuda.synchronize()
    check_rhs_jac(o, mech, field, host(f).reshape(n, nn), host(J).reshape(n, nn, nn), name)


@pytest.mark.parametrize("name,field", _fields())
def test_single_rodas_step_matches_oracle(name, field):
    from tests.gpu_util import chem_for, dev, host, say
    mech = synth.mechanism(name)
    o = Oracle(mech)
    c = chem_for(mech)
    n, nn = field.n_cells, mech.n_species + 1
    for hstep in (1e-12, 1e-9, 1e-7):
        say("rodas_step", name, n, hstep)
        yn = torch.zeros(n * nn, dtype=torch.float64, device="cuda")
        er = torch.zeros(n * nn, dtype=torch.float64, device="cuda")
        c.rodas_step(dev(field.T), dev(field.p), dev(field.Y), hstep, yn, er)
        torch.cuda.synchronize()
        yn = host(yn).reshape(n, nn)
        er = host(er).reshape(n, nn)
        worst = 0.0
        for i in range(n):
            y = np.concatenate([[field.T[i]], field.Y[:, i]])
            yo, eo, rc = o.rodas4_step(field.p[i], y, hstep)
            assert rc == 0
            if not np.all(np.isfinite(yo)):
                continue
            # one step solves six systems with M = I/(gamma h) - J; a backward-
            # stable solve has a forward error of at most about cond(M) eps
            # (growth factor ~1 with partial pivoting), once on each side; the
            # 4 covers the two sides and the stage sums (worst cells measured
            # at 0.2 of this bound)
            Mo = np.eye(nn) / (0.25 * hstep) - o.jac(field.p[i], y)
            bound = max(1e-12, 4 * 2.2e-16 * np.linalg.cond(Mo))
            scale = np.abs(y) + np.abs(yo) + 1e-12
            r_y = np.max(np.abs(yn[i] - yo) / scale) / bound
            # the error estimate is the last stage's solution: per component, to
            # the same bound on the same scale
            r_e = np.max(np.abs(er[i] - eo) / scale) / bound
            worst = max(worst, r_y, r_e)
        print("rodas step", name, hstep, "worst / bound", worst)
        assert worst <= 1.0
