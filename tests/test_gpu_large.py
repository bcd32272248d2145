"""Large-mechanism path (130 species, 1000 reactions; 131 unknowns): the
workgroup-per-cell kernel with the iteration matrix in LDS and the blocked LU
on the FP64 matrix cores, against the CPU oracle at the same bar as the
wavefront kernel: rates and Jacobian, one fixed Rodas4 step, and adaptive
integration of flame-field cells (|dT|/T <= 1e-6, |dY| <= 1e-8)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle  # noqa: E402
from paper_2011_07978_amd import synth  # noqa: E402
from paper_2011_07978_amd.chem import CHEM_SCHED_BLOCKS, CHEM_SCHED_PLAIN, CHEM_SCHED_QUEUE  # noqa: E402

pytestmark = pytest.mark.gpu


def _cells(n_hot, n_cold, seed=104):
    f = synth.field_bimodal("mech130", 16384, seed=seed, dt=2e-6)
    n_h = 16384 // 10
    idx = np.r_[np.arange(0, n_h)[:: n_h // n_hot][:n_hot],
                np.arange(n_h, 16384)[:: (16384 - n_h) // n_cold][:n_cold]]
    return synth.subsample(f, idx)


@pytest.fixture(scope="module")
def mech():
    return synth.mechanism("mech130")


def test_rhs_and_jacobian_match_oracle(mech):
    from tests.gpu_util import chem_for, dev, host, say
    f = _cells(12, 12)
    o = Oracle(mech)
    c = chem_for(mech)
    n, nn = f.n_cells, mech.n_species + 1
    say("large rhs_jac", n)
    fv = torch.zeros(n * nn, dtype=torch.float64, device="cuda")
    J = torch.zeros(n * nn * nn, dtype=torch.float64, device="cuda")
    c.eval_rhs_jac(dev(f.T), dev(f.p), dev(f.Y), fv, J)
    torch.cuda.synchronize()
    fv = host(fv).reshape(n, nn)
    J = host(J).reshape(n, nn, nn)
    from tests.gpu_util import check_rhs_jac
    check_rhs_jac(o, mech, f, fv, J, "mech130")


def test_single_rodas_step_matches_oracle(mech):
    from tests.gpu_util import chem_for, dev, host, say
    f = _cells(8, 8)
    o = Oracle(mech)
    c = chem_for(mech)
    n, nn = f.n_cells, mech.n_species + 1
    for hstep in (1e-12, 1e-9, 1e-7):
        say("large rodas_step", n, hstep)
        yn = torch.zeros(n * nn, dtype=torch.float64, device="cuda")
        er = torch.zeros(n * nn, dtype=torch.float64, device="cuda")
        c.rodas_step(dev(f.T), dev(f.p), dev(f.Y), hstep, yn, er)
        torch.cuda.synchronize()
        yn = host(yn).reshape(n, nn)
        er = host(er).reshape(n, nn)
        worst = 0.0
        for i in range(n):
            y = np.concatenate([[f.T[i]], f.Y[:, i]])
            yo, eo, rc = o.rodas4_step(f.p[i], y, hstep)
            assert rc == 0
            if not np.all(np.isfinite(yo)):
                continue
            Mo = np.eye(nn) / (0.25 * hstep) - o.jac(f.p[i], y)
            bound = max(1e-12, 4 * 2.2e-16 * np.linalg.cond(Mo))
            scale = np.abs(y) + np.abs(yo) + 1e-12
            r_y = np.max(np.abs(yn[i] - yo) / scale) / bound
            r_e = np.max(np.abs(er[i] - eo) / scale) / bound
            worst = max(worst, r_y, r_e)
        print("large rodas step", hstep, "worst / bound", worst)
        assert worst <= 1.0


def test_flame_cells_match_oracle_and_schedules_agree(mech):
    from tests.gpu_util import chem_for, compare_to_oracle, run_integrate, say
    f = _cells(16, 48)
    o = Oracle(mech)
    ref = o.integrate_batch(f.T, f.p, f.Y, f.dt, threads=16, schedule=1)
    assert np.all(ref[3] == 0)
    c = chem_for(mech)
    outs = []
    for sched in (CHEM_SCHED_QUEUE, CHEM_SCHED_PLAIN, CHEM_SCHED_BLOCKS):
        say("large integrate", f.n_cells, "schedule", sched)
        out = run_integrate(c, f, schedule=sched)
        assert np.all(out["status"] == 0)
        rep = compare_to_oracle(out, ref[0], ref[1], ref[4], ref[5])
        print(rep, out["stats"])
        assert rep["ok"], rep
        assert rep["step_sequence_differs"] <= 2
        outs.append(out)
    for o in outs[1:]:
        assert np.array_equal(outs[0]["T"], o["T"]) and np.array_equal(outs[0]["Y"], o["Y"])
