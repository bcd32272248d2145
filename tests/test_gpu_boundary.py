"""Both sides of the size boundary between the two integrators: 63 species
(n = 64, the largest the one-wavefront kernel takes, 64-row register LU) and
64 species (n = 65, the smallest the workgroup kernel takes, LDS matrix and
blocked MFMA LU).  RHS and Jacobian against the oracle's complex-step
Jacobian, and a flow step of hot and cold cells against the oracle, under the
three launch schedules (bit-identical to each other)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle  # noqa: E402
from paper_2011_07978_amd import synth  # noqa: E402
from paper_2011_07978_amd.chem import (CHEM_SCHED_BLOCKS, CHEM_SCHED_PLAIN,  # noqa: E402
                                       CHEM_SCHED_QUEUE)

pytestmark = pytest.mark.gpu

MECHS = ["mech63", "mech64"]


def _cells(name, n_hot, n_cold):
    f = synth.field_bimodal(name, 1000, seed=21)
    idx = np.concatenate([np.arange(n_hot), 1000 - 1 - np.arange(n_cold)])
    return synth.subsample(f, idx)


@pytest.mark.parametrize("name", MECHS)
def test_rhs_and_jacobian_at_the_boundary(name):
    from tests.gpu_util import chem_for, dev, host, say
    mech = synth.mechanism(name)
    f = _cells(name, 12, 12)
    o = Oracle(mech)
    c = chem_for(mech)
    n, nn = f.n_cells, mech.n_species + 1
    say("boundary rhs_jac", name, n)
    fd = torch.zeros(n * nn, dtype=torch.float64, device="cuda")
    J = torch.zeros(n * nn * nn, dtype=torch.float64, device="cuda")
    c.eval_rhs_jac(dev(f.T), dev(f.p), dev(f.Y), fd, J)
    torch.cuda.synchronize()
    fd = host(fd).reshape(n, nn)
    J = host(J).reshape(n, nn, nn)
    from tests.gpu_util import check_rhs_jac
    check_rhs_jac(o, mech, f, fd, J, "boundary " + name)


@pytest.mark.parametrize("name", MECHS)
def test_flow_step_at_the_boundary(name):
    from tests.gpu_util import chem_for, compare_to_oracle, run_integrate, say
    mech = synth.mechanism(name)
    f = _cells(name, 16, 32)
    o = Oracle(mech)
    ref = o.integrate_batch(f.T, f.p, f.Y, f.dt, threads=16, schedule=1)
    assert np.all(ref[3] == 0)
    c = chem_for(mech)
    outs = []
    for sched in (CHEM_SCHED_QUEUE, CHEM_SCHED_PLAIN, CHEM_SCHED_BLOCKS):
        say("boundary integrate", name, f.n_cells, "schedule", sched)
        out = run_integrate(c, f, schedule=sched)
        assert np.all(out["status"] == 0)
        rep = compare_to_oracle(out, ref[0], ref[1], ref[4], ref[5])
        print(name, sched, rep, out["stats"])
        assert rep["ok"], rep
        assert rep["step_sequence_differs"] <= 2
        outs.append(out)
    for other in outs[1:]:
        assert np.array_equal(outs[0]["T"], other["T"]) and np.array_equal(outs[0]["Y"], other["Y"])
