"""Fall-off kinetics (Lindemann and Troe forms) on both integrators: 53 species
(one-wavefront kernel) and 64 species (workgroup kernel), with half of the
third-body reactions in fall-off form.  RHS and the analytic Jacobian against
the oracle's complex-step Jacobian, and a flow step of hot and cold cells
against the oracle under the three launch schedules (bit-identical to each
other)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle  # noqa: E402
from paper_2011_07978_amd import synth  # noqa: E402
from tests.test_gpu_boundary import test_flow_step_at_the_boundary as _flow  # noqa: E402
from tests.test_gpu_boundary import test_rhs_and_jacobian_at_the_boundary as _rhs  # noqa: E402

pytestmark = pytest.mark.gpu

MECHS = ["mech53fo", "mech64fo"]


def test_mechanisms_have_both_forms():
    for name in MECHS:
        m = synth.mechanism(name)
        assert (m.falloff == 1).sum() >= 8 and (m.falloff == 2).sum() >= 8


@pytest.mark.parametrize("name", MECHS)
def test_rhs_and_jacobian_with_falloff(name):
    _rhs(name)


@pytest.mark.parametrize("name", MECHS)
def test_flow_step_with_falloff(name):
    _flow(name)
