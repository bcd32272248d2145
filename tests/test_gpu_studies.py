"""The load-balancing benchmark (Sec. 3) and the mapping study (App. A) run
end to end through the public calls on small sizes."""
import math

import pytest

torch = pytest.importorskip("torch")

from paper_2011_07978_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


def test_unit_benchmark_small():
    from paper_2011_07978_amd import studies
    from paper_2011_07978_amd.chem import Chem
    from tests.gpu_util import say
    mech = synth.mechanism("mech53")
    c = Chem(0)
    c.set_mechanism(mech)
    say("unit benchmark C1/C4, 4 problems per slot")
    res = studies.unit_benchmark(c, torch, synth, mech, n_per_slot=4, reps=1, layouts=("C1", "C4"))
    assert res["slots"] >= 256
    for name in ("C1", "C4"):
        r = res["layouts"][name]
        assert r["cells"] == res["slots"] * 4
        assert r["xi_attempts"] > 1.0
        for k in ("ms_unbalanced_blocks", "ms_balanced_queue", "chi_su", "chi_su_bound"):
            assert math.isfinite(r[k]) and r[k] > 0.0, (name, k)
    assert res["layouts"]["C4"]["chi_su_bound"] == pytest.approx(1.0, rel=1e-12)


def test_mapping_study_small():
    from paper_2011_07978_amd import studies
    from paper_2011_07978_amd.chem import Chem
    from tests.gpu_util import say
    mech = synth.mechanism("mech53")
    c = Chem(0)
    c.set_mechanism(mech)
    say("mapping study 4096 cells, 2 steps")
    res = studies.mapping_study(c, torch, synth, mech, n_cells=4096, steps=2, z_tols=(1e-2, 1e-6))
    runs = {(r["Z_tol"], r["use_T"]): r for r in res["runs"]}
    assert runs[(1e-2, False)]["mapped_per_step"] >= runs[(1e-6, False)]["mapped_per_step"]
    assert runs[(1e-2, False)]["mapped_per_step"] > 0
    for r in res["runs"]:
        assert math.isfinite(r["mean_abs_dT"]) and math.isfinite(r["heat_release_rel_err"])
