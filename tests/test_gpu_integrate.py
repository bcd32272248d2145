"""Integration parity of the HIP path with the CPU oracle.

Bar: |dT|/T <= 1e-6 and |dY| <= 1e-8 per cell at rtol 1e-8, atol 1e-12; the
static launch and the work-queue launch agree bit for bit (the load balancer
changes where a cell runs, never what it computes); mapping flags are exact."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle  # noqa: E402
from paper_2011_07978_amd import synth  # noqa: E402
from paper_2011_07978_amd.chem import CHEM_SCHED_BLOCKS, CHEM_SCHED_PLAIN, CHEM_SCHED_QUEUE  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small_case():
    mech = synth.mechanism("small")
    f = synth.field_small(4096)
    o = Oracle(mech)
    ref = o.integrate_batch(f.T, f.p, f.Y, f.dt, threads=16)
    return mech, f, ref


def _flame_subset(n_hot=48, n_cold=80):
    f = synth.field_bimodal("mech53", 65536)
    idx = np.r_[np.arange(0, 6553)[:: 6553 // n_hot][:n_hot],
                np.arange(6553, 65536)[:: (65536 - 6553) // n_cold][:n_cold]]
    return synth.subsample(f, idx)


@pytest.fixture(scope="module")
def flame_case():
    mech = synth.mechanism("mech53")
    f = _flame_subset()
    o = Oracle(mech)
    ref = o.integrate_batch(f.T, f.p, f.Y, f.dt, threads=16, schedule=1)
    return mech, f, ref


@pytest.mark.parametrize("schedule", [CHEM_SCHED_PLAIN, CHEM_SCHED_QUEUE])
def test_small_mechanism_full_field(small_case, schedule):
    from tests.gpu_util import chem_for, compare_to_oracle, say
    mech, f, ref = small_case
    say("integrate small 4096 cells schedule", schedule)
    from tests.gpu_util import run_integrate
    c = chem_for(mech)
    out = run_integrate(c, f, schedule=schedule)
    assert np.all(out["status"] == 0)
    assert np.all(ref[3] == 0)
    rep = compare_to_oracle(out, ref[0], ref[1], ref[4], ref[5])
    print(rep)
    assert rep["ok"], rep
    assert rep["step_sequence_differs"] <= f.n_cells // 100
    s = out["stats"]
    assert s["cells_integrated"] == f.n_cells and s["cells_failed"] == 0
    assert s["steps_accepted"] == int(out["nacc"].sum())
    assert s["steps_rejected"] == int(out["nrej"].sum())


def test_flame_cells_match_oracle(flame_case):
    from tests.gpu_util import chem_for, compare_to_oracle, run_integrate, say
    mech, f, ref = flame_case
    say("integrate flame subset", f.n_cells)
    c = chem_for(mech)
    out = run_integrate(c, f, schedule=CHEM_SCHED_QUEUE)
    assert np.all(out["status"] == 0)
    rep = compare_to_oracle(out, ref[0], ref[1], ref[4], ref[5])
    print(rep)
    assert rep["ok"], rep
    np.testing.assert_allclose(out["h"], ref[2], rtol=1e-3)


def test_plain_and_queue_bitwise_identical():
    """Paper App. A: balancing without mapping gives results identical to the
    standard model.  Here: the queue launch equals the static launches (one
    cell per workgroup, and one contiguous block per slot) bit for bit."""
    from tests.gpu_util import chem_for, dev, host, say
    mech = synth.mechanism("mech53")
    f = synth.field_bimodal("mech53", 4096, seed=77, shuffle=True)
    c = chem_for(mech)
    outs = []
    for sched, chunk in ((CHEM_SCHED_PLAIN, 0), (CHEM_SCHED_QUEUE, 1), (CHEM_SCHED_QUEUE, 4),
                         (CHEM_SCHED_BLOCKS, 0)):
        say("bitwise", sched, chunk)
        c.set_options(schedule=sched, queue_chunk=chunk)
        T, Y = dev(f.T), dev(f.Y)
        cost = torch.zeros(f.n_cells, dtype=torch.int32, device="cuda")
        if sched == CHEM_SCHED_QUEUE:
            # a heavy-first order from a previous call's cost
            cost = dev(np.random.default_rng(1).integers(0, 5000, f.n_cells), torch.int32)
        c.integrate(T, dev(f.p), Y, f.dt, cost=cost)
        torch.cuda.synchronize()
        outs.append((host(T), host(Y)))
    for T, Y in outs[1:]:
        assert np.array_equal(T, outs[0][0])
        assert np.array_equal(Y, outs[0][1])


def test_static_blocks_cover_every_cell_once():
    """The static-partition launch (each slot owns a contiguous block) integrates
    every non-mapped cell exactly once, also when the cell count is not a
    multiple of the slot count and when there are fewer cells than slots."""
    from tests.gpu_util import chem_for, run_integrate, say
    mech = synth.mechanism("small")
    for n in (5000, 37, 1):
        f = synth.field_small(n)
        c = chem_for(mech, schedule=CHEM_SCHED_BLOCKS)
        say("static blocks", n)
        out = run_integrate(c, f)
        assert out["stats"]["cells_integrated"] == n
        assert np.array_equal(out["cost"].cpu().numpy(), out["nacc"] + out["nrej"])
        ref = run_integrate(chem_for(mech, schedule=CHEM_SCHED_QUEUE), f)
        assert np.array_equal(out["T"], ref["T"]) and np.array_equal(out["Y"], ref["Y"])


def test_every_cell_processed_once_and_cost_feedback():
    from tests.gpu_util import chem_for, run_integrate, say
    mech = synth.mechanism("small")
    f = synth.field_small(5000)
    c = chem_for(mech, schedule=CHEM_SCHED_QUEUE, queue_chunk=3)
    say("queue exactly once")
    out = run_integrate(c, f)
    s = out["stats"]
    assert s["cells_integrated"] == f.n_cells
    cost = out["cost"]
    assert np.array_equal(cost.cpu().numpy(), out["nacc"] + out["nrej"])
    # second call ordered by the first call's cost: same cells, same results
    out2 = run_integrate(c, f, cost=cost)
    assert out2["stats"]["cells_integrated"] == f.n_cells
    assert np.array_equal(out2["T"], out["T"]) and np.array_equal(out2["Y"], out["Y"])


def test_failure_codes_from_host_inputs():
    from tests.gpu_util import chem_for, run_integrate, say
    mech = synth.mechanism("small")
    f = synth.field_small(64)
    f.T[3] = -10.0
    f.Y[2, 5] = np.nan
    f.p[7] = 0.0
    c = chem_for(mech)
    say("bad inputs")
    out = run_integrate(c, f)
    assert out["status"][3] == 4 and out["status"][5] == 4 and out["status"][7] == 4
    assert out["T"][3] == -10.0                       # left untouched
    good = np.setdiff1d(np.arange(64), [3, 5, 7])
    assert np.all(out["status"][good] == 0)
    assert out["stats"]["cells_failed"] == 3
    c.set_options(max_steps=1)
    out = run_integrate(c, synth.field_small(16))
    assert np.all(out["status"] == 1)
    c.set_options(max_steps=100000, hmin_frac=0.5)
    out = run_integrate(c, synth.field_small(16))
    assert np.all(out["status"] == 2)


def test_empty_and_tiny_inputs():
    from tests.gpu_util import chem_for, dev, say
    mech = synth.mechanism("small")
    c = chem_for(mech)
    say("empty")
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    st = c.integrate(e, e, torch.zeros(0, dtype=torch.float64, device="cuda"), 1e-6, stats=True)
    assert st["cells_integrated"] == 0
    f = synth.field_small(1)
    o = Oracle(mech)
    ref = o.integrate_batch(f.T, f.p, f.Y, f.dt)
    T, Y = dev(f.T), dev(f.Y)
    c.integrate(T, dev(f.p), Y, f.dt)
    torch.cuda.synchronize()
    assert abs(T.item() - ref[0][0]) <= 1e-6 * ref[0][0]


def test_mapping_flags_exact_full_field():
    """Sec. 2.3 criterion on the 262144-cell mapped workload: flags bit-exact."""
    from tests.gpu_util import chem_for, dev, host, say
    mech = synth.mechanism("mech53")
    f = synth.field_mapped(262144)
    o = Oracle(mech)
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    c = chem_for(mech)
    for Z_tol, use_T in ((1e-4, False), (1e-4, True), (1e-2, False), (1e-6, True), (-1.0, False)):
        say("map", Z_tol, use_T)
        flags_o, ref_o = o.map_reference(f.T, f.Y, Yf, Yo, Z_tol, 1.0, use_T)
        flags, ref = c.map_reference(dev(f.T), dev(f.p), dev(f.Y), Yf, Yo, Z_tol, 1.0, use_T)
        torch.cuda.synchronize()
        assert int(host(ref)[0]) == ref_o
        assert np.array_equal(host(flags), flags_o)


def test_mapped_step_matches_oracle():
    """Map, integrate flags 0/1, give flag-2 cells the reference increment with
    an enthalpy-consistent temperature; compare with the oracle's own step."""
    from tests.gpu_util import chem_for, compare_to_oracle, dev, host, say
    mech = synth.mechanism("mech53")
    full = synth.field_mapped(262144)
    idx = synth.stratified_indices(full, 40, seed=3)
    f = synth.subsample(full, idx)
    o = Oracle(mech)
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    flags_o, ref_o = o.map_reference(f.T, f.Y, Yf, Yo, 1e-4)
    assert ref_o >= 0 and (flags_o == 2).sum() >= 30
    refo = o.step_mapped(f.T, f.p, f.Y, f.dt, flags_o, ref_o, threads=16)
    c = chem_for(mech)
    say("mapped step", f.n_cells)
    T, p, Y = dev(f.T), dev(f.p), dev(f.Y)
    flags, ref = c.map_reference(T, p, Y, Yf, Yo, 1e-4)
    st = torch.zeros(f.n_cells, dtype=torch.uint8, device="cuda")
    s = c.integrate(T, p, Y, f.dt, flags=flags, ref_index=ref, status=st, stats=True)
    torch.cuda.synchronize()
    assert np.array_equal(host(flags), flags_o)
    out = dict(T=host(T), Y=host(Y))
    rep = compare_to_oracle(out, refo[0], refo[1])
    print(rep, s)
    assert rep["ok"], rep
    assert s["cells_mapped"] == int((flags_o == 2).sum())
    assert np.all(host(st)[flags_o == 2] == 5)


def test_full_size_field_sampled_parity():
    """The 1,048,576-cell field of the headline workload, mapped (Z_tol 1e-4)
    and integrated in the launch configuration the benchmark times (heavy-first
    work queue); a stratified sample of cells is recomputed by the oracle one
    by one: integrated cells from their own state, mapped cells from the
    reference cell's increment (Sec. 2.3)."""
    from tests.gpu_util import chem_for, compare_to_oracle, dev, host, say
    mech = synth.mechanism("mech53")
    full = synth.WORKLOADS["surrogate"]["field"]()
    assert full.n_cells == 1048576
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    c = chem_for(mech, schedule=CHEM_SCHED_QUEUE)
    say("full-size field", full.n_cells)
    T, p, Y = dev(full.T), dev(full.p), dev(full.Y)
    flags, ref = c.map_reference(T, p, Y, Yf, Yo, 1e-4)
    s = c.integrate(T, p, Y, full.dt, flags=flags, ref_index=ref, stats=True)
    torch.cuda.synchronize()
    fl, r0 = host(flags), int(host(ref)[0])
    assert r0 >= 0 and s["cells_failed"] == 0
    assert s["cells_mapped"] + s["cells_integrated"] == full.n_cells
    idx = synth.stratified_indices(full, 24, seed=11)
    idx = idx[idx != r0]
    sub = synth.subsample(full, np.concatenate([[r0], idx]))
    sub_flags = np.concatenate([[1], fl[idx]]).astype(np.uint8)
    o = Oracle(mech)
    say("oracle on", sub.n_cells, "sampled cells")
    refo = o.step_mapped(sub.T, sub.p, sub.Y, sub.dt, sub_flags, 0, threads=16)
    keep = np.concatenate([[r0], idx])
    out = dict(T=host(T)[keep], Y=host(Y)[:, keep])
    rep = compare_to_oracle(out, refo[0], refo[1])
    print(rep, s, "mapped in sample", int((sub_flags == 2).sum()))
    assert rep["ok"], rep
    assert (sub_flags == 2).sum() > 0 and (sub_flags == 0).sum() > 0


def test_static_blocks_with_mapping_and_slot_query():
    """CHEM_SCHED_BLOCKS skips mapped cells like the other launches (results
    equal the queue's bit for bit); the slot count needs a mechanism."""
    from paper_2011_07978_amd.chem import Chem, ChemError
    from tests.gpu_util import chem_for, dev, host, say
    with pytest.raises(ChemError):
        Chem(0).slots()
    mech = synth.mechanism("mech53")
    f = synth.field_mapped(20000, seed=41)
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    outs = []
    for sched in (CHEM_SCHED_QUEUE, CHEM_SCHED_BLOCKS):
        c = chem_for(mech, schedule=sched)
        assert c.slots() >= 256
        say("mapped + schedule", sched)
        T, p, Y = dev(f.T), dev(f.p), dev(f.Y)
        flags, ref = c.map_reference(T, p, Y, Yf, Yo, 1e-4)
        s = c.integrate(T, p, Y, f.dt, flags=flags, ref_index=ref, stats=True)
        torch.cuda.synchronize()
        assert s["cells_mapped"] > 0 and s["cells_mapped"] + s["cells_integrated"] == f.n_cells
        outs.append((host(T), host(Y)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
