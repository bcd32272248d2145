"""HIP-graph capture of consecutive flow steps and launch autotuning.

A recorded graph of ten steps (mapping, heavy-first queue, integration,
mapped update) replays to the same bits as the eager calls, on every replay,
with eager copies and synchronisations between replays.  The autotuner keeps
the fastest measured configuration, and no configuration changes results."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2011_07978_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _state(f):
    from tests.gpu_util import dev
    n = f.n_cells
    return dict(T=dev(f.T), p=dev(f.p), Y=dev(f.Y),
                h=torch.zeros(n, dtype=torch.float64, device="cuda"),
                cost=torch.zeros(n, dtype=torch.int32, device="cuda"),
                flags=torch.zeros(n, dtype=torch.uint8, device="cuda"),
                ref=torch.zeros(1, dtype=torch.int64, device="cuda"),
                status=torch.zeros(n, dtype=torch.uint8, device="cuda"))


def _step(c, S, mech, dt, surrogate):
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    c.map_reference(S["T"], S["p"], S["Y"], Yf, Yo, 1e-4, flags=S["flags"], ref_index=S["ref"])
    if surrogate:
        c.integrate_surrogate(S["T"], S["p"], S["Y"], dt, S["flags"], S["ref"],
                              gate=dict(tau_T=1e9, y_min=-1.0, max_dT=1e30, T_max=1e30), h=S["h"], cost=S["cost"],
                              status=S["status"])
    else:
        c.integrate(S["T"], S["p"], S["Y"], dt, flags=S["flags"], ref_index=S["ref"], h=S["h"],
                    cost=S["cost"], status=S["status"])


@pytest.mark.parametrize("surrogate", [False, True])
def test_graph_of_ten_steps_replays_bitwise(surrogate):
    from paper_2011_07978_amd.chem import Chem
    from tests.gpu_util import host, say
    mech = synth.mechanism("mech53")
    f = synth.field_mapped(6000, seed=81)
    n_steps = 10 if not surrogate else 3
    P = synth.surrogate_params(mech.n_species, seed=82, zero_output_weights=True, out_sd=(1.0, 1.0),
                               out_bias=synth.surrogate_increment_bias(mech.n_species, 83, 1e-8, 0.01)
                               ) if surrogate else None
    stream = torch.cuda.Stream()
    keys = ("T", "Y", "h", "cost", "flags", "status")
    say("graph eager reference, surrogate", surrogate)
    with torch.cuda.stream(stream):
        c = Chem(0, stream=stream)
        c.set_mechanism(mech)
        c.reserve(f.n_cells)
        if surrogate:
            c.surrogate_set_params(P)
        S = _state(f)
        for _ in range(n_steps):
            _step(c, S, mech, f.dt, surrogate)
        stream.synchronize()
        want = {k: host(S[k]).copy() for k in keys}
        say("graph capture, surrogate", surrogate)
        G = _state(f)
        pristine = {k: v.clone() for k, v in G.items()}
        _step(c, G, mech, f.dt, surrogate)          # warm every workspace eagerly
        stream.synchronize()
        c.graph_begin()
        for _ in range(n_steps):
            _step(c, G, mech, f.dt, surrogate)
        g = c.graph_end()
        for rep in range(3):
            for k in G:                               # eager work between replays
                G[k].copy_(pristine[k])
            stream.synchronize()
            say("graph replay", rep)
            g.launch()
            stream.synchronize()
            for k in keys:
                assert np.array_equal(host(G[k]), want[k]), (rep, k)
        g.close()
    if surrogate:
        assert (want["flags"] == 3).any()


def test_capture_refuses_allocation():
    from paper_2011_07978_amd.chem import Chem, ChemError
    from tests.gpu_util import say
    mech = synth.mechanism("mech53")
    f = synth.field_mapped(512, seed=83)
    stream = torch.cuda.Stream()
    say("capture without reserved workspace")
    with torch.cuda.stream(stream):
        c = Chem(0, stream=stream)
        c.set_mechanism(mech)
        S = _state(f)
        stream.synchronize()
        c.graph_begin()
        with pytest.raises(ChemError):
            c.integrate(S["T"], S["p"], S["Y"], f.dt, h=S["h"])   # queue workspace not reserved
        with pytest.raises(ChemError):
            c.graph_end()
    with pytest.raises(ChemError):
        Chem(0).graph_begin()                        # null stream cannot be captured


def test_autotune_keeps_fastest_and_never_changes_results():
    from paper_2011_07978_amd.chem import CHEM_SCHED_QUEUE
    from tests.gpu_util import chem_for, dev, host, run_integrate, say
    mech = synth.mechanism("mech53")
    f = synth.field_bimodal("mech53", 8192, seed=84)
    say("autotune mech53 8192 cells")
    c = chem_for(mech)
    T, p, Y = dev(f.T), dev(f.p), dev(f.Y)
    T0, Y0 = host(T).copy(), host(Y).copy()
    res = c.autotune(T, p, Y, f.dt, remeasure=True)
    print(res)
    # the plain launch, then queue_chunk 1, 2, 4, 8 for each distinct slots_per_cu
    # (one when a single workgroup of the integration kernel fills a CU)
    slots = sorted({r[2] for r in res[1:]})
    assert res[0][:3] == (0, 0, 0) and 1 <= len(slots) <= 2
    assert [r[:3] for r in res[1:]] == [(1, k, s) for s in slots for k in (1, 2, 4, 8)]
    assert np.array_equal(host(T), T0) and np.array_equal(host(Y), Y0)   # input untouched
    best = min(res, key=lambda r: r[3])
    o = c.options()
    assert (o.schedule, o.queue_chunk, o.slots_per_cu) == best[:3]
    # kept for the process: a second context with the same mechanism and sample
    # size gets the same timings and choice back without measuring
    say("autotune kept timings, second context")
    c2 = chem_for(mech)
    assert c2.autotune(T, p, Y, f.dt) == res
    o2 = c2.options()
    assert (o2.schedule, o2.queue_chunk, o2.slots_per_cu) == best[:3]
    say("autotune remeasure")
    again = c2.autotune(T, p, Y, f.dt, remeasure=True)
    assert [r[:3] for r in again] == [r[:3] for r in res]
    tuned = run_integrate(c, f)
    c.set_options(schedule=CHEM_SCHED_QUEUE, queue_chunk=0, slots_per_cu=0)
    default = run_integrate(c, f)
    assert np.array_equal(tuned["T"], default["T"]) and np.array_equal(tuned["Y"], default["Y"])
