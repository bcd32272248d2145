"""Consecutive flow steps against the oracle (Sec. 2.3, App. B): ten steps of
reference mapping and integration on a stratified sample of the
262,144-cell mapped field, with step sizes and per-cell costs carried from
step to step, eagerly, replayed from one recorded HIP graph, and in the
launch configuration the autotuner picks; a reference cell whose own
integration fails is not copied; mechanism rejection through the context."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle  # noqa: E402
from paper_2011_07978_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

Z_TOL = 1e-4
N_STEPS = 10


@pytest.fixture(scope="module")
def c3():
    """Stratified sample (64 cells per class) of the 262,144-cell mapped
    field, sorted, with the field's reference cell (its lowest-index mapping
    candidate) included; the oracle's ten steps on it."""
    mech = synth.mechanism("mech53")
    full = synth.field_mapped()
    o = Oracle(mech)
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    _, ref_full = o.map_reference(full.T, full.Y, Yf, Yo, Z_TOL)
    idx = np.union1d(synth.stratified_indices(full, 64, seed=91), [ref_full])
    f = synth.subsample(full, idx)
    w, bf, bo = o.map_weights(Yf, Yo)
    T, Y, h = f.T.copy(), f.Y.copy(), np.zeros(f.n_cells)
    steps = []
    for _ in range(N_STEPS):
        flags, ref = o.map_reference(T, Y, Yf, Yo, Z_TOL)
        Z = o.mixture_fraction(Y, w, bf, bo)
        T, Y, h, st, na, nr = o.step_mapped(T, f.p, Y, f.dt, flags, ref, h=h, threads=16)
        steps.append(dict(flags=flags, ref=ref, Z=Z, T=T.copy(), Y=Y.copy(), status=st.copy(),
                          nacc=na, nrej=nr))
    assert int(np.searchsorted(idx, ref_full)) == steps[0]["ref"]
    return mech, f, steps


def _state(f):
    from tests.gpu_util import dev
    n = f.n_cells
    return dict(T=dev(f.T), p=dev(f.p), Y=dev(f.Y),
                h=torch.zeros(n, dtype=torch.float64, device="cuda"),
                cost=torch.zeros(n, dtype=torch.int32, device="cuda"),
                flags=torch.zeros(n, dtype=torch.uint8, device="cuda"),
                ref=torch.zeros(1, dtype=torch.int64, device="cuda"),
                status=torch.zeros(n, dtype=torch.uint8, device="cuda"),
                steps=torch.zeros(2 * n, dtype=torch.int32, device="cuda"))


def _step(c, S, mech, dt):
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    c.map_reference(S["T"], S["p"], S["Y"], Yf, Yo, Z_TOL, flags=S["flags"], ref_index=S["ref"])
    c.integrate(S["T"], S["p"], S["Y"], dt, flags=S["flags"], ref_index=S["ref"], h=S["h"],
                cost=S["cost"], status=S["status"], steps=S["steps"])


def _snapshot(S):
    from tests.gpu_util import host
    st = host(S["steps"]).reshape(-1, 2)
    return dict(flags=host(S["flags"]).copy(), ref=int(host(S["ref"])[0]), T=host(S["T"]).copy(),
                Y=host(S["Y"]).copy(), status=host(S["status"]).copy(), nacc=st[:, 0].copy(),
                nrej=st[:, 1].copy())


def _compare(got, want, k):
    """Flags exact (apart from cells whose mixture fraction lies within 1e-9
    of the threshold, where the two sides' states, equal to the step
    tolerance, may fall either way), parity at |dT|/T <= 1e-6 and
    |dY| <= 1e-8, statuses exact."""
    marginal = np.abs(want["Z"] - Z_TOL) <= 1e-9 * Z_TOL
    assert got["ref"] == want["ref"], k
    assert np.array_equal(got["flags"][~marginal], want["flags"][~marginal]), k
    assert np.array_equal(got["status"], want["status"]), k
    dT = np.max(np.abs(got["T"] - want["T"]) / want["T"])
    dY = np.max(np.abs(got["Y"] - want["Y"]))
    differs = int(((got["nacc"] != want["nacc"]) | (got["nrej"] != want["nrej"]))[want["flags"] != 2].sum())
    print(f"step {k + 1}: max|dT|/T {dT:.2e} max|dY| {dY:.2e} mapped {(got['flags'] == 2).sum()} "
          f"step sequence differs {differs}")
    assert dT <= 1e-6 and dY <= 1e-8, (k, dT, dY)
    assert differs <= 2, (k, differs)
    return marginal.sum()


def test_ten_steps_eager_match_oracle(c3):
    from tests.gpu_util import chem_for, say
    mech, f, want = c3
    c = chem_for(mech)
    S = _state(f)
    for k in range(N_STEPS):
        say("C3 ten steps eager, step", k + 1, "cells", f.n_cells)
        _step(c, S, mech, f.dt)
        torch.cuda.synchronize()
        _compare(_snapshot(S), want[k], k)


def test_ten_steps_graph_replay_match_oracle(c3):
    from paper_2011_07978_amd.chem import Chem
    from tests.gpu_util import say
    mech, f, want = c3
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        c = Chem(0, stream=stream)
        c.set_mechanism(mech)
        c.reserve(f.n_cells)
        G = _state(f)
        pristine = {k: v.clone() for k, v in G.items()}
        say("C3 graph: eager warm-up step")
        _step(c, G, mech, f.dt)
        stream.synchronize()
        c.graph_begin()
        for _ in range(N_STEPS):
            _step(c, G, mech, f.dt)
        g = c.graph_end()
        for rep in range(2):
            for key in G:
                G[key].copy_(pristine[key])
            stream.synchronize()
            say("C3 graph replay", rep)
            g.launch()
            stream.synchronize()
            _compare(_snapshot(G), want[-1], N_STEPS - 1)
        g.close()


def test_ten_steps_autotuned_match_oracle(c3):
    from tests.gpu_util import chem_for, dev, say
    mech, f, want = c3
    c = chem_for(mech)
    say("C3 autotune on the pristine sample")
    res = c.autotune(dev(f.T), dev(f.p), dev(f.Y), f.dt)
    o = c.options()
    print("autotune", res, "->", o.schedule, o.queue_chunk, o.slots_per_cu)
    S = _state(f)
    for k in range(N_STEPS):
        say("C3 ten steps autotuned, step", k + 1)
        _step(c, S, mech, f.dt)
        torch.cuda.synchronize()
        _compare(_snapshot(S), want[k], k)


@pytest.mark.parametrize("case", ["step_limit", "bad_input"])
def test_failed_reference_is_not_copied(case):
    """One attempted step over dt = 1e-2 s stops the reference at the step
    limit (status 1); a reference with T = -1 is refused (status 4).  Either
    way mapped cells keep their state with status 7 and count as failed,
    as the oracle does."""
    from tests.gpu_util import chem_for, dev, host, say
    mech = synth.mechanism("mech53")
    o = Oracle(mech)
    f = synth.field_mapped(2000, seed=31)
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    flags_o, ref_o = o.map_reference(f.T, f.Y, Yf, Yo, Z_TOL)
    T0 = f.T.copy()
    dt, kw = (1e-2, dict(max_steps=1)) if case == "step_limit" else (1e-6, {})
    if case == "bad_input":
        T0[ref_o] = -1.0
    Tw, Yw, _, st_o = o.step_mapped(T0, f.p, f.Y, dt, flags_o, ref_o, **kw)[:4]
    mapped = flags_o == 2
    assert np.all(st_o[mapped] == 7)
    say("failed reference", case, f.n_cells, "cells")
    c = chem_for(mech, **kw)
    T, p, Y = dev(T0), dev(f.p), dev(f.Y)
    flags, ref = c.map_reference(T, p, Y, Yf, Yo, Z_TOL)
    status = torch.full((f.n_cells,), 255, dtype=torch.uint8, device="cuda")
    s = c.integrate(T, p, Y, dt, flags=flags, ref_index=ref, status=status, stats=True)
    torch.cuda.synchronize()
    fl, st, Tg, Yg = host(flags), host(status), host(T), host(Y)
    assert np.array_equal(fl, flags_o) and int(host(ref)[0]) == ref_o
    assert st[ref_o] == st_o[ref_o] == (1 if case == "step_limit" else 4)
    assert np.all(st[mapped] == 7)
    assert np.array_equal(Tg[mapped], T0[mapped]) and np.array_equal(Yg[:, mapped], f.Y[:, mapped])
    assert s["cells_mapped"] == 0
    assert s["cells_failed"] == int((st != 0).sum()) >= int(mapped.sum()) + 1


def test_context_refuses_bad_mechanism():
    """chem_set_mechanism runs the same validation as the host-only check and
    leaves the context without a mechanism."""
    import copy

    from paper_2011_07978_amd.chem import Chem, ChemError
    from tests.gpu_util import say
    mech = synth.mechanism("mech53")
    bad = copy.deepcopy(mech)
    bad.W = mech.W.copy()
    bad.W[7] *= 1.001
    say("bad mechanism through the context")
    c = Chem(0)
    with pytest.raises(ChemError, match="W inconsistent"):
        c.set_mechanism(bad)
    c.set_mechanism(mech)          # a good one afterwards is accepted
