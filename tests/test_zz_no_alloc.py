"""chem_integrate_noalloc (the integration entry point for callers that cannot
allocate) against chem_integrate: same results bit for bit on two calls in a
row, the second smaller, with mapping on the first; no device memory is
allocated by the calls; sizes beyond the fixed workspace and mechanisms it
does not cover are refused on the host."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2011_07978_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

MAX_CELLS = 1 << 21


def _free_device_bytes():
    hip = ctypes.CDLL("libamdhip64.so")
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


def _state(f):
    from tests.gpu_util import dev
    n = f.n_cells
    return dict(T=dev(f.T), p=dev(f.p), Y=dev(f.Y),
                h=torch.zeros(n, dtype=torch.float64, device="cuda"),
                cost=torch.zeros(n, dtype=torch.int32, device="cuda"),
                status=torch.full((n,), 255, dtype=torch.uint8, device="cuda"),
                steps=torch.zeros(2 * n, dtype=torch.int32, device="cuda"),
                flags=torch.zeros(n, dtype=torch.uint8, device="cuda"),
                ref=torch.zeros(1, dtype=torch.int64, device="cuda"))


def _call(c, S, dt, mapped, noalloc):
    mech = c.mech
    if mapped:
        c.map_reference(S["T"], S["p"], S["Y"], synth.stream_fuel(mech), synth.stream_oxidiser(mech),
                        1e-4, flags=S["flags"], ref_index=S["ref"])
    fn = c.integrate_noalloc if noalloc else c.integrate
    return fn(S["T"], S["p"], S["Y"], dt, flags=S["flags"] if mapped else None,
              ref_index=S["ref"] if mapped else None, h=S["h"], cost=S["cost"], status=S["status"],
              steps=S["steps"], stats=True)


def test_noalloc_equals_integrate_on_two_calls():
    from tests.gpu_util import chem_for, host, say
    mech = synth.mechanism("mech53")
    big = synth.field_mapped(6000, seed=131)
    small = synth.subsample(synth.field_mapped(4000, seed=132), np.arange(0, 4000, 2))
    calls = [(big, True), (small, False)]
    say("no-alloc reference path (chem_integrate), two calls")
    ref_ctx = chem_for(mech)
    want = []
    for f, mapped in calls:
        S = _state(f)
        st = _call(ref_ctx, S, f.dt, mapped, noalloc=False)
        torch.cuda.synchronize()
        want.append(({k: host(v).copy() for k, v in S.items()}, st))
    ctx = chem_for(mech)                  # a fresh context: its own queue was never allocated
    states = [_state(f) for f, _ in calls]
    torch.cuda.synchronize()
    free0 = _free_device_bytes()
    for q, ((f, mapped), S) in enumerate(zip(calls, states)):
        say("chem_integrate_noalloc call", q + 1, f.n_cells, "cells, mapped", mapped)
        st = _call(ctx, S, f.dt, mapped, noalloc=True)
        torch.cuda.synchronize()
        got = {k: host(v) for k, v in S.items()}
        w, wst = want[q]
        for k in ("T", "Y", "h", "cost", "status", "steps", "flags", "ref"):
            assert np.array_equal(got[k], w[k]), (q, k)
        for k in ("cells_integrated", "cells_mapped", "cells_failed", "steps_accepted",
                  "steps_rejected", "max_cell_steps"):
            assert st[k] == wst[k], (q, k)
        assert st["cells_failed"] == 0
    assert want[0][1]["cells_mapped"] > 1000
    free1 = _free_device_bytes()
    print("device bytes free before / after the no-alloc calls:", free0, free1)
    assert free1 >= free0


def test_noalloc_refuses_what_it_cannot_hold():
    from paper_2011_07978_amd.chem import Chem
    from tests.gpu_util import say
    say("no-alloc limits (host-side refusals)")
    c = Chem(0)
    c.set_mechanism(synth.mechanism("mech53"))
    t = torch.ones(4, dtype=torch.float64, device="cuda")
    P = lambda x: ctypes.c_void_p(x.data_ptr())
    L = c.L
    # one cell beyond the fixed workspace: refused before anything is enqueued
    assert L.chem_integrate_noalloc(c.h, MAX_CELLS + 1, P(t), P(t), P(t), 1e-6, None, None, None,
                                    None, None, None, None) == -1
    assert "2097152" in L.chem_last_error(c.h).decode()
    assert L.chem_integrate_noalloc(c.h, -1, P(t), P(t), P(t), 1e-6, None, None, None, None, None,
                                    None, None) == -1
    # the large-mechanism integrator needs device-sized Jacobian slots
    c.set_mechanism(synth.mechanism("mech130"))
    assert L.chem_integrate_noalloc(c.h, 4, P(t), P(t), P(t), 1e-6, None, None, None, None, None,
                                    None, None) == -5
    # zero cells is a valid, empty call
    c.set_mechanism(synth.mechanism("mech53"))
    assert L.chem_integrate_noalloc(c.h, 0, None, None, None, 1e-6, None, None, None, None, None,
                                    None, None) == 0
