"""Surrogate parity of the HIP path with the CPU oracle.

Forward pass: the BF16-MFMA network against the oracle's bfloat16-emulated
FP64 forward (same roundings of inputs, weights and activations; FP32 versus
FP64 accumulation), within bfloat16 bounds.  Backpropagation: gradients
against the oracle's.  Projection, enthalpy temperature and gate: with the
output layer's weights zero the network output is its bias exactly on both
sides, so the post-processing is compared tightly and the gate's decisions
exactly.  Cells the gate rejects go through the Rosenbrock solver at the
integrator's parity bar.  Training: the loss decreases and parameters
survive a save/load round trip."""
import os
import tempfile

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import Oracle  # noqa: E402
from paper_2011_07978_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _features(N, f, dt):
    return np.stack([oracle.mlp_features(N, f.T[i], f.p[i], f.Y[:, i], dt[i])
                     for i in range(f.n_cells)])


def _cells(n, seed):
    f = synth.field_mapped(4 * n, seed=seed)
    return synth.subsample(f, np.arange(n))


def _norm_block(P):
    nb = P[-6 * 64:].astype(np.float64).reshape(6, 64)
    return dict(mu_x=nb[0], sd_x=nb[1], mu_o=nb[2], sd_o=nb[3], xmin=nb[4], xmax=nb[5])


def test_forward_matches_bf16_oracle():
    from tests.gpu_util import chem_for, dev, host, say
    mech = synth.mechanism("mech53")
    N = mech.n_species
    n = 1000                                   # 15 full 64-row tiles and a ragged tail
    f = _cells(n, 31)
    dt = synth.surrogate_dt(n, 32)
    P = synth.surrogate_params(N, seed=33)
    say("surrogate forward mech53", n, "cells")
    c = chem_for(mech)
    c.surrogate_set_params(P)
    out = host(c.surrogate_forward(dev(f.T), dev(f.p), dev(f.Y), dev(dt)))
    X = _features(N, f, dt)
    emu = oracle.mlp_forward(P, X, N + 3, bf16_emulation=True)
    exact = oracle.mlp_forward(P, X, N + 3, bf16_emulation=False)
    live = slice(0, N + 1)
    err = np.abs(out[:, live] - emu[:, live])
    scale = np.abs(emu[:, live]).max()
    print("forward: max", err.max() / scale, "median", np.median(err) / scale,
          "bf16 effect", np.abs(exact - emu)[:, live].mean() / scale)
    assert np.all(out[:, N + 1:] == 0.0)           # padded outputs: zero rows, zero bias
    # FP32 accumulation against FP64: differences far below a bfloat16 ulp,
    # except where that changes the rounding of an activation to bfloat16
    assert err.max() <= 5e-3 * scale
    assert np.median(err) <= 1e-7 * scale
    # the kernel rounds like the emulation, not like FP64
    assert err.mean() < 0.25 * np.abs(exact - emu)[:, live].mean()


@pytest.mark.parametrize("n", [256, 4096])
def test_loss_gradient_matches_oracle(n):
    """256 rows: weight gradients in two K slices; 4096 rows (the training
    batch): sixteen slices and 1024 per-block loss sums."""
    from tests.gpu_util import chem_for, dev, say
    mech = synth.mechanism("mech53")
    N = mech.n_species
    f = _cells(n, 41)
    dt = synth.surrogate_dt(n, 42)
    rng = np.random.default_rng(43)
    T1 = f.T + rng.normal(0.0, 20.0, n)
    Y1 = f.Y + rng.normal(0.0, 1e-4, f.Y.shape)
    P = synth.surrogate_params(N, seed=44)
    say("surrogate loss gradient mech53", n, "pairs")
    c = chem_for(mech)
    c.surrogate_set_params(P)
    loss_g, grad_g = c.surrogate_loss_grad(dev(f.T), dev(f.p), dev(f.Y), dev(dt), dev(T1), dev(Y1))
    nb = _norm_block(P)
    tgt = np.zeros((n, 64))
    # targets in the output scale: asinh(dY / 1e-12), asinh(dT / 1e-6 K)
    tgt[:, :N] = (np.arcsinh((Y1 - f.Y).T / 1e-12) - nb["mu_o"][:N]) / nb["sd_o"][:N]
    tgt[:, N] = (np.arcsinh((T1 - f.T) / 1e-6) - nb["mu_o"][N]) / nb["sd_o"][N]
    loss_o, grad_o = oracle.mlp_loss_grad(P, _features(N, f, dt), tgt, N + 3, N + 1,
                                          bf16_emulation=True)
    print("loss", loss_g, loss_o)
    assert abs(loss_g - loss_o) <= 1e-2 * loss_o
    dims = synth.SUR_DIMS
    o = 0
    for l in range(5):
        ni, no = dims[l], dims[l + 1]
        for name, size in (("W", no * ni), ("b", no)):
            g, r = grad_g[o:o + size].astype(np.float64), grad_o[o:o + size]
            o += size
            cos = g @ r / (np.linalg.norm(g) * np.linalg.norm(r))
            rel = np.linalg.norm(g - r) / np.linalg.norm(r)
            print(f"layer {l} {name}: cos {cos:.6f} rel {rel:.2e}")
            assert cos >= 0.999 and rel <= 3e-2, (l, name, cos, rel)
    assert np.all(grad_g[o:] == 0.0)


def _gate_case(o, f, P, dt, tau_T=None, y_min=-1e-10):
    """The oracle's gate decisions and states for every cell; chooses tau_T
    between two neighbouring temperature gaps near the median, so that no
    decision is marginal."""
    N = f.Y.shape[0]
    nb = _norm_block(P)
    # the output layer is its bias alone (zero weights): known exactly
    d = synth.SUR_DIMS
    off = sum(d[l] * d[l + 1] + d[l + 1] for l in range(4)) + d[4] * d[5]
    b5 = P[off:off + d[5]]
    # output scale: dY_k = 1e-12 sinh(t_k), dT = 1e-6 K sinh(t_N)
    dY = 1e-12 * np.sinh(b5[:N].astype(np.float64) * nb["sd_o"][:N] + nb["mu_o"][:N])
    dT = 1e-6 * np.sinh(float(b5[N]) * nb["sd_o"][N] + nb["mu_o"][N])
    gaps = np.full(f.n_cells, np.inf)
    miny = np.full(f.n_cells, -np.inf)
    for i in range(f.n_cells):
        Yc = oracle.conserve(o, f.Y[:, i], np.maximum(f.Y[:, i] + dY, 0.0))
        if Yc is None:
            continue
        miny[i] = Yc.min()
        Th, _ = o.temperature_from_enthalpy(o.enthalpy(f.T[i], f.Y[:, i]), Yc, f.T[i] + dT)
        gaps[i] = abs(f.T[i] + dT - Th)
    if tau_T is None:
        s = np.sort(gaps[np.isfinite(gaps)])
        k = s.size // 2
        tau_T = 0.5 * (s[k - 1] + s[k])
    marginal = np.abs(gaps - tau_T) <= 1e-9 * tau_T
    marginal |= np.abs(miny - y_min) <= 1e-9 * abs(y_min)
    res = [oracle.surrogate_cell(o, P, f.p[i], f.T[i], f.Y[:, i], dt, tau_T=tau_T, y_min=y_min)
           for i in range(f.n_cells)]
    ok = np.array([r[0] for r in res])
    T1 = np.array([r[1] for r in res])
    Y1 = np.stack([r[2] for r in res], axis=1)
    return tau_T, ok, T1, Y1, marginal


def test_projection_gate_and_fallback_match_oracle():
    from tests.gpu_util import chem_for, compare_to_oracle, dev, host, say
    mech = synth.mechanism("mech53")
    N = mech.n_species
    full = synth.field_mapped(20000, seed=51)
    f = synth.subsample(full, synth.stratified_indices(full, 100, seed=52)[:290])
    n = f.n_cells
    # box on ln T rejects the coldest and hottest cells
    box = (np.r_[np.log(350.0), -1e30 * np.ones(N + 2)], np.r_[np.log(2400.0), 1e30 * np.ones(N + 2)])
    P = synth.surrogate_params(N, seed=53, zero_output_weights=True, out_sd=(1.0, 1.0), box=box,
                               out_bias=synth.surrogate_increment_bias(N, 54, 1e-5, 0.5))
    y_min = -1e-10
    o = Oracle(mech)
    tau, ok_o, T_o, Y_o, marginal = _gate_case(o, f, P, f.dt, y_min=y_min)
    print("oracle accepts", ok_o.sum(), "of", n)
    assert 0 < ok_o.sum() < n and not marginal.any()
    say("surrogate gate + fallback mech53", n, "cells, tau", tau)
    c = chem_for(mech)
    c.surrogate_set_params(P)
    T, p, Y = dev(f.T), dev(f.p), dev(f.Y)
    flags = torch.zeros(n, dtype=torch.uint8, device="cuda")
    status = torch.full((n,), 255, dtype=torch.uint8, device="cuda")
    h = torch.zeros(n, dtype=torch.float64, device="cuda")
    s = c.integrate_surrogate(T, p, Y, f.dt, flags, gate=dict(tau_T=tau, y_min=y_min, max_dT=1e30, T_max=1e30),
                              h=h, status=status, stats=True)
    torch.cuda.synchronize()
    fl, stt, Tg, Yg = host(flags), host(status), host(T), host(Y)
    acc = fl == 3
    print("accepted", acc.sum(), "of", n, s)
    assert np.array_equal(acc, ok_o)
    assert np.all(fl[~acc] == 0)
    assert np.all(stt[acc] == 6) and np.all(stt[~acc] == 0)
    assert s["cells_surrogate"] == acc.sum() and s["cells_rejected"] == n - acc.sum()
    assert s["cells_integrated"] == n - acc.sum()
    # surrogate cells: projection and enthalpy temperature
    assert np.max(np.abs(Tg[acc] - T_o[acc]) / T_o[acc]) <= 1e-12
    assert np.max(np.abs(Yg[:, acc] - Y_o[:, acc])) <= 1e-15
    E = mech.composition.T / mech.W[None, :]
    assert np.abs(E @ (Yg[:, acc] - f.Y[:, acc])).max() <= 1e-15
    # rejected cells: the Rosenbrock solver at the integrator's bar
    rej = np.nonzero(~acc)[0]
    sub = synth.subsample(f, rej)
    ref = o.integrate_batch(sub.T, sub.p, sub.Y, sub.dt, threads=16, schedule=1)
    rep = compare_to_oracle(dict(T=Tg[rej], Y=Yg[:, rej]), ref[0], ref[1])
    print(rep)
    assert rep["ok"], rep
    # a largest-|dT| bound below the (common) predicted increment rejects every cell
    nb = _norm_block(P)
    d = synth.SUR_DIMS
    off = sum(d[l] * d[l + 1] + d[l + 1] for l in range(4)) + d[4] * d[5]
    dT = 1e-6 * np.sinh(float(P[off + N]) * nb["sd_o"][N] + nb["mu_o"][N])
    i0 = int(np.nonzero(ok_o)[0][0])
    assert not oracle.surrogate_cell(o, P, f.p[i0], f.T[i0], f.Y[:, i0], f.dt, tau_T=tau, y_min=y_min,
                                     max_dT=0.5 * abs(dT))[0]
    flags.zero_()
    s = c.integrate_surrogate(dev(f.T), p, dev(f.Y), f.dt, flags,
                              gate=dict(tau_T=tau, y_min=y_min, max_dT=0.5 * abs(dT), T_max=1e30),
                              stats=True)
    assert s["cells_surrogate"] == 0 and s["cells_integrated"] == n


def test_surrogate_leaves_mapped_and_reference_cells_alone():
    from tests.gpu_util import chem_for, dev, host, say
    mech = synth.mechanism("mech53")
    N = mech.n_species
    f = synth.field_mapped(3000, seed=61)
    n = f.n_cells
    P = synth.surrogate_params(N, seed=62, zero_output_weights=True, out_sd=(1.0, 1.0),
                               out_bias=synth.surrogate_increment_bias(N, 63, 1e-7, 0.2))
    say("surrogate with mapping mech53", n, "cells")
    c = chem_for(mech)
    c.surrogate_set_params(P)
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    outs = []
    for use_sur in (False, True):
        T, p, Y = dev(f.T), dev(f.p), dev(f.Y)
        flags, ref = c.map_reference(T, p, Y, Yf, Yo, 1e-4)
        f0 = host(flags).copy()
        st = torch.zeros(n, dtype=torch.uint8, device="cuda")
        if use_sur:
            s = c.integrate_surrogate(T, p, Y, f.dt, flags, ref, gate=dict(tau_T=1e9, y_min=-1.0, max_dT=1e30, T_max=1e30), status=st,
                                      stats=True)
        else:
            s = c.integrate(T, p, Y, f.dt, flags=flags, ref_index=ref, status=st, stats=True)
        torch.cuda.synchronize()
        outs.append((f0, host(flags), host(T), host(Y), host(st), s))
    (f0, fa, Ta, Ya, sa, _), (f0b, fb, Tb, Yb, sb, s) = outs
    assert np.array_equal(f0, f0b) and np.array_equal(f0, fa)
    keep = f0 != 0
    assert np.array_equal(fb[keep], f0[keep])             # flags 1 and 2 untouched
    assert np.all(np.isin(fb[~keep], (0, 3)))
    assert np.array_equal(Ta[keep], Tb[keep]) and np.array_equal(Ya[:, keep], Yb[:, keep])
    assert np.all(sb[fb == 3] == 6) and np.all(sb[fb == 2] == 5)
    same = (fb == 0)                                       # rejected: solver, bit for bit
    assert np.array_equal(Ta[same], Tb[same]) and np.array_equal(Ya[:, same], Yb[:, same])
    assert s["cells_mapped"] == int((f0 == 2).sum())
    assert s["cells_surrogate"] == int((fb == 3).sum()) > 0


def test_training_reduces_loss_and_roundtrips():
    from paper_2011_07978_amd import surrogate
    from tests.gpu_util import chem_for, dev, host, say
    mech = synth.mechanism("mech53")
    say("surrogate pairs + training mech53 16384 x 2")
    c = chem_for(mech)
    pairs = surrogate.generate_pairs(c, n_cells=16384, n_steps=2, seed=71)
    assert pairs.n >= 30000
    hist = surrogate.train(c, pairs, epochs=8, batch=1024, seed=72)
    print("loss history", hist)
    assert np.all(np.isfinite(hist)) and hist[-1] < 0.5 * hist[0]
    P = c.surrogate_get_params()
    assert np.all(np.isfinite(P))
    sub = pairs.take(np.arange(700))
    out1 = host(c.surrogate_forward(sub.T0, sub.p, sub.Y0, sub.dt))
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "sur.bin")
        c.surrogate_save(path)
        c2 = chem_for(mech)
        c2.surrogate_load(path)
    assert np.array_equal(c2.surrogate_get_params(), P)
    out2 = host(c2.surrogate_forward(sub.T0, sub.p, sub.Y0, sub.dt))
    assert np.array_equal(out1, out2)
    # a file for another mechanism is refused
    c3 = chem_for(synth.mechanism("small"))
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "sur.bin")
        c.surrogate_save(path)
        with pytest.raises(Exception):
            c3.surrogate_load(path)
