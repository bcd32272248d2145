"""Pins of the surrogate oracle: bfloat16 rounding, the MLP forward pass,
backpropagation and the element-conservation projection (CPU only)."""
import numpy as np
import pytest
import torch
from scipy.special import erf

import oracle
from oracle import Oracle
from paper_2011_07978_amd import synth

IN, HID, OUT = 64, 256, 64
DIMS = [IN, HID, HID, HID, HID, OUT]


def random_params(seed=0, nfeat=56, scale=1.0):
    rng = np.random.default_rng(seed)
    P = []
    for l in range(5):
        ni, no = DIMS[l], DIMS[l + 1]
        P.append((rng.standard_normal((no, ni)) * scale / np.sqrt(ni)).ravel())
        P.append(rng.standard_normal(no) * 0.1)
    mu = np.zeros(IN)
    sd = np.ones(IN)
    mu[:nfeat] = rng.standard_normal(nfeat) * 0.1
    sd[:nfeat] = rng.uniform(0.5, 2.0, nfeat)
    P += [mu, sd, np.zeros(IN), np.ones(IN), -np.ones(IN) * 1e9, np.ones(IN) * 1e9]
    P = np.concatenate(P).astype(np.float32)
    assert P.size == oracle.mlp_param_count()
    return P


def unpack(P):
    out, o = [], 0
    for l in range(5):
        ni, no = DIMS[l], DIMS[l + 1]
        W = P[o:o + no * ni].reshape(no, ni).astype(np.float64)
        o += no * ni
        b = P[o:o + no].astype(np.float64)
        o += no
        out.append((W, b))
    nb = P[o:].reshape(6, IN).astype(np.float64)
    return out, nb


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(5)
    vals = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-8, 8, 2000),
                           [0.0, -0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 65504.0, 1e-40]])
    ref = torch.tensor(vals.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([oracle.bf16(v) for v in vals.astype(np.float32)])
    assert np.array_equal(got, ref)


def test_forward_fp64_matches_matrix_products():
    P = random_params(1)
    layers, nb = unpack(P)
    rng = np.random.default_rng(2)
    X = np.zeros((7, IN))
    X[:, :56] = rng.standard_normal((7, 56))
    out = oracle.mlp_forward(P, X, 56, bf16_emulation=False)
    h = (X - nb[0]) / nb[1]
    h[:, 56:] = 0.0
    for l, (W, b) in enumerate(layers):
        z = h @ W.T + b
        h = 0.5 * z * (1 + erf(z / np.sqrt(2))) if l < 4 else z
    np.testing.assert_allclose(out, h, rtol=1e-12, atol=1e-12)


def test_bf16_forward_close_to_fp64():
    P = random_params(3)
    X = np.zeros((5, IN))
    X[:, :56] = np.random.default_rng(4).standard_normal((5, 56))
    a = oracle.mlp_forward(P, X, 56, bf16_emulation=False)
    b = oracle.mlp_forward(P, X, 56, bf16_emulation=True)
    err = np.abs(a - b).max() / np.abs(a).max()
    assert 1e-5 < err < 5e-2      # bfloat16 has an 8-bit mantissa


def test_backprop_matches_central_differences():
    P = random_params(6)
    rng = np.random.default_rng(7)
    X = np.zeros((4, IN))
    X[:, :56] = rng.standard_normal((4, 56))
    target = rng.standard_normal((4, OUT))
    loss, g = oracle.mlp_loss_grad(P, X, target, 56, 54, bf16_emulation=False)
    nparam = P.size - 6 * IN
    idx = np.concatenate([rng.choice(nparam, 40, replace=False),
                          [0, 64 * 256 + 3, nparam - 1, nparam - 64 - 5]])
    for i in idx:
        eps = 1e-3 * max(1.0, abs(float(P[i])))
        Pp, Pm = P.copy(), P.copy()
        Pp[i] = np.float32(P[i] + eps)
        Pm[i] = np.float32(P[i] - eps)
        d = float(Pp[i]) - float(Pm[i])
        lp, _ = oracle.mlp_loss_grad(Pp, X, target, 56, 54)
        lm, _ = oracle.mlp_loss_grad(Pm, X, target, 56, 54)
        fd = (lp - lm) / d
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])
    assert np.all(g[nparam:] == 0)


def test_conservation_of_clipped_prediction():
    mech = synth.mechanism("mech53")
    o = Oracle(mech)
    N = mech.n_species
    E = (mech.composition.T / mech.W[None, :])          # [elements, species]
    rng = np.random.default_rng(8)
    f = synth.field_mapped(400, seed=9)
    for i in range(0, 400, 40):
        Y0 = f.Y[:, i]
        Y1 = np.maximum(Y0 + rng.standard_normal(N) * 1e-4, 0.0)
        Y2 = oracle.conserve(o, Y0, Y1)
        scale = np.abs(E).max() * 1e-3
        assert np.abs(E @ (Y2 - Y0)).max() <= 1e-14 * scale * 100
        assert abs((Y2 - Y0).sum()) <= 1e-15
        assert np.all(Y2[Y1 == 0.0] == 0.0)              # clipped species stay at zero
        # the correction is Y1_k (E^T lam)_k: weighted minimum norm
        pos = Y1 > 0
        d = (Y1 - Y2)[pos] / Y1[pos]
        lam, *_ = np.linalg.lstsq(E.T[pos], d, rcond=None)
        np.testing.assert_allclose(E.T[pos] @ lam, d, atol=1e-12 * max(1.0, np.abs(d).max()))
        # idempotent
        np.testing.assert_allclose(oracle.conserve(o, Y0, Y2), Y2, rtol=0, atol=1e-15)
    # a uniform rescaling is undone exactly: the correction (c - 1) / c is the
    # constant vector E^T (m_e (c - 1) / c), m_e the element masses
    Y0 = f.Y[:, 7]
    for c in (0.9, 1.05, 1.3):
        np.testing.assert_allclose(oracle.conserve(o, Y0, c * Y0), Y0, rtol=1e-13, atol=1e-19)


def test_surrogate_cell_gate_and_conservation():
    mech = synth.mechanism("mech53")
    o = Oracle(mech)
    N = mech.n_species
    P = random_params(9, scale=1e-3)       # tiny network: small increments
    layers, nb = unpack(P)
    f = synth.field_mapped(2000, seed=4)
    i = int(np.nonzero(f.cls == 1)[0][0])
    T, Y = f.T[i], f.Y[:, i].copy()
    ok, T1, Y1 = oracle.surrogate_cell(o, P, f.p[i], T, Y, 1e-6, tau_T=1e9, y_min=-1.0)
    assert ok
    E = (mech.composition.T / mech.W[None, :])
    assert np.abs(E @ (Y1 - Y)).max() <= 1e-15
    assert abs(o.enthalpy(T1, Y1) - o.enthalpy(T, Y)) <= 1e-12 * o.cp(T, Y) * T
    # a predicted |dT| above max_dT is rejected, the state untouched
    ok3, T3, Y3 = oracle.surrogate_cell(o, P, f.p[i], T, Y, 1e-6, tau_T=1e9, y_min=-1.0, max_dT=0.0)
    dT_pred = abs(T1 - T)
    assert (not ok3 and T3 == T and np.array_equal(Y3, Y)) or dT_pred == 0.0
    # a cell hotter than T_max is not offered
    ok4, T4, Y4 = oracle.surrogate_cell(o, P, f.p[i], T, Y, 1e-6, tau_T=1e9, y_min=-1.0, T_max=T - 1.0)
    assert not ok4 and T4 == T and np.array_equal(Y4, Y)
    # out-of-box input is rejected
    P2 = P.copy()
    base = P2.size - 6 * IN
    P2[base + 4 * IN: base + 5 * IN] = 0.0      # xmin
    P2[base + 5 * IN: base + 6 * IN] = 0.0      # xmax: empty box
    ok, T2, Y2 = oracle.surrogate_cell(o, P2, f.p[i], T, Y, 1e-6, tau_T=1e9, y_min=-1.0)
    assert not ok and T2 == T and np.array_equal(Y2, Y)
