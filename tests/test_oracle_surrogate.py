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


# --------------------------------------------------- closed-form forward pins
# Standard normal distribution function at 1 and 2 (textbook values): the
# erf-form GELU is z Phi(z), so GELU(1) = Phi(1) and GELU(2) = 2 Phi(2); for
# |z| >= 9 the tail is below FP64 resolution, GELU(z) = z (z > 0) or -0 (z < 0).
PHI1 = 0.8413447460685429
PHI2 = 0.9772498680518208
# the same values rounded to bfloat16 by hand (8 significant bits):
# Phi(1) = 215.38 / 256 -> 215 / 256; 2 Phi(2) = 250.18 / 128 -> 250 / 128
PHI1_BF16 = 215.0 / 256.0
TWO_PHI2_BF16 = 250.0 / 128.0


def blank_params(nfeat=56):
    """Every weight and bias zero; identity normalisation; an unbounded box."""
    P = np.zeros(oracle.mlp_param_count(), np.float32)
    base = P.size - 6 * IN
    P[base + IN: base + 2 * IN] = 1.0            # sd_x
    P[base + 3 * IN: base + 4 * IN] = 1.0        # sd_o
    P[base + 4 * IN: base + 5 * IN] = -1e30      # xmin
    P[base + 5 * IN: base + 6 * IN] = 1e30       # xmax
    return P


def layer_views(P):
    """Writable views W_l [out x in], b_l [out] into the blob."""
    out, o = [], 0
    for l in range(5):
        ni, no = DIMS[l], DIMS[l + 1]
        W = P[o:o + no * ni].reshape(no, ni)
        o += no * ni
        b = P[o:o + no]
        o += no
        out.append((W, b))
    return out, P[o:].reshape(6, IN)


@pytest.mark.parametrize("bf16", [False, True])
def test_forward_zero_hidden_weights_is_output_layer_of_gelu_bias(bf16):
    """W_1..W_4 = 0: every hidden layer is GELU of its bias alone, so the
    output is W_5 GELU(b_4) + b_5 whatever b_1..b_3 are.  b_4 holds 0, 40,
    -40, 1 and 2, whose GELU values are known without evaluating erf."""
    P = blank_params()
    L, _ = layer_views(P)
    rng = np.random.default_rng(11)
    for l in range(3):
        L[l][1][:] = rng.standard_normal(HID).astype(np.float32)   # ignored: W_{l+1} = 0
    b4 = L[3][1]
    b4[:] = 0.0
    b4[3], b4[7], b4[11], b4[20] = 40.0, -40.0, 1.0, 2.0
    g = {3: 40.0, 11: PHI1_BF16 if bf16 else PHI1, 20: TWO_PHI2_BF16 if bf16 else 2 * PHI2}
    W5, b5 = L[4]
    # weights and biases that bfloat16 represents exactly (k / 8, |k| <= 64)
    W5[:, :] = rng.integers(-64, 65, W5.shape).astype(np.float32) / 8.0
    b5[:] = rng.integers(-64, 65, OUT).astype(np.float32) / 8.0
    X = np.zeros((3, IN))
    X[:, :56] = rng.standard_normal((3, 56))
    out = oracle.mlp_forward(P, X, 56, bf16_emulation=bf16)
    want = b5.astype(np.float64).copy()
    for i, gi in g.items():
        want += W5[:, i].astype(np.float64) * gi
    for r in range(3):
        np.testing.assert_allclose(out[r], want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("bf16", [False, True])
def test_forward_one_hot_through_identity_layers(bf16):
    """Normalisation (x - mu) / sd maps the raw one-hot value 3 of feature j
    (mu 1, sd 2) to 1; identity first layer: GELU(1) = Phi(1) on unit j, 0
    elsewhere (GELU(0) = 0); second layer 16 I lifts it to 16 Phi(1) > 9,
    where GELU is the identity, so layers three and four and the identity
    output layer pass it through: out = 16 Phi(1) e_j."""
    nfeat = 56
    P = blank_params(nfeat)
    L, nb = layer_views(P)
    L[0][0][:IN, :IN] = np.eye(IN, dtype=np.float32)
    L[1][0][:, :] = 16.0 * np.eye(HID, dtype=np.float32)
    L[2][0][:, :] = np.eye(HID, dtype=np.float32)
    L[3][0][:, :] = np.eye(HID, dtype=np.float32)
    L[4][0][:, :IN] = np.eye(OUT, dtype=np.float32)
    for j in (0, 17, nfeat - 1):
        nb[0][:] = 0.0
        nb[1][:] = 1.0
        nb[0][j], nb[1][j] = 1.0, 2.0
        X = np.zeros((1, IN))
        X[0, j] = 3.0
        out = oracle.mlp_forward(P, X, nfeat, bf16_emulation=bf16)[0]
        want = np.zeros(OUT)
        want[j] = 16.0 * (PHI1_BF16 if bf16 else PHI1)
        np.testing.assert_allclose(out, want, rtol=1e-15, atol=0)
    # features past nfeat never enter, whatever their raw value
    nb[0][:] = 0.0
    nb[1][:] = 1.0
    X = np.zeros((1, IN))
    X[0, nfeat + 2] = 5.0
    assert np.all(oracle.mlp_forward(P, X, nfeat, bf16_emulation=bf16) == 0.0)


# ------------------------------------------------------ gate threshold pins
def gate_setup(dT_target=0.3):
    """A network whose output is zero (all weights and biases zero), so the
    increments are fixed by the de-normalisation alone: mu_o = 0 for the
    species gives dY = 0 exactly, mu_o[N] = asinh(dT / 1e-6 K) gives dT.
    With dY = 0 the conserved state is the input state, T' = T (enthalpy
    unchanged), so the residual |T + dT - T'| is |dT|."""
    mech = synth.mechanism("mech53")
    o = Oracle(mech)
    N = mech.n_species
    P = blank_params(N + 3)
    _, nb = layer_views(P)
    nb[2][N] = np.float32(np.arcsinh(dT_target / 1e-6))
    dT = 1e-6 * np.sinh(float(nb[2][N]))
    f = synth.field_mapped(400, seed=4)
    i = int(np.nonzero(f.cls == 1)[0][0])
    return o, P, nb, f.p[i], f.T[i], f.Y[:, i].copy(), dT, N


def run_gate(o, P, p, T, Y, **kw):
    args = dict(tau_T=1e9, y_min=-1.0, margin=0.0, max_dT=np.inf, T_max=np.inf)
    args.update(kw)
    return oracle.surrogate_cell(o, P, p, T, Y, 1e-6, **args)


def assert_accept(res, T, Y):
    ok, T1, Y1 = res
    assert ok
    assert abs(T1 - T) <= 1e-9 and np.array_equal(Y1, Y)


def assert_reject(res, T, Y):
    ok, T1, Y1 = res
    assert not ok and T1 == T and np.array_equal(Y1, Y)


def test_gate_residual_threshold_tau_T():
    o, P, _, p, T, Y, dT, _ = gate_setup(0.3)
    assert 0.29 < dT < 0.31
    assert_accept(run_gate(o, P, p, T, Y, tau_T=dT + 1e-6), T, Y)
    assert_reject(run_gate(o, P, p, T, Y, tau_T=dT - 1e-6), T, Y)


def test_gate_residual_with_a_changed_composition():
    """Mass moved between two species (dY != 0), so the conserved state Y'
    has another enthalpy-temperature relation and T' differs from T.  The
    gate's residual is then |T + dT - T'| with T' the temperature at which Y'
    holds the input's enthalpy; it is rebuilt here from the separately pinned
    conservation and enthalpy inversion, and the threshold must fall exactly
    there (accept just above, reject just below), the accepted state being
    (T', Y')."""
    o, P, nb, p, T, Y, dT, N = gate_setup(0.3)
    a, b = (int(k) for k in np.argsort(Y)[-2:])
    for k, delta in ((a, -1e-3), (b, 1e-3)):
        nb[2][k] = np.float32(np.arcsinh(delta / 1e-12))
    dY = np.zeros(N)
    for k in (a, b):
        dY[k] = 1e-12 * np.sinh(float(nb[2][k]))
    Yc = oracle.conserve(o, Y, np.maximum(Y + dY, 0.0))
    assert Yc is not None
    Tp, _ = o.temperature_from_enthalpy(o.enthalpy(T, Y), Yc, T + dT)
    r = abs(T + dT - Tp)
    # the composition change moves T' by far more than the threshold window below
    assert abs(Tp - T) > 100 * 1e-6 * r
    ok, T1, Y1 = run_gate(o, P, p, T, Y, tau_T=r * (1 + 1e-6))
    assert ok and T1 == Tp and np.array_equal(Y1, Yc)
    assert_reject(run_gate(o, P, p, T, Y, tau_T=r * (1 - 1e-6)), T, Y)


def test_gate_predicted_dT_threshold():
    o, P, _, p, T, Y, dT, _ = gate_setup(0.3)
    assert_accept(run_gate(o, P, p, T, Y, max_dT=dT * (1 + 1e-9)), T, Y)
    assert_reject(run_gate(o, P, p, T, Y, max_dT=dT * (1 - 1e-9)), T, Y)


def test_gate_negative_mass_fraction_threshold_y_min():
    """dY = 0: the conserved state equals the input, so its smallest mass
    fraction is min Y exactly; y_min at that value passes (>=), the next
    double above it fails."""
    o, P, _, p, T, Y, _, _ = gate_setup(1e-3)
    ymin = float(Y.min())
    assert_accept(run_gate(o, P, p, T, Y, y_min=ymin), T, Y)
    assert_reject(run_gate(o, P, p, T, Y, y_min=np.nextafter(ymin, np.inf)), T, Y)


def test_gate_hottest_cell_threshold_T_max():
    o, P, _, p, T, Y, _, _ = gate_setup(1e-3)
    assert_accept(run_gate(o, P, p, T, Y, T_max=T), T, Y)
    assert_reject(run_gate(o, P, p, T, Y, T_max=np.nextafter(T, -np.inf)), T, Y)


def test_gate_training_box_margin():
    """ln T lies a distance d below a box of span s: the margin reaches it
    exactly when margin s >= d."""
    o, P, nb, p, T, Y, _, N = gate_setup(1e-3)
    x0 = np.log(T)
    nb[4][:] = -1e30
    nb[5][:] = 1e30
    nb[4][0] = np.float32(x0 + 0.5)
    nb[5][0] = np.float32(x0 + 1.5)
    d = float(nb[4][0]) - x0
    s = float(nb[5][0]) - float(nb[4][0])
    assert d > 0.4 and s > 0.9
    assert_accept(run_gate(o, P, p, T, Y, margin=d / s * (1 + 1e-9)), T, Y)
    assert_reject(run_gate(o, P, p, T, Y, margin=d / s * (1 - 1e-9)), T, Y)
    assert_reject(run_gate(o, P, p, T, Y, margin=0.0), T, Y)
    # above the box, symmetrically
    nb[4][0] = np.float32(x0 - 1.5)
    nb[5][0] = np.float32(x0 - 0.5)
    d = x0 - float(nb[5][0])
    s = float(nb[5][0]) - float(nb[4][0])
    assert_accept(run_gate(o, P, p, T, Y, margin=d / s * (1 + 1e-9)), T, Y)
    assert_reject(run_gate(o, P, p, T, Y, margin=d / s * (1 - 1e-9)), T, Y)
