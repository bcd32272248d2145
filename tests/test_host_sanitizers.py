"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle's C sources and the host load-balancing planner (csrc/balance.cpp)
are compiled with gcc / g++ -fsanitize=address,undefined, and the host side of
csrc/api.cpp (for its mechanism check) with the same sanitizers through
-Xarch_host, every finding fatal, together with small drivers
(tests/sanitize/) that call each entry point on small synthetic inputs.  A
driver must exit cleanly, and the values it prints must equal those of the
regular builds (the oracle through its ctypes binding, the planner and the
mechanism check through the library), which shows that the sanitized runs
went through the same paths.  No GPU code is built with a sanitizer, and
nothing here runs on a GPU.
"""
import copy
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2011_07978_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
# the regular oracle build's floating-point flags, so that results agree bit for bit
FP = ["-march=x86-64-v3", "-ffp-contract=off", "-fno-math-errno"]


def _env(leaks=True):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = f"detect_leaks={int(leaks)}:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "2"
    return env


def _exec(cmd, timeout):
    """Run a sanitized driver; where LeakSanitizer cannot run at all (it needs
    to stop the process's threads, which some sandboxes forbid), run again
    without leak checking rather than report a finding that is not one."""
    r = subprocess.run(cmd, capture_output=True, text=True, env=_env(), timeout=timeout)
    if r.returncode != 0 and "LeakSanitizer has encountered a fatal error" in r.stderr:
        r = subprocess.run(cmd, capture_output=True, text=True, env=_env(False), timeout=timeout)
    return r


def _compile(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        if "asan" in r.stderr.lower() or "ubsan" in r.stderr.lower():
            pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
        raise AssertionError("build failed:\n" + " ".join(cmd) + "\n" + r.stderr[-3000:])


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    from oracle.build import SOURCES
    osrc = [os.path.join(REPO, "oracle", s) for s in SOURCES]
    od = str(d / "oracle_driver")
    _compile(["gcc", "-std=gnu11", "-fopenmp", "-Wall", "-Wno-unused-function"] + FP + SAN +
             ["-o", od, os.path.join(HERE, "sanitize", "oracle_driver.c")] + osrc + ["-lm"])
    bd = str(d / "balance_driver")
    _compile(["g++", "-std=c++17", "-Wall"] + SAN +
             ["-o", bd, os.path.join(HERE, "sanitize", "balance_driver.cpp"),
              os.path.join(REPO, "paper_2011_07978_amd", "csrc", "balance.cpp")])
    return d, od, bd


def _run(exe, arg):
    r = _exec([exe, arg], 600)
    report = r.stderr
    assert r.returncode == 0, f"{os.path.basename(exe)} exited {r.returncode}:\n{report[-4000:]}"
    for bad in ("ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:"):
        assert bad not in report, report[-4000:]
    out = {}
    for line in r.stdout.splitlines():
        parts = line.split()
        if not parts:
            continue
        out.setdefault(parts[0], []).append(parts[1:])
    return out


def _vec(out, key, dtype=float):
    (row,) = out[key]
    n = int(row[0])
    v = np.array([dtype(x) for x in row[1:]])
    assert v.size == n
    return v


def _write_input(path, mech, T, p, Y, dt, Yfuel, Yox, P):
    N, R = mech.n_species, mech.n_reactions
    fo_t = getattr(mech, "falloff", None)
    fo_p = getattr(mech, "fo_params", None)
    if fo_t is None:
        fo_t, fo_p = np.zeros(R, np.int32), np.zeros((R, 7))
    pl_n = getattr(mech, "plog_count", None)
    i32 = lambda a: np.ascontiguousarray(a, np.int32).tobytes()
    f64 = lambda a: np.ascontiguousarray(a, np.float64).tobytes()
    with open(path, "wb") as f:
        f.write(i32([mech.n_elements, N, R, len(mech.eff_value), int(pl_n is not None),
                     T.size, P.size]))
        f.write(f64(mech.elem_mass) + i32(mech.composition) + f64(mech.W) + f64(mech.nasa))
        f.write(i32(mech.reactants) + i32(mech.products) + f64(mech.A) + f64(mech.b) + f64(mech.Ea))
        f.write(i32(mech.third_body) + i32(mech.eff_reaction) + i32(mech.eff_species))
        f.write(f64(mech.eff_value) + i32(fo_t) + f64(fo_p))
        if pl_n is not None:
            f.write(i32(pl_n) + f64(mech.plog_params))
        f.write(f64([p, dt]) + f64(T) + f64(Y) + f64(Yfuel) + f64(Yox))
        f.write(np.ascontiguousarray(P, np.float32).tobytes())


def _cells(mech, n, seed):
    rng = np.random.default_rng(seed)
    N = mech.n_species
    Z = rng.uniform(0.05, 0.95, size=n)
    Yf, Yo = synth.stream_fuel(mech), synth.stream_oxidiser(mech)
    Y = 0.7 * (np.outer(Yf, Z) + np.outer(Yo, 1.0 - Z)) + 0.3 * rng.dirichlet(np.full(N, 0.5), n).T
    T = rng.uniform(800.0, 1600.0, size=n)
    return T, Y / Y.sum(axis=0), Yf, Yo


@pytest.mark.parametrize("name", ["small", "mech53fo", "mech53pl"])
def test_oracle_clean_under_sanitizers(drivers, name):
    d, od, _ = drivers
    mech = synth.mechanism(name)
    N = mech.n_species
    T, Y, Yf, Yo = _cells(mech, 4, seed=11)
    p, dt = synth.P_ATM, 1e-7
    P = synth.surrogate_params(N, seed=3, weight_scale=1.0)
    path = str(d / f"in_{name}.bin")
    _write_input(path, mech, T, p, Y, dt, Yf, Yo, P)
    out = _run(od, path)

    o = oracle.Oracle(mech)
    y0 = np.concatenate([[T[0]], Y[:, 0]])
    assert np.array_equal(_vec(out, "rhs"), o.rhs(p, y0))
    assert np.array_equal(_vec(out, "jac"), o.jac(p, y0).ravel())
    assert np.array_equal(_vec(out, "jac_cs"), o.jac_cs(p, y0).ravel())
    yc, hc, st = o.integrate_cell(p, y0, dt)
    assert np.array_equal(_vec(out, "cell_y"), yc)
    assert _vec(out, "cell_h")[0] == hc
    assert list(_vec(out, "cell_stats", int)) == [st.n_accept, st.n_reject, st.n_jac, st.n_lu,
                                                   st.n_rhs, st.status]
    for sched, tag in ((0, "static"), (1, "dyn")):
        Tb, Yb, _, sb, na, nr = o.integrate_batch(T, np.full(T.size, p), Y, dt, threads=2,
                                                  schedule=sched)
        assert np.array_equal(_vec(out, "batch_T_" + tag), Tb)
        assert np.array_equal(_vec(out, "batch_Y_" + tag), Yb.ravel())
        assert list(_vec(out, "batch_steps_" + tag, int)) == list(na + nr + 1000 * sb.astype(int))
    flags, ref = o.map_reference(T, Y, Yf, Yo, 1e-2, 1.0, False)
    assert list(_vec(out, "map_flags", int)) == list(flags) + [ref]
    X = np.stack([oracle.mlp_features(N, T[c], p, Y[:, c], dt) for c in range(T.size)])
    assert np.array_equal(_vec(out, "mlp_x"), X.ravel())
    assert np.array_equal(_vec(out, "mlp_out_bf16"), oracle.mlp_forward(P, X, N + 3, True).ravel())
    assert np.array_equal(_vec(out, "mlp_out_f64"), oracle.mlp_forward(P, X, N + 3, False).ravel())
    gates = [oracle.surrogate_cell(o, P, p, T[c], Y[:, c], dt, 0.5, -1e-10, 0.0, 1.0, 1000.0)
             for c in range(T.size)]
    assert list(_vec(out, "gate", int)) == [int(g[0]) for g in gates]
    assert np.array_equal(_vec(out, "gate_T"), np.array([g[1] for g in gates]))


def test_planner_clean_under_sanitizers(drivers):
    from paper_2011_07978_amd import chem
    try:
        chem.load_library()
    except RuntimeError:
        pytest.skip("libchem.so not built")
    d, _, bd = drivers
    rng = np.random.default_rng(5)
    cases = []
    for n_proc in (1, 2, 3, 7, 16, 64):
        n_prob = rng.integers(0, 40, size=n_proc)
        cost = rng.exponential(1.0, size=int(n_prob.sum())) * rng.choice([1.0, 9.0], size=int(n_prob.sum()))
        cases.append((n_proc, 0.01, 2 * n_proc, n_prob, cost))
    cases.append((4, 0.01, 8, np.array([0, 0, 3, 3]), np.full(6, 2.0)))        # hand-worked case
    cases.append((4, 0.0, 8, np.zeros(4, np.int64), np.zeros(0)))              # no load at all
    cases.append((5, 0.01, 1, np.array([1, 1, 1, 1, 20]), np.ones(24)))        # too few slots
    path = str(d / "cases.txt")
    with open(path, "w") as f:
        f.write(f"{len(cases)}\n")
        for n_proc, mf, mo, n_prob, cost in cases:
            f.write(f"{n_proc} {mf!r} {mo}\n")
            at = 0
            for k in n_prob:
                f.write(" ".join([str(int(k))] + [repr(float(c)) for c in cost[at:at + k]]) + "\n")
                at += int(k)
    r = _exec([bd, path], 300)
    assert r.returncode == 0, r.stderr[-4000:]
    for bad in ("ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:"):
        assert bad not in r.stderr, r.stderr[-4000:]
    blocks, cur = [], None
    for line in r.stdout.splitlines():
        w = line.split()
        if w[0] == "case":
            cur = {"rc": int(w[3]), "n_ops": int(w[5]), "ops": [], "loads": None}
            blocks.append(cur)
        elif w[0] == "op":
            cur["ops"].append((int(w[1]), int(w[2]), int(w[3]), int(w[4]), float(w[5]), float(w[6])))
        elif w[0] == "loads":
            cur["loads"] = [float(x) for x in w[1:]]
    assert len(blocks) == len(cases)
    for (n_proc, mf, mo, n_prob, cost), got in zip(cases, blocks):
        if mo < 2 * n_proc:
            assert got["rc"] != 0 and got["n_ops"] > mo     # refused after filling the slots
            continue
        assert got["rc"] == 0
        ops, after = chem.plan_balance(n_prob, cost, mf)
        assert got["ops"] == ops
        assert got["loads"] == list(after)


# ------------------------------------------------ the library's mechanism check
def _write_desc(path, mech):
    R = mech.n_reactions
    fo_t = getattr(mech, "falloff", None)
    pl_n = getattr(mech, "plog_count", None)
    i32 = lambda a: np.ascontiguousarray(a, np.int32).tobytes()
    f64 = lambda a: np.ascontiguousarray(a, np.float64).tobytes()
    with open(path, "wb") as f:
        f.write(i32([mech.n_elements, mech.n_species, R, len(mech.eff_value),
                     int(fo_t is not None), int(pl_n is not None)]))
        f.write(f64(mech.elem_mass) + i32(mech.composition) + f64(mech.W) + f64(mech.nasa))
        f.write(i32(mech.reactants) + i32(mech.products) + f64(mech.A) + f64(mech.b) + f64(mech.Ea))
        f.write(i32(mech.third_body) + i32(mech.eff_reaction) + i32(mech.eff_species))
        f.write(f64(mech.eff_value))
        if fo_t is not None:
            f.write(i32(fo_t) + f64(mech.fo_params))
        if pl_n is not None:
            f.write(i32(pl_n) + f64(mech.plog_params))


def _broken(m, **kw):
    b = copy.deepcopy(m)
    for k, v in kw.items():
        setattr(b, k, v)
    return b


def test_mechanism_check_clean_under_sanitizers(tmp_path):
    from paper_2011_07978_amd import chem
    try:
        chem.load_library()
    except RuntimeError:
        pytest.skip("libchem.so not built")
    bdir = os.path.join(REPO, "paper_2011_07978_amd", "_build")
    others = [os.path.join(bdir, f) for f in ("balance.cpp.o", "integrate.hip.o",
                                              "integrate_fo.hip.o", "integrate_big.hip.o",
                                              "map_queue.hip.o", "mlp.hip.o")]
    if not all(os.path.exists(o) for o in others):
        pytest.skip("library objects not built")
    rocm = "/opt/rocm"
    api_o, drv_o, exe = str(tmp_path / "api_san.o"), str(tmp_path / "drv.o"), str(tmp_path / "vd")
    host_san = []
    for flag in SAN[:3]:
        host_san += ["-Xarch_host", flag]
    _compile([f"{rocm}/bin/hipcc", "-x", "hip", "-std=c++17", "-O1", "-g", "-fPIC",
              "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wno-unused-command-line-argument"] + host_san +
             ["-c", os.path.join(REPO, "paper_2011_07978_amd", "csrc", "api.cpp"), "-o", api_o])
    clang = f"{rocm}/llvm/bin/clang++"
    _compile([clang, "-std=c++17", "-O1", "-g"] + SAN[:3] +
             ["-c", os.path.join(HERE, "sanitize", "validate_driver.cpp"), "-o", drv_o])
    _compile([clang] + SAN[:3] + ["-o", exe, drv_o, api_o] + others +
             [f"-L{rocm}/lib", "-lamdhip64", f"-Wl,-rpath,{rocm}/lib"])

    base = synth.mechanism("mech53")
    fo, pl = synth.mechanism("mech53fo"), synth.mechanism("mech53pl")
    prod = base.products.copy()
    k = int(prod[17, 0])
    prod[17, 0] = next(q for q in range(base.n_species)
                       if not np.array_equal(base.composition[q], base.composition[k]))
    W = base.W.copy()
    W[5] *= 1.0 + 1e-6
    nasa = base.nasa.copy()
    nasa[3, 1] = -1e-2
    A = base.A.copy()
    A[9] = 0.0
    rea = base.reactants.copy()
    rea[3, 0] = base.n_species
    er = base.eff_reaction.copy()
    er[0] = int(np.nonzero(base.third_body == 0)[0][0])
    t = fo.falloff.copy()
    t[int(np.nonzero(fo.third_body == 0)[0][0])] = 2
    j = int(np.nonzero(pl.plog_count)[0][0])
    Pp = pl.plog_params.copy()
    Pp[j, 1, 0] = Pp[j, 0, 0]
    cases = [synth.mechanism("small"), base, fo, pl, synth.mechanism("mech130"),
             _broken(base, products=prod), _broken(base, W=W), _broken(base, nasa=nasa),
             _broken(base, A=A), _broken(base, reactants=rea), _broken(base, eff_reaction=er),
             _broken(fo, falloff=t), _broken(pl, plog_params=Pp)]
    paths = []
    for i, m in enumerate(cases):
        paths.append(str(tmp_path / f"m{i}.bin"))
        _write_desc(paths[-1], m)
    r = _exec([exe] + paths, 300)
    assert r.returncode == 0, r.stderr[-4000:]
    for bad in ("ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:"):
        assert bad not in r.stderr, r.stderr[-4000:]
    lines = r.stdout.splitlines()
    assert len(lines) == len(cases)
    for m, line in zip(cases, lines):
        rc, why = chem.validate_mechanism(m)
        assert line == f"rc {rc} {why}"
    assert [int(l.split()[1]) for l in lines] == [0] * 5 + [-7] * 8
