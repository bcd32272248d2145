"""CPU oracle (FP64, serial per cell) — TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding) never
does.  The C sources next to this file implement, in plain serial FP64, every
computation of the chemistry hot path; see oracle.h for the formulas and the
paper passages they follow.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

_lib = None

_d = C.POINTER(C.c_double)
_i32 = C.POINTER(C.c_int32)
_u8 = C.POINTER(C.c_uint8)


class OOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("max_steps", C.c_int),
                ("hmin_frac", C.c_double), ("use_cs_jac", C.c_int)]


class OStats(C.Structure):
    _fields_ = [("n_accept", C.c_int), ("n_reject", C.c_int), ("n_jac", C.c_int),
                ("n_lu", C.c_int), ("n_rhs", C.c_int), ("status", C.c_int)]


def lib():
    global _lib
    if _lib is None:
        # ORACLE_LIB names another build of these sources (the mutation tests
        # load deliberately broken copies through it); by default the library
        # next to this file, built on first use
        path = os.environ.get("ORACLE_LIB", "")
        if not path:
            path = LIB
            if not os.path.exists(LIB):
                build()
        L = C.CDLL(path)
        L.orc_mech_create.restype = C.c_int
        L.orc_map_reference.restype = C.c_int64
        L.orc_enthalpy_mass.restype = C.c_double
        L.orc_cp_mass.restype = C.c_double
        L.orc_density.restype = C.c_double
        L.orc_temperature_from_enthalpy.restype = C.c_double
        L.orc_integrate_cell.restype = C.c_int
        L.orc_rodas4_step.restype = C.c_int
        L.orc_lu.restype = C.c_int
        L.orc_mlp_param_count.restype = C.c_int64
        L.orc_bf16.restype = C.c_double
        L.orc_bf16.argtypes = [C.c_double]
        L.orc_mlp_loss_grad.restype = C.c_double
        L.orc_surrogate_cell.restype = C.c_int
        _lib = L
    return _lib


def _p(a, t=_d):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class Oracle:
    """Oracle bound to one mechanism (synth.Mechanism or anything with its fields)."""

    RTOL, ATOL = 1e-8, 1e-12

    def __init__(self, mech):
        L = lib()
        self.mech = mech
        self.N = int(mech.n_species)
        self.n = self.N + 1
        self.R = int(mech.n_reactions)
        fo_t = getattr(mech, "falloff", None)
        fo_p = getattr(mech, "fo_params", None)
        if fo_t is None:
            fo_t, fo_p = np.zeros(self.R, np.int32), np.zeros((self.R, 7))
        self._keep = [_f64(mech.elem_mass), _i(mech.composition), _f64(mech.W), _f64(mech.nasa),
                      _i(mech.reactants), _i(mech.products), _f64(mech.A), _f64(mech.b),
                      _f64(mech.Ea), _i(mech.third_body), _i(mech.eff_reaction),
                      _i(mech.eff_species), _f64(mech.eff_value), _i(fo_t), _f64(fo_p)]
        k = self._keep
        h = C.c_void_p()
        rc = L.orc_mech_create(C.byref(h), int(mech.n_elements), self.N, self.R,
                               _p(k[0]), _p(k[1], _i32), _p(k[2]), _p(k[3]), _p(k[4], _i32),
                               _p(k[5], _i32), _p(k[6]), _p(k[7]), _p(k[8]), _p(k[9], _i32),
                               int(len(k[12])), _p(k[10], _i32), _p(k[11], _i32), _p(k[12]),
                               _p(k[13], _i32), _p(k[14]))
        if rc != 0:
            raise RuntimeError("orc_mech_create failed")
        self.h = h
        pl_n = getattr(mech, "plog_count", None)
        if pl_n is not None:
            self._keep += [_i(pl_n), _f64(mech.plog_params)]
            if L.orc_mech_set_plog(h, _p(self._keep[-2], _i32), _p(self._keep[-1])) != 0:
                raise RuntimeError("orc_mech_set_plog failed")

    def __del__(self):
        try:
            lib().orc_mech_destroy(self.h)
        except Exception:
            pass

    # -- thermo / kinetics -------------------------------------------------
    def thermo(self, T):
        cp, h, s = (np.zeros(self.N) for _ in range(3))
        lib().orc_thermo(self.h, C.c_double(T), _p(cp), _p(h), _p(s))
        return cp, h, s

    def ln_kf(self, j, T, p):
        """ln k_f of reaction j at (T, p): Arrhenius, or for a PLOG reaction
        the interpolation in ln p of its tabulated rate expressions."""
        f = lib().orc_ln_kf
        f.restype = C.c_double
        return f(self.h, C.c_int(int(j)), C.c_double(T), C.c_double(p))

    def falloff_factor(self, j, T, M):
        """G of reaction j (its rate constant is k_inf G); [M] itself when j has
        no fall-off form."""
        f = lib().orc_falloff_factor
        f.restype = C.c_double
        return f(self.h, C.c_int(int(j)), C.c_double(T), C.c_double(M))

    def kinetics(self, T, p, Y):
        Y = _f64(Y)
        kf, kr, q = (np.zeros(self.R) for _ in range(3))
        om = np.zeros(self.N)
        lib().orc_kinetics(self.h, C.c_double(T), C.c_double(p), _p(Y), _p(kf), _p(kr), _p(q), _p(om))
        return kf, kr, q, om

    def rhs(self, p, y):
        y = _f64(y)
        f = np.zeros(self.n)
        lib().orc_rhs(self.h, C.c_double(p), _p(y), _p(f))
        return f

    def rhs_cs_dir(self, p, y, v, hstep=1e-30):
        y, v = _f64(y), _f64(v)
        fr, fi = np.zeros(self.n), np.zeros(self.n)
        lib().orc_rhs_cs_dir(self.h, C.c_double(p), _p(y), _p(v), C.c_double(hstep), _p(fr), _p(fi))
        return fr, fi

    def jac(self, p, y):
        y = _f64(y)
        J = np.zeros((self.n, self.n))
        lib().orc_jac(self.h, C.c_double(p), _p(y), _p(J))
        return J

    def jac_cs(self, p, y):
        y = _f64(y)
        J = np.zeros((self.n, self.n))
        lib().orc_jac_cs(self.h, C.c_double(p), _p(y), _p(J))
        return J

    def enthalpy(self, T, Y):
        return lib().orc_enthalpy_mass(self.h, C.c_double(T), _p(_f64(Y)))

    def cp(self, T, Y):
        return lib().orc_cp_mass(self.h, C.c_double(T), _p(_f64(Y)))

    def density(self, T, p, Y):
        return lib().orc_density(self.h, C.c_double(T), C.c_double(p), _p(_f64(Y)))

    def temperature_from_enthalpy(self, h, Y, T_guess):
        it = C.c_int()
        T = lib().orc_temperature_from_enthalpy(self.h, C.c_double(h), _p(_f64(Y)),
                                                C.c_double(T_guess), C.byref(it))
        return T, it.value

    # -- integration -------------------------------------------------------
    def opts(self, rtol=None, atol=None, max_steps=100000, hmin_frac=1e-14, cs_jac=False):
        return OOpts(self.RTOL if rtol is None else rtol, self.ATOL if atol is None else atol,
                     max_steps, hmin_frac, 1 if cs_jac else 0)

    def rodas4_step(self, p, y, h, J=None):
        y = _f64(y)
        f0 = self.rhs(p, y)
        J = self.jac(p, y) if J is None else _f64(J)
        yn, err = np.zeros(self.n), np.zeros(self.n)
        rc = lib().orc_rodas4_step(self.h, C.c_double(p), _p(y), _p(f0), _p(J), C.c_double(h),
                                   _p(yn), _p(err))
        return yn, err, rc

    def integrate_cell(self, p, y, dt, h0=0.0, **kw):
        y = _f64(y).copy()
        hh = C.c_double(h0)
        st = OStats()
        o = self.opts(**kw)
        lib().orc_integrate_cell(self.h, C.c_double(p), _p(y), C.c_double(dt), C.byref(o),
                                 C.byref(hh), C.byref(st))
        return y, hh.value, st

    def integrate_batch(self, T, p, Y, dt, h=None, flags=None, threads=0, schedule=0, **kw):
        """Returns (T, Y, h, status, n_acc, n_rej); inputs are not modified."""
        T = _f64(T).copy()
        p = _f64(p)
        Y = _f64(Y).copy()
        ncells = T.shape[0]
        h = np.zeros(ncells) if h is None else _f64(h).copy()
        st = np.zeros(ncells, np.uint8)
        na = np.zeros(ncells, np.int32)
        nr = np.zeros(ncells, np.int32)
        fl = None if flags is None else np.ascontiguousarray(flags, dtype=np.uint8)
        o = self.opts(**kw)
        lib().orc_integrate_batch(self.h, C.c_int64(ncells), _p(T), _p(p), _p(Y), C.c_double(dt),
                                  C.byref(o), _p(h), None if fl is None else _p(fl, _u8),
                                  _p(st, _u8), _p(na, _i32), _p(nr, _i32), int(threads), int(schedule))
        return T, Y, h, st, na, nr

    def rk4(self, p, y, t_end, nsteps):
        y = _f64(y).copy()
        lib().orc_rk4(self.h, C.c_double(p), _p(y), C.c_double(t_end), C.c_int64(nsteps))
        return y

    # -- mapping -----------------------------------------------------------
    def map_weights(self, Yfuel, Yox):
        w = np.zeros(self.N)
        bf, bo = C.c_double(), C.c_double()
        lib().orc_map_weights(self.h, _p(_f64(Yfuel)), _p(_f64(Yox)), _p(w), C.byref(bf), C.byref(bo))
        return w, bf.value, bo.value

    def mixture_fraction(self, Y, w, beta_f, beta_ox):
        Y = _f64(Y)
        ncells = Y.shape[1]
        Z = np.zeros(ncells)
        lib().orc_mixture_fraction(self.h, C.c_int64(ncells), _p(Y), _p(_f64(w)),
                                   C.c_double(beta_f), C.c_double(beta_ox), _p(Z))
        return Z

    def map_reference(self, T, Y, Yfuel, Yox, Z_tol, T_tol=1.0, use_T=False):
        w, bf, bo = self.map_weights(Yfuel, Yox)
        T, Y = _f64(T), _f64(Y)
        ncells = T.shape[0]
        flags = np.zeros(ncells, np.uint8)
        ref = lib().orc_map_reference(self.h, C.c_int64(ncells), _p(T), _p(Y), _p(w),
                                      C.c_double(bf), C.c_double(bo), C.c_double(Z_tol),
                                      C.c_double(T_tol), int(bool(use_T)), _p(flags, _u8))
        return flags, int(ref)

    def map_scatter(self, T, Y, flags, Yref_old, Yref_new):
        T, Y = _f64(T).copy(), _f64(Y).copy()
        lib().orc_map_scatter(self.h, C.c_int64(T.shape[0]), _p(T), _p(Y),
                              _p(np.ascontiguousarray(flags, np.uint8), _u8),
                              _p(_f64(Yref_old)), _p(_f64(Yref_new)))
        return T, Y

    def step_mapped(self, T, p, Y, dt, flags, ref, h=None, threads=0, **kw):
        """Full oracle step with reference mapping (Sec. 2.3): integrate flags
        0/1, then give flag-2 cells the reference's increment (status 5).  If
        the reference's own integration failed (status != 0) there is no
        solution to copy: flag-2 cells keep their state and take status 7.
        Returns (T, Y, h, status, n_acc, n_rej)."""
        if ref < 0:
            return self.integrate_batch(T, p, Y, dt, h=h, threads=threads, **kw)
        Yref_old = _f64(Y)[:, ref].copy()
        out = self.integrate_batch(T, p, Y, dt, h=h, flags=flags, threads=threads, **kw)
        T2, Y2, h2, st = out[0], out[1], out[2], out[3].copy()
        mapped = np.asarray(flags) == 2
        if st[ref] != 0:
            st[mapped] = 7
            return (T2, Y2, h2, st) + tuple(out[4:])
        Yref_new = Y2[:, ref].copy()
        T3, Y3 = self.map_scatter(T2, Y2, flags, Yref_old, Yref_new)
        st[mapped] = 5
        return (T3, Y3, h2, st) + tuple(out[4:])


# ----------------------------------------------------------------- surrogate
MLP_IN, MLP_HID, MLP_OUT = 64, 256, 64


def mlp_param_count():
    return int(lib().orc_mlp_param_count())


def bf16(x):
    return lib().orc_bf16(float(x))


def mlp_features(N, T, p, Y, dt):
    x = np.zeros(MLP_IN)
    lib().orc_mlp_features(int(N), C.c_double(T), C.c_double(p), _p(_f64(Y)), C.c_double(dt), _p(x))
    return x


def mlp_forward(params, X, nfeat, bf16_emulation=True, want_acts=False):
    P = np.ascontiguousarray(params, np.float32)
    X = _f64(X)
    n = X.shape[0]
    out = np.zeros((n, MLP_OUT))
    acts = np.zeros((n, 4, MLP_HID)) if want_acts else None
    lib().orc_mlp_forward(P.ctypes.data_as(C.POINTER(C.c_float)), C.c_int64(n), int(nfeat), _p(X),
                          int(bool(bf16_emulation)), _p(out),
                          _p(acts) if acts is not None else None, None)
    return (out, acts) if want_acts else out


def mlp_loss_grad(params, X, target, nfeat, nout, bf16_emulation=False):
    P = np.ascontiguousarray(params, np.float32)
    X, target = _f64(X), _f64(target)
    g = np.zeros(mlp_param_count())
    loss = lib().orc_mlp_loss_grad(P.ctypes.data_as(C.POINTER(C.c_float)), C.c_int64(X.shape[0]),
                                   int(nfeat), int(nout), _p(X), _p(target),
                                   int(bool(bf16_emulation)), _p(g))
    return loss, g


def conserve(o, Y0, Y1):
    """Clipped prediction Y1 corrected to conserve the elements of Y0; None if
    the weighted element matrix is singular."""
    y = _f64(Y1).copy()
    rc = lib().orc_conserve(o.h, _p(_f64(Y0)), _p(y))
    return None if rc else y


def surrogate_cell(o, params, p, T, Y, dt, tau_T=0.5, y_min=-1e-10, margin=0.0, max_dT=np.inf,
                   T_max=np.inf):
    P = np.ascontiguousarray(params, np.float32)
    Tc = C.c_double(T)
    Yc = _f64(Y).copy()
    ok = lib().orc_surrogate_cell(o.h, P.ctypes.data_as(C.POINTER(C.c_float)), C.c_double(p),
                                  C.byref(Tc), _p(Yc), C.c_double(dt), C.c_double(tau_T),
                                  C.c_double(y_min), C.c_double(margin), C.c_double(max_dT),
                                  C.c_double(T_max))
    return bool(ok), Tc.value, Yc


def rodas4_coefficients():
    a = np.zeros((6, 6))
    c = np.zeros((6, 6))
    g = C.c_double()
    lib().orc_rodas4_coeffs(_p(a), _p(c), C.byref(g))
    return a, c, g.value


def lu(A):
    A = _f64(A).copy()
    n = A.shape[0]
    piv = np.zeros(n, np.int32)
    rc = lib().orc_lu(n, _p(A), _p(piv, _i32))
    return A, piv, rc


def lu_solve(LU, piv, b):
    b = _f64(b).copy()
    lib().orc_lu_solve(LU.shape[0], _p(_f64(LU)), _p(np.ascontiguousarray(piv, np.int32), _i32), _p(b))
    return b
