"""Python binding of libchem (ctypes).  Argument marshalling only.

Every computation runs in the HIP kernels of libchem.so; PyTorch tensors only
provide device memory and the HIP stream.  Names follow the C ABI in
include/chem.h (chem_set_mechanism -> Chem.set_mechanism, ...).  There is no
CPU fallback: without the built library or a HIP device the constructor raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchem.so")

CHEM_SCHED_PLAIN, CHEM_SCHED_QUEUE, CHEM_SCHED_BLOCKS = 0, 1, 2
(CELL_OK, CELL_MAX_STEPS, CELL_H_UNDERFLOW, CELL_NONFINITE, CELL_BAD_INPUT, CELL_MAPPED,
 CELL_SURROGATE, CELL_REF_FAILED) = range(8)
FLAG_SOLVE, FLAG_REFERENCE, FLAG_MAPPED, FLAG_SURROGATE = range(4)

_d = C.POINTER(C.c_double)
_i32 = C.POINTER(C.c_int32)


class MechDesc(C.Structure):
    _fields_ = [("n_elements", C.c_int32), ("n_species", C.c_int32), ("n_reactions", C.c_int32),
                ("elem_mass", _d), ("composition", _i32), ("W", _d), ("nasa", _d),
                ("reactants", _i32), ("products", _i32), ("A", _d), ("b", _d), ("Ea", _d),
                ("third_body", _i32), ("n_eff", C.c_int32), ("eff_reaction", _i32),
                ("eff_species", _i32), ("eff_value", _d), ("falloff", _i32),
                ("falloff_params", _d), ("plog_count", _i32), ("plog_params", _d)]


class Options(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("max_steps", C.c_int32),
                ("hmin_frac", C.c_double), ("schedule", C.c_int32), ("queue_chunk", C.c_int32),
                ("slots_per_cu", C.c_int32), ("order_by_cost", C.c_int32)]


class BalanceOp(C.Structure):
    _fields_ = [("sender", C.c_int32), ("receiver", C.c_int32), ("first", C.c_int64),
                ("count", C.c_int64), ("load", C.c_double), ("planned", C.c_double)]


def plan_balance(n_prob, t_cost, min_frac=0.01):
    """Algorithm 1 (Sec. 2.2) on the host: returns (operations, loads_after).
    operations: list of (sender, receiver, first, count, load, planned);
    n_prob[k] problems per process, t_cost their costs concatenated in list
    order.  Needs no GPU."""
    import numpy as np
    L = load_library()
    n_prob = np.ascontiguousarray(n_prob, dtype=np.int64)
    t_cost = np.ascontiguousarray(t_cost, dtype=np.float64)
    n_proc = int(n_prob.size)
    max_ops = max(1, 2 * n_proc)
    ops = (BalanceOp * max_ops)()
    n_ops = C.c_int64(0)
    after = np.zeros(max(n_proc, 1), dtype=np.float64)
    rc = L.chem_plan_balance(n_proc, n_prob.ctypes.data_as(C.POINTER(C.c_int64)),
                             t_cost.ctypes.data_as(C.POINTER(C.c_double)), float(min_frac), ops,
                             max_ops, C.byref(n_ops), after.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != 0:
        raise ChemError(f"chem_plan_balance failed ({rc})")
    out = [(o.sender, o.receiver, o.first, o.count, o.load, o.planned) for o in ops[:n_ops.value]]
    return out, after[:n_proc]


class MapParams(C.Structure):
    _fields_ = [("Z_tol", C.c_double), ("T_tol", C.c_double), ("use_T", C.c_int32),
                ("Y_fuel", _d), ("Y_ox", _d)]


class Stats(C.Structure):
    _fields_ = [("cells_integrated", C.c_int64), ("cells_mapped", C.c_int64),
                ("cells_failed", C.c_int64), ("steps_accepted", C.c_int64),
                ("steps_rejected", C.c_int64), ("max_cell_steps", C.c_int32),
                ("reserved", C.c_int32), ("ms_total", C.c_double), ("ms_integrate", C.c_double),
                ("cells_surrogate", C.c_int64), ("cells_rejected", C.c_int64),
                ("ms_surrogate", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class TrainParams(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr_max", C.c_double),
                ("lr_min", C.c_double), ("seed", C.c_uint64), ("verbose", C.c_int32)]


class GateParams(C.Structure):
    _fields_ = [("tau_T", C.c_double), ("y_min", C.c_double), ("margin", C.c_double),
                ("max_dT", C.c_double), ("T_max", C.c_double)]


class TuneEntry(C.Structure):
    _fields_ = [("schedule", C.c_int32), ("queue_chunk", C.c_int32), ("slots_per_cu", C.c_int32),
                ("ms", C.c_double)]


EXPORTS = ["chem_create", "chem_destroy", "chem_set_stream", "chem_last_error",
           "chem_set_mechanism", "chem_validate_mechanism", "chem_max_species", "chem_set_options", "chem_get_options",
           "chem_query_slots", "chem_plan_balance", "chem_integrate_noalloc",
           "chem_default_options", "chem_reserve", "chem_map_reference", "chem_integrate",
           "chem_eval_rhs_jac", "chem_rodas_step", "chem_integrate_surrogate",
           "chem_default_train_params", "chem_default_gate_params", "chem_surrogate_param_count",
           "chem_surrogate_train", "chem_surrogate_get_params", "chem_surrogate_set_params",
           "chem_surrogate_save", "chem_surrogate_load", "chem_surrogate_forward",
           "chem_surrogate_forward_fused",
           "chem_surrogate_loss_grad", "chem_graph_begin", "chem_graph_end", "chem_graph_launch",
           "chem_graph_destroy", "chem_autotune", "chem_autotune_forget"]
_VOID = ("chem_destroy", "chem_default_options", "chem_last_error", "chem_default_train_params",
         "chem_default_gate_params", "chem_surrogate_param_count", "chem_graph_destroy",
         "chem_autotune_forget")

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libchem.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libchem.so not built ({path}); run __graft_entry__.build()")
    L = C.CDLL(path)
    vp = C.c_void_p
    L.chem_create.argtypes = [C.POINTER(vp), C.c_int, vp]
    L.chem_destroy.argtypes = [vp]
    L.chem_destroy.restype = None
    L.chem_set_stream.argtypes = [vp, vp]
    L.chem_last_error.argtypes = [vp]
    L.chem_last_error.restype = C.c_char_p
    L.chem_set_mechanism.argtypes = [vp, C.POINTER(MechDesc)]
    L.chem_validate_mechanism.argtypes = [C.POINTER(MechDesc), C.c_char_p, C.c_int32]
    L.chem_max_species.argtypes = []
    L.chem_set_options.argtypes = [vp, C.POINTER(Options)]
    L.chem_get_options.argtypes = [vp, C.POINTER(Options)]
    L.chem_query_slots.argtypes = [vp, C.POINTER(C.c_int64)]
    L.chem_plan_balance.argtypes = [C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                    C.c_double, C.POINTER(BalanceOp), C.c_int64,
                                    C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    L.chem_default_options.argtypes = [C.POINTER(Options)]
    L.chem_default_options.restype = None
    L.chem_reserve.argtypes = [vp, C.c_int64]
    L.chem_map_reference.argtypes = [vp, C.c_int64, vp, vp, vp, C.POINTER(MapParams), vp, vp]
    L.chem_integrate.argtypes = [vp, C.c_int64, vp, vp, vp, C.c_double, vp, vp, vp, vp, vp, vp,
                                 C.POINTER(Stats)]
    L.chem_integrate_noalloc.argtypes = L.chem_integrate.argtypes
    L.chem_eval_rhs_jac.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp]
    L.chem_rodas_step.argtypes = [vp, C.c_int64, vp, vp, vp, C.c_double, vp, vp]
    L.chem_integrate_surrogate.argtypes = [vp, C.c_int64, vp, vp, vp, C.c_double, vp, vp,
                                           C.POINTER(GateParams), vp, vp, vp, vp, C.POINTER(Stats)]
    L.chem_default_train_params.argtypes = [C.POINTER(TrainParams)]
    L.chem_default_train_params.restype = None
    L.chem_default_gate_params.argtypes = [C.POINTER(GateParams)]
    L.chem_default_gate_params.restype = None
    L.chem_surrogate_param_count.argtypes = []
    L.chem_surrogate_param_count.restype = C.c_int64
    L.chem_surrogate_train.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp, vp,
                                       C.POINTER(TrainParams), vp]
    L.chem_surrogate_get_params.argtypes = [vp, vp]
    L.chem_surrogate_set_params.argtypes = [vp, vp]
    L.chem_surrogate_save.argtypes = [vp, C.c_char_p]
    L.chem_surrogate_load.argtypes = [vp, C.c_char_p]
    L.chem_surrogate_forward.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp]
    L.chem_surrogate_forward_fused.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp]
    L.chem_surrogate_loss_grad.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp, vp, vp,
                                           C.POINTER(C.c_double)]
    L.chem_graph_begin.argtypes = [vp]
    L.chem_graph_end.argtypes = [vp, C.POINTER(vp)]
    L.chem_graph_launch.argtypes = [vp, vp]
    L.chem_graph_destroy.argtypes = [vp]
    L.chem_graph_destroy.restype = None
    L.chem_autotune.argtypes = [vp, C.c_int64, vp, vp, vp, C.c_double, vp, vp,
                                C.POINTER(TuneEntry), C.c_int32, C.POINTER(C.c_int32)]
    L.chem_autotune_forget.argtypes = []
    L.chem_autotune_forget.restype = None
    for name in EXPORTS:
        if name not in _VOID:
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return C.c_void_p(t.data_ptr())


def _np(a, dtype):
    import numpy as np
    return np.ascontiguousarray(a, dtype=dtype)


class ChemError(RuntimeError):
    pass


def mech_desc(mech):
    """chem_mech_desc of a mechanism object (synth.Mechanism or anything with
    its fields), and the host arrays it points into (keep them alive)."""
    import numpy as np
    k = [_np(mech.elem_mass, np.float64), _np(mech.composition, np.int32), _np(mech.W, np.float64),
         _np(mech.nasa, np.float64), _np(mech.reactants, np.int32), _np(mech.products, np.int32),
         _np(mech.A, np.float64), _np(mech.b, np.float64), _np(mech.Ea, np.float64),
         _np(mech.third_body, np.int32), _np(mech.eff_reaction, np.int32),
         _np(mech.eff_species, np.int32), _np(mech.eff_value, np.float64)]
    P = lambda a, t: a.ctypes.data_as(t)
    fo_t = getattr(mech, "falloff", None)
    fo_p = getattr(mech, "fo_params", None)
    if fo_t is not None:
        k += [_np(fo_t, np.int32), _np(fo_p, np.float64)]
    pl_n = getattr(mech, "plog_count", None)
    pl = []
    if pl_n is not None:
        pl = [_np(pl_n, np.int32), _np(mech.plog_params, np.float64)]
        k += pl
    d = MechDesc(int(mech.n_elements), int(mech.n_species), int(mech.n_reactions),
                 P(k[0], _d), P(k[1], _i32), P(k[2], _d), P(k[3], _d), P(k[4], _i32),
                 P(k[5], _i32), P(k[6], _d), P(k[7], _d), P(k[8], _d), P(k[9], _i32),
                 int(k[12].size), P(k[10], _i32), P(k[11], _i32), P(k[12], _d),
                 P(k[13], _i32) if fo_t is not None else None,
                 P(k[14], _d) if fo_t is not None else None,
                 P(pl[0], _i32) if pl else None, P(pl[1], _d) if pl else None)
    return d, k


def validate_mechanism(mech):
    """chem_validate_mechanism (host only, no GPU): (return code, reason)."""
    L = load_library()
    d, keep = mech_desc(mech)
    buf = C.create_string_buffer(512)
    rc = L.chem_validate_mechanism(C.byref(d), buf, 512)
    del keep
    return rc, buf.value.decode()


class Chem:
    """A libchem context on one HIP device, enqueueing on torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("libchem needs a HIP device; none is visible")
        self.L = load_library()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        rc = self.L.chem_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise ChemError(f"chem_create failed ({rc})")
        self.h = h
        self.mech = None
        self._keep = []

    def close(self):
        if getattr(self, "h", None):
            self.L.chem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc < 0:
            raise ChemError(f"{what} failed ({rc}): {self.L.chem_last_error(self.h).decode()}")
        return rc

    # ---------------------------------------------------------------- setup
    def set_mechanism(self, mech):
        d, keep = mech_desc(mech)
        self._check(self.L.chem_set_mechanism(self.h, C.byref(d)), "chem_set_mechanism")
        del keep
        self.mech = mech
        return self

    def options(self) -> Options:
        o = Options()
        self._check(self.L.chem_get_options(self.h, C.byref(o)), "chem_get_options")
        return o

    def set_options(self, **kw):
        o = self.options()
        for key, v in kw.items():
            setattr(o, key, v)
        self._check(self.L.chem_set_options(self.h, C.byref(o)), "chem_set_options")
        return o

    def reserve(self, max_cells: int):
        self._check(self.L.chem_reserve(self.h, int(max_cells)), "chem_reserve")

    def slots(self) -> int:
        """Cells integrated at once by the persistent launches (see chem_query_slots)."""
        v = C.c_int64(0)
        self._check(self.L.chem_query_slots(self.h, C.byref(v)), "chem_query_slots")
        return int(v.value)

    # ------------------------------------------------------------ hot path
    def map_reference(self, T, p, Y, Y_fuel, Y_ox, Z_tol, T_tol=1.0, use_T=False,
                      flags=None, ref_index=None):
        import numpy as np
        n = T.shape[0]
        if flags is None:
            flags = torch.empty(n, dtype=torch.uint8, device=T.device)
        if ref_index is None:
            ref_index = torch.empty(1, dtype=torch.int64, device=T.device)
        yf, yo = _np(Y_fuel, np.float64), _np(Y_ox, np.float64)
        mp = MapParams(float(Z_tol), float(T_tol), 1 if use_T else 0,
                       yf.ctypes.data_as(_d), yo.ctypes.data_as(_d))
        self._check(self.L.chem_map_reference(self.h, n, _ptr(T), _ptr(p), _ptr(Y), C.byref(mp),
                                              _ptr(flags), _ptr(ref_index)), "chem_map_reference")
        return flags, ref_index

    def integrate_noalloc(self, T, p, Y, dt, flags=None, ref_index=None, h=None, cost=None,
                          status=None, steps=None, stats=False):
        """chem_integrate_noalloc: chem_integrate with the library's fixed
        device workspace (no allocation; at most 2097152 cells)."""
        n = T.shape[0]
        st = Stats() if stats else None
        rc = self.L.chem_integrate_noalloc(self.h, n, _ptr(T), _ptr(p), _ptr(Y), float(dt),
                                           _ptr(flags), _ptr(ref_index), _ptr(h), _ptr(cost),
                                           _ptr(status), _ptr(steps),
                                           C.byref(st) if st is not None else None)
        self._check(rc, "chem_integrate_noalloc")
        return st.as_dict() if st is not None else None

    def integrate(self, T, p, Y, dt, flags=None, ref_index=None, h=None, cost=None,
                  status=None, steps=None, stats=False):
        n = T.shape[0]
        st = Stats() if stats else None
        rc = self.L.chem_integrate(self.h, n, _ptr(T), _ptr(p), _ptr(Y), float(dt), _ptr(flags),
                                   _ptr(ref_index), _ptr(h), _ptr(cost), _ptr(status),
                                   _ptr(steps), C.byref(st) if st is not None else None)
        self._check(rc, "chem_integrate")
        return st.as_dict() if st is not None else None

    def eval_rhs_jac(self, T, p, Y, f=None, J=None):
        self._check(self.L.chem_eval_rhs_jac(self.h, T.shape[0], _ptr(T), _ptr(p), _ptr(Y),
                                             _ptr(f), _ptr(J)), "chem_eval_rhs_jac")
        return f, J

    def rodas_step(self, T, p, Y, h, ynew, err):
        self._check(self.L.chem_rodas_step(self.h, T.shape[0], _ptr(T), _ptr(p), _ptr(Y), float(h),
                                           _ptr(ynew), _ptr(err)), "chem_rodas_step")
        return ynew, err

    # ------------------------------------------------------------ surrogate
    def integrate_surrogate(self, T, p, Y, dt, flags, ref_index=None, gate=None, h=None,
                            cost=None, status=None, steps=None, stats=False):
        """chem_integrate_surrogate; gate: dict of chem_gate_params fields."""
        g = GateParams()
        self.L.chem_default_gate_params(C.byref(g))
        for key, v in (gate or {}).items():
            setattr(g, key, v)
        st = Stats() if stats else None
        rc = self.L.chem_integrate_surrogate(self.h, T.shape[0], _ptr(T), _ptr(p), _ptr(Y),
                                             float(dt), _ptr(flags), _ptr(ref_index), C.byref(g),
                                             _ptr(h), _ptr(cost), _ptr(status), _ptr(steps),
                                             C.byref(st) if st is not None else None)
        self._check(rc, "chem_integrate_surrogate")
        return st.as_dict() if st is not None else None

    def surrogate_param_count(self) -> int:
        return int(self.L.chem_surrogate_param_count())

    def surrogate_train(self, T0, p, Y0, dt, T1, Y1, **kw):
        """chem_surrogate_train; returns the per-epoch loss (numpy float32)."""
        import numpy as np
        tp = TrainParams()
        self.L.chem_default_train_params(C.byref(tp))
        for key, v in kw.items():
            setattr(tp, key, v)
        hist = np.zeros(tp.epochs, np.float32)
        self._check(self.L.chem_surrogate_train(self.h, T0.shape[0], _ptr(T0), _ptr(p), _ptr(Y0),
                                                _ptr(dt), _ptr(T1), _ptr(Y1), C.byref(tp),
                                                hist.ctypes.data_as(C.c_void_p)),
                    "chem_surrogate_train")
        return hist

    def surrogate_get_params(self):
        import numpy as np
        P = np.zeros(self.surrogate_param_count(), np.float32)
        self._check(self.L.chem_surrogate_get_params(self.h, P.ctypes.data_as(C.c_void_p)),
                    "chem_surrogate_get_params")
        return P

    def surrogate_set_params(self, P):
        import numpy as np
        P = _np(P, np.float32)
        if P.size != self.surrogate_param_count():
            raise ValueError("parameter blob has the wrong size")
        self._check(self.L.chem_surrogate_set_params(self.h, P.ctypes.data_as(C.c_void_p)),
                    "chem_surrogate_set_params")

    def surrogate_save(self, path):
        self._check(self.L.chem_surrogate_save(self.h, os.fsencode(path)), "chem_surrogate_save")

    def surrogate_load(self, path):
        self._check(self.L.chem_surrogate_load(self.h, os.fsencode(path)), "chem_surrogate_load")

    def surrogate_forward(self, T, p, Y, dt, out=None):
        n = T.shape[0]
        if out is None:
            out = torch.empty((n, 64), dtype=torch.float32, device=T.device)
        self._check(self.L.chem_surrogate_forward(self.h, n, _ptr(T), _ptr(p), _ptr(Y), _ptr(dt),
                                                  _ptr(out)), "chem_surrogate_forward")
        return out

    def surrogate_forward_fused(self, T, p, Y, dt, out=None):
        n = T.shape[0]
        if out is None:
            out = torch.empty((n, 64), dtype=torch.float32, device=T.device)
        self._check(self.L.chem_surrogate_forward_fused(self.h, n, _ptr(T), _ptr(p), _ptr(Y),
                                                        _ptr(dt), _ptr(out)),
                    "chem_surrogate_forward_fused")
        return out

    def surrogate_loss_grad(self, T0, p, Y0, dt, T1, Y1):
        import numpy as np
        g = np.zeros(self.surrogate_param_count(), np.float32)
        loss = C.c_double(0.0)
        self._check(self.L.chem_surrogate_loss_grad(self.h, T0.shape[0], _ptr(T0), _ptr(p),
                                                    _ptr(Y0), _ptr(dt), _ptr(T1), _ptr(Y1),
                                                    g.ctypes.data_as(C.c_void_p), C.byref(loss)),
                    "chem_surrogate_loss_grad")
        return float(loss.value), g

    # ------------------------------------------------------ graphs, tuning
    def graph_begin(self):
        self._check(self.L.chem_graph_begin(self.h), "chem_graph_begin")

    def graph_end(self):
        g = C.c_void_p()
        self._check(self.L.chem_graph_end(self.h, C.byref(g)), "chem_graph_end")
        return Graph(self, g)

    def autotune(self, T, p, Y, dt, flags=None, ref_index=None, remeasure=False):
        """chem_autotune; returns [(schedule, queue_chunk, slots_per_cu, ms)] and
        leaves the fastest configuration in the context's options.  Timings
        kept from an earlier call with the same key are reused unless
        remeasure (chem_autotune_forget first)."""
        if remeasure:
            self.L.chem_autotune_forget()
        res = (TuneEntry * 16)()
        cnt = C.c_int32(0)
        self._check(self.L.chem_autotune(self.h, T.shape[0], _ptr(T), _ptr(p), _ptr(Y), float(dt),
                                         _ptr(flags), _ptr(ref_index), res, 16, C.byref(cnt)),
                    "chem_autotune")
        return [(r.schedule, r.queue_chunk, r.slots_per_cu, r.ms) for r in res[:cnt.value]]


class Graph:
    """A recorded sequence of libchem calls (chem_graph)."""

    def __init__(self, chem, handle):
        self.chem, self.h = chem, handle

    def launch(self):
        self.chem._check(self.chem.L.chem_graph_launch(self.chem.h, self.h), "chem_graph_launch")

    def close(self):
        if getattr(self, "h", None):
            self.chem.L.chem_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
