"""The C-ABI library loads and exports every entry point include/chem.h declares
(no compute call: this runs without a GPU)."""
import os
import re
import ctypes

from paper_2011_07978_amd import chem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"\b(chem_[a-z_]+)\s*\(", txt)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = chem.load_library()
    declared = _declared()
    assert len(declared) >= 14
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(chem.EXPORTS)


def test_no_compute_without_context():
    L = chem.load_library()
    assert L.chem_max_species() == 137
    o = chem.Options()
    L.chem_default_options(ctypes.byref(o))
    assert o.rtol == 1e-8 and o.atol == 1e-12 and o.schedule == chem.CHEM_SCHED_QUEUE
    # null context pointers are rejected, never dereferenced
    assert L.chem_set_options(None, ctypes.byref(o)) == -1
    assert L.chem_integrate(None, 0, None, None, None, 1e-6, None, None, None, None, None,
                            None, None) == -1


def test_surrogate_defaults_without_gpu():
    L = chem.load_library()
    assert L.chem_surrogate_param_count() == 230848
    tp = chem.TrainParams()
    L.chem_default_train_params(ctypes.byref(tp))
    assert tp.batch % 64 == 0 and tp.epochs >= 1 and tp.lr_max > tp.lr_min >= 0
    g = chem.GateParams()
    L.chem_default_gate_params(ctypes.byref(g))
    assert g.tau_T == 0.5 and g.y_min == -1e-10 and g.margin == 0.01 and g.max_dT == 1.0 and g.T_max == 1000.0
    assert L.chem_surrogate_train(None, 0, None, None, None, None, None, None,
                                  ctypes.byref(tp), None) == -1
    assert L.chem_surrogate_load(None, b"/nonexistent") == -1
