"""The C ABI without a GPU: the library loads, exports every symbol the header
declares, and rejects bad arguments on the host before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "redo.h")
LIB = os.path.join(ROOT, "paper_1707_02162_amd", "libredo.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libredo.so not built")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(redo_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    lib = ctypes.CDLL(LIB)
    names = header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_1707_02162_amd import redo as R
    assert set(header_functions()) == set(R.exported_symbols())


def _lib():
    from paper_1707_02162_amd import redo as R
    return R, R.lib()


def test_bad_descriptors_rejected_on_host():
    R, lib = _lib()
    good = dict(d=4, K=1, base=16, digits=2, dt=1e-6, eps=1.0, phased=0, drift_is_diag=1, n_drift=1, splitting=0)
    bad = [dict(d=3), dict(d=96), dict(K=0), dict(K=17), dict(base=1), dict(digits=0), dict(base=65536, digits=2),
           dict(dt=0.0), dict(eps=-1.0), dict(phased=2), dict(n_drift=0), dict(splitting=2)]
    dummy = ctypes.c_void_p(16)
    for b in bad:
        f = dict(good)
        f.update(b)
        desc = R._Desc(**f)
        h = ctypes.c_void_p()
        st = lib.redo_build_table(ctypes.byref(desc), dummy, dummy, dummy, None, ctypes.byref(h))
        assert st == 1, (b, st)
        assert h.value is None
        assert len(lib.redo_last_error()) > 0
    # the Strang splitting is provided for diagonal drifts only
    f = dict(good, splitting=1, drift_is_diag=0)
    desc = R._Desc(**f)
    h = ctypes.c_void_p()
    assert lib.redo_build_table(ctypes.byref(desc), dummy, dummy, None, None, ctypes.byref(h)) == 6
    assert h.value is None
    # NULL operands and missing phase generators
    desc = R._Desc(**good)
    h = ctypes.c_void_p()
    assert lib.redo_build_table(ctypes.byref(desc), None, dummy, None, None, ctypes.byref(h)) == 1
    f = dict(good, phased=1)
    desc = R._Desc(**f)
    assert lib.redo_build_table(ctypes.byref(desc), dummy, dummy, None, None, ctypes.byref(h)) == 1
    assert lib.redo_build_table(None, dummy, dummy, None, None, ctypes.byref(h)) == 1


def test_calls_without_table_rejected():
    R, lib = _lib()
    d = ctypes.c_void_p(16)
    assert lib.redo_quantise(None, d, 1, 1, d, d, None) == 1
    assert lib.redo_compose_steps(None, 0, d, 1, 1, d, None, 0, None) == 1
    assert lib.redo_chain_propagator(None, 0, d, None, 1, 1, 0, 0, None, d, None, None, None, 0, None,
                                     None, 0, None) == 1
    assert lib.redo_grape_fidelity_grad(None, 0, d, None, 1, 1, d, 0, d, None, d, None, 0, None) == 1
    assert lib.redo_workspace_bytes(None, 0, 1, 1) == 0
    assert lib.redo_table_destroy(None) == 0
    assert lib.redo_unitary_fidelity(0, 1, d, d, None, None, None) == 1
    assert lib.redo_status_string(100) == b"amplitudes clamped"
    assert lib.redo_grape_state_fidelity_grad(None, 0, d, None, 1, 1, d, d, d, None, d, None, 0, None) == 1
    assert lib.redo_kron_chain(None, 1, d, None, 1, 1, 0, 0, None, d, None, None, 0, None, None, 0, None) == 1
    n = ctypes.c_int32(-1)
    assert lib.redo_table_spins(None, ctypes.byref(n)) == 1 and n.value == -1
    # launch timing: two kinds; reading with nothing recorded touches no device
    assert lib.redo_profile_read_kind(2, None, None, 0) == 1
    assert lib.redo_profile_read_kind(-1, None, None, 0) == 1
    ms, cnt = ctypes.c_double(-1.0), ctypes.c_int64(-1)
    assert lib.redo_profile_read_kind(1, ctypes.byref(ms), ctypes.byref(cnt), 1) == 0
    assert ms.value == 0.0 and cnt.value == 0
