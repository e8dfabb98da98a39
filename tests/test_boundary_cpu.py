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
    # launch timing: three kinds; reading with nothing recorded touches no device
    assert lib.redo_profile_read_kind(3, None, None, 0) == 1
    assert lib.redo_profile_read_kind(-1, None, None, 0) == 1
    ms, cnt = ctypes.c_double(-1.0), ctypes.c_int64(-1)
    assert lib.redo_profile_read_kind(1, ctypes.byref(ms), ctypes.byref(cnt), 1) == 0
    assert ms.value == 0.0 and cnt.value == 0


def test_walsh_spectrum_collective_x_closed_form():
    """sum_q I_x^(q) (f = 1/2 at the single-bit offsets): D_k = (n - 2 popcount(k)) / 2."""
    import numpy as np
    from paper_1707_02162_amd import redo as R, workloads as W
    for n in (3, 7, 10):
        d = 2 ** n
        D = R.walsh_spectrum(*W.observable_ell(W.collective(n, range(n), "x")))
        pc = np.array([bin(k).count("1") for k in range(d)])
        assert np.array_equal(D, 0.5 * (n - 2 * pc))


def test_walsh_spectrum_reconstructs_dyadic_observables():
    """A random real f on a few offsets, M_ij = f(i XOR j) written out, its row lists
    shuffled and one entry split in two: Hn diag(D) Hn (scipy's Hadamard matrix) is M."""
    import math
    import numpy as np
    from scipy.linalg import hadamard
    from paper_1707_02162_amd import redo as R
    rng = np.random.default_rng(41)
    d = 64
    f = np.zeros(d)
    f[rng.choice(d, 6, replace=False)] = rng.normal(size=6)
    M = np.array([[f[i ^ j] for j in range(d)] for i in range(d)])
    w = 7
    cols = np.zeros((d, w), np.int32)
    vals = np.zeros((d, w), np.complex64)
    for i in range(d):
        nz = [j for j in range(d) if M[i, j] != 0]
        rng.shuffle(nz)
        cols[i, :len(nz)] = nz
        vals[i, :len(nz)] = M[i, nz]
        cols[i, len(nz):] = i          # padding: value 0
    # one entry as two halves of the same column
    cols[5, 6] = cols[5, 0]
    vals[5, 0] = vals[5, 6] = np.float32(M[5, cols[5, 0]]) / 2
    D = R.walsh_spectrum(cols, vals)
    Hn = hadamard(d) / math.sqrt(d)
    assert np.abs(Hn @ np.diag(D) @ Hn - M.astype(np.float32)).max() < 1e-6


def test_walsh_spectrum_rejections():
    """Not a function of i XOR j (collective I_z; one entry missing; a complex f) gives
    None; bad sizes and column indices are argument errors."""
    import numpy as np
    from paper_1707_02162_amd import redo as R, workloads as W
    n, d = 5, 32
    assert R.walsh_spectrum(*W.observable_ell(np.diag(W.collective_z_diag(n, range(n))).astype(complex))) is None
    cols, vals = W.observable_ell(W.collective(n, range(n), "x"))
    v = np.array(vals).copy()
    v[3, 0] = 0
    assert R.walsh_spectrum(cols, v) is None
    assert R.walsh_spectrum(cols, np.array(vals) * 1j) is None
    with pytest.raises(R.RedoError, match="power of two"):
        R.walsh_spectrum(np.zeros((24, 2), np.int32), np.zeros((24, 2), np.complex64))
    c = np.array(cols).copy()
    c[2, 1] = d
    with pytest.raises(R.RedoError, match="outside"):
        R.walsh_spectrum(c, vals)


def test_walsh_observable_refused_before_any_device_work():
    """A Walsh observable is only created from lists that pass the analysis: the same
    refusals as the spectrum (None for a non-XOR observable, argument errors for bad
    sizes or columns), decided on the host before the library touches the device."""
    import numpy as np
    from paper_1707_02162_amd import redo as R, workloads as W
    n, d = 5, 32
    assert R.walsh_observable(*W.observable_ell(np.diag(W.collective_z_diag(n, range(n))).astype(complex))) is None
    cols, vals = W.observable_ell(W.collective(n, range(n), "x"))
    assert R.walsh_observable(cols, np.array(vals) * 1j) is None
    with pytest.raises(R.RedoError, match="power of two"):
        R.walsh_observable(np.zeros((24, 2), np.int32), np.zeros((24, 2), np.complex64))
    c = np.array(cols).copy()
    c[2, 1] = d
    with pytest.raises(R.RedoError, match="outside"):
        R.walsh_observable(c, vals)
    lib = R.lib()
    assert lib.redo_walsh_observable_destroy(None) == 0
