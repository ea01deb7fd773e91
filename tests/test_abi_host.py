"""Host-side checks of the C ABI (no GPU needed).

* the built library exports every function ``include/pw_api.h`` declares;
* its host-only sphere enumeration agrees with the oracle's: the same set
  bit for bit, and an order whose kinetic energies never decrease;
* argument checks that return before any device work.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import gsphere as gs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pw_api.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pw_[a-z0-9_]+)\s*\(", src)))


def _lib():
    from paper_1709_10010_amd import _lib
    return _lib


def test_header_declares_entry_points():
    names = _declared()
    for n in ("pw_hpsi", "pw_precond", "pw_problem_create", "pw_gsphere"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib().LIBPATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("cfg,ik", [(1, 0), (2, 0), (2, 3), (0, 0)])
def test_gsphere_matches_oracle(cfg, ik):
    L = _lib()
    c = synth.make_cell(cfg)
    m_lib = L.pw_gsphere(c.A, c.kpts[ik], c.ecut_ha)
    m_or = gs.gsphere(c.A, c.kpts[ik], c.ecut_ha)
    assert m_lib.shape == m_or.shape
    key = lambda m: np.lexsort((m[:, 2], m[:, 1], m[:, 0]))
    assert np.array_equal(m_lib[key(m_lib)], m_or[key(m_or)])
    t = gs.kinetic(c.A, c.kpts[ik], m_lib)
    assert np.all(np.diff(t) >= -1e-12 * t.max())


def test_gsphere_general_cell_kpoint():
    L = _lib()
    A = np.array([[5.0, 0.3, -0.2], [0.7, 6.1, 0.4], [-0.5, 0.2, 4.4]])
    k = np.array([0.21, -0.37, 0.08])
    m_lib = L.pw_gsphere(A, k, 4.0)
    m_or = gs.gsphere(A, k, 4.0)
    assert set(map(tuple, m_lib.tolist())) == set(map(tuple, m_or.tolist()))


def test_gsphere_rejects_bad_cutoff():
    L = _lib()
    with pytest.raises(L.PwError) as e:
        L.pw_gsphere(np.eye(3) * 10, np.zeros(3), -1.0)
    assert e.value.status == -1


def test_problem_create_rejects_null_desc():
    L = _lib()
    h = ctypes.c_void_p()
    st = L.LIB.pw_problem_create(None, 1, None, 0, None, ctypes.byref(h))
    assert st == -1 and b"null" in L.LIB.pw_last_error()


def test_problem_create_rejects_bad_grid_before_device_work():
    L = _lib()
    d = L._Desc()
    d.cell[:] = list(np.eye(3).reshape(9) * 10)
    d.ecut = 7.5
    d.nr[:] = [24, 24, 7]           # 7 is not 2^a 3^b 5^c
    mill = np.zeros((1, 3), dtype=np.int32)
    d.npw = 1
    d.miller = mill.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.vloc = ctypes.c_void_p(1)     # never dereferenced: the grid check fails first
    h = ctypes.c_void_p()
    st = L.LIB.pw_problem_create(ctypes.byref(d), 4, None, 0, None, ctypes.byref(h))
    assert st == -2 and b"grid" in L.LIB.pw_last_error()


def _config1_desc(L, keep):
    """Descriptor of the config-1 cell whose device pointers are never
    dereferenced (only host-side checks run on it)."""
    c = synth.make_cell(1)
    m = np.ascontiguousarray(gs.gsphere(c.A, c.kpts[0], c.ecut_ha), dtype=np.int32)
    po = np.ascontiguousarray(c.proj_offset, dtype=np.int32)
    dj = np.ascontiguousarray(c.dij_concat(), dtype=np.float64)
    keep += [m, po, dj]
    d = L._Desc()
    d.cell[:] = list(np.asarray(c.A, dtype=np.float64).reshape(9))
    d.kpt[:] = [0.0, 0.0, 0.0]
    d.ecut = c.ecut_ha
    d.nr[:] = [int(x) for x in c.nr]
    d.npw = m.shape[0]
    d.miller = m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.vloc = ctypes.c_void_p(256)
    d.nproj = int(po[-1])
    d.natom = po.shape[0] - 1
    d.proj_offset = po.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.dij = dj.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.beta = ctypes.c_void_p(256)
    d.ld_beta = (m.shape[0] + 63) // 64 * 64
    return d, m.shape[0], int(po[-1]), c


def test_workspace_size_counts_the_per_band_buffers():
    # per extra band: one band of sticks (FP64, N2 * nst_pad values), P and
    # D P (2 * nproj complex128), 32 * nproj of split-K partials, and four
    # per-band words; 256-byte rounding of each region aside
    L = _lib()
    keep = []
    d, npw, nproj, c = _config1_desc(L, keep)
    b16, b32 = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.LIB.pw_workspace_size(ctypes.byref(d), 16, ctypes.byref(b16)) == 0
    assert L.LIB.pw_workspace_size(ctypes.byref(d), 32, ctypes.byref(b32)) == 0
    nst = len({(h % c.nr[0], k % c.nr[1]) for h, k, _ in gs.gsphere(c.A, c.kpts[0], c.ecut_ha).tolist()})
    nst_pad = (nst + 15) // 16 * 16
    # split-K partials are min(32 * P bytes, 512 MiB): 32 * nproj * 16 per band here
    per_band = c.nr[2] * nst_pad * 16 + 2 * nproj * 16 + 32 * nproj * 16 + 2 * 8 + 2 * 4
    diff = b32.value - b16.value
    assert abs(diff - 16 * per_band) <= 10 * 256, (diff, 16 * per_band)
    assert b16.value >= np.prod(c.nr) * 8 + nproj * d.ld_beta * 16


def test_problem_create_rejects_small_or_misaligned_workspace():
    L = _lib()
    keep = []
    d, npw, nproj, c = _config1_desc(L, keep)
    need = ctypes.c_size_t()
    assert L.LIB.pw_workspace_size(ctypes.byref(d), 16, ctypes.byref(need)) == 0
    h = ctypes.c_void_p()
    # the pointers are never dereferenced: the workspace check fails first
    st = L.LIB.pw_problem_create(ctypes.byref(d), 16, ctypes.c_void_p(1 << 20), need.value - 1, None,
                                 ctypes.byref(h))
    assert st == -1 and b"workspace" in L.LIB.pw_last_error() and not h.value
    st = L.LIB.pw_problem_create(ctypes.byref(d), 16, ctypes.c_void_p((1 << 20) + 64), need.value, None,
                                 ctypes.byref(h))
    assert st == -1 and b"aligned" in L.LIB.pw_last_error() and not h.value
    st = L.LIB.pw_problem_create(ctypes.byref(d), 16, None, need.value, None, ctypes.byref(h))
    assert st == -1 and b"workspace" in L.LIB.pw_last_error() and not h.value


def test_stick_order_is_a_permutation_listed_by_stick():
    """The front end's G order: the sphere's set unchanged, listed by
    (h mod N0, k mod N1) and then l mod N2 ascending, so each z-stick's
    points are consecutive."""
    from paper_1709_10010_amd.problems import stick_order
    c = synth.make_cell(1)
    m0 = gs.gsphere(c.A, c.kpts[0], c.ecut_ha)
    m = stick_order(m0, c.nr)
    assert sorted(map(tuple, m.tolist())) == sorted(map(tuple, np.asarray(m0).tolist()))
    key = [((h % c.nr[0]) * c.nr[1] + k % c.nr[1], l % c.nr[2]) for h, k, l in m.tolist()]
    assert key == sorted(key)
    assert len(set(key)) == len(key)
