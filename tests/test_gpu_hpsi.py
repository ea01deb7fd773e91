"""GPU parity of H*psi (pw_hpsi, FP64 form) against the FP64 oracle.

Element-by-element on the same seeded inputs, at sizes the oracle finishes
in seconds and that span several stick tiles, plane groups, band chunks and
GEMM tiles with ragged tails; at the full config-2 size on sampled bands.
Tolerance: the FP64 path reorders sums (FFT butterflies, split-K GEMM), so
each output element carries a few ulps of the largest term it sums;
max|d| <= 1e-12 * max|ref| bounds that with a wide margin (observed ~1e-15).
"""
import numpy as np
import pytest

import synth
from oracle import davidson as odv
from oracle import hamiltonian as ham

from gpu_util import from_gpu_block, log, problems, rel_err, start_block, to_gpu_block

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_1709_10010_amd import _lib
    return _lib


def _run(lib, pl, psi, terms=7, ld_pad=64):
    import torch
    x = to_gpu_block(psi, ld_pad)
    y = torch.full_like(x, complex(np.nan, np.nan))
    lib.pw_hpsi(pl, x, y, terms=terms)
    return from_gpu_block(y, psi.shape[1])


@pytest.mark.parametrize("terms", [1, 2, 4, 7])
def test_hpsi_terms_config1(lib, terms):
    c = synth.make_cell(1)
    log("hpsi cfg1 terms", terms)
    po, pl = problems(c)
    psi = start_block(c, 16, po.npw)
    got = _run(lib, pl, psi, terms)
    ref = np.zeros_like(psi)
    if terms & 1:
        ref += po.kinetic()[None, :] * psi
    if terms & 2:
        ref += np.array([ham.apply_local(po, p) for p in psi])
    if terms & 4:
        ref += ham.apply_nonlocal(po, psi)
    assert rel_err(got, ref) < TOL


@pytest.mark.parametrize("nb", [1, 5, 13, 16])
def test_hpsi_ragged_band_counts(lib, nb):
    c = synth.make_cell(1)
    log("hpsi cfg1 nb", nb)
    po, pl = problems(c, max_bands=16)
    psi = start_block(c, nb, po.npw)
    assert rel_err(_run(lib, pl, psi), ham.hpsi(po, psi)) < TOL


def test_hpsi_zero_bands_is_noop(lib):
    import torch
    c = synth.make_cell(1)
    po, pl = problems(c)
    x = torch.zeros((0, 960), dtype=torch.complex128, device="cuda")
    lib.pw_hpsi(pl, x, x.clone())


def test_hpsi_unpadded_ld_and_tiny_grid(lib):
    c = synth.make_cell(0)
    log("hpsi tiny 9^3 unpadded")
    po, pl = problems(c, ld_pad=1)
    psi = start_block(c, 8, po.npw)
    assert rel_err(_run(lib, pl, psi, ld_pad=1), ham.hpsi(po, psi)) < TOL


def test_hpsi_kpoint_full_d_matches_dense_h(lib):
    """s+p+d projectors, full symmetric D, k != 0: compare with the dense matrix too."""
    c = synth.make_cell(0, seed=19)
    c.lmax = np.full(c.natom, 2, dtype=np.int32)
    c.dij = synth.cells._dij(np.random.default_rng(5), c.lmax, full=True)
    c.kpts = np.array([[0.31, -0.17, 0.05]])
    log("hpsi tiny spd kpoint")
    po, pl = problems(c)
    psi = start_block(c, 6, po.npw)
    got = _run(lib, pl, psi)
    assert rel_err(got, ham.hpsi(po, psi)) < TOL
    assert rel_err(got, (ham.dense_h(po) @ psi.T).T) < TOL


def test_hpsi_non_cubic_grid(lib):
    """N0 != N1 != N2 (3*5*8-like shapes exercise every radix and the pruned rows)."""
    c = synth.make_cell(0, seed=23)
    c.nr = (10, 12, 15)
    log("hpsi grid 10x12x15")
    po, pl = problems(c)
    psi = start_block(c, 8, po.npw)
    assert rel_err(_run(lib, pl, psi), ham.hpsi(po, psi)) < TOL


def test_projections_match_oracle(lib):
    import torch
    c = synth.make_cell(1)
    po, pl = problems(c)
    psi = start_block(c, 16, po.npw)
    x = to_gpu_block(psi)
    P = torch.zeros((16, po.nproj), dtype=torch.complex128, device="cuda")
    lib.pw_projections(pl, x, P)
    torch.cuda.synchronize()
    ref = ham.projections(po, psi).T
    assert rel_err(P.cpu().numpy(), ref) < TOL


def test_hpsi_config2_kpoint_bands(lib):
    """Config-2 k-point 1 (72^3, s+p+d, 576 projectors): 24 bands, all checked."""
    c = synth.make_cell(2)
    log("hpsi cfg2 k1 24 bands")
    po, pl = problems(c, ik=1, max_bands=24)
    psi = start_block(c, 24, po.npw, ik=1)
    got = _run(lib, pl, psi)
    ref = ham.hpsi(po, psi)
    assert rel_err(got, ref) < TOL


def test_hpsi_config2_full_block_sampled(lib):
    """Full config-2 launch (256 bands, one k-point): sampled bands vs the oracle,
    plus Hermiticity <phi|H psi> = <H phi|psi>^* over pairs of GPU bands."""
    c = synth.make_cell(2)
    log("hpsi cfg2 gamma 256 bands")
    po, pl = problems(c, ik=0, max_bands=256)
    psi = start_block(c, 256, po.npw, ik=0)
    got = _run(lib, pl, psi)
    for n in (0, 97, 200, 255):
        ref = ham.hpsi(po, psi[n:n + 1])[0]
        assert rel_err(got[n], ref) < TOL, n
    a = psi.conj() @ got.T           # <psi_m | H psi_n>
    assert np.abs(a - a.conj().T).max() <= 1e-12 * np.abs(a).max()


def _by_stick(miller, nr):
    """The Miller list re-listed by z-stick: (h mod N0, k mod N1), then l mod N2."""
    m = np.asarray(miller)
    return m[np.lexsort((m[:, 2] % nr[2], m[:, 1] % nr[1], m[:, 0] % nr[0]))]


@pytest.mark.parametrize("cfg,ik,nb,prec", [(1, 0, 16, 0), (1, 0, 16, 1), (2, 1, 24, 0)])
def test_hpsi_stick_ordered_sphere(lib, cfg, ik, nb, prec):
    """G listed by stick: the z passes then read psi and write H psi in order
    (no gather).  Same check as above on that order; the FP32-FFT form at the
    precision-form bound."""
    c = synth.make_cell(cfg)
    log("hpsi stick order cfg", cfg, "k", ik, "prec", prec)
    m = _by_stick(ham.problem_from_cell(c, ik).miller, c.nr)
    po, pl = problems(c, ik=ik, precision=prec, max_bands=nb, miller=m)
    psi = start_block(c, nb, po.npw, ik=ik)
    got = _run(lib, pl, psi)
    ref = ham.hpsi(po, psi)
    assert rel_err(got, ref) < (TOL if prec == 0 else 5e-6)


def test_precond_tpa_matches_oracle(lib):
    import torch
    c = synth.make_cell(1)
    po, pl = problems(c)
    rng = np.random.default_rng(8)
    X = start_block(c, 16, po.npw)
    R = rng.standard_normal(X.shape) + 1j * rng.standard_normal(X.shape)
    xg, rg = to_gpu_block(X), to_gpu_block(R)
    tg = torch.zeros_like(xg)
    lib.pw_precond(pl, lib.PW_PRECOND_TPA, None, xg, rg, tg)
    got = from_gpu_block(tg, po.npw)
    ref = odv.tpa_apply(po.kinetic(), X.T, R.T).T
    assert rel_err(got, ref) < TOL


def test_sphere_outside_grid_is_shape_error(lib):
    import torch
    c = synth.make_cell(1)
    po = ham.problem_from_cell(c)
    v = torch.zeros((8, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.PwError) as e:
        lib.pw_problem_create(po.A, po.kfrac, c.ecut_ha, (8, 8, 8), po.miller, v, None, None, None)
    assert e.value.status == -2


# every cubic grid size with compile-time FFT plans (odd ones have no
# register plane instance and fall back to the LDS kernel)
PLANE_SIZES = [24, 36, 40, 45, 48, 50, 54, 60, 64, 72, 81, 90]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", PLANE_SIZES)
def test_hpsi_every_plane_kernel_and_size(lib, n, prec):
    """The tiny cell on an n^3 grid through each plane kernel (register,
    wave-local, LDS), one and four bands per plane workgroup, and sweeps of
    four bands (nine bands: ragged groups and a ragged last sweep).  FP64
    against the oracle at 1e-12; the complex64-FFT form at 5e-6 (the
    precision-form bound)."""
    c = synth.make_cell(0, seed=31)
    c.nr = (n, n, n)
    log("plane kernels n", n, "prec", prec)
    po, pl = problems(c, precision=prec, max_bands=9)
    psi = start_block(c, 9, po.npw)
    ref = ham.hpsi(po, psi)
    tol = TOL if prec == 0 else 5e-6
    for kernel in (lib.PW_PLANE_REGISTER, lib.PW_PLANE_WAVE, lib.PW_PLANE_LDS):
        for group, chunk in ((1, 9), (4, 4)):
            lib.pw_problem_set_tuning(pl, group, chunk, 0, kernel)
            err = rel_err(_run(lib, pl, psi), ref)
            assert err < tol, (kernel, group, chunk, err)


def test_set_tuning_rejects_out_of_range(lib):
    c = synth.make_cell(0)
    po, pl = problems(c, max_bands=8)
    before = lib.pw_problem_tuning(pl)
    for bad in ((0, 8, 0, 0), (2, 9, 0, 0), (2, 8, 65, 0), (2, 8, 0, 3), (2, 0, 0, 0)):
        with pytest.raises(lib.PwError):
            lib.pw_problem_set_tuning(pl, *bad)
    assert lib.pw_problem_tuning(pl) == before


def test_caller_workspace_is_never_read_before_written(lib, monkeypatch):
    """The problem and Davidson handles keep their large buffers in the
    caller's workspace.  Filled with NaN bytes before create, it must still
    give H*psi at 1e-12 against the oracle and the dense eigenvalues from a
    Davidson solve (nothing in it is read before the library writes it)."""
    import torch
    real = lib._workspace

    def nan_workspace(nbytes, device=None):
        ws = real(nbytes, device)
        ws.fill_(0xFF)           # every double in it is a NaN
        return ws

    monkeypatch.setattr(lib, "_workspace", nan_workspace)
    c = synth.make_cell(1)
    po, pl = problems(c)
    assert pl.workspace is not None and int(pl.workspace.numel()) > 0
    psi = start_block(c, 16, po.npw)
    assert rel_err(_run(lib, pl, psi), ham.hpsi(po, psi)) < TOL
    res = lib.davidson_solve(pl, to_gpu_block(psi), tol=5e-9)
    w, _ = ham.eigh_lowest(po, 16)
    log("nan-filled workspaces: davidson iterations", res["iterations"],
        "max |theta - eigh|", float(np.abs(res["theta"] - w).max()))
    assert res["converged"] and np.abs(res["theta"] - w).max() < 5e-9
    torch.cuda.synchronize()


def test_davidson_rejects_small_workspace(lib):
    import ctypes
    import torch
    c = synth.make_cell(0)
    po, pl = problems(c, max_bands=8)
    need = ctypes.c_size_t()
    lib._check(lib.LIB.pw_davidson_workspace_size(pl.handle, 8, 0, ctypes.byref(need)))
    ws = torch.empty(int(need.value), dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    st = lib.LIB.pw_davidson_create(pl.handle, 8, 0, 5e-9, ctypes.c_void_p(ws.data_ptr()), need.value - 1,
                                    None, ctypes.byref(h))
    assert st == -1 and b"workspace" in lib.LIB.pw_last_error() and not h.value
