"""Reduced-precision forms of H*psi against the FP64 oracle.

Forms: complex64 FFTs (FP32 twiddles, FP32 V) with projector GEMMs in FP32
MFMA (PW_MIXED_FP32) or BF16 inputs / FP32 accumulation (PW_MIXED_BF16);
inputs and outputs stay complex128, the kinetic term stays FP64.

Tolerances (max |d| over max |ref| of the term):
  FP32 FFT: each radix pass adds ~u = 6e-8 relative; 3 passes per axis,
  6 axes, plus the V product -> a few 1e-7; bound 5e-6.
  FP32 GEMM: K-term dot products accumulate ~sqrt(K) u -> ~2e-6 at
  K = 949; bound 5e-6.
  BF16 GEMM: inputs rounded to 2^-9 relative (u_bf16 = 2e-3), so a
  projection and the update carry ~1e-3 relative each; bound 2e-2.
Ragged band counts (5, 13) make a wrong accumulator lane layout an O(1)
error, not a rounding one.
"""
import numpy as np
import pytest

import synth
from oracle import hamiltonian as ham

from gpu_util import from_gpu_block, log, problems, rel_err, start_block, to_gpu_block

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_1709_10010_amd import _lib
    return _lib


def _term(lib, pl, psi, terms):
    import torch
    x = to_gpu_block(psi)
    y = torch.full_like(x, complex(np.nan, np.nan))
    lib.pw_hpsi(pl, x, y, terms=terms)
    return from_gpu_block(y, psi.shape[1])


@pytest.mark.parametrize("prec,tol_nl", [(1, 5e-6), (2, 2e-2)])
@pytest.mark.parametrize("nb", [5, 13, 16])
def test_mixed_terms_config1(lib, prec, tol_nl, nb):
    c = synth.make_cell(1)
    log("mixed prec", prec, "nb", nb)
    po, pl = problems(c, precision=prec, max_bands=16)
    psi = start_block(c, nb, po.npw)
    loc = _term(lib, pl, psi, 2)
    nl = _term(lib, pl, psi, 4)
    kin = _term(lib, pl, psi, 1)
    ref_loc = np.array([ham.apply_local(po, p) for p in psi])
    ref_nl = ham.apply_nonlocal(po, psi)
    assert rel_err(kin, po.kinetic()[None, :] * psi) < 1e-15
    assert rel_err(loc, ref_loc) < 5e-6
    assert rel_err(nl, ref_nl) < tol_nl
    full = _term(lib, pl, psi, 7)
    assert rel_err(full, ham.hpsi(po, psi)) < max(tol_nl, 5e-6)


@pytest.mark.parametrize("prec", [1, 2])
def test_mixed_projections_layout(lib, prec):
    import torch
    c = synth.make_cell(2)
    po, pl = problems(c, ik=2, precision=prec, max_bands=24)
    psi = start_block(c, 21, po.npw, ik=2)
    x = to_gpu_block(psi)
    P = torch.zeros((21, po.nproj), dtype=torch.complex128, device="cuda")
    lib.pw_projections(pl, x, P)
    torch.cuda.synchronize()
    ref = ham.projections(po, psi).T
    assert rel_err(P.cpu().numpy(), ref) < (1e-5 if prec == 1 else 2e-2)


def test_mixed_fp32_config2_kpoint(lib):
    c = synth.make_cell(2)
    log("mixed fp32 cfg2 k3")
    po, pl = problems(c, ik=3, precision=1, max_bands=16)
    psi = start_block(c, 16, po.npw, ik=3)
    assert rel_err(_term(lib, pl, psi, 7), ham.hpsi(po, psi)) < 5e-6


@pytest.mark.parametrize("prec,loose", [(1, 1e-5), (2, 1e-3)])
def test_mixed_davidson_then_fp64_refinement(lib, prec, loose):
    """Iterate with the reduced-precision operator, switch the solve to the FP64
    operator, finish to 1e-8 Ry: eigenvalues equal dense eigh to 5e-9 Ha."""
    c = synth.make_cell(1)
    log("mixed davidson prec", prec)
    po, pm = problems(c, precision=prec)
    _, pd = problems(c, precision=0)
    x0 = to_gpu_block(start_block(c, 16, po.npw))
    res = lib.davidson_solve(pm, x0, tol=loose, refine=pd, refine_tol=5e-9, want_vectors=True)
    w, _ = ham.eigh_lowest(po, 16)
    log("iterations mixed", res["iterations_first"], "total", res["iterations"],
        "max |theta-eigh|", np.abs(res["theta"] - w).max())
    assert res["converged"]
    assert np.abs(res["theta"] - w).max() < 5e-9
    X = from_gpu_block(res["X"], po.npw)
    R = ham.hpsi(po, X) - res["theta"][:, None] * X
    assert np.sqrt((np.abs(R) ** 2).sum(axis=1)).max() < 5e-9 * 1.001


def test_mixed_fp32_davidson_alone(lib):
    """FP32 operator only, residual target 5e-7 Ha (1e-6 Ry): the eigenvalues of
    the reduced-precision operator stay within 1e-6 Ry of the FP64 ones."""
    c = synth.make_cell(1)
    po, pm = problems(c, precision=1)
    x0 = to_gpu_block(start_block(c, 16, po.npw))
    res = lib.davidson_solve(pm, x0, tol=5e-7, max_iter=120)
    w, _ = ham.eigh_lowest(po, 16)
    err = np.abs(res["theta"] - w).max()
    log("fp32 alone converged", res["converged"], "iterations", res["iterations"], "max err Ha", err,
        "max rho", res["rho"].max())
    assert res["converged"]
    assert err < 5e-7
