"""Learned preconditioner kernels against the FP64 oracle network.

The GPU network is FP32; the oracle is FP64 on the same (float32) inputs.
Tolerances: forward 1e-5 relative (FP32 dot products of length <= 64 and
transcendental functions, ~1e-6 each); gradient 1e-4 of the largest
gradient entry (FP32 sums over ~1e3 samples); Adam 1e-6.
"""
import numpy as np
import pytest

import synth
from oracle import davidson as odv
from oracle import hamiltonian as ham
from oracle import mlp as omlp

from gpu_util import from_gpu_block, log, problems, rel_err, start_block, to_gpu_block

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_1709_10010_amd import _lib
    return _lib


def _f32params(seed):
    p = omlp.init_params(seed)
    p["b1"] = np.random.default_rng(seed + 1).uniform(-0.5, 0.5, 64)
    p["b2"] = np.random.default_rng(seed + 2).uniform(-0.5, 0.5, 64)
    p["b3"] = np.array([0.3])
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def test_forward_matches_oracle(lib):
    import torch
    p = _f32params(4)
    rng = np.random.default_rng(5)
    Fraw = rng.standard_normal((5000, 4)).astype(np.float32) * 3 + 1
    scaler = np.array([1.0, 1.0, 1.0, 1.0, 1 / 3, 1 / 3, 1 / 3, 1 / 3], dtype=np.float32)
    net = lib.Mlp(lib.pack_params(p), scaler)
    F = torch.from_numpy(Fraw).cuda()
    s = torch.zeros(5000, dtype=torch.float32, device="cuda")
    lib.pw_mlp_forward(net, F, s)
    torch.cuda.synchronize()
    Fstd = (Fraw.astype(np.float64) - scaler[:4].astype(np.float64)) * scaler[4:].astype(np.float64)
    ref, _ = omlp.forward(p, Fstd)
    got = s.cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()


def _batch(seed, nbd, npw):
    rng = np.random.default_rng(seed)
    Fraw = (rng.standard_normal((nbd * npw, 4)) * [2, 1, 0.5, 1] + [3, -1, 1, -0.5]).astype(np.float32)
    R = rng.standard_normal((npw, nbd)) + 1j * rng.standard_normal((npw, nbd))
    D = R * (0.3 + rng.uniform(0, 1, (npw, nbd))) + 0.2 * (rng.standard_normal((npw, nbd)) + 0j)
    return Fraw, R, D


def _gpu_batch(Fraw, R, D, nbd, npw):
    import torch
    F = torch.from_numpy(Fraw).cuda()
    Rg = torch.from_numpy(np.ascontiguousarray(R.T).reshape(-1)).cuda()
    Dg = torch.from_numpy(np.ascontiguousarray(D.T).reshape(-1)).cuda()
    off = torch.arange(0, nbd * npw + 1, npw, dtype=torch.int64, device="cuda")
    band_of = torch.repeat_interleave(torch.arange(nbd, dtype=torch.int32), npw).cuda()
    s = torch.zeros(nbd * npw, dtype=torch.float32, device="cuda")
    return F, Rg, Dg, off, band_of, s


def test_gradient_matches_oracle(lib):
    nbd, npw = 3, 700
    p = _f32params(7)
    Fraw, R, D = _batch(8, nbd, npw)
    scaler = np.array([3, -1, 1, -0.5, 0.5, 1, 2, 1], dtype=np.float32)
    net = lib.Mlp(lib.pack_params(p), scaler)
    F, Rg, Dg, off, band_of, s = _gpu_batch(Fraw, R, D, nbd, npw)
    loss = lib.pw_mlp_train_step(net, F, Rg, Dg, off, band_of, s, update=False)
    _, _, g = net.get()
    Fstd = (Fraw.astype(np.float64) - scaler[:4]) * scaler[4:]
    lref, gref = omlp.batch_loss_grad(p, Fstd, R, D)
    assert abs(loss - lref) < 1e-5
    gv = lib.unpack_params(g)
    gmax = max(np.abs(v).max() for v in gref.values())
    for k in gref:
        err = np.abs(gv[k] - gref[k]).max()
        assert err <= 1e-4 * gmax, (k, err, gmax)


def test_adam_step_matches_oracle(lib):
    nbd, npw = 2, 300
    p = _f32params(9)
    Fraw, R, D = _batch(10, nbd, npw)
    scaler = np.array([3, -1, 1, -0.5, 0.5, 1, 2, 1], dtype=np.float32)
    net = lib.Mlp(lib.pack_params(p), scaler)
    F, Rg, Dg, off, band_of, s = _gpu_batch(Fraw, R, D, nbd, npw)
    lib.pw_mlp_train_step(net, F, Rg, Dg, off, band_of, s, lr=1e-2, update=True)
    pg, _, g = net.get()
    ref = dict(p)
    omlp.adam_step(ref, lib.unpack_params(g), {}, lr=1e-2)
    got = lib.unpack_params(pg)
    for k in ref:
        assert np.abs(got[k] - ref[k]).max() < 1e-6, k


def test_targets_and_features_match_oracle(lib):
    import torch
    c = synth.make_cell(1)
    po, pl = problems(c)
    w, V = ham.eigh_lowest(po, 16)
    rng = np.random.default_rng(3)
    Xit = V + 0.05 * (rng.standard_normal(V.shape) + 1j * rng.standard_normal(V.shape))
    Xit = np.linalg.qr(Xit.T)[0].T          # orthonormal iterate block, as Ritz vectors are
    # clusters: bands with eigenvalue gaps < 1e-6 Ha share an id
    cid = np.zeros(16, dtype=np.int32)
    for i in range(1, 16):
        cid[i] = cid[i - 1] + (0 if w[i] - w[i - 1] < 1e-6 else 1)
    Xc_g, Xi_g = to_gpu_block(V), to_gpu_block(Xit)
    Dg = torch.zeros_like(Xc_g)
    work = torch.zeros(17 * 16 * 16, dtype=torch.complex128, device="cuda")
    lib.pw_mlp_targets(pl, Xc_g, torch.from_numpy(cid).cuda(), Xi_g, Dg, work)
    got = from_gpu_block(Dg, po.npw)
    for n in range(16):
        members = np.nonzero(cid == cid[n])[0]
        ref = omlp.target_correction(Xit[n], V[members].T, Xit.T)
        assert np.abs(got[n] - ref).max() < 1e-12
    # features
    theta = torch.from_numpy(w.copy()).cuda()
    Rr = rng.standard_normal(V.shape) + 1j * rng.standard_normal(V.shape)
    rn = np.linalg.norm(Rr, axis=1)
    F = torch.zeros(16 * po.npw * 4, dtype=torch.float32, device="cuda")
    lib.pw_mlp_features(pl, theta, Xi_g, to_gpu_block(Rr), torch.from_numpy(rn).cuda(), F)
    torch.cuda.synchronize()
    ref = omlp.features(po.kinetic(), w, Xit.T, Rr.T, float(po.vloc.mean()))
    assert np.abs(F.cpu().numpy().reshape(-1, 4) - ref).max() <= 1e-6 * np.abs(ref).max()


def test_davidson_with_untrained_network_converges(lib):
    """A zero network (s = 1/4 + 15/8 everywhere, a constant multiple of TPA) is a valid preconditioner:
    the solve must still reach the dense eigenvalues."""
    c = synth.make_cell(0)
    po, pl = problems(c, max_bands=8)
    net = lib.Mlp(np.zeros(lib.MLP_NPARAM, dtype=np.float32))
    res = lib.davidson_solve(pl, to_gpu_block(start_block(c, 8, po.npw)), tol=5e-9, precond=2, net=net)
    w, _ = ham.eigh_lowest(po, 8)
    assert res["converged"] and np.abs(res["theta"] - w).max() < 5e-9


def test_nan_network_falls_back_to_tpa(lib):
    """NaN weights poison every s: every band must fall back to TPA, so the solve
    repeats the TPA solve exactly (same iteration count, same Ritz values)."""
    c = synth.make_cell(1)
    po, pl = problems(c)
    x0 = start_block(c, 16, po.npw)
    bad = np.full(lib.MLP_NPARAM, np.nan, dtype=np.float32)
    net = lib.Mlp(bad)
    r_mlp = lib.davidson_solve(pl, to_gpu_block(x0), tol=5e-9, precond=2, net=net)
    r_tpa = lib.davidson_solve(pl, to_gpu_block(x0), tol=5e-9, precond=1)
    log("nan-net iterations", r_mlp["iterations"], "tpa", r_tpa["iterations"])
    assert r_mlp["converged"] and r_mlp["iterations"] == r_tpa["iterations"]
    assert np.array_equal(r_mlp["theta"], r_tpa["theta"])


def test_precond_mlp_kind_matches_oracle(lib):
    """pw_precond with the learned kind: T = s(G, n) K_TPA(G, n) R_n(G), the
    features computed from the iterate (T_n), the residual's own norm, the
    Ritz value and <V_LOC>; FP32 network against the FP64 oracle network on
    the same weights (1e-5 of the largest entry, as the forward test).  A
    NaN network gives TPA in every band."""
    import torch
    c = synth.make_cell(1)
    po, pl = problems(c)
    npw, nbd = po.npw, 16
    rng = np.random.default_rng(11)
    X = start_block(c, nbd, npw)
    R = rng.standard_normal((nbd, npw)) + 1j * rng.standard_normal((nbd, npw))
    theta = rng.uniform(-1.0, 1.0, nbd)
    p = _f32params(12)
    scaler = np.array([1.0, -0.2, 1.0, -0.4, 0.5, 2.0, 1.0, 1.5], dtype=np.float32)
    net = lib.Mlp(lib.pack_params(p), scaler)
    xg, rg = to_gpu_block(X), to_gpu_block(R)
    tg = torch.zeros_like(xg)
    th = torch.from_numpy(theta).cuda()
    lib.pw_precond(pl, lib.PW_PRECOND_MLP, th, xg, rg, tg, net=net)
    got = from_gpu_block(tg, npw)
    t = po.kinetic()
    F = omlp.features(t, theta, X.T, R.T, float(po.vloc.mean()))
    Fstd = (F.astype(np.float32).astype(np.float64) - scaler[:4].astype(np.float64)) * scaler[4:].astype(np.float64)
    s, _ = omlp.forward(p, Fstd)
    ref = s.reshape(nbd, npw) * odv.tpa_apply(t, X.T, R.T).T
    err = np.abs(got - ref).max() / np.abs(ref).max()
    log("pw_precond MLP kind: max rel err", err)
    assert err <= 1e-5
    bad = lib.Mlp(np.full(lib.MLP_NPARAM, np.nan, dtype=np.float32))
    lib.pw_precond(pl, lib.PW_PRECOND_MLP, th, xg, rg, tg, net=bad)
    got_nan = from_gpu_block(tg, npw)
    assert rel_err(got_nan, odv.tpa_apply(t, X.T, R.T).T) < 1e-12
