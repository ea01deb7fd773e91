"""Learned diagonal preconditioner: data from the solver, training, evaluation.

Sequencing only: every arithmetic step (Davidson, H*psi, targets, features,
network forward / backward / Adam) runs in libpwhip.so's kernels; torch
holds device memory and concatenates the collected samples.

Data: for a training cell, a reference TPA solve gives converged vectors and
their degenerate clusters; a second TPA solve from the same start block is
snapshotted at a few iterations, and for the unconverged bands of each
snapshot the library builds the features and the target correction
d = P_c x / ||P_c x|| - x (P_c: projector on the band's converged cluster).
"""
from __future__ import annotations

import time

import numpy as np

import synth

from . import _lib
from .problems import band_block, build_problem

SNAP_ITERS = (2, 4, 7, 11, 16, 22, 29, 37, 46)
# output map s = 1/4 + 15/4 sigmoid(z): s = 1 at z = log(1/4)
B3_TPA = float(np.log(0.25))


def cluster_ids(theta: np.ndarray, gap: float = 1e-6) -> np.ndarray:
    """Consecutive Ritz values closer than `gap` (Ha) share a cluster id."""
    cid = np.zeros(len(theta), dtype=np.int32)
    for i in range(1, len(theta)):
        cid[i] = cid[i - 1] + (0 if theta[i] - theta[i - 1] < gap else 1)
    return cid


def collect(cell, ik: int = 0, precision: int = _lib.PW_FP64, tol: float = 5e-7,
            snap_iters=SNAP_ITERS, bands_per_snap: int | None = 64, seed: int = 0):
    """Samples (F, R, D, band sizes) from one cell; tensors stay on the GPU."""
    import torch
    nb = cell.nbands
    prob, _ = build_problem(cell, ik, precision=precision, max_bands=nb)
    npw = prob.npw
    x0 = band_block(nb, npw)
    x0[:, :npw] = torch.from_numpy(synth.psi_start(cell.seed, nb, npw, ik)).cuda()
    ref = _lib.davidson_solve(prob, x0, tol=tol * 1e-2, want_vectors=True)
    if not ref["converged"]:
        raise RuntimeError(f"reference solve of {cell.name} did not converge")
    Xc = ref["X"]
    cid = torch.from_numpy(cluster_ids(ref["theta"])).cuda()
    d = _lib.Davidson(prob, nb, 0, tol)
    _lib.pw_davidson_init(d, x0)
    X = torch.zeros_like(x0)
    R = torch.zeros_like(x0)
    Dt = torch.zeros_like(x0)
    RK = torch.zeros_like(x0)
    th = torch.zeros(nb, dtype=torch.float64, device="cuda")
    rh = torch.zeros(nb, dtype=torch.float64, device="cuda")
    work = torch.zeros(17 * nb * nb, dtype=torch.complex128, device="cuda")
    F = torch.zeros(nb * npw * 4, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(seed)
    Fs, Rs, Ds, sizes = [], [], [], []
    for it in range(1, max(snap_iters) + 1):
        conv = _lib.pw_davidson_step(d, _lib.PW_PRECOND_TPA)
        if it in snap_iters:
            _lib.pw_davidson_snapshot(d, X, R, th, rh)
            _lib.pw_mlp_targets(prob, Xc, cid, X, Dt, work)
            _lib.pw_mlp_features(prob, th, X, R, rh, F)
            # the network scales the TPA correction: its residual samples are K_TPA R
            _lib.pw_precond(prob, _lib.PW_PRECOND_TPA, None, X, R, RK)
            torch.cuda.synchronize()
            rho = rh.cpu().numpy()
            bands = np.nonzero(rho >= tol)[0]
            if bands_per_snap and len(bands) > bands_per_snap:
                bands = np.sort(rng.choice(bands, bands_per_snap, replace=False))
            if len(bands):
                bi = torch.from_numpy(bands).cuda()
                Fs.append(F.view(nb, npw, 4)[bi].reshape(-1, 4))
                Rs.append(RK[bi, :npw].reshape(-1))
                Ds.append(Dt[bi, :npw].reshape(-1))
                sizes += [npw] * len(bands)
        if conv:
            break
    d.close()
    return Fs, Rs, Ds, sizes


def build_dataset(parts):
    import torch
    Fs, Rs, Ds, sizes = [], [], [], []
    for f, r, d, s in parts:
        Fs += f
        Rs += r
        Ds += d
        sizes += s
    F = torch.cat(Fs).contiguous()
    R = torch.cat(Rs).contiguous()
    D = torch.cat(Ds).contiguous()
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    band_of = np.repeat(np.arange(len(sizes), dtype=np.int32), sizes)
    return dict(F=F, R=R, D=D, off=off, band_of=band_of, nbands=len(sizes))


def train(ds, epochs: int = 30, bands_per_batch: int = 64, lr: float = 1e-3, seed: int = 0,
          net=None, log=print, validate=None, val_every: int = 2):
    """Adam over minibatches of whole bands; returns the network and the loss history.

    With ``validate`` (a function of the network returning a score, lower is
    better) the network is scored every ``val_every`` epochs and the
    parameters with the best score are the ones returned; the history of
    (epoch, score) pairs is in ``net.val_history``."""
    import torch
    init = init_params(seed)
    if net is None:
        net = _lib.Mlp(init)
    _lib.pw_mlp_fit_scaler(net, ds["F"])
    rng = np.random.default_rng(seed)
    off = ds["off"]
    nbd = ds["nbands"]
    hist, val_hist, best = [], [], None
    smax = int(max(off[b + 1] - off[b] for b in range(nbd))) * bands_per_batch
    s_work = torch.zeros(smax, dtype=torch.float32, device="cuda")
    for ep in range(epochs):
        order = rng.permutation(nbd)
        tot, nbat = 0.0, 0
        for b0 in range(0, nbd, bands_per_batch):
            sel = np.sort(order[b0:b0 + bands_per_batch])
            idx = np.concatenate([np.arange(off[b], off[b + 1]) for b in sel])
            sizes = off[sel + 1] - off[sel]
            boff = torch.from_numpy(np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)).cuda()
            bof = torch.from_numpy(np.repeat(np.arange(len(sel), dtype=np.int32), sizes)).cuda()
            ii = torch.from_numpy(idx).cuda()
            loss = _lib.pw_mlp_train_step(net, ds["F"][ii].contiguous(), ds["R"][ii].contiguous(),
                                          ds["D"][ii].contiguous(), boff, bof, s_work, lr=lr)
            tot += loss
            nbat += 1
        hist.append(tot / max(nbat, 1))
        if log:
            log(f"epoch {ep}: mean band loss {hist[-1]:.4f}")
        if validate is not None and ((ep + 1) % val_every == 0 or ep + 1 == epochs):
            score = validate(net)
            val_hist.append((ep + 1, score))
            if log:
                log(f"epoch {ep}: validation score {score:.4f}")
            if best is None or score < best[0]:
                p, sc, _ = net.get()
                best = (score, p.copy(), sc.copy())
    if best is not None:
        net.set(params=best[1], scaler=best[2])
    net.val_history = val_hist
    return net, hist


def baseline_loss(ds, bands_per_batch: int = 64) -> float:
    """Mean band loss of s = 1 everywhere, i.e. of plain TPA on the same samples."""
    import torch
    p = np.zeros(_lib.MLP_NPARAM, dtype=np.float32)
    p[-1] = B3_TPA
    net = _lib.Mlp(p)
    off, nbd = ds["off"], ds["nbands"]
    smax = int(max(off[b + 1] - off[b] for b in range(nbd))) * bands_per_batch
    s_work = torch.zeros(smax, dtype=torch.float32, device="cuda")
    tot, n = 0.0, 0
    for b0 in range(0, nbd, bands_per_batch):
        sel = np.arange(b0, min(nbd, b0 + bands_per_batch))
        sizes = off[sel + 1] - off[sel]
        lo, hi = int(off[sel[0]]), int(off[sel[-1] + 1])
        boff = torch.from_numpy(np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)).cuda()
        bof = torch.from_numpy(np.repeat(np.arange(len(sel), dtype=np.int32), sizes)).cuda()
        l = _lib.pw_mlp_train_step(net, ds["F"][lo:hi].contiguous(), ds["R"][lo:hi].contiguous(),
                                   ds["D"][lo:hi].contiguous(), boff, bof, s_work, update=False)
        tot += l * len(sel)
        n += len(sel)
    net.close()
    return tot / n


def init_params(seed: int) -> np.ndarray:
    """Kaiming-uniform weights (bound sqrt(6 / fan_in)), zero biases, packed float32;
    the last layer starts small with b3 = B3_TPA, so s ~ 1 (plain TPA) at the start."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in (("W1", (64, 4)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
                      ("W3", (1, 64)), ("b3", (1,))):
        p[name] = rng.uniform(-np.sqrt(6.0 / shp[1]), np.sqrt(6.0 / shp[1]), size=shp) \
            if name.startswith("W") else np.zeros(shp)
    p["W3"] *= 0.1
    p["b3"][:] = B3_TPA
    return _lib.pack_params(p)


def save(net, path: str) -> None:
    p, s, _ = net.get()
    np.savez(path, params=p, scaler=s)


def load(path: str):
    z = np.load(path, allow_pickle=False)
    return _lib.Mlp(z["params"], z["scaler"])


def evaluate(cell, net, ik: int = 0, precision: int = _lib.PW_MIXED_FP32, tol: float = 5e-7,
             max_iter: int = 300, prob=None, which=("tpa", "mlp")):
    """TPA vs MLP solves of one cell from the same start: iterations, wall time, eigenvalues."""
    import torch
    nb = cell.nbands
    if prob is None:
        prob, _ = build_problem(cell, ik, precision=precision, max_bands=nb)
    npw = prob.npw
    out = {}
    for name, kind, nt in (("tpa", _lib.PW_PRECOND_TPA, None), ("mlp", _lib.PW_PRECOND_MLP, net)):
        if name not in which:
            continue
        x0 = band_block(nb, npw)
        x0[:, :npw] = torch.from_numpy(synth.psi_start(cell.seed, nb, npw, ik)).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = _lib.davidson_solve(prob, x0, tol=tol, precond=kind, net=nt, max_iter=max_iter)
        torch.cuda.synchronize()
        r["seconds"] = time.perf_counter() - t0
        out[name] = r
    if "tpa" in out and "mlp" in out:
        out["max_theta_diff_Ha"] = float(np.abs(out["tpa"]["theta"] - out["mlp"]["theta"]).max())
    return out
