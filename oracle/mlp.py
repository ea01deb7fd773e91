"""Learned diagonal preconditioner: network, loss and optimiser (FP64 oracle).

The paper has no learned component; the workload defines it.  The reading:
  * per sample (G, n) four features
      f = (t(G) / T_n, theta_n, |R_n(G)| sqrt(npw) / ||R_n||, <V_loc>),
    T_n = <x_n|t|x_n> / <x_n|x_n> the band's kinetic energy (the TPA argument);
    standardised with stored mean / std;
  * three linear layers 4 -> 64 -> 64 -> 1, SiLU after the first two, and
    the output z mapped to s = S_LO + (S_HI - S_LO) sigmoid(z) with
    S_LO = 1/4, S_HI = 4, so the scale is positive and bounded;
  * correction T_n(G) = s(G, n) K_n(G) R_n(G) with K_n the Teter-Payne-Allan
    diagonal (the residual samples handed to the loss are K_n R_n);
  * loss for one band sample (n, iteration): 1 - |<d, sR>|^2 / (||d||^2 ||sR||^2)
    where d is the target correction, the part outside the iterate block of
    the move to the converged cluster (scale invariant, since the Davidson
    update uses only span(T));
  * Adam (Kingma & Ba 2015) with bias correction.

Parameters are a dict of W1 (64,4) b1 (64) W2 (64,64) b2 (64) W3 (1,64) b3 (1),
row-major, y = W x + b.

TEST INFRASTRUCTURE ONLY (see package header).
"""
from __future__ import annotations

import numpy as np

H = 64
NF = 4
PARAM_SHAPES = (("W1", (H, NF)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
                ("W3", (1, H)), ("b3", (1,)))


def init_params(seed: int) -> dict:
    """Kaiming-uniform weights (bound sqrt(6/fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in PARAM_SHAPES:
        if name.startswith("W"):
            bound = np.sqrt(6.0 / shp[1])
            p[name] = rng.uniform(-bound, bound, size=shp)
        else:
            p[name] = np.zeros(shp)
    return p


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


S_LO, S_HI = 0.25, 4.0


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def scale_out(z):
    return S_LO + (S_HI - S_LO) * sigmoid(z)


def forward(p: dict, F: np.ndarray):
    """F (ns, 4) standardised features -> s (ns,), cache for backward."""
    z1 = F @ p["W1"].T + p["b1"]
    a1 = silu(z1)
    z2 = a1 @ p["W2"].T + p["b2"]
    a2 = silu(z2)
    z3 = a2 @ p["W3"].T + p["b3"]
    s = scale_out(z3[:, 0])
    return s, (F, z1, a1, z2, a2, z3)


def backward(p: dict, cache, ds: np.ndarray) -> dict:
    """Gradients of sum_i ds_i * s_i with respect to every parameter."""
    F, z1, a1, z2, a2, z3 = cache
    q = sigmoid(z3[:, 0])
    g3 = (ds * (S_HI - S_LO) * q * (1.0 - q))[:, None]   # d/dz3
    gW3 = g3.T @ a2
    gb3 = g3.sum(axis=0)
    g2 = (g3 @ p["W3"]) * dsilu(z2)
    gW2 = g2.T @ a1
    gb2 = g2.sum(axis=0)
    g1 = (g2 @ p["W2"]) * dsilu(z1)
    gW1 = g1.T @ F
    gb1 = g1.sum(axis=0)
    return dict(W1=gW1, b1=gb1, W2=gW2, b2=gb2, W3=gW3, b3=gb3)


def features(t: np.ndarray, theta: np.ndarray, X: np.ndarray, R: np.ndarray,
             vavg: float) -> np.ndarray:
    """Raw features for every (G, n) of iterates X and residuals R (npw x nbands),
    band-major rows; the kinetic feature is t(G) / T_n with T_n the band's
    kinetic energy <x|t|x> / <x|x>."""
    npw, nbd = R.shape
    amp = np.abs(R) * np.sqrt(npw) / np.sqrt((np.abs(R) ** 2).sum(axis=0))[None, :]
    w = np.abs(X) ** 2
    tn = (t[:, None] * w).sum(axis=0) / w.sum(axis=0)
    f = np.empty((nbd, npw, NF))
    f[:, :, 0] = (t[:, None] / tn[None, :]).T
    f[:, :, 1] = theta[:, None]
    f[:, :, 2] = amp.T
    f[:, :, 3] = vavg
    return f.reshape(-1, NF)


def band_loss_grad(s: np.ndarray, R: np.ndarray, d: np.ndarray):
    """Loss 1 - |<d, sR>|^2/(|d|^2 |sR|^2) for one band and dL/ds (real, per G)."""
    u = s * R
    a = np.vdot(d, u)
    nd = np.vdot(d, d).real
    nu = np.vdot(u, u).real
    loss = 1.0 - abs(a) ** 2 / (nd * nu)
    da2 = 2.0 * np.real(np.conj(a) * np.conj(d) * R)
    dnu = 2.0 * s * np.abs(R) ** 2
    ds = -(da2 * nu - abs(a) ** 2 * dnu) / (nd * nu * nu)
    return loss, ds


def batch_loss_grad(p: dict, F: np.ndarray, R: np.ndarray, D: np.ndarray):
    """Mean band loss over a batch and its parameter gradients.

    F (nbd*npw, 4) standardised features, band-major; R, D (npw, nbd).
    """
    npw, nbd = R.shape
    s, cache = forward(p, F)
    S = s.reshape(nbd, npw)
    ds = np.empty_like(S)
    tot = 0.0
    for n in range(nbd):
        l, g = band_loss_grad(S[n], R[:, n], D[:, n])
        tot += l
        ds[n] = g / nbd
    return tot / nbd, backward(p, cache, ds.reshape(-1))


def adam_step(p: dict, g: dict, state: dict, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8) -> None:
    """One Adam update in place; ``state`` holds m, v and the step count."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1 - b1) * g[k]
        v[...] = b2 * v + (1 - b2) * g[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def target_correction(Xn: np.ndarray, Pc: np.ndarray, X: np.ndarray | None = None) -> np.ndarray:
    """d = P_c x / ||P_c x|| - x: the move from iterate x to the converged cluster
    (Pc: orthonormal columns spanning the cluster).  With the iterate block X
    (npw x nb, orthonormal columns) given, the part inside span(X) is removed,
    d - X X^H d, since the Rayleigh-Ritz step supplies that part itself."""
    y = Pc @ (Pc.conj().T @ Xn)
    d = y / np.linalg.norm(y) - Xn
    if X is not None:
        d = d - X @ (X.conj().T @ d)
    return d
