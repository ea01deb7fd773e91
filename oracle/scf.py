"""Self-consistent field loop around the eigensolver.

The Kohn-Sham potential is the sum of the local ionic, Hartree and
exchange-correlation potentials (the paper writes V_LOC that way in its
relativistic PAW section), and the exact-exchange section describes the
outer loop that rebuilds the operator from the bands until it stops
changing.  On the scalar, spin-unpolarised path, in Hartree atomic units:

  n(r)    = Omega^-1 sum_k w_k sum_n f_n |u_nk(r)|^2,   u_nk(r) = sum_G psi_nk(G) e^{iG.r}
            (the Bloch phase e^{ik.r} drops out of |psi|^2; bands normalised
            so that sum_G |psi(G)|^2 = 1)
  V_H(G)  = 4 pi n(G) / |G|^2 for G != 0, V_H(0) = 0
            (Poisson's equation in G space, the way the exact-exchange section
            solves it for pair densities; the G = 0 term is cancelled by the
            compensating background of the ions)
  V_x(r)  = -(3 n(r) / pi)^{1/3}   (local-density exchange of the uniform gas)
  V_eff   = V_ion + V_H + V_x
  mixing  : n_in <- n_in + alpha (n_out - n_in)   (linear), or with the Kerker
            weight on each Fourier component of the residual:
            n_in(G) <- n_in(G) + alpha G^2 / (G^2 + q0^2) (n_out - n_in)(G)
            (alpha alone at G = 0), which damps the long-wavelength charge
            oscillations linear mixing sets off in large cells

Readings where the paper is silent: exchange-only local-density functional;
Fermi-Dirac occupations f_nk = 2 / (1 + exp((eps_nk - mu) / sigma)) with the
chemical potential mu fixed by sum_k w_k sum_n f_nk = N_el (bisection; with
integer occupations the synthetic cells' near-degenerate levels swap places
from one step to the next and the loop never settles); linear mixing of the
density, Kerker-weighted when q0 > 0; the first step solves with V_ion alone and its output density is
the first input density; convergence when int |n_out - n_in| dr / N_el falls
below the tolerance.  The energy reported is the Harris-Foulkes form at the
input density, E = sum f eps - E_H + E_x - int v_x n, and the free energy
F = E - sigma S with S = -sum_k w_k sum_n 2 [g ln g + (1 - g) ln(1 - g)],
g = f / 2.

Grid conventions are those of ``grid``: n(G) = N^-3 sum_r n(r) e^{-iG.r},
so that int f g dr = Omega sum_G f(G)^* g(G).

TEST INFRASTRUCTURE ONLY (see package header).
"""
from __future__ import annotations

import numpy as np

from . import grid as _grid
from . import gsphere as _gs
from . import hamiltonian as _ham


def volume(A: np.ndarray) -> float:
    return float(abs(np.linalg.det(np.asarray(A, dtype=np.float64))))


def g_squared(A: np.ndarray, nr) -> np.ndarray:
    """|G|^2 of every grid point, G = h b_0 + k b_1 + l b_2 with the signed
    index h = j for j <= N/2, j - N above (the alias of the grid point)."""
    B = _gs.reciprocal(A)
    idx = [np.where(np.arange(n) <= n // 2, np.arange(n), np.arange(n) - n) for n in nr]
    h, k, l = np.meshgrid(*idx, indexing="ij")
    m = np.stack([h, k, l], axis=-1).astype(np.float64)
    g = m @ B
    return np.einsum("...i,...i->...", g, g)


def density(p: "_ham.Problem", psi: np.ndarray, f: np.ndarray) -> np.ndarray:
    """n(r) = Omega^-1 sum_n f_n |u_n(r)|^2 for the bands psi ([nb][npw]) of
    one k-point; f carries occupation times k-point weight."""
    psi = np.atleast_2d(psi)
    n = np.zeros(tuple(p.nr))
    for b in range(psi.shape[0]):
        u = _grid.inv_fft(_grid.sphere_to_grid(psi[b], p.miller, p.nr))
        n += f[b] * (u.real ** 2 + u.imag ** 2)
    return n / volume(p.A)


def hartree(n: np.ndarray, A: np.ndarray):
    """V_H(r) and E_H = (1/2) int V_H n dr for the density n on the grid."""
    ng = _grid.fwd_fft(n.astype(np.complex128))
    g2 = g_squared(A, n.shape)
    vg = np.zeros_like(ng)
    nz = g2 > 0
    vg[nz] = 4.0 * np.pi * ng[nz] / g2[nz]
    vh = _grid.inv_fft(vg).real
    eh = 0.5 * volume(A) * float(np.real(np.vdot(vg, ng)))
    return vh, eh


def lda_exchange(n: np.ndarray):
    """eps_x(n) = -(3/4)(3n/pi)^{1/3} per electron and v_x = d(n eps_x)/dn =
    -(3n/pi)^{1/3}; zero where n <= 0."""
    c = np.cbrt(3.0 * np.maximum(n, 0.0) / np.pi)
    return -0.75 * c, -c


def potential(vion: np.ndarray, n: np.ndarray, A: np.ndarray):
    """V_eff = V_ion + V_H[n] + V_x[n] and the energies that go with it:
    E_H, E_x = int n eps_x and int n v_x (grid sums times Omega / N^3)."""
    vh, eh = hartree(n, A)
    ex, vx = lda_exchange(n)
    dv = volume(A) / n.size
    e = {"hartree": eh, "xc": float(np.sum(n * ex) * dv), "vxc_n": float(np.sum(n * vx) * dv)}
    return vion + vh + vx, e


def fermi_occupations(eps, kweights, nel: float, sigma: float):
    """Occupations f_nk = 2 g((eps_nk - mu) / sigma), g(x) = 1 / (1 + e^x), and
    mu such that sum_k w_k sum_n f_nk = nel, by bisection on mu (the count
    is monotone in mu) to 1e-14 Ha; returns (f per k-point, mu, entropy S)."""
    eps = [np.asarray(e, dtype=np.float64) for e in eps]
    kweights = np.asarray(kweights, dtype=np.float64)

    def occ(mu):
        return [2.0 / (1.0 + np.exp(np.clip((e - mu) / sigma, -700.0, 700.0))) for e in eps]

    def count(mu):
        return float(sum(w * np.sum(f) for w, f in zip(kweights, occ(mu))))

    lo = min(float(e.min()) for e in eps) - 50.0 * sigma
    hi = max(float(e.max()) for e in eps) + 50.0 * sigma
    while hi - lo > 1e-14:
        mid = 0.5 * (lo + hi)
        if count(mid) < nel:
            lo = mid
        else:
            hi = mid
        if mid == lo and mid == hi:
            break
    mu = 0.5 * (lo + hi)
    f = occ(mu)
    ent = 0.0
    for w, fk in zip(kweights, f):
        g = np.clip(fk / 2.0, 1e-300, 1.0)
        h = np.clip(1.0 - fk / 2.0, 1e-300, 1.0)
        ent -= w * 2.0 * float(np.sum(g * np.log(g) + h * np.log(h)))
    return f, mu, ent


def mix(n_in: np.ndarray, n_out: np.ndarray, alpha: float, q0: float = 0.0, A=None) -> np.ndarray:
    """Next input density: linear (q0 = 0) or Kerker-weighted (q0 > 0, cell A)."""
    if q0 <= 0.0:
        return n_in + alpha * (n_out - n_in)
    rg = _grid.fwd_fft((n_out - n_in).astype(np.complex128))
    g2 = g_squared(A, n_in.shape)
    w = np.where(g2 > 0, alpha * g2 / (g2 + q0 * q0), alpha)
    return n_in + _grid.inv_fft(w * rg).real


def scf(probs, kweights, vion: np.ndarray, nel: float, nbands: int, sigma: float, alpha: float,
        tol: float, max_iter: int, q0: float = 0.0):
    """SCF loop over the k-point problems ``probs`` (their vloc is replaced by
    V_eff at every step), nbands eigenpairs per k-point from dense
    diagonalisation.  Step 0 solves with V_ion; step i >= 1 with V_eff[n_in].
    Returns the input density of the last step solved (n_in, zero at step 0),
    its output density, eigenvalues, occupations, mu and energies, and the
    history of int |n_out - n_in| dr / N_el over steps 1, 2, ..."""
    kweights = np.asarray(kweights, dtype=np.float64)
    A = probs[0].A
    dv = volume(A) / vion.size
    n_next = None
    hist = []
    for it in range(max_iter + 1):
        if n_next is None:
            n_in = np.zeros(vion.shape)
            v, e = vion.copy(), {"hartree": 0.0, "xc": 0.0, "vxc_n": 0.0}
        else:
            n_in = n_next
            v, e = potential(vion, n_in, A)
        eps, vecs = [], []
        for p in probs:
            p.vloc = v
            w, X = _ham.eigh_lowest(p, nbands)
            eps.append(w)
            vecs.append(X)
        f, mu, ent = fermi_occupations(eps, kweights, nel, sigma)
        n_out = np.zeros(vion.shape)
        for p, wk, X, fk in zip(probs, kweights, vecs, f):
            n_out += density(p, X, wk * fk)
        if it == 0:
            n_next = n_out
            continue
        d = float(np.sum(np.abs(n_out - n_in)) * dv) / nel
        hist.append(d)
        if d < tol:
            break
        n_next = mix(n_in, n_out, alpha, q0, A)
    eband = float(sum(wk * np.sum(fk * w) for wk, fk, w in zip(kweights, f, eps)))
    e["band"] = eband
    e["total"] = eband - e["hartree"] + e["xc"] - e["vxc_n"]
    e["free"] = e["total"] - sigma * ent
    return {"n_in": n_in, "n_out": n_out, "eigenvalues": eps, "occupations": f, "mu": mu,
            "energies": e, "history": hist, "converged": bool(hist and hist[-1] < tol), "veff": v}
