"""Exact (Fock) exchange and its adaptively compressed form (ACE).

The Fock operator on a state phi (paper, exact-exchange section, eq. Vx),
spin-unpolarised, Hartree units (e^2 = 1):

  (V_x phi)(r) = - sum_j w_j psi_j(r) v_j(r),
  v_j(r) = int dr' rho_j(r') / |r - r'|,   rho_j(r) = psi_j^*(r) phi(r)   (eq. Poisson)

with the sum over the occupied states psi_j (w_j = 1 for a fully occupied
spatial orbital; a fractional occupation scales its term).  The Poisson
equation is solved in reciprocal space, as the paper does:
v_j(G) = 4 pi rho_j(G) / |G|^2.  ACE (eq. Vxace) replaces V_x by

  V_x phi ~ sum_jm xi_j (M^-1)_jm <xi_m | phi>,   xi_i = V_x psi_i,  M_jm = <psi_j | xi_m>,

exact for phi in the span of the occupied states.

Readings where the paper is silent: Gamma-point sampling only (the pair
densities then carry no Bloch phase and the kernel is 4 pi / |G|^2); the
G = 0 term of the kernel is dropped, as for the Hartree potential (a
compensating background; the integrable divergence is not corrected); the
Poisson solves run on the full FFT grid (G up to 2 G_c, the exact rule of
the paper's ecutfock paragraph).  Plane-wave coefficients are normalised as
in ``hamiltonian``: psi(r) = Omega^-1/2 sum_G c(G) e^{iG.r}, so that in
coefficients (V_x phi)(G) = N^-3 sum_r [- sum_j w_j u_j(r) v_j(r)] e^{-iG.r}
with u = sum_G c(G) e^{iG.r} and rho_j = conj(u_j) u_phi / Omega.

TEST INFRASTRUCTURE ONLY (see package header).
"""
from __future__ import annotations

import numpy as np

from . import grid as _grid
from . import hamiltonian as _ham
from . import scf as _scf


def coulomb_kernel(A: np.ndarray, nr) -> np.ndarray:
    """4 pi / |G|^2 on the grid of G (signed indices), 0 at G = 0."""
    g2 = _scf.g_squared(A, nr)
    k = np.zeros_like(g2)
    k[g2 > 0] = 4.0 * np.pi / g2[g2 > 0]
    return k


def vx(p: "_ham.Problem", psi_occ: np.ndarray, w_occ: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """V_x applied to each band of phi ([nphi][npw]) for the occupied bands
    psi_occ ([nocc][npw]) with weights w_occ; Gamma point only."""
    if np.any(np.asarray(p.kfrac) != 0):
        raise ValueError("exchange: Gamma point only")
    psi_occ = np.atleast_2d(psi_occ)
    phi = np.atleast_2d(phi)
    omega = _scf.volume(p.A)
    kern = coulomb_kernel(p.A, p.nr)
    u_occ = [_grid.inv_fft(_grid.sphere_to_grid(c, p.miller, p.nr)) for c in psi_occ]
    out = np.zeros_like(phi, dtype=np.complex128)
    for i in range(phi.shape[0]):
        u_i = _grid.inv_fft(_grid.sphere_to_grid(phi[i], p.miller, p.nr))
        acc = np.zeros(tuple(p.nr), dtype=np.complex128)
        for wj, u_j in zip(w_occ, u_occ):
            rho = np.conj(u_j) * u_i / omega
            v = _grid.inv_fft(kern * _grid.fwd_fft(rho))
            acc -= wj * u_j * v
        out[i] = _grid.grid_to_sphere(_grid.fwd_fft(acc), p.miller, p.nr)
    return out


def ace(p: "_ham.Problem", psi_occ: np.ndarray, w_occ: np.ndarray):
    """xi = V_x psi_occ ([nocc][npw]) and M_jm = <psi_j | xi_m>."""
    xi = vx(p, psi_occ, w_occ, psi_occ)
    M = np.conj(psi_occ) @ xi.T
    return xi, M


def ace_apply(xi: np.ndarray, M: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """sum_jm xi_j (M^-1)_jm <xi_m | phi_i> for each band of phi."""
    phi = np.atleast_2d(phi)
    C = np.conj(xi) @ phi.T            # C[m, i] = <xi_m | phi_i>
    Y = np.linalg.solve(M, C)          # M^-1 C
    return (xi.T @ Y).T


def exchange_energy(p: "_ham.Problem", psi_occ: np.ndarray, w_occ: np.ndarray) -> float:
    """Exchange energy of doubly occupied spatial orbitals: the pair sum
    -(1/2) sum_ij (ij|ji) once per spin, so E_x = sum_i w_i <psi_i | V_x psi_i>."""
    xi = vx(p, psi_occ, w_occ, psi_occ)
    return float(np.real(np.sum(np.asarray(w_occ) * np.einsum("ig,ig->i", np.conj(psi_occ), xi))))


def ace_matrix(xi: np.ndarray, M: np.ndarray) -> np.ndarray:
    """The compressed operator xi M^-1 xi^H as a dense npw x npw matrix."""
    return xi.T @ np.linalg.solve(M, np.conj(xi))


def scf_hybrid(p: "_ham.Problem", vion: np.ndarray, nel: float, nbands: int, sigma: float, alpha: float,
               tol: float, max_iter: int, exx_alpha: float, exx_tol: float, max_outer: int, q0: float = 0.0):
    """The paper's double loop for a hybrid functional, Gamma point, one k-point.

    Inner loop: the SCF loop of ``scf`` (Fermi occupations, linear or Kerker
    mixing, convergence in int |n_out - n_in| / N_el) with the Fock
    operator fixed as exx_alpha V_ace and the local exchange scaled by
    1 - exx_alpha.  Outer loop: rebuild V_ace from the occupied orbitals of
    the converged inner loop (those with f/2 > 1e-8, weights f/2) until the
    exchange energy e_xx = sum_i w_i <psi_i | V_ace psi_i> changes by less
    than exx_tol.  The first inner loop runs the plain local functional
    (no Fock term, full local exchange).  Reported energy:
    E = sum f eps - exx_alpha e_xx - E_H + (1 - exx_alpha) (E_x - int v_x n)
    (the band energy counts the Fock term twice), F = E - sigma S."""
    if np.any(np.asarray(p.kfrac) != 0):
        raise ValueError("hybrid SCF: Gamma point only")
    A = p.A
    dv = _scf.volume(A) / vion.size
    vion = np.asarray(vion, dtype=np.float64)
    xfrac, hx, e_xx = 1.0, None, 0.0
    n_next = None
    hist, exx_hist = [], []
    first = True
    for outer in range(max_outer + 1):
        for it in range(max_iter + 1):
            if n_next is None:
                n_in = np.zeros(vion.shape)
                v, e = vion.copy(), {"hartree": 0.0, "xc": 0.0, "vxc_n": 0.0}
            else:
                n_in = n_next
                vh, eh = _scf.hartree(n_in, A)
                ex, vx = _scf.lda_exchange(n_in)
                v = vion + vh + xfrac * vx
                e = {"hartree": eh, "xc": xfrac * float(np.sum(n_in * ex) * dv),
                     "vxc_n": xfrac * float(np.sum(n_in * vx) * dv)}
            p.vloc = v
            H = _ham.dense_h(p)
            if hx is not None:
                H = H + exx_alpha * hx
            w, U = np.linalg.eigh((H + H.conj().T) / 2)
            eps, X = w[:nbands], U[:, :nbands].T.copy()
            f, mu, ent = _scf.fermi_occupations([eps], [1.0], nel, sigma)
            n_out = _scf.density(p, X, f[0])
            if first:
                first = False
                n_next = n_out
                continue
            d = float(np.sum(np.abs(n_out - n_in)) * dv) / nel
            hist.append(d)
            if d < tol:
                break
            n_next = _scf.mix(n_in, n_out, alpha, q0, A)
        if exx_alpha == 0.0:
            break
        occ = f[0] / 2.0 > 1e-8
        xi, M = ace(p, X[occ], f[0][occ] / 2.0)
        e_new = float(np.real(np.sum(f[0][occ] / 2.0 * np.diag(M))))
        exx_hist.append(e_new)
        if outer >= 1 and abs(e_new - e_xx) < exx_tol:
            e_xx = e_new
            break
        hx, e_xx, xfrac = ace_matrix(xi, M), e_new, 1.0 - exx_alpha
        n_next = n_in
    eband = float(np.sum(f[0] * eps))
    e["band"] = eband
    e["exx"] = e_xx
    e["total"] = eband - exx_alpha * e_xx - e["hartree"] + e["xc"] - e["vxc_n"]
    e["free"] = e["total"] - sigma * ent
    return {"n_in": n_in, "n_out": n_out, "eigenvalues": eps, "vectors": X, "occupations": f[0], "mu": mu,
            "energies": e, "history": hist, "exx_history": exx_hist,
            "converged": bool(hist and hist[-1] < tol)}
