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
