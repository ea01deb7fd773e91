"""Lanczos recursion on H and the continued fraction of its resolvent (oracle).

The paper's section on dynamic perturbations (optical, EEL and magnetic
spectroscopies) computes a diagonal matrix element of a resolvent,
g_v(w) = <v | (w - L)^{-1} v> (eq. resolvent), from a Lanczos chain
(eqs. rec1 - rec4):

  q_0 = 0,  q_1 = v,
  alpha_n = <q_n | L q_n>,
  beta_{n+1} q_{n+1} = (L - alpha_n) q_n - beta_n q_{n-1},

with beta_{n+1} fixed by <q_{n+1}|q_{n+1}> = 1.  In the basis of the first M
vectors L is the tridiagonal T_M (eq. tridiagonal: alpha on the diagonal,
beta_2 .. beta_M beside it), and g_v(w) ~ <v|(w - T_M)^{-1} v> is the
continued fraction 1 / (w - alpha_1 - beta_2^2 / (w - alpha_2 - ...))
(eq. continuedfraction).  The paper states it for a Hermitian operator
(Haydock, Heine and Kelly); here L = H, the Kohn-Sham Hamiltonian the rest
of the oracle applies, and q_1 = v / ||v|| so that a start vector of any
norm works: g_v = ||v||^2 times the fraction (beta_1 = ||v|| is returned
beside the chain).

A chain whose beta_{n+1} vanishes has found an invariant subspace.  In
floating point it never vanishes exactly, so the chain ends (beta_{n+1} and
q_{n+1} set to zero, and every later alpha and beta zero, which ends the
fraction there) once beta_{n+1} <= BREAKDOWN ||H q_n||: the rest of the
residual is then rounding error, and normalising it would start a chain of
noise.  The paper is silent on breakdown; this threshold is a reading.

TEST INFRASTRUCTURE ONLY (see package header).
"""
from __future__ import annotations

import numpy as np

from . import hamiltonian as _ham

BREAKDOWN = 1e-12


def lanczos(p: "_ham.Problem", v: np.ndarray, steps: int, apply_h=None):
    """Chain of `steps` Lanczos steps from v (npw complex).

    Returns (alpha[steps], beta[steps + 1]) with beta[0] = ||v|| (the
    paper's beta_1 slot, which the recursion multiplies by q_0 = 0) and
    beta[n] = beta_{n+1} for n >= 1, i.e. alpha[n-1] = alpha_n.
    apply_h: optional callable x -> H x (default: the oracle's FFT H*psi).
    """
    h = apply_h if apply_h is not None else (lambda x: _ham.hpsi(p, x[None, :])[0])
    v = np.asarray(v, dtype=np.complex128)
    alpha = np.zeros(steps)
    beta = np.zeros(steps + 1)
    beta[0] = np.linalg.norm(v)
    q_prev = np.zeros_like(v)
    q = v / beta[0] if beta[0] > 0 else np.zeros_like(v)
    b = 0.0                                     # beta_n multiplying q_{n-1}; q_0 = 0
    for n in range(steps):
        hq = h(q)
        a = float(np.real(np.vdot(q, hq)))      # alpha_n = <q_n | H q_n>, real for Hermitian H
        w = hq - a * q - b * q_prev
        bn = float(np.linalg.norm(w))           # beta_{n+1}: <q_{n+1}|q_{n+1}> = 1
        if bn <= BREAKDOWN * float(np.linalg.norm(hq)):
            bn = 0.0                            # invariant subspace: the chain ends
        alpha[n] = a
        beta[n + 1] = bn
        q_prev, q = q, (w / bn if bn > 0 else np.zeros_like(w))
        b = bn
    return alpha, beta


def tridiagonal(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """T_M of the chain (eq. tridiagonal): alpha_1..M on the diagonal,
    beta_2..beta_M on the first off-diagonals (beta[1 .. M-1] here)."""
    m = len(alpha)
    t = np.diag(np.asarray(alpha, dtype=np.float64))
    for n in range(m - 1):
        t[n, n + 1] = t[n + 1, n] = beta[n + 1]
    return t


def continued_fraction(alpha: np.ndarray, beta: np.ndarray, z) -> np.ndarray:
    """g(z) = ||v||^2 / (z - alpha_1 - beta_2^2 / (z - alpha_2 - ... - beta_M^2 / (z - alpha_M)))
    for each complex z (eq. continuedfraction), evaluated from the bottom up."""
    z = np.asarray(z, dtype=np.complex128)
    m = len(alpha)
    g = 1.0 / (z - alpha[m - 1])
    for n in range(m - 2, -1, -1):
        g = 1.0 / (z - alpha[n] - beta[n + 1] ** 2 * g)
    return beta[0] ** 2 * g
