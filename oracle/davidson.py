"""Block Davidson for the lowest eigenpairs of H, FP64 (oracle).

The paper names a Davidson-like algorithm (Davidson 1975, cited for
turbo_davidson) and "subspace diagonalization used in PWscf in the
iterative diagonalization" (section on new parallelization levels); it
does not spell the iteration out.  The reading implemented here is the
standard block form, in this order:

  1. V = orthonormalised start block, W = H V, Hs = V^H W (Hermitised).
  2. eigh(Hs): Ritz values theta (ascending) and vectors Y, lowest nb kept.
  3. X = V Y, HX = W Y, R = HX - X diag(theta), rho_n = ||R_n||_2.
  4. All rho_n < tol: stop.
  5. Unconverged set U (soft locking); T_n = K(R_n) by the preconditioner.
  6. Restart when m + |U| > m_max: V = X, W = HX, Hs = diag(theta).
  7. Classical Gram-Schmidt twice against V, then Cholesky-QR of T;
     columns that are numerically dependent are dropped.  The pair is
     applied twice: once the corrections are small, one pass leaves V
     orthonormal only to ~1e-9, which lets Ritz values drop below the
     true eigenvalues.
  8. V = [V T], W = [W HT], Hs bordered with V^H (H T).  Back to 2.

The Teter-Payne-Allan (1989) preconditioner scales each residual
component by K(x) = (27+18x+12x^2+8x^3)/(27+18x+12x^2+8x^3+16x^4),
x = t(G)/T_n with T_n the band's kinetic energy <x_n|t|x_n>.

Matrices here are column-major in the mathematical sense: V is npw x m.

TEST INFRASTRUCTURE ONLY (see package header).  Iteration counts and
timings are "parity unpinned": the paper prints none.
"""
from __future__ import annotations

import numpy as np

from . import hamiltonian as _ham


def tpa_k(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    num = 27.0 + x * (18.0 + x * (12.0 + x * 8.0))
    return num / (num + 16.0 * x ** 4)


def tpa_apply(t: np.ndarray, X: np.ndarray, R: np.ndarray) -> np.ndarray:
    """T_n(G) = K(t(G)/T_n) R_n(G), T_n = sum_G t(G)|X_n(G)|^2 / ||X_n||^2."""
    tn = (t[:, None] * np.abs(X) ** 2).sum(axis=0) / (np.abs(X) ** 2).sum(axis=0)
    return tpa_k(t[:, None] / tn[None, :]) * R


def orthonormalize(T: np.ndarray, rel_drop: float = 1e-12) -> np.ndarray:
    """Cholesky-QR of T (npw x k); dependent columns dropped via eigh of T^H T."""
    if T.shape[1] == 0:
        return T
    S = T.conj().T @ T
    S = 0.5 * (S + S.conj().T)
    try:
        L = np.linalg.cholesky(S)
        d = np.abs(np.diag(L)) ** 2
        if np.min(d) > rel_drop * np.max(np.real(np.diag(S))):
            return np.linalg.solve(L.conj(), T.T).T  # T L^{-H}
    except np.linalg.LinAlgError:
        pass
    w, U = np.linalg.eigh(S)
    keep = w > rel_drop * max(w[-1], 0.0)
    return (T @ U[:, keep]) / np.sqrt(w[keep])[None, :]


def davidson(p: "_ham.Problem", psi0: np.ndarray, nb: int, tol: float,
             m_max: int | None = None, max_iter: int = 200,
             precond=None, record=None):
    """Lowest nb eigenpairs of H to residual 2-norm < tol (Hartree).

    psi0 : [nb][npw] start block (any full-rank block).
    precond : None -> TPA; "none" -> identity; callable(t, X, R, theta) -> T.
    record : optional list; per iteration a dict(X, R, theta, rho) is appended.
    Returns dict(theta, X (npw x nb), iterations, rho, n_hpsi, history).
    """
    t = p.kinetic()
    m_max = 3 * nb if m_max is None else int(m_max)
    V = orthonormalize(np.asarray(psi0, dtype=np.complex128).T.copy())
    if V.shape[1] < nb:
        raise ValueError("start block is rank deficient")
    W = _ham.hpsi(p, V.T).T
    n_hpsi = V.shape[1]
    Hs = V.conj().T @ W
    Hs = 0.5 * (Hs + Hs.conj().T)
    history = []
    for it in range(1, max_iter + 1):
        m = V.shape[1]
        w, Y = np.linalg.eigh(Hs)
        theta, Y = w[:nb], Y[:, :nb]
        X = V @ Y
        HX = W @ Y
        R = HX - X * theta[None, :]
        rho = np.sqrt((np.abs(R) ** 2).sum(axis=0))
        history.append((theta.copy(), rho.copy(), m))
        if record is not None:
            record.append(dict(X=X.copy(), R=R.copy(), theta=theta.copy(), rho=rho.copy()))
        if np.max(rho) < tol:
            return dict(theta=theta, X=X, iterations=it, rho=rho, n_hpsi=n_hpsi,
                        history=history, converged=True)
        U = np.nonzero(rho >= tol)[0]
        if precond is None:
            T = tpa_apply(t, X[:, U], R[:, U])
        elif precond == "none":
            T = R[:, U].copy()
        else:
            T = precond(t, X[:, U], R[:, U], theta[U])
        if m + len(U) > m_max:
            V, W = X, HX
            Hs = np.diag(theta).astype(np.complex128)
        for _ in range(2):
            for _ in range(2):
                T = T - V @ (V.conj().T @ T)
            T = orthonormalize(T)
        HT = _ham.hpsi(p, T.T).T
        n_hpsi += T.shape[1]
        Hvt = V.conj().T @ HT
        Htt = T.conj().T @ HT
        Htt = 0.5 * (Htt + Htt.conj().T)
        Hs = np.block([[Hs, Hvt], [Hvt.conj().T, Htt]])
        V = np.concatenate([V, T], axis=1)
        W = np.concatenate([W, HT], axis=1)
    return dict(theta=theta, X=X, iterations=max_iter, rho=rho, n_hpsi=n_hpsi,
                history=history, converged=False)


# ---------------------------------------------------------------- generalized problem
# With ultrasoft / PAW augmentation the paper's equation reads
# (H - eps S) psi = 0 (eq. pauli_ks).  The block Davidson then keeps the
# space S-orthonormal (V^H S V = 1), so the Rayleigh-Ritz problem V^H H V
# stays a standard Hermitian one, and the residual is H x - theta S x.
# The same steps as `davidson`, in the S inner product:
#   1. V = S-orthonormalised start block; W = H V, SV = S V; Hs = V^H W.
#   2. eigh(Hs) -> theta, Y; X = V Y, HX = W Y, SX = SV Y; R = HX - SX theta.
#   3. all |R_n| < tol: stop.  Else T = K(R) for the open bands.
#   4. restart when the space is full: V, W, SV = X, HX, SX; Hs = diag(theta).
#   5. twice: T <- T - V (SV^H T) (twice), then S-Cholesky-QR of T.
#   6. V, W, SV grow by T, H T, S T; Hs is bordered with V^H H T.

def orthonormalize_s(T: np.ndarray, ST: np.ndarray, rel_drop: float = 1e-12):
    """S-orthonormal basis of span(T) from T and ST = S T (npw x k): Cholesky
    of the Gram matrix T^H S T = L L^H, T <- T L^{-H} (ST likewise); with a
    (numerically) dependent column, eigh of the Gram matrix drops the
    directions below rel_drop of the largest."""
    if T.shape[1] == 0:
        return T, ST
    G = T.conj().T @ ST
    G = 0.5 * (G + G.conj().T)
    try:
        L = np.linalg.cholesky(G)
        d = np.abs(np.diag(L)) ** 2
        if np.min(d) > rel_drop * np.max(np.real(np.diag(G))):
            return np.linalg.solve(L.conj(), T.T).T, np.linalg.solve(L.conj(), ST.T).T
    except np.linalg.LinAlgError:
        pass
    w, U = np.linalg.eigh(G)
    keep = w > rel_drop * max(w[-1], 0.0)
    scale = U[:, keep] / np.sqrt(w[keep])[None, :]
    return T @ scale, ST @ scale


def davidson_generalized(p: "_ham.Problem", psi0: np.ndarray, nb: int, tol: float,
                         m_max: int | None = None, max_iter: int = 200):
    """Lowest nb eigenpairs of H x = theta S x to |H x - theta S x| < tol (Ha).
    Returns dict(theta, X (npw x nb, S-orthonormal), iterations, rho, converged)."""
    t = p.kinetic()
    m_max = 3 * nb if m_max is None else int(m_max)
    sop = lambda X: _ham.spsi(p, X.T).T          # noqa: E731
    hop = lambda X: _ham.hpsi(p, X.T).T          # noqa: E731
    V = np.asarray(psi0, dtype=np.complex128).T.copy()
    V, SV = orthonormalize_s(V, sop(V))
    if V.shape[1] < nb:
        raise ValueError("start block is rank deficient")
    W = hop(V)
    Hs = V.conj().T @ W
    Hs = 0.5 * (Hs + Hs.conj().T)
    for it in range(1, max_iter + 1):
        w, Y = np.linalg.eigh(Hs)
        theta, Y = w[:nb], Y[:, :nb]
        X, HX, SX = V @ Y, W @ Y, SV @ Y
        R = HX - SX * theta[None, :]
        rho = np.sqrt((np.abs(R) ** 2).sum(axis=0))
        if np.max(rho) < tol:
            return dict(theta=theta, X=X, iterations=it, rho=rho, converged=True)
        U = np.nonzero(rho >= tol)[0]
        T = tpa_apply(t, X[:, U], R[:, U])
        if V.shape[1] + len(U) > m_max:
            V, W, SV = X, HX, SX
            Hs = np.diag(theta).astype(np.complex128)
        for _ in range(2):
            for _ in range(2):
                T = T - V @ (SV.conj().T @ T)
            T, ST = orthonormalize_s(T, sop(T))
        HT = hop(T)
        Hvt = V.conj().T @ HT
        Htt = T.conj().T @ HT
        Htt = 0.5 * (Htt + Htt.conj().T)
        Hs = np.block([[Hs, Hvt], [Hvt.conj().T, Htt]])
        V = np.concatenate([V, T], axis=1)
        W = np.concatenate([W, HT], axis=1)
        SV = np.concatenate([SV, ST], axis=1)
    return dict(theta=theta, X=X, iterations=max_iter, rho=rho, converged=False)
