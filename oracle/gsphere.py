"""Plane-wave sphere {G : |k+G|^2/2 < E_cut} and kinetic energies.

Bands are expanded as c_{k,n}(G) (paper, section on new parallelization
levels); the G-set is the set of reciprocal-lattice vectors inside the
kinetic-energy cutoff sphere centred at -k.  The ordering is the
reproducible one the paper asks for in its large-record data file section:
ascending kinetic energy, ties (same shell) broken by the Miller triple.

TEST INFRASTRUCTURE ONLY (see package header).
"""
from __future__ import annotations

import math

import numpy as np


def reciprocal(A: np.ndarray) -> np.ndarray:
    """B with rows b_i such that a_i . b_j = 2 pi delta_ij."""
    return 2.0 * np.pi * np.linalg.inv(np.asarray(A, dtype=np.float64)).T


def kinetic(A: np.ndarray, kfrac, miller: np.ndarray) -> np.ndarray:
    """t(G) = |k + G|^2 / 2 in Hartree, k and G from crystal coordinates."""
    q = (np.asarray(miller, dtype=np.float64) + np.asarray(kfrac, dtype=np.float64)[None, :]) @ reciprocal(A)
    return 0.5 * np.einsum("ij,ij->i", q, q)


def gsphere(A: np.ndarray, kfrac, ecut_ha: float) -> np.ndarray:
    """Miller triples (int32 [npw][3]) with |k+G|^2/2 < ecut_ha, canonical order.

    Search box: G . a_i = 2 pi h_i, so |h_i + k_i| <= |k+G| |a_i| / (2 pi).
    Canonical order: kinetic energy rounded to 12 significant digits,
    then h, then k, then l (all ascending).
    """
    A = np.asarray(A, dtype=np.float64)
    kfrac = np.asarray(kfrac, dtype=np.float64)
    qmax = math.sqrt(2.0 * ecut_ha)
    rng = []
    for i in range(3):
        span = qmax * np.linalg.norm(A[i]) / (2.0 * np.pi)
        lo = int(math.floor(-kfrac[i] - span)) - 1
        hi = int(math.ceil(-kfrac[i] + span)) + 1
        rng.append(np.arange(lo, hi + 1))
    h, k, l = np.meshgrid(rng[0], rng[1], rng[2], indexing="ij")
    m = np.stack([h.ravel(), k.ravel(), l.ravel()], axis=1)
    t = kinetic(A, kfrac, m)
    keep = t < ecut_ha
    m, t = m[keep], t[keep]
    key = np.array([float(f"{x:.11e}") for x in t])
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0], key))
    return np.ascontiguousarray(m[order].astype(np.int32))
