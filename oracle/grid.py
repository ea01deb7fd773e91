"""Sphere <-> real-space grid and the grid Fourier transforms.

Conventions (the paper's Poisson / exchange paragraph solves on an FFT
grid holding G up to a modulus 2 G_c; the transform signs are not stated,
the reading used here is):
  u(r_j) = sum_G c(G) exp(+i G.r_j)                      (inverse, unnormalised)
  c(G)   = N^-3 sum_j w(r_j) exp(-i G.r_j)               (forward, 1/N^3)
with r_j = (j0/N0, j1/N1, j2/N2) in crystal coordinates, so
G.r_j = 2 pi (h j0/N0 + k j1/N1 + l j2/N2).  A Miller triple maps to the
grid point (h mod N0, k mod N1, l mod N2); that map is one-to-one when
|h_i| < N_i/2 on every axis.

TEST INFRASTRUCTURE ONLY (see package header).
"""
from __future__ import annotations

import numpy as np


def grid_index(miller: np.ndarray, nr) -> tuple:
    m = np.asarray(miller, dtype=np.int64)
    return (m[:, 0] % nr[0], m[:, 1] % nr[1], m[:, 2] % nr[2])


def fits(miller: np.ndarray, nr) -> bool:
    m = np.abs(np.asarray(miller, dtype=np.int64))
    return all(2 * int(m[:, i].max(initial=0)) < int(nr[i]) for i in range(3))


def sphere_to_grid(c: np.ndarray, miller: np.ndarray, nr) -> np.ndarray:
    g = np.zeros(tuple(int(x) for x in nr), dtype=np.complex128)
    g[grid_index(miller, nr)] = c
    return g


def grid_to_sphere(g: np.ndarray, miller: np.ndarray, nr) -> np.ndarray:
    return g[grid_index(miller, nr)].copy()


def inv_fft(g: np.ndarray) -> np.ndarray:
    """u(r) = sum_G c(G) e^{+iG.r}: numpy's ifftn carries 1/N, undo it."""
    return np.fft.ifftn(g) * g.size


def fwd_fft(u: np.ndarray) -> np.ndarray:
    """c(G) = N^-3 sum_r u(r) e^{-iG.r}."""
    return np.fft.fftn(u) / u.size


def dft_direct(g: np.ndarray, sign: int) -> np.ndarray:
    """Direct O(N^6) sum  out[j] = sum_m g[m] exp(sign 2 pi i m.j / N), no scaling.

    Used only to pin ``inv_fft`` / ``fwd_fft`` on tiny grids.
    """
    n0, n1, n2 = g.shape
    out = np.zeros_like(g, dtype=np.complex128)
    m0, m1, m2 = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij")
    for j0 in range(n0):
        for j1 in range(n1):
            for j2 in range(n2):
                ph = 2.0 * np.pi * (m0 * j0 / n0 + m1 * j1 / n1 + m2 * j2 / n2)
                out[j0, j1, j2] = np.sum(g * np.exp(sign * 1j * ph))
    return out
