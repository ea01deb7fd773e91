"""Seeded Gaussian-well cells (inputs only; no method arithmetic).

Problem statement followed: the scalar, norm-conserving reduction of the
Kohn-Sham equation in the paper's fully relativistic PAW section (eq.
pauli_ks): kinetic p^2/2m on the FFT mesh, a local potential V_LOC(r) and a
separable nonlocal term sum_I,mn D_I,mn |beta_m^I><beta_n^I| with S = 1.

Readings (the paper gives no pseudopotential data for synthetic cells):
  * local potential  V(r) = -sum_a A_a sum_L exp(-|r - R_a - L|^2 / (2 s^2)),
    s = 0.8 bohr, A_a ~ U[0.5, 2] Ha, all periodic images L;
  * projectors  beta_{a,lm}(q) = (-i)^l Y_lm(q) q^l exp(-s_b^2 q^2 / 2)
    exp(-i q.R_a), q = k + G, s_b = 0.8 bohr, real harmonics
    (s: 1; p: x, y, z; d: xy, yz, zx, x^2-y^2, 3z^2-r^2), each normalised
    to unit 2-norm on the discrete sphere it is sampled on;
  * D per atom: diagonal U[0.1, 1] Ha, or (s+p+d cells) Q diag(lambda) Q^T
    with lambda ~ U[0.1, 1] Ha and Q a sign-fixed Haar orthogonal matrix.

Draw order from ``numpy.random.default_rng(seed)``: atom count / cell size /
cutoff / band count (ragged configs only), positions, depths, D, k-points.
Starting bands use an independent stream ``default_rng([seed, 7919, ik])``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BOHR_SIGMA_WELL = 0.8
BOHR_SIGMA_PROJ = 0.8


@dataclasses.dataclass
class Cell:
    """One synthetic cell: everything needed to build H at any k-point."""

    name: str
    seed: int
    A: np.ndarray            # (3,3) bohr, rows a1, a2, a3
    ecut_ha: float           # sphere: |k+G|^2 / 2 < ecut_ha
    nr: tuple                # FFT grid (N0, N1, N2)
    pos: np.ndarray          # (nat,3) bohr, Cartesian
    depth: np.ndarray        # (nat,) Ha, well depths A_a (> 0)
    lmax: np.ndarray         # (nat,) 1 = s+p (4 proj), 2 = s+p+d (9 proj)
    dij: list                # per-atom (np_a, np_a) real symmetric, Ha
    kpts: np.ndarray         # (nk,3) crystal (fractions of b1,b2,b3)
    nbands: int
    sigma_well: float = BOHR_SIGMA_WELL
    sigma_proj: float = BOHR_SIGMA_PROJ
    qij: list | None = None  # per-atom augmentation blocks of S (None: S = 1)

    @property
    def natom(self) -> int:
        return len(self.depth)

    @property
    def proj_offset(self) -> np.ndarray:
        n = np.array([(lm + 1) ** 2 for lm in self.lmax], dtype=np.int32)
        return np.concatenate([[0], np.cumsum(n)]).astype(np.int32)

    @property
    def nproj(self) -> int:
        return int(self.proj_offset[-1])

    def dij_concat(self) -> np.ndarray:
        """Row-major per-atom blocks, concatenated (library layout)."""
        return np.concatenate([d.reshape(-1) for d in self.dij]).astype(np.float64)

    def qij_concat(self) -> np.ndarray | None:
        """The augmentation blocks in the layout of dij_concat (None: S = 1)."""
        if self.qij is None:
            return None
        return np.concatenate([q.reshape(-1) for q in self.qij]).astype(np.float64)


def with_augmentation(cell: Cell, lo: float = 0.1, hi: float = 0.6) -> Cell:
    """A copy of `cell` with overlap augmentation: per atom a real symmetric
    block q, diagonal U[lo, hi] for s+p atoms, Q diag(mu) Q^T with mu ~
    U[lo, hi] and Q a sign-fixed Haar orthogonal matrix for s+p+d atoms
    (positive, so S = 1 + sum q |beta><beta| is positive definite).  Drawn
    from its own stream default_rng([seed, 2718]), so every other input of
    the cell is unchanged."""
    rng = np.random.default_rng([cell.seed, 2718])
    qs = []
    for lm in cell.lmax:
        n = (int(lm) + 1) ** 2
        mu = rng.uniform(lo, hi, size=n)
        if lm >= 2:
            o = _haar_orthogonal(rng, n)
            q = (o * mu[None, :]) @ o.T
            q = 0.5 * (q + q.T)
        else:
            q = np.diag(mu)
        qs.append(np.ascontiguousarray(q))
    out = dataclasses.replace(cell)
    out.qij = qs
    out.name = cell.name + ".aug"
    return out


def _is_smooth(n: int) -> bool:
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def smooth_grid(nmin: int) -> int:
    """Smallest 2*3*5-smooth integer >= nmin."""
    n = max(1, int(nmin))
    while not _is_smooth(n):
        n += 1
    return n


def alias_free_min(a_bohr: float, ecut_ry: float) -> int:
    """Grid size holding G up to 2*G_c for a cubic cell (cutoff 4*E_c).

    G_c = sqrt(ecut_Ry) bohr^-1; the largest Miller index on an axis is
    floor(G_c a / 2 pi), and products of two bands need twice that range.
    """
    hmax = int(math.floor(math.sqrt(ecut_ry) * a_bohr / (2.0 * math.pi)))
    return 4 * hmax + 1


def _positions(rng, nat: int, a: float, min_sep: float | None) -> np.ndarray:
    if not min_sep:
        return rng.uniform(0.0, a, size=(nat, 3))
    pos = np.zeros((nat, 3))
    placed = 0
    tries = 0
    while placed < nat:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place atoms with the requested separation")
        p = rng.uniform(0.0, a, size=3)
        if placed:
            d = pos[:placed] - p
            d -= a * np.round(d / a)
            if np.min(np.einsum("ij,ij->i", d, d)) < min_sep * min_sep:
                continue
        pos[placed] = p
        placed += 1
    return pos


def _min_sep(nat: int, a: float, want: float = 3.0) -> float:
    """Requested separation, capped at 0.7x the mean spacing (a^3/nat)^(1/3) so that
    random sequential placement stays feasible in dense cells."""
    return min(want, 0.7 * (a ** 3 / nat) ** (1.0 / 3.0))


def _haar_orthogonal(rng, n: int) -> np.ndarray:
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def _dij(rng, lmax: np.ndarray, full: bool) -> list:
    out = []
    for lm in lmax:
        n = (int(lm) + 1) ** 2
        lam = rng.uniform(0.1, 1.0, size=n)
        if full:
            q = _haar_orthogonal(rng, n)
            d = (q * lam[None, :]) @ q.T
            d = 0.5 * (d + d.T)
        else:
            d = np.diag(lam)
        out.append(np.ascontiguousarray(d))
    return out


def _cubic(a: float) -> np.ndarray:
    return np.eye(3) * float(a)


def make_cell(config: int, index: int = 0, seed: int | None = None) -> Cell:
    """Seeded cell for one of the five workloads.

    config 1 / 3 : a=10, 15 Ry, 24^3, 8 atoms s+p, diagonal D, 16 bands, Gamma.
    config 2     : a=20, 30 Ry, 72^3, 64 atoms (sep >= 3) s+p+d, full SPD D,
                   256 bands, Gamma + 4 k-points ~ U[-1/2, 1/2)^3.
    config 4     : ragged cell ``index`` of 64: a~U[10,18], ecut~U[20,40] Ry,
                   atoms U{8..48} s+p, bands U{32..192}, Gamma.
    config 5     : index < 200: training cell a~U[16,24], atoms U{32..96},
                   15 Ry, 4 bands per atom; index = -1: evaluation cell
                   a=24, 128 atoms, 30 Ry, 512 bands.
    config 0     : tiny cell a=6, 6 Ry, s+p, 4 atoms, 8 bands (brute-force size).
    """
    if config in (1, 3):
        s = 1001 if seed is None else seed
        rng = np.random.default_rng(s)
        a, ecut_ry, nat, nb, n = 10.0, 15.0, 8, 16, 24
        pos = _positions(rng, nat, a, None)
        depth = rng.uniform(0.5, 2.0, size=nat)
        lmax = np.ones(nat, dtype=np.int32)
        dij = _dij(rng, lmax, full=False)
        kpts = np.zeros((1, 3))
        return Cell(f"cfg{config}", s, _cubic(a), ecut_ry / 2, (n, n, n), pos,
                    depth, lmax, dij, kpts, nb)
    if config == 2:
        s = 2001 if seed is None else seed
        rng = np.random.default_rng(s)
        a, ecut_ry, nat, nb = 20.0, 30.0, 64, 256
        n = smooth_grid(alias_free_min(a, ecut_ry))
        pos = _positions(rng, nat, a, _min_sep(nat, a))
        depth = rng.uniform(0.5, 2.0, size=nat)
        lmax = np.full(nat, 2, dtype=np.int32)
        dij = _dij(rng, lmax, full=True)
        kpts = np.vstack([np.zeros((1, 3)), rng.uniform(-0.5, 0.5, size=(4, 3))])
        return Cell("cfg2", s, _cubic(a), ecut_ry / 2, (n, n, n), pos, depth,
                    lmax, dij, kpts, nb)
    if config == 4:
        s = 4000 + index if seed is None else seed
        rng = np.random.default_rng(s)
        a = rng.uniform(10.0, 18.0)
        ecut_ry = rng.uniform(20.0, 40.0)
        nat = int(rng.integers(8, 49))
        nb = int(rng.integers(32, 193))
        n = smooth_grid(alias_free_min(a, ecut_ry))
        pos = _positions(rng, nat, a, _min_sep(nat, a))
        depth = rng.uniform(0.5, 2.0, size=nat)
        lmax = np.ones(nat, dtype=np.int32)
        dij = _dij(rng, lmax, full=False)
        kpts = np.zeros((1, 3))
        return Cell(f"cfg4.{index}", s, _cubic(a), ecut_ry / 2, (n, n, n), pos,
                    depth, lmax, dij, kpts, nb)
    if config == 5:
        if index < 0:
            s = 5999 if seed is None else seed
            rng = np.random.default_rng(s)
            a, ecut_ry, nat, nb = 24.0, 30.0, 128, 512
        else:
            s = 5000 + index if seed is None else seed
            rng = np.random.default_rng(s)
            a = rng.uniform(16.0, 24.0)
            ecut_ry = 15.0
            nat = int(rng.integers(32, 97))
            nb = 4 * nat
        n = smooth_grid(alias_free_min(a, ecut_ry))
        pos = _positions(rng, nat, a, _min_sep(nat, a))
        depth = rng.uniform(0.5, 2.0, size=nat)
        lmax = np.ones(nat, dtype=np.int32)
        dij = _dij(rng, lmax, full=False)
        kpts = np.zeros((1, 3))
        name = "cfg5.eval" if index < 0 else f"cfg5.train{index}"
        return Cell(name, s, _cubic(a), ecut_ry / 2, (n, n, n), pos, depth,
                    lmax, dij, kpts, nb)
    if config == 0:
        s = 7 if seed is None else seed
        rng = np.random.default_rng(s)
        a, ecut_ry, nat, nb = 6.0, 6.0, 4, 8
        n = smooth_grid(alias_free_min(a, ecut_ry))
        pos = _positions(rng, nat, a, None)
        depth = rng.uniform(0.5, 2.0, size=nat)
        lmax = np.ones(nat, dtype=np.int32)
        dij = _dij(rng, lmax, full=False)
        kpts = np.zeros((1, 3))
        return Cell("tiny", s, _cubic(a), ecut_ry / 2, (n, n, n), pos, depth,
                    lmax, dij, kpts, nb)
    raise ValueError(f"unknown config {config}")


CONFIGS = {
    1: "a=10 bohr, 15 Ry, 24^3, 8 atoms s+p, 16 bands, Gamma",
    2: "a=20 bohr, 30 Ry, 72^3, 64 atoms s+p+d, 256 bands, Gamma + 4 k",
    3: "config 1 inputs, reduced-precision forms",
    4: "64 ragged cells a=10-18 bohr, 20-40 Ry, 8-48 atoms, 32-192 bands",
    5: "learned preconditioner: 200 training cells, eval a=24, 128 atoms, 30 Ry, 512 bands",
}


def _axis_profile(n: int, a: float, centre: float, sigma: float) -> np.ndarray:
    """sum_L exp(-(x_i - c - L a)^2 / (2 sigma^2)) on the grid x_i = i a / n."""
    x = np.arange(n) * (a / n)
    d = x - centre
    d -= a * np.round(d / a)
    acc = np.zeros(n)
    nimg = int(math.ceil(12.0 * sigma / a)) + 1
    for L in range(-nimg, nimg + 1):
        acc += np.exp(-((d - L * a) ** 2) / (2.0 * sigma * sigma))
    return acc


def vloc_on_grid(cell: Cell) -> np.ndarray:
    """Gaussian wells sampled on the grid, layout [N0][N1][N2] (N2 fastest).

    Orthorhombic cells only: the periodic Gaussian then factorises into a
    product of three 1D periodic profiles, summed over enough images that
    the truncated tail is below 1e-30 of a well depth.
    """
    A = cell.A
    if np.any(np.abs(A - np.diag(np.diag(A))) > 0):
        raise ValueError("vloc_on_grid: orthorhombic cells only")
    a = np.diag(A)
    n0, n1, n2 = cell.nr
    v = np.zeros((n0, n1, n2))
    for p, dep in zip(cell.pos, cell.depth):
        gx = _axis_profile(n0, a[0], p[0], cell.sigma_well)
        gy = _axis_profile(n1, a[1], p[1], cell.sigma_well)
        gz = _axis_profile(n2, a[2], p[2], cell.sigma_well)
        v -= dep * (gx[:, None, None] * gy[None, :, None] * gz[None, None, :])
    return v


def projectors(cell: Cell, kfrac, miller: np.ndarray) -> np.ndarray:
    """beta_{a,lm}(k+G) on the given Miller set: complex128 [nproj][npw].

    Evaluated at q = (k + m) @ B, B = 2 pi inv(A)^T; each row is scaled to
    unit 2-norm over the supplied set.  The ordering of ``miller`` is kept.
    """
    B = 2.0 * np.pi * np.linalg.inv(cell.A).T
    q = (np.asarray(miller, dtype=np.float64) + np.asarray(kfrac, dtype=np.float64)[None, :]) @ B
    qx, qy, qz = q[:, 0], q[:, 1], q[:, 2]
    q2 = qx * qx + qy * qy + qz * qz
    rad = np.exp(-0.5 * cell.sigma_proj ** 2 * q2)
    s3 = math.sqrt(3.0)
    ang = {
        0: [np.ones_like(qx)],
        1: [qx, qy, qz],
        2: [s3 * qx * qy, s3 * qy * qz, s3 * qz * qx,
            0.5 * s3 * (qx * qx - qy * qy), 0.5 * (3.0 * qz * qz - q2)],
    }
    rows = []
    for p, lm in zip(cell.pos, cell.lmax):
        phase = np.exp(-1j * (q @ p))
        for l in range(int(lm) + 1):
            for f in ang[l]:
                b = ((-1j) ** l) * f * rad * phase
                nrm = np.sqrt(np.sum(np.abs(b) ** 2))
                rows.append(b / nrm if nrm > 0 else b)
    return np.ascontiguousarray(np.array(rows, dtype=np.complex128))


def psi_start(seed: int, nbands: int, npw: int, ik: int = 0) -> np.ndarray:
    """Complex normal (x + i y)/sqrt(2) starting bands, [nbands][npw], NOT orthonormalised."""
    rng = np.random.default_rng([int(seed), 7919, int(ik)])
    z = rng.standard_normal((nbands, npw, 2))
    return np.ascontiguousarray((z[..., 0] + 1j * z[..., 1]) / math.sqrt(2.0))
