"""H*psi and the dense Hamiltonian on the plane-wave sphere.

Operator (paper, eq. pauli_ks, scalar norm-conserving reduction: one spin
component, no augmentation, S = 1):

  H = p^2/2m + V_LOC(r) + sum_I sum_mn D_I,mn |beta_m^I><beta_n^I|

in Hartree units, on the basis {e^{i(k+G).r}} with G in the cutoff sphere.
The kinetic operator is diagonal in G; the local potential acts on the FFT
mesh (the paper states that the kinetic energy acts "in the mesh defined by
the FFT grid"); the nonlocal term is built from the scalar products
<beta_j|psi_n> (the paper's p_ij arrays).

On the grid the local part is exactly the matrix
  V~(G - G' mod N),   V~(q) = N^-3 sum_r V(r) e^{-i q.r}
which ``dense_h`` writes out element by element and ``hpsi`` applies
through two FFTs.  The factor e^{ik.r} of a Bloch state cancels in V(r)psi.

TEST INFRASTRUCTURE ONLY (see package header).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import grid as _grid
from . import gsphere as _gs


@dataclasses.dataclass
class Problem:
    A: np.ndarray          # (3,3) bohr, rows a_i
    kfrac: np.ndarray      # (3,) crystal coordinates
    nr: tuple              # grid
    miller: np.ndarray     # (npw,3) int
    vloc: np.ndarray       # (N0,N1,N2) real, Ha
    beta: np.ndarray       # (nproj,npw) complex
    proj_offset: np.ndarray  # (natom+1,) int
    dij: list              # per-atom real symmetric blocks, Ha
    qij: list | None = None  # per-atom real symmetric augmentation blocks (S != 1), or None (S = 1)

    @property
    def npw(self) -> int:
        return int(self.miller.shape[0])

    @property
    def nproj(self) -> int:
        return int(self.beta.shape[0])

    def kinetic(self) -> np.ndarray:
        return _gs.kinetic(self.A, self.kfrac, self.miller)

    def d_matrix(self) -> np.ndarray:
        """Block-diagonal D (nproj x nproj) assembled from the per-atom blocks."""
        return self._blocks(self.dij)

    def q_matrix(self) -> np.ndarray:
        """Block-diagonal q of the overlap S (zeros when S = 1)."""
        return self._blocks(self.qij) if self.qij is not None else np.zeros((self.nproj, self.nproj))

    def _blocks(self, blocks) -> np.ndarray:
        d = np.zeros((self.nproj, self.nproj))
        for a, blk in enumerate(blocks):
            o0, o1 = int(self.proj_offset[a]), int(self.proj_offset[a + 1])
            d[o0:o1, o0:o1] = blk
        return d


def problem_from_cell(cell, ik: int = 0, miller=None) -> Problem:
    """Assemble a Problem from a synthetic cell (inputs from ``synth``)."""
    import synth

    kf = np.asarray(cell.kpts[ik], dtype=np.float64)
    if miller is None:
        miller = _gs.gsphere(cell.A, kf, cell.ecut_ha)
    return Problem(
        A=np.asarray(cell.A, dtype=np.float64),
        kfrac=kf,
        nr=tuple(int(x) for x in cell.nr),
        miller=np.asarray(miller, dtype=np.int32),
        vloc=synth.vloc_on_grid(cell),
        beta=synth.projectors(cell, kf, miller),
        proj_offset=cell.proj_offset,
        dij=[np.asarray(d, dtype=np.float64) for d in cell.dij],
        qij=None if getattr(cell, "qij", None) is None else [np.asarray(q, dtype=np.float64) for q in cell.qij],
    )


def apply_local(p: Problem, c: np.ndarray) -> np.ndarray:
    """(V psi)(G) for one band: scatter, inverse FFT, multiply, forward FFT, gather."""
    g = _grid.sphere_to_grid(c, p.miller, p.nr)
    u = _grid.inv_fft(g)
    w = p.vloc * u
    return _grid.grid_to_sphere(_grid.fwd_fft(w), p.miller, p.nr)


def projections(p: Problem, psi: np.ndarray) -> np.ndarray:
    """P[j, n] = <beta_j | psi_n> = sum_G beta_j(G)^* psi_n(G)."""
    return p.beta.conj() @ psi.T


def apply_nonlocal(p: Problem, psi: np.ndarray) -> np.ndarray:
    """sum_ij beta_i(G) D_ij <beta_j|psi_n>, returned band-major [nb][npw]."""
    q = p.d_matrix() @ projections(p, psi)
    return (p.beta.T @ q).T


def hpsi(p: Problem, psi: np.ndarray) -> np.ndarray:
    """H applied to each band of psi ([nb][npw] complex) through the FFT grid."""
    psi = np.atleast_2d(np.asarray(psi, dtype=np.complex128))
    if not _grid.fits(p.miller, p.nr):
        raise ValueError("sphere does not fit the FFT grid")
    t = p.kinetic()
    out = t[None, :] * psi
    for n in range(psi.shape[0]):
        out[n] += apply_local(p, psi[n])
    out += apply_nonlocal(p, psi)
    return out


def vtilde(p: Problem) -> np.ndarray:
    """V~(q) = N^-3 sum_r V(r) e^{-i q.r} on the whole grid of q."""
    return _grid.fwd_fft(p.vloc.astype(np.complex128))


def dense_h(p: Problem) -> np.ndarray:
    """H_{GG'} = t(G) delta + V~(G - G' mod N) + sum_ij beta_i(G) D_ij beta_j(G')^*."""
    vt = vtilde(p)
    m = np.asarray(p.miller, dtype=np.int64)
    dm = m[:, None, :] - m[None, :, :]
    h = vt[dm[..., 0] % p.nr[0], dm[..., 1] % p.nr[1], dm[..., 2] % p.nr[2]].astype(np.complex128)
    h[np.diag_indices(p.npw)] += p.kinetic()
    h += p.beta.T @ p.d_matrix() @ p.beta.conj()
    return h


def eigh_lowest(p: Problem, nb: int):
    """nb lowest eigenvalues (ascending) and eigenvectors of dense_h (LAPACK).
    With S != 1: the generalized problem H x = eps S x (eigenvectors
    S-orthonormal)."""
    if p.qij is not None:
        import scipy.linalg
        w, v = scipy.linalg.eigh(dense_h(p), dense_s(p))
        return w[:nb], v[:, :nb].T.copy()
    w, v = np.linalg.eigh(dense_h(p))
    return w[:nb], v[:, :nb].T.copy()


# ---------------------------------------------------------------- overlap S
# The paper's general Kohn-Sham equation (eq. pauli_ks) carries -eps_i S:
# with ultrasoft or PAW augmentation the overlap is
#   S = 1 + sum_I sum_mn q_I,mn |beta_m^I><beta_n^I|,
# built from the same projectors as the nonlocal term (the paper rewrites
# the overlap in terms of projector functions), so that H psi = eps S psi.

def spsi(p: Problem, psi: np.ndarray) -> np.ndarray:
    """S applied to each band of psi ([nb][npw]): psi + sum_ij beta_i q_ij <beta_j|psi>."""
    psi = np.atleast_2d(np.asarray(psi, dtype=np.complex128))
    if p.qij is None:
        return psi.copy()
    q = p.q_matrix() @ projections(p, psi)
    return psi + (p.beta.T @ q).T


def dense_s(p: Problem) -> np.ndarray:
    """S_{GG'} = delta_{GG'} + sum_ij beta_i(G) q_ij beta_j(G')^*."""
    s = np.eye(p.npw, dtype=np.complex128)
    if p.qij is not None:
        s += p.beta.T @ p.q_matrix() @ p.beta.conj()
    return s
