"""Library problems from seeded synthetic cells (product path, no oracle).

The sphere comes from the library's own ``pw_gsphere``; the potential and
projectors are sampled by the input generator ``synth``; everything else is
computed by the library.
"""
from __future__ import annotations

import numpy as np

import synth

from . import _lib


def stick_order(miller, nr):
    """The same G set listed by z-stick: (h mod N0, k mod N1) ascending, then
    l mod N2.  In this order the library's z passes read psi and write H psi
    in sequence instead of through a gather (any order gives the same H psi)."""
    m = np.asarray(miller, dtype=np.int32).reshape(-1, 3)
    key = np.lexsort((m[:, 2] % nr[2], m[:, 1] % nr[1], m[:, 0] % nr[0]))
    return np.ascontiguousarray(m[key])


def build_problem(cell, ik: int = 0, precision: int = _lib.PW_FP64, max_bands: int | None = None,
                  miller=None, ld_pad: int = 64, device="cuda", stream=None):
    """Create a library problem for k-point ``ik`` of ``cell``.

    Without ``miller`` the sphere is the library's ``pw_gsphere`` set listed
    by stick (``stick_order``).  Returns (Problem, miller) with the device
    copies of V and beta released once the handle has copied them.
    """
    import torch
    kf = np.asarray(cell.kpts[ik], dtype=np.float64)
    if miller is None:
        miller = stick_order(_lib.pw_gsphere(cell.A, kf, cell.ecut_ha), cell.nr)
    npw = miller.shape[0]
    v = torch.from_numpy(synth.vloc_on_grid(cell)).to(device)
    beta_h = synth.projectors(cell, kf, miller)
    ld = (npw + ld_pad - 1) // ld_pad * ld_pad
    beta = torch.zeros((beta_h.shape[0], ld), dtype=torch.complex128, device=device)
    beta[:, :npw] = torch.from_numpy(beta_h).to(device)
    prob = _lib.pw_problem_create(cell.A, kf, cell.ecut_ha, cell.nr, miller, v, beta,
                                  cell.proj_offset, cell.dij_concat(), precision=precision,
                                  max_bands=max_bands or cell.nbands, stream=stream,
                                  qij=cell.qij_concat())
    return prob, miller


def band_block(nb: int, npw: int, ld_pad: int = 64, device="cuda"):
    """Zeroed complex128 [nb][ld] block with ld = npw rounded up to ld_pad."""
    import torch
    ld = (npw + ld_pad - 1) // ld_pad * ld_pad
    return torch.zeros((nb, ld), dtype=torch.complex128, device=device)
