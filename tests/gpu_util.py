"""Helpers shared by the GPU tests: identical inputs for the oracle and the library."""
import sys

import numpy as np

import synth
from oracle import hamiltonian as ham


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def problems(cell, ik=0, precision=0, max_bands=None, miller=None, ld_pad=64):
    """Oracle Problem and library Problem built from the same inputs.

    The Miller set is the oracle's (so no oracle input comes from the GPU
    path); V and beta are sampled once by the generator and fed to both.
    """
    import torch
    from paper_1709_10010_amd import _lib

    po = ham.problem_from_cell(cell, ik, miller=miller)
    npw = po.npw
    ld = (npw + ld_pad - 1) // ld_pad * ld_pad
    v = torch.from_numpy(po.vloc).cuda()
    beta = torch.zeros((po.nproj, ld), dtype=torch.complex128, device="cuda")
    if po.nproj:
        beta[:, :npw] = torch.from_numpy(po.beta).cuda()
    dij = np.concatenate([d.reshape(-1) for d in po.dij]) if po.dij else np.zeros(0)
    qij = np.concatenate([q.reshape(-1) for q in po.qij]) if po.qij is not None else None
    pl = _lib.pw_problem_create(po.A, po.kfrac, cell.ecut_ha, po.nr, po.miller, v,
                                beta if po.nproj else None, po.proj_offset, dij,
                                precision=precision, max_bands=max_bands or cell.nbands, qij=qij)
    return po, pl


def to_gpu_block(x, ld_pad=64):
    import torch
    nb, npw = x.shape
    ld = (npw + ld_pad - 1) // ld_pad * ld_pad
    t = torch.zeros((nb, ld), dtype=torch.complex128, device="cuda")
    t[:, :npw] = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return t


def from_gpu_block(t, npw):
    import torch
    torch.cuda.synchronize()
    return t[:, :npw].cpu().numpy()


def rel_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def start_block(cell, nb, npw, ik=0):
    return synth.psi_start(cell.seed, nb, npw, ik)
