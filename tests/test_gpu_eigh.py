"""GPU Jacobi eigensolver (pw_eigh) against LAPACK eigh on random Hermitian
matrices, in both code paths (m <= 64: one workgroup in LDS; larger: block
Jacobi over pairs of 16-index blocks, 4 to 64 blocks here).  Eigenvalues to
1e-12 relative of the spectral radius; eigenvectors through the residual
||A z - w z|| and orthonormality."""
import numpy as np
import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_1709_10010_amd import _lib
    return _lib


@pytest.mark.parametrize("m", [1, 2, 7, 48, 64, 65, 130, 288, 501, 1000])
def test_eigh_random_hermitian(lib, m):
    import time
    import torch
    rng = np.random.default_rng(m)
    X = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    A = (X + X.conj().T) / 2
    if m > 3:
        A[:, 2] = A[:, 1]  # a repeated column pair gives a near-degenerate spectrum
        A[2, :] = A[1, :]
        A = (A + A.conj().T) / 2
    At = torch.from_numpy(A).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w, Z = lib.pw_eigh(At)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    w, Z = w.cpu().numpy(), Z.cpu().numpy()
    ref = np.linalg.eigvalsh(A)
    scale = np.abs(ref).max()
    log("eigh m", m, "seconds", round(dt, 4), "max |w - ref|/scale", np.abs(w - ref).max() / scale)
    assert np.abs(w - ref).max() <= 1e-12 * scale
    assert np.abs(A @ Z - Z * w[None, :]).max() <= 1e-11 * scale
    assert np.abs(Z.conj().T @ Z - np.eye(m)).max() <= 1e-11
