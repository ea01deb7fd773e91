"""pw_eigh_noalloc (static device scratch, no allocation) against pw_eigh
(caller workspace) through the C ABI: calls in a row on one GPU, each
smaller than the one before, so every call reuses scratch the previous one
left; each is checked against pw_eigh on the same matrix and against LAPACK.
Eigenvalues to 1e-12 of the spectral radius (as pw_eigh's own test);
eigenvectors through |<z_noalloc, z_eigh>| = 1 per column (the spectra are
simple) and the residual ||A z - w z||."""
import ctypes

import numpy as np
import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu


def _noalloc(lib, A):
    import torch
    m = int(A.shape[0])
    At = A.t().contiguous()
    w = torch.empty(m, dtype=torch.float64, device=A.device)
    Zt = torch.empty((m, m), dtype=torch.complex128, device=A.device)
    f = lib.LIB.pw_eigh_noalloc
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    f.restype = ctypes.c_int32
    f.argtypes = [vp, i64, ctypes.c_int32, vp, vp, i64, vp]
    st = f(vp(At.data_ptr()), m, m, vp(w.data_ptr()), vp(Zt.data_ptr()), m, lib._stream(None))
    if st != 0:
        raise lib.PwError(st, lib.LIB.pw_last_error().decode())
    torch.cuda.synchronize()
    return w, Zt.t()


def test_noalloc_matches_workspace_form_on_shrinking_calls():
    import torch
    from paper_1709_10010_amd import _lib as lib
    assert torch.cuda.is_available()
    for m in (512, 288, 40):
        log("pw_eigh_noalloc: m", m, "seed", 1000 + m)
        rng = np.random.default_rng(1000 + m)
        X = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
        A = (X + X.conj().T) / 2
        At = torch.from_numpy(A).cuda()
        w0, Z0 = lib.pw_eigh(At)
        w1, Z1 = _noalloc(lib, At)
        w0, Z0, w1, Z1 = (t.cpu().numpy() for t in (w0, Z0, w1, Z1))
        scale = np.abs(w0).max()
        ref = np.linalg.eigvalsh(A)
        log("  max |w_noalloc - w_eigh| / scale", np.abs(w1 - w0).max() / scale,
            " max |w_noalloc - lapack| / scale", np.abs(w1 - ref).max() / scale)
        assert np.abs(w1 - w0).max() <= 1e-12 * scale
        assert np.abs(w1 - ref).max() <= 1e-12 * scale
        ov = np.abs(np.einsum("gi,gi->i", Z0.conj(), Z1))
        assert np.abs(ov - 1.0).max() <= 1e-9, np.abs(ov - 1.0).max()
        assert np.abs(A @ Z1 - Z1 * w1[None, :]).max() <= 1e-11 * scale


def test_noalloc_rejects_size_beyond_maximum():
    import torch
    from paper_1709_10010_amd import _lib as lib
    A = torch.eye(513, dtype=torch.complex128, device="cuda")
    with pytest.raises(lib.PwError) as e:
        _noalloc(lib, A)
    assert e.value.status == -1 and "512" in str(e.value)
