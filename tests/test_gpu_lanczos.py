"""GPU Lanczos recursion on H (pw_lanczos_*) against the FP64 oracle chain.

Many chains run in lockstep on the GPU; each is compared with the oracle's
chain from the same start vector (oracle/lanczos.py, the FFT H*psi path).
Early coefficients agree to rounding (1e-10 relative: the GPU reorders the
sums of H*psi and of the dot products); later ones drift as the chain loses
orthogonality in finite precision on both sides, so long chains are checked
through what is stable: the continued fraction off the real axis against a
dense solve of <v|(z - H)^{-1}|v> and against the oracle's own fraction.
Breakdown: a start in a two-eigenvector subspace ends at beta_3 = 0.
"""
import numpy as np
import pytest

import synth
from oracle import hamiltonian as ham
from oracle import lanczos as olz

from gpu_util import log, problems, to_gpu_block

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_1709_10010_amd import _lib
    return _lib


def _starts(seed, nch, npw):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((nch, npw)) + 1j * rng.standard_normal((nch, npw))
    if nch > 1:
        v[1] *= 3.7       # chains of different norms
    return v


@pytest.mark.parametrize("cfg,nch,steps", [(0, 5, 25), (1, 9, 30)])
def test_lanczos_coefficients_match_oracle(lib, cfg, nch, steps):
    import torch
    c = synth.make_cell(cfg)
    po, pl = problems(c, max_bands=nch)
    v = _starts(70 + cfg, nch, po.npw)
    lz = lib.Lanczos(pl, nch, steps + 5)
    lz.start(to_gpu_block(v))
    lz.run(steps)
    a, b, n = lz.coefficients()
    torch.cuda.synchronize()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert n == steps
    assert np.all(a[:, steps:] == 0) and np.all(b[:, steps + 1:] == 0)
    worst = 0.0
    for ch in range(nch):
        ra, rb = olz.lanczos(po, v[ch], steps)
        k = min(steps, 20)
        ea = np.abs(a[ch, :k] - ra[:k]).max() / np.abs(ra).max()
        eb = np.abs(b[ch, :k + 1] - rb[:k + 1]).max() / np.abs(rb).max()
        worst = max(worst, ea, eb)
    log(f"cfg{cfg}: {nch} chains x {steps} steps, worst rel err of the first 20 coefficients {worst:.2e}")
    assert worst < 1e-10


def test_lanczos_resolvent_long_chain_against_dense_solve(lib):
    """Config-1 cell (949 plane waves), 4 chains of 200 steps: the GPU's
    continued fraction against <v|(z - H)^{-1}|v> from a dense solve, at
    points 0.05-0.5 Ha off the real axis."""
    import torch
    c = synth.make_cell(1)
    po, pl = problems(c, max_bands=4)
    v = _starts(75, 4, po.npw)
    lz = lib.Lanczos(pl, 4, 200)
    lz.start(to_gpu_block(v))
    lz.run(200)
    H = ham.dense_h(po)
    w = np.linalg.eigvalsh(H)
    z = np.array([w[0] - 0.1 + 0.05j, w[3] + 0.1j, w[40] + 0.2j, 0.5 * (w[0] + w[-1]) + 0.5j])
    g = lz.resolvent(torch.from_numpy(z).cuda()).cpu().numpy()
    for ch in range(4):
        exact = np.array([np.vdot(v[ch], np.linalg.solve(zk * np.eye(po.npw) - H, v[ch])) for zk in z])
        err = np.abs(g[ch] - exact).max() / np.abs(exact).max()
        log(f"chain {ch}: |g_gpu - dense| / |g| = {err:.2e}")
        assert err < 1e-7
    # the same chain on the oracle side gives the same fraction
    ra, rb = olz.lanczos(po, v[0], 200)
    ro = olz.continued_fraction(ra, rb, z)
    assert np.abs(g[0] - ro).max() <= 1e-7 * np.abs(ro).max()


def test_lanczos_breakdown_in_invariant_subspace(lib):
    import torch
    c = synth.make_cell(0)
    po, pl = problems(c, max_bands=2)
    _, U = np.linalg.eigh(ham.dense_h(po))
    v = np.zeros((2, po.npw), dtype=complex)
    v[0] = (0.6 - 0.3j) * U[:, 2] + 1.1j * U[:, 7]
    v[1] = _starts(77, 1, po.npw)[0]
    lz = lib.Lanczos(pl, 2, 6)
    lz.start(to_gpu_block(v))
    lz.run(6)
    a, b, _ = lz.coefficients()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    ra, rb = olz.lanczos(po, v[0], 6)
    log("breakdown chain: beta", b[0], "oracle", rb)
    assert b[0, 2] == 0.0 and np.all(b[0, 3:] == 0.0) and np.all(a[0, 2:] == 0.0)
    assert np.abs(a[0, :2] - ra[:2]).max() <= 1e-12 * np.abs(ra).max()
    assert np.all(b[1, 1:] > 0)          # the other chain runs on
    z = torch.tensor([0.3 + 0.05j, -1.0 + 0.2j], dtype=torch.complex128, device="cuda")
    assert np.all(np.isfinite(lz.resolvent(z).cpu().numpy()))


def test_lanczos_zero_start_and_limits(lib):
    import torch
    c = synth.make_cell(0)
    po, pl = problems(c, max_bands=3)
    v = np.zeros((3, po.npw), dtype=complex)
    v[2] = _starts(78, 1, po.npw)[0]
    lz = lib.Lanczos(pl, 3, 4)
    lz.start(to_gpu_block(v))
    lz.run(4)
    a, b, _ = lz.coefficients()
    assert torch.all(a[:2] == 0) and torch.all(b[:2] == 0)
    with pytest.raises(lib.PwError):
        lz.run(1)                         # past max_steps
    with pytest.raises(lib.PwError):
        lib.Lanczos(pl, 4, 4)             # more chains than the problem's max_bands


def test_lanczos_config2_sampled_chains(lib):
    """Full size: 256 chains on the medium workload's k-point 0 (npw 22119,
    72^3, 576 projectors), 30 steps; chains 0 and 201 against the oracle."""
    import time
    import torch
    c = synth.make_cell(2)
    po, pl = problems(c, max_bands=256)
    rng = np.random.default_rng(79)
    v = rng.standard_normal((256, po.npw)) + 1j * rng.standard_normal((256, po.npw))
    lz = lib.Lanczos(pl, 256, 30)
    lz.start(to_gpu_block(v))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lz.run(30)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"256 chains x 30 steps at npw {po.npw}: {dt:.4f} s, {256 * 30 / dt:.0f} chain-steps/s")
    a, b, _ = lz.coefficients()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    for ch in (0, 201):
        ra, rb = olz.lanczos(po, v[ch], 12)
        assert np.abs(a[ch, :12] - ra).max() <= 1e-10 * np.abs(ra).max()
        assert np.abs(b[ch, :13] - rb).max() <= 1e-10 * np.abs(rb).max()
