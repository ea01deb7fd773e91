"""Batched H*psi over ragged cells: graph replay vs eager sweep vs oracle; autotuner."""
import numpy as np
import pytest

import synth
from oracle import hamiltonian as ham

from gpu_util import from_gpu_block, log, problems, rel_err, start_block, to_gpu_block

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_1709_10010_amd import _lib
    return _lib


def test_graph_replays_match_eager_and_oracle(lib):
    import torch
    cells = [synth.make_cell(4, i) for i in (0, 3, 7)] + [synth.make_cell(1)]
    probs, pos, xs, ys = [], [], [], []
    for c in cells:
        nb = min(c.nbands, 24)
        po, pl = problems(c, max_bands=nb)
        log("batch cell", c.name, "npw", po.npw, "grid", c.nr, "nb", nb)
        x = to_gpu_block(start_block(c, nb, po.npw))
        probs.append(pl)
        pos.append(po)
        xs.append(x)
        ys.append(torch.zeros_like(x))
    b = lib.Batch(probs, xs, ys)
    lib.pw_batch_hpsi(b)
    torch.cuda.synchronize()
    eager = [y.clone() for y in ys]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        lib.pw_batch_capture(b, s)
    s.synchronize()
    for rep in range(3):
        for y in ys:
            y.zero_()                      # eager work between replays
        torch.cuda.synchronize()
        lib.pw_batch_launch(b, s)
        s.synchronize()
        for y, e in zip(ys, eager):
            assert torch.equal(y, e), rep
    # one cell against the oracle
    po, x, y = pos[1], xs[1], ys[1]
    psi = from_gpu_block(x, po.npw)
    assert rel_err(from_gpu_block(y, po.npw), ham.hpsi(po, psi)) < 1e-12


def test_autotune_keeps_results(lib):
    import torch
    c = synth.make_cell(2)
    po, pl = problems(c, ik=0, max_bands=64)
    psi = start_block(c, 64, po.npw)
    x = to_gpu_block(psi)
    y0 = torch.zeros_like(x)
    lib.pw_hpsi(pl, x, y0)
    ms = lib.pw_problem_autotune(pl, 64, reps=2)
    tun = lib.pw_problem_tuning(pl)
    log("autotune cfg2 k0 64 bands: best ms", ms, tun)
    y1 = torch.zeros_like(x)
    lib.pw_hpsi(pl, x, y1)
    torch.cuda.synchronize()
    a, b = from_gpu_block(y0, po.npw), from_gpu_block(y1, po.npw)
    assert rel_err(b, a) < 1e-13
    assert rel_err(b[:3], ham.hpsi(po, psi[:3])) < 1e-12
