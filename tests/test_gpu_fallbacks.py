"""GPU parity of the variants that environment switches select.

The library reads its switches once per process, so each set of variants
runs in a child process:
  - PW_GEMM_3M=0 / PW_PLANE_HALVES=0: FP64 complex GEMMs with four real MFMA
    products per complex product, and the register plane kernel with
    quad-permutation lane joins where the exchange-of-halves form applies;
    H (FP64) on nine bands of the tiny cell on 48^3 and 72^3 grids (N / 4
    even) against the oracle at the 1e-12 bound of the default variants;
  - the eigensolver and Davidson switches (full pair solves in every block
    Jacobi round, unblocked Cholesky and triangular inverse, two Gram-Schmidt
    passes in the first orthonormalisation round, the stop test over the pairs
    that touch the wanted diagonal entries,
    no active-space restart, the register plane kernel's scatter / gather
    form instead of its pipelined direct-I/O form) and, in a second child, the FFT and
    orthonormalisation switches (runtime FFT plans at compile-time sizes, a
    non-default stick tile, always two orthonormalisation rounds, a tighter
    eigensolver stop level): H on the tiny cell at 48^3 and 72^3 (1e-12),
    pw_eigh against LAPACK at m = 40, 130, 288 (1e-12 of the spectral
    radius), and a 32-band Davidson on the config-1 cell (subspaces up to
    96, so the block solver runs) against dense eigh (5e-9 Ha).
"""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[1] + "/tests")
import numpy as np, torch
import synth
from oracle import hamiltonian as ham
from gpu_util import from_gpu_block, problems, rel_err, start_block, to_gpu_block
from paper_1709_10010_amd import _lib
out = {}
for n in (48, 72):
    c = synth.make_cell(0, seed=31)
    c.nr = (n, n, n)
    po, pl = problems(c, max_bands=9)
    _lib.pw_problem_set_tuning(pl, 2, 9, 0, _lib.PW_PLANE_REGISTER)
    psi = start_block(c, 9, po.npw)
    x = to_gpu_block(psi)
    y = torch.full_like(x, complex(np.nan, np.nan))
    _lib.pw_hpsi(pl, x, y)
    out[str(n)] = rel_err(from_gpu_block(y, po.npw), ham.hpsi(po, psi))
    # projections alone exercise the split-K CN GEMM
    P = torch.zeros((9, po.nproj), dtype=torch.complex128, device="cuda")
    _lib.pw_projections(pl, x, P)
    torch.cuda.synchronize()
    out["proj" + str(n)] = rel_err(P.cpu().numpy(), ham.projections(po, psi).T)
print("RESULT " + json.dumps(out), flush=True)
"""


def test_four_product_gemm_and_quad_joins_match_oracle():
    env = dict(os.environ, PW_GEMM_3M="0", PW_PLANE_HALVES="0")
    print("child: PW_GEMM_3M=0 PW_PLANE_HALVES=0, tiny cell on 48^3 and 72^3", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True, text=True,
                       timeout=240)
    line = [s for s in r.stdout.splitlines() if s.startswith("RESULT ")]
    assert r.returncode == 0 and line, (r.returncode, r.stdout[-2000:], r.stderr[-2000:])
    errs = json.loads(line[-1][len("RESULT "):])
    print(errs, flush=True)
    for k, e in errs.items():
        assert e < 1e-12, (k, e)


CHILD2 = r"""
import json, sys
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[1] + "/tests")
import numpy as np, torch
import synth
from oracle import hamiltonian as ham
from gpu_util import from_gpu_block, problems, rel_err, start_block, to_gpu_block
from paper_1709_10010_amd import _lib
out = {}
for n in (48, 72):
    c = synth.make_cell(0, seed=31)
    c.nr = (n, n, n)
    po, pl = problems(c, max_bands=9)
    psi = start_block(c, 9, po.npw)
    x = to_gpu_block(psi)
    y = torch.full_like(x, complex(np.nan, np.nan))
    _lib.pw_hpsi(pl, x, y)
    out["hpsi" + str(n)] = rel_err(from_gpu_block(y, po.npw), ham.hpsi(po, psi))
for m in (40, 130, 288):
    rng = np.random.default_rng(m)
    X = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    A = (X + X.conj().T) / 2
    w, Z = _lib.pw_eigh(torch.from_numpy(A).cuda())
    w = w.cpu().numpy()
    out["eigh" + str(m)] = float(np.abs(w - np.linalg.eigvalsh(A)).max() / np.abs(w).max())
c = synth.make_cell(1)
po, pl = problems(c, max_bands=32)
res = _lib.davidson_solve(pl, to_gpu_block(start_block(c, 32, po.npw)), tol=5e-9)
wd, _ = ham.eigh_lowest(po, 32)
out["davidson_converged"] = bool(res["converged"])
out["davidson_iterations"] = int(res["iterations"])
out["davidson_theta"] = float(np.abs(res["theta"] - wd).max())
print("RESULT " + json.dumps(out), flush=True)
"""

VARIANT_SETS = [
    {"PW_BJ_CROSS": "0", "PW_CHOL_IMPL": "1", "PW_DAV_GS_FIRST": "2", "PW_EIG_WANTED": "1",
     "PW_DAV_ACT_MUL": "0", "PW_PLANE_PIPE": "0"},
    {"PW_FFT_GENERIC": "1", "PW_STICK_TILE": "8", "PW_DAV_ORTHO_SKIP": "0", "PW_DAV_OFF_FACTOR": "1"},
]


@pytest.mark.parametrize("variants", VARIANT_SETS, ids=["eigensolver", "fft_ortho"])
def test_switch_selected_variants_match_oracle(variants):
    env = dict(os.environ, **variants)
    print("child:", " ".join(f"{k}={v}" for k, v in variants.items()), flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD2, ROOT], env=env, capture_output=True, text=True,
                       timeout=300)
    line = [s for s in r.stdout.splitlines() if s.startswith("RESULT ")]
    assert r.returncode == 0 and line, (r.returncode, r.stdout[-2000:], r.stderr[-2000:])
    out = json.loads(line[-1][len("RESULT "):])
    print(out, flush=True)
    for k, e in out.items():
        if k.startswith("hpsi") or k.startswith("eigh"):
            assert e < 1e-12, (k, e)
    assert out["davidson_converged"] and out["davidson_theta"] < 5e-9
