"""GPU parity of the launch variants that are off by default.

The library reads PW_GEMM_3M and PW_PLANE_HALVES once per process, so the
variants they select -- FP64 complex GEMMs with four real MFMA products per
complex product, and the register plane kernel with quad-permutation lane
joins at sizes where the exchange-of-halves form applies -- run in one child
process.  It applies H (FP64 form) to nine bands of the tiny cell on 48^3
and 72^3 grids (N / 4 even) and compares with the oracle at the 1e-12
bound of the default variants.
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
