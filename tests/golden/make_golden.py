#!/usr/bin/env python3
"""Writes the stored expected values under tests/golden/ from the FP64 oracle
alone (dense diagonalisation of the discrete Hamiltonian of eq. pauli_ks on
the sphere basis; sphere sizes from the cutoff inequality; the oracle's
block Davidson at the medium workload's full size).

    python tests/golden/make_golden.py               # everything (~20 min)
    python tests/golden/make_golden.py --quick       # without the Davidson goldens
    python tests/golden/make_golden.py --config4     # only the two ragged-batch cells
    python tests/golden/make_golden.py --augmented   # only the medium workload with S != 1
    python tests/golden/make_golden.py --scf         # only the SCF loops of the config-1 cell
    python tests/golden/make_golden.py --hybrid      # only its hybrid double loop

Regression fixtures: tests/test_golden.py recomputes them with the oracle,
and the GPU tests compare the library against them.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import gsphere  # noqa: E402
from oracle import hamiltonian as ham  # noqa: E402


def eig_fixture(cfg, nlow):
    c = synth.make_cell(cfg)
    po = ham.problem_from_cell(c)
    w, _ = ham.eigh_lowest(po, nlow)
    return c, po, w


def sphere_rows():
    rows = []
    for cfg, idx in ((0, 0), (1, 0), (2, 0), (5, -1)):
        c = synth.make_cell(cfg, idx)
        for ik in range(len(c.kpts)):
            m = gsphere.gsphere(c.A, c.kpts[ik], c.ecut_ha)
            rows.append((c.name, ik, len(m)))
    return rows


def davidson_config2(ik):
    """Oracle block Davidson (TPA, soft locking, m_max = 3 nb) on the medium
    workload at k-point ik, all 256 bands, to a residual 2-norm of 5e-9 Ha
    (1e-8 Ry) on every band."""
    from oracle import davidson as odv
    c = synth.make_cell(2)
    po = ham.problem_from_cell(c, ik)
    r = odv.davidson(po, synth.psi_start(c.seed, c.nbands, po.npw, ik), c.nbands, 5e-9)
    assert r["converged"], "oracle Davidson did not converge"
    fname = f"config2_k{ik}_davidson256_Ha.txt"
    with open(os.path.join(HERE, fname), "w") as f:
        f.write(f"# {c.name} k-point {ik} (crystal {np.round(c.kpts[ik], 6).tolist()}): npw {po.npw}, grid "
                f"{c.nr[0]}^3, {c.nbands} bands; oracle block Davidson to |Hx - theta x| < 5e-9 Ha "
                f"({r['iterations']} iterations); columns: theta (Ha), residual 2-norm (Ha); "
                f"written by make_golden.py (oracle only)\n")
        for t, rho in zip(r["theta"], r["rho"]):
            f.write(f"{t:.17e} {rho:.3e}\n")


def davidson_config4(index):
    """Oracle block Davidson on one cell of the ragged batch (its own band
    count, Gamma point) to 5e-9 Ha on every band."""
    from oracle import davidson as odv
    c = synth.make_cell(4, index)
    po = ham.problem_from_cell(c)
    r = odv.davidson(po, synth.psi_start(c.seed, c.nbands, po.npw), c.nbands, 5e-9)
    assert r["converged"], "oracle Davidson did not converge"
    fname = f"config4_cell{index}_davidson_Ha.txt"
    with open(os.path.join(HERE, fname), "w") as f:
        f.write(f"# {c.name}: a {c.A[0, 0]:.4f} bohr, ecut {c.ecut_ha:.6f} Ha, npw {po.npw}, grid {c.nr[0]}^3, "
                f"{c.natom} atoms, {c.nbands} bands; oracle block Davidson to |Hx - theta x| < 5e-9 Ha "
                f"({r['iterations']} iterations); columns: theta (Ha), residual 2-norm (Ha); "
                f"written by make_golden.py (oracle only)\n")
        for t, rho in zip(r["theta"], r["rho"]):
            f.write(f"{t:.17e} {rho:.3e}\n")


def davidson_config2_augmented(ik):
    """Oracle S-orthonormal block Davidson for H x = eps S x on the medium
    workload with overlap augmentation (synth.with_augmentation), k-point ik,
    all 256 bands, to |H x - theta S x| < 5e-9 Ha."""
    from oracle import davidson as odv
    c = synth.with_augmentation(synth.make_cell(2))
    po = ham.problem_from_cell(c, ik)
    r = odv.davidson_generalized(po, synth.psi_start(c.seed, c.nbands, po.npw, ik), c.nbands, 5e-9)
    assert r["converged"], "oracle generalized Davidson did not converge"
    fname = f"config2aug_k{ik}_davidson256_Ha.txt"
    with open(os.path.join(HERE, fname), "w") as f:
        f.write(f"# {c.name} k-point {ik}: npw {po.npw}, grid {c.nr[0]}^3, {c.nbands} bands, overlap "
                f"augmentation; oracle S-orthonormal block Davidson to |Hx - theta Sx| < 5e-9 Ha "
                f"({r['iterations']} iterations); columns: theta (Ha), residual 2-norm (Ha); "
                f"written by make_golden.py (oracle only)\n")
        for t, rho in zip(r["theta"], r["rho"]):
            f.write(f"{t:.17e} {rho:.3e}\n")


# SCF workload on the config-1 cell: 12 electrons in 16 bands per k-point,
# Fermi width 0.02 Ha, linear mixing 0.5, converged to int |n_out - n_in| /
# N_el < 1e-11 (the GPU tests stop at 1e-9)
SCF_PARAMS = dict(nel=12.0, nbands=16, sigma=0.02, alpha=0.5)
SCF_KPOINTS = {"gamma": ([[0.0, 0.0, 0.0]], [1.0], {}),
               "2k": ([[0.0, 0.0, 0.0], [0.25, 0.1, -0.3]], [0.5, 0.5], {}),
               "gamma_kerker": ([[0.0, 0.0, 0.0]], [1.0], dict(alpha=0.8, q0=1.0))}


def scf_config1(tag):
    """Oracle SCF loop (dense diagonalisation per step) on the config-1 cell
    at the k-points of SCF_KPOINTS[tag]: mu, energies, eigenvalues and the
    converged input density at 256 seeded grid points, and the density
    distance of every step."""
    from oracle import scf as osc
    c = synth.make_cell(1)
    kpts, kw, extra = SCF_KPOINTS[tag]
    c.kpts = np.asarray(kpts, dtype=np.float64)
    probs = [ham.problem_from_cell(c, ik) for ik in range(len(kpts))]
    vion = synth.vloc_on_grid(c)
    r = osc.scf(probs, kw, vion, tol=1e-11, max_iter=200, **dict(SCF_PARAMS, **extra))
    assert r["converged"], "oracle SCF did not converge"
    rng = np.random.default_rng(314)
    pts = rng.integers(0, c.nr[0], size=(256, 3))
    e = r["energies"]
    with open(os.path.join(HERE, f"config1_scf_{tag}.txt"), "w") as f:
        f.write(f"# {c.name} SCF, k-points {kpts} weights {kw}, {dict(SCF_PARAMS, **extra)}; oracle loop converged to "
                f"int|n_out - n_in|/N_el = {r['history'][-1]:.2e} in {len(r['history']) + 1} steps; "
                f"written by make_golden.py (oracle only)\n")
        f.write(f"mu {r['mu']:.17e}\n")
        for key in ("band", "hartree", "xc", "vxc_n", "total", "free"):
            f.write(f"energy {key} {float(e[key]):.17e}\n")
        for ik, w in enumerate(r["eigenvalues"]):
            f.write(f"eig {ik} " + " ".join(f"{x:.17e}" for x in w) + "\n")
        f.write("hist " + " ".join(f"{x:.17e}" for x in r["history"]) + "\n")
        for p_ in pts:
            f.write(f"n {p_[0]} {p_[1]} {p_[2]} {r['n_in'][tuple(p_)]:.17e}\n")


HYBRID_PARAMS = dict(exx_alpha=0.25, exx_tol=1e-10)


def scf_config1_hybrid():
    """Oracle double loop of a hybrid functional (ACE, exx_alpha 0.25) on the
    config-1 cell at Gamma, with SCF_PARAMS: mu, energies (with e_xx),
    eigenvalues, the e_xx of every outer step and the converged input density
    at 256 seeded grid points."""
    from oracle import exx as oex
    c = synth.make_cell(1)
    p = ham.problem_from_cell(c, 0)
    assert not np.any(p.kfrac)
    vion = synth.vloc_on_grid(c)
    r = oex.scf_hybrid(p, vion, tol=1e-11, max_iter=200, max_outer=60, **SCF_PARAMS, **HYBRID_PARAMS)
    assert r["converged"], "oracle hybrid SCF did not converge"
    rng = np.random.default_rng(314)
    pts = rng.integers(0, c.nr[0], size=(256, 3))
    e = r["energies"]
    with open(os.path.join(HERE, "config1_scf_gamma_hybrid.txt"), "w") as f:
        f.write(f"# {c.name} hybrid SCF at Gamma, {dict(SCF_PARAMS, **HYBRID_PARAMS)}; oracle double loop, inner "
                f"loops to int|n_out - n_in|/N_el < 1e-11, {len(r['exx_history'])} ACE builds, "
                f"{len(r['history'])} inner steps; written by make_golden.py (oracle only)\n")
        f.write(f"mu {r['mu']:.17e}\n")
        for key in ("band", "hartree", "xc", "vxc_n", "exx", "total", "free"):
            f.write(f"energy {key} {float(e[key]):.17e}\n")
        f.write("eig 0 " + " ".join(f"{x:.17e}" for x in r["eigenvalues"]) + "\n")
        f.write("exx_hist " + " ".join(f"{x:.17e}" for x in r["exx_history"]) + "\n")
        for p_ in pts:
            f.write(f"n {p_[0]} {p_[1]} {p_[2]} {r['n_in'][tuple(p_)]:.17e}\n")


def main():
    if "--scf" in sys.argv:
        for tag in SCF_KPOINTS:
            scf_config1(tag)
        scf_config1_hybrid()
        return
    if "--hybrid" in sys.argv:
        scf_config1_hybrid()
        return
    if "--augmented" in sys.argv:
        davidson_config2_augmented(0)
        return
    if "--config4" in sys.argv:
        for index in (10, 19):
            davidson_config4(index)
        return
    if "--quick" not in sys.argv:
        for ik in (0, 1):
            davidson_config2(ik)
        for index in (10, 19):
            davidson_config4(index)
        davidson_config2_augmented(0)
        for tag in SCF_KPOINTS:
            scf_config1(tag)
        scf_config1_hybrid()
    for cfg, nlow, fname in ((0, 8, "tiny_cell_lowest8_Ha.txt"), (1, 16, "config1_lowest16_Ha.txt")):
        c, po, w = eig_fixture(cfg, nlow)
        with open(os.path.join(HERE, fname), "w") as f:
            f.write(f"# {c.name}: lowest {nlow} eigenvalues (Ha) of the dense FP64 Hamiltonian, npw {po.npw},"
                    f" grid {c.nr[0]}^3; written by make_golden.py (oracle only)\n")
            for v in w:
                f.write(f"{v:.17e}\n")
    with open(os.path.join(HERE, "sphere_sizes.txt"), "w") as f:
        f.write("# cell  k-point  npw: |k+G|^2/2 < ecut (strict, FP64); written by make_golden.py (oracle only)\n")
        for name, ik, n in sphere_rows():
            f.write(f"{name} {ik} {n}\n")


if __name__ == "__main__":
    main()
