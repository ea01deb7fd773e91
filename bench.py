#!/usr/bin/env python3
"""Benchmark: band-H*psi/s of the plane-wave Hamiltonian on one MI355X, and
Davidson time-to-solution of the plain FP64 form against the mixed, batched
and learned forms at equal accuracy.

The headline step applies H to the whole band block of the medium workload:
a cubic cell a = 20 bohr, 30 Ry (npw ~ 22.1-22.2k), 72^3 grid, 64 atoms with
s+p+d projectors (576), 256 bands at Gamma + 4 k-points = 1280 band-H*psi per
step, inputs resident in HBM, launch choices fixed (the autotuner's pick at
this workload) so that the kernel profiles under profiles/ describe exactly
the launches timed here.  Prints one JSON line (N = 1).

The dominant kernel's roofline figures come from HIP events the library
records around each of its launches on the launch stream over the timed
steps; the CPU baseline times the FP64 oracle on a bounded sample of the
same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
GOLDEN = os.path.join(ROOT, "tests", "golden")

PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}       # dense MFMA
# vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz for FP64;
# FP32 counts the packed (two-wide) rate
PEAK_VALU_TFLOPS = {"f64": 78.6, "f32": 157.3}

# launch choices of the headline step per precision form: (plane_group,
# band_chunk, ksplit, plane_kernel); 0 = PW_PLANE_REGISTER
PINNED = {"fp64": (4, 256, 0, 0), "fp32": (2, 256, 0, 0), "bf16": (2, 256, 0, 0)}

# HBM bytes per launch measured with rocprofv3 (FETCH_SIZE x 2.0 + WRITE_SIZE
# x 1.0, factors from a plain device copy); valid only for the kernel source
# and launch choices they were taken with
MEASURED_TRAFFIC = {
    "plane": {"source": "paper_1709_10010_amd/csrc/fft.hip", "sha256_16": "15f0210dfd7ae295",
              "precision": 0, "band_chunk": 256, "plane_group": 4, "plane_kernel": 0,
              "bytes_per_launch": 566932696.2},
}


def note(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def source_hash(rel):
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel, prec, tuning):
    """Counter-measured bytes per launch of `kernel`, or None once the kernel
    source or its launch choices differ from those of the measurement."""
    m = MEASURED_TRAFFIC.get(kernel)
    if m is None or tuning is None or prec != m["precision"] or not m["bytes_per_launch"]:
        return None
    if (tuning.get("band_chunk"), tuning.get("plane_group"), tuning.get("plane_kernel_id")) != \
            (m["band_chunk"], m["plane_group"], m["plane_kernel"]):
        return None
    try:
        return m["bytes_per_launch"] if source_hash(m["source"]) == m["sha256_16"] else None
    except OSError:
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16"], default="fp64")
    ap.add_argument("--kpoints", type=int, default=5)
    ap.add_argument("--autotune", action="store_true", help="search the launch choices instead of the pinned ones")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-davidson", action="store_true")
    ap.add_argument("--davidson-reps", type=int, default=3)
    ap.add_argument("--no-davidson-medium", action="store_true")
    ap.add_argument("--davidson-medium-kpoints", type=int, default=5)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-cells", type=int, default=64)
    ap.add_argument("--streams", type=int, default=4, help="streams of the batched forms")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-cells", type=int, default=10)
    ap.add_argument("--no-lanczos", action="store_true")
    ap.add_argument("--lanczos-steps", type=int, default=40)
    ap.add_argument("--no-scf", action="store_true")
    ap.add_argument("--no-exx", action="store_true")
    ap.add_argument("--scf-steps", type=int, default=30, help="at most this many SCF steps on the medium workload")
    ap.add_argument("--profile-davidson", action="store_true",
                    help="only run one FP64 Davidson solve of k-point 0 of the medium workload (256 bands, "
                         "1e-8 Ry) after a warm-up solve, for kernel profiles, and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (the reference "
                         "kernel that scales HBM byte counters) and exit")
    return ap.parse_args()


def stage_model(info, nb, prec):
    """Algorithmic work of each H*psi stage for one call (one k-point, nb bands):
    HBM bytes for the memory-bound stages, flops for the arithmetic-bound ones.

    z passes: each band's sphere in (16 B per G) and its z-sticks out (nst * n
    values), and back.  Plane pass (arithmetic intensity ~16 flop/B in FP64,
    above the ridge 78.6e12 / 8e12): per band the FFT lines of a plane pass --
    nx columns inverse and forward along y, n rows inverse and forward along x,
    on each of n planes -- at 5 m log2(m) flops per m-point line, plus the
    V(r) product (2 flops per grid point).  Projector GEMMs: 8 real flops per
    complex multiply-add, the usual complex GEMM count (the FP64 kernels
    execute 6 of them on MFMA, three real products; see mfma_executed)."""
    npw, nst, nproj, n, nx = info["npw"], info["nsticks"], info["nproj"], info["n"], info["nx"]
    s = 16 if prec == 0 else 8
    col = nst * n * s                       # one band's z-sticks
    fft_line = 5.0 * n * np.log2(n)
    return {
        "zfft_inv": ("hbm", nb * (16 * npw + col)),
        "plane": ("alu", nb * (n * (2 * nx + 2 * n) * fft_line + 2.0 * n ** 3)),
        "zfft_fwd": ("hbm", nb * (col + 32 * npw)),
        "proj": ("mfma", 8.0 * npw * nproj * nb),
        "nlupd": ("mfma", 8.0 * npw * nproj * nb),
        "dmat": ("hbm", nb * nproj * 32),
    }


def mfma_executed(prec):
    """MFMA flops executed per counted complex-GEMM flop: 6/8 for the FP64
    kernels in the three-product form (PW_GEMM_3M, on unless 0), else 1."""
    import re
    v = os.environ.get("PW_GEMM_3M", "")
    m = re.match(r"\s*[+-]?\d+", v)          # read as the library reads it (atoi)
    on = True if not v else (int(m.group()) != 0 if m else False)
    return 0.75 if prec == 0 and on else 1.0


def golden(name):
    a = np.loadtxt(os.path.join(GOLDEN, name), comments="#")
    return a if a.ndim == 2 else a[:, None]


def host_info():
    """Host cores this process may use, CPU model, BLAS library and threads."""
    info = {"affinity_cores": len(os.sched_getaffinity(0)), "cpu_model": None, "blas": None}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        info["blas"] = [{"api": d.get("internal_api"), "version": d.get("version"),
                         "threads": d.get("num_threads")} for d in threadpool_info()
                        if d.get("user_api") == "blas"]
    except Exception:
        pass
    return info


def cpu_baseline(cell, ik, budget_s):
    """FP64 oracle H*psi on the host: bands of one k-point for about budget_s
    with the BLAS threads the process has, and again with one thread."""
    from oracle import hamiltonian as ham
    import synth
    from threadpoolctl import threadpool_limits
    hi = host_info()
    po = ham.problem_from_cell(cell, ik)
    psi = synth.psi_start(cell.seed, cell.nbands, po.npw, ik)
    ham.hpsi(po, psi[:2])                      # warm-up

    def run(limit):
        done, chunk = 0, 8
        with threadpool_limits(limits=limit, user_api="blas"):
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < budget_s and done + chunk <= cell.nbands:
                ham.hpsi(po, psi[done:done + chunk])
                done += chunk
            return done, time.perf_counter() - t0

    n_all, t_all = run(hi["affinity_cores"])
    n_one, t_one = run(1)
    blas_threads = max([b["threads"] or 1 for b in hi["blas"] or [{"threads": 1}]])
    return {"value": n_all / t_all, "unit": "band-H*psi/s", "cores": int(min(blas_threads, hi["affinity_cores"])),
            "kind": "oracle",
            "sample": f"{n_all} bands of k-point {ik} of the medium workload (npw={po.npw}, 72^3 grid, "
                      f"576 projectors) in {t_all:.1f} s; numpy FFT (one thread) per band, BLAS for the "
                      f"projector products",
            "one_thread": {"value": n_one / t_one, "sample": f"{n_one} bands in {t_one:.1f} s, BLAS limited to 1 thread"},
            "host": hi}


def fixed_tuning(p, name):
    from paper_1709_10010_amd import _lib
    g, c, k, pk = PINNED[name]
    c = min(c, _lib.pw_problem_tuning(p)["band_chunk"])
    _lib.pw_problem_set_tuning(p, g, c, k, pk)


def davidson_small_section(reps: int):
    """Config-1 cell (npw 949, 24^3, 32 projectors, 16 bands, Gamma):
    time-to-solution of each form and, per band, the eigenvalue error against
    the oracle's dense diagonalisation (tests/golden, written by the oracle)
    and the residual.  Forms: FP64 to 1e-8 Ry; FP32 (complex64 FFTs, FP32
    GEMMs) and BF16 (complex64 FFTs, BF16 GEMMs) alone to 1e-6 Ry, and each
    followed by FP64 iterations to 1e-8 Ry."""
    import torch
    import synth
    from paper_1709_10010_amd import _lib
    from paper_1709_10010_amd.problems import band_block, build_problem

    cell = synth.make_cell(1)
    nb = cell.nbands
    p64, miller = build_problem(cell, 0, precision=_lib.PW_FP64, max_bands=nb)
    p32, _ = build_problem(cell, 0, precision=_lib.PW_MIXED_FP32, max_bands=nb, miller=miller)
    p16, _ = build_problem(cell, 0, precision=_lib.PW_MIXED_BF16, max_bands=nb, miller=miller)
    npw = p64.npw
    x0 = band_block(nb, npw)
    x0[:, :npw] = torch.from_numpy(synth.psi_start(cell.seed, nb, npw)).cuda()
    exact = golden("config1_lowest16_Ha.txt")[:, 0]
    out = {"workload": "a=10 bohr, 15 Ry, npw 949, 24^3, 8 atoms s+p (32 proj), 16 bands, Gamma; residual "
                       "2-norm of every band; errors against the oracle's dense eigenvalues"}
    forms = {"fp64_1e-8Ry": dict(prob=p64, tol=5e-9),
             "fp32_1e-6Ry": dict(prob=p32, tol=5e-7),
             "bf16_1e-6Ry": dict(prob=p16, tol=5e-7),
             "fp32_then_fp64_1e-8Ry": dict(prob=p32, tol=1e-5, refine=p64, refine_tol=5e-9),
             "bf16_then_fp64_1e-8Ry": dict(prob=p16, tol=1e-3, refine=p64, refine_tol=5e-9)}
    for name, kw in forms.items():
        best = None
        for _ in range(reps + 1):          # the first run warms up the kernels
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = _lib.davidson_solve(kw["prob"], x0, tol=kw["tol"], refine=kw.get("refine"),
                                    refine_tol=kw.get("refine_tol"), max_iter=300)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if best is None or dt < best[0]:
                best = (dt, r)
        dt, r = best
        err = np.abs(r["theta"] - exact)
        o = {"seconds": round(dt, 5), "iterations": r["iterations"], "n_hpsi": r["n_hpsi"],
             "converged": bool(r["converged"]), "max_residual_Ry": float(2 * r["rho"].max()),
             "max_abs_theta_minus_oracle_Ry": float(2 * err.max()),
             "per_band_abs_theta_minus_oracle_Ry": [float(f"{2 * e:.3e}") for e in err],
             "per_band_residual_Ry": [float(f"{2 * e:.3e}") for e in r["rho"]]}
        if "iterations_first" in r:
            o["iterations_reduced_precision"] = r["iterations_first"]
        out[name] = o
    out["speedup_fp32_then_fp64_over_fp64_at_1e-8Ry"] = round(
        out["fp64_1e-8Ry"]["seconds"] / out["fp32_then_fp64_1e-8Ry"]["seconds"], 3)
    for p in (p64, p32, p16):
        p.close()
    return out


def davidson_medium_section(nk: int):
    """Config-2 time-to-solution, every k-point in turn (256 bands each): plain
    FP64 to 1e-8 Ry; the FP32 form to 1e-6 Ry alone; the FP32 form to 1e-5 Ha
    followed by FP64 iterations to 1e-8 Ry from the same subspace.  k-points 0
    and 1 are compared band by band with the oracle's own Davidson at full
    size (tests/golden).  Then one profiled FP64 solve of k-point 0: time per
    stage (library HIP events), eigensolver share, ms per iteration."""
    import torch
    import synth
    from paper_1709_10010_amd import _lib
    from paper_1709_10010_amd.problems import band_block, build_problem

    cell = synth.make_cell(2)
    nb = cell.nbands
    nk = max(1, min(nk, len(cell.kpts)))
    out = {"workload": f"a=20 bohr, 30 Ry, 72^3, 64 atoms s+p+d (576 proj), {nb} bands, {nk} k-points "
                       f"solved one after another; residual 2-norm of every band"}
    forms = {"fp64_1e-8Ry": dict(tol=5e-9), "fp32_1e-6Ry": dict(tol=5e-7, mixed=True),
             "fp32_then_fp64_1e-8Ry": dict(tol=1e-5, mixed=True, refine=True)}
    res = {k: {"seconds": 0.0, "iterations": 0, "n_hpsi": 0, "converged": True, "max_residual_Ry": 0.0,
               "theta": []} for k in forms}
    gold = {ik: golden(f"config2_k{ik}_davidson256_Ha.txt") for ik in (0, 1)}
    stage = None
    for ik in range(nk):
        p64, miller = build_problem(cell, ik, precision=_lib.PW_FP64, max_bands=nb)
        p32, _ = build_problem(cell, ik, precision=_lib.PW_MIXED_FP32, max_bands=nb, miller=miller)
        fixed_tuning(p64, "fp64")
        fixed_tuning(p32, "fp32")
        npw = p64.npw
        x0 = band_block(nb, npw)
        x0[:, :npw] = torch.from_numpy(synth.psi_start(cell.seed, nb, npw, ik)).cuda()
        for name, kw in forms.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = _lib.davidson_solve(p32 if kw.get("mixed") else p64, x0, tol=kw["tol"],
                                    refine=p64 if kw.get("refine") else None, refine_tol=5e-9)
            torch.cuda.synchronize()
            o = res[name]
            o["seconds"] += time.perf_counter() - t0
            o["iterations"] += r["iterations"]
            o["n_hpsi"] += r["n_hpsi"]
            o["converged"] &= bool(r["converged"])
            o["max_residual_Ry"] = max(o["max_residual_Ry"], float(2 * r["rho"].max()))
            o["theta"].append(r["theta"])
            if ik in gold:
                d = np.abs(r["theta"] - gold[ik][:, 0])
                o.setdefault("max_abs_theta_minus_oracle_Ry", {})[f"k{ik}"] = float(2 * d.max())
        if ik == 0:
            _lib.pw_profile_enable(p64, True)
            _lib.pw_profile_read(p64, reset=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = _lib.davidson_solve(p64, x0, tol=5e-9)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            st = _lib.pw_profile_read(p64, reset=True)
            _lib.pw_profile_enable(p64, False)
            tot = sum(v[0] for v in st.values())
            stage = {"kpoint": 0, "iterations": r["iterations"], "wall_s_profiled": round(wall, 4),
                     "ms_per_iteration": round(wall * 1e3 / r["iterations"], 3),
                     "gpu_busy_fraction": round(tot * 1e-3 / wall, 3),
                     "stages_ms": {k: round(v[0], 2) for k, v in sorted(st.items(), key=lambda kv: -kv[1][0])},
                     "eigensolver_share": round(st.get("eig", (0, 0))[0] / max(tot, 1e-9), 3),
                     "hpsi_share": round(sum(st.get(k, (0, 0))[0] for k in ("zfft_inv", "plane", "zfft_fwd",
                                                                            "proj", "dmat", "nlupd")) / max(tot, 1e-9), 3),
                     "subspace_gemm_share": round((st.get("subgemm", (0, 0))[0] + st.get("updgemm", (0, 0))[0])
                                                  / max(tot, 1e-9), 3)}
        p64.close()
        p32.close()
    ref = np.concatenate(res["fp64_1e-8Ry"]["theta"])
    for name, o in res.items():
        th = np.concatenate(o.pop("theta"))
        o["seconds"] = round(o["seconds"], 3)
        o["max_abs_theta_minus_fp64_Ry"] = float(2.0 * np.abs(th - ref).max())
        out[name] = o
    base = res["fp64_1e-8Ry"]["seconds"]
    out["speedup_fp32_then_fp64_over_fp64_at_1e-8Ry"] = round(base / res["fp32_then_fp64_1e-8Ry"]["seconds"], 3)
    out["speedup_fp32_over_fp64_1e-6Ry_vs_1e-8Ry"] = round(base / res["fp32_1e-6Ry"]["seconds"], 3)
    out["fp64_stage_breakdown"] = stage
    # the k-points are independent problems: solved side by side, one stream each
    p64s, p32s, xs = [], [], []
    for ik in range(nk):
        p64, miller = build_problem(cell, ik, precision=_lib.PW_FP64, max_bands=nb)
        p32, _ = build_problem(cell, ik, precision=_lib.PW_MIXED_FP32, max_bands=nb, miller=miller)
        fixed_tuning(p64, "fp64")
        fixed_tuning(p32, "fp32")
        x0 = band_block(nb, p64.npw)
        x0[:, :p64.npw] = torch.from_numpy(synth.psi_start(cell.seed, nb, p64.npw, ik)).cuda()
        p64s.append(p64)
        p32s.append(p32)
        xs.append(x0)
    kforms = {"fp64_kpoints_batched_1e-8Ry": dict(probs=p64s, tol=5e-9),
              "fp32_then_fp64_kpoints_batched_1e-8Ry": dict(probs=p32s, tol=1e-5, refine=p64s, refine_tol=5e-9),
              "fp32_kpoints_batched_1e-6Ry": dict(probs=p32s, tol=5e-7)}
    for name, kw in kforms.items():
        # best of two runs: the first can carry the allocator's growth by the
        # solves' workspaces (5.4 GB for the five states)
        best = None
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rs = _lib.batch_davidson_solve(kw["probs"], xs, tol=kw["tol"], nstreams=nk, refine=kw.get("refine"),
                                           refine_tol=kw.get("refine_tol"))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        o = {"seconds": round(best, 3), "runs": 2, "streams": nk,
             "converged": all(r["converged"] for r in rs),
             "iterations": int(sum(r["iterations"] for r in rs)),
             "max_residual_Ry": float(2 * max(r["rho"].max() for r in rs)),
             "max_abs_theta_minus_fp64_Ry": float(2 * np.abs(np.concatenate([r["theta"] for r in rs]) - ref).max()),
             "max_abs_theta_minus_oracle_Ry": {f"k{ik}": float(2 * np.abs(rs[ik]["theta"] - gold[ik][:, 0]).max())
                                               for ik in gold if ik < nk}}
        o["speedup_over_fp64_one_after_another_1e-8Ry"] = round(base / o["seconds"], 3)
        out[name] = o
    for p in p64s + p32s:
        p.close()
    return out


def batched_section(ncells: int, steps: int, nstreams: int, learned_net=None):
    """The 64 ragged cells (a 10-18 bohr, 20-40 Ry, 8-48 atoms s+p, 32-192
    bands).  H*psi sweep: in order on one stream, over side streams, and the
    side-stream sweep captured in one HIP graph.  Davidson time-to-solution
    of the whole batch: plain FP64 one cell after another (the baseline)
    against the batched forms side by side on the streams: FP64 to 1e-8 Ry,
    FP32 then FP64 to 1e-8 Ry, FP32 alone to 1e-6 Ry, and the FP32 form with
    the learned preconditioner to 1e-6 Ry."""
    import torch
    import synth
    from paper_1709_10010_amd import _lib
    from paper_1709_10010_amd.problems import band_block, build_problem

    cells = [synth.make_cell(4, i) for i in range(ncells)]
    p64s, p32s, xs, nbs = [], [], [], []
    for c in cells:
        p, miller = build_problem(c, 0, max_bands=c.nbands)
        q, _ = build_problem(c, 0, precision=_lib.PW_MIXED_FP32, max_bands=c.nbands, miller=miller)
        x = band_block(c.nbands, p.npw)
        x[:, :p.npw] = torch.from_numpy(synth.psi_start(c.seed, c.nbands, p.npw)).cuda()
        p64s.append(p)
        p32s.append(q)
        xs.append(x)
        nbs.append(c.nbands)
    kinds = {}
    for p, q, nb in zip(p64s, p32s, nbs):              # launch choices, outside the timed regions
        _lib.pw_problem_autotune(p, nb, reps=2)
        _lib.pw_problem_autotune(q, nb, reps=2)
        k = _lib.pw_problem_tuning(p)["plane_kernel"]
        kinds[k] = kinds.get(k, 0) + 1
    ys = [torch.zeros_like(x) for x in xs]
    b = _lib.Batch(p64s, xs, ys)
    s = torch.cuda.Stream()
    out = {"cells": ncells, "bands": int(sum(nbs)), "npw_range": [min(p.npw for p in p64s), max(p.npw for p in p64s)],
           "streams": nstreams,
           "plane_kernels": {("register", "wave", "lds")[k]: v for k, v in kinds.items()}}

    def timed(fn):
        with torch.cuda.stream(s):
            fn()
            s.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                fn()
            s.synchronize()
            return (time.perf_counter() - t0) / steps

    te = timed(lambda: _lib.pw_batch_hpsi(b, s))
    _lib.pw_batch_set_streams(b, [torch.cuda.Stream() for _ in range(nstreams)])
    ts = timed(lambda: _lib.pw_batch_hpsi(b, s))
    with torch.cuda.stream(s):
        _lib.pw_batch_capture(b, s)
    tg = timed(lambda: _lib.pw_batch_launch(b, s))
    b.close()
    nbt = sum(nbs)
    out["hpsi_sweep"] = {"in_order_eager": {"ms": round(te * 1e3, 3), "band-H*psi/s": round(nbt / te, 1)},
                         "side_streams_eager": {"ms": round(ts * 1e3, 3), "band-H*psi/s": round(nbt / ts, 1)},
                         "side_streams_graph": {"ms": round(tg * 1e3, 3), "band-H*psi/s": round(nbt / tg, 1),
                                                "launches_per_sweep": 1}}

    def summarise(rs, dt):
        return {"seconds": round(dt, 3), "converged": all(r["converged"] for r in rs),
                "iterations_total": int(sum(r["iterations"] for r in rs)),
                "max_residual_Ry": float(2 * max(r["rho"].max() for r in rs))}

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [_lib.davidson_solve(p, x, tol=5e-9) for p, x in zip(p64s, xs)]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    dav = {"fp64_one_after_another_1e-8Ry": summarise(seq, t_seq)}
    ref = [r["theta"] for r in seq]
    forms = {"fp64_batched_1e-8Ry": dict(probs=p64s, tol=5e-9),
             "fp32_then_fp64_batched_1e-8Ry": dict(probs=p32s, tol=1e-5, refine=p64s, refine_tol=5e-9),
             "fp32_batched_1e-6Ry": dict(probs=p32s, tol=5e-7)}
    if learned_net is not None:
        forms["fp32_batched_learned_1e-6Ry"] = dict(probs=p32s, tol=5e-7, precond=_lib.PW_PRECOND_MLP,
                                                     net=learned_net)
    for name, kw in forms.items():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = _lib.batch_davidson_solve(kw["probs"], xs, tol=kw["tol"], nstreams=nstreams,
                                       refine=kw.get("refine"), refine_tol=kw.get("refine_tol"),
                                       precond=kw.get("precond", _lib.PW_PRECOND_TPA), net=kw.get("net"),
                                       max_iter=300)
        torch.cuda.synchronize()
        o = summarise(rs, time.perf_counter() - t0)
        o["max_abs_theta_minus_fp64_Ry"] = float(2 * max(np.abs(r["theta"] - t).max() for r, t in zip(rs, ref)))
        o["speedup_over_fp64_one_after_another"] = round(t_seq / o["seconds"], 3)
        dav[name] = o
    out["davidson_time_to_solution"] = dav
    for p in p64s + p32s:
        p.close()
    return out


def learned_section(ncells: int):
    """TPA against the trained network (FP32 form, 1e-6 Ry): cells of the
    training family that took no part in training or in the choice of the
    kept weights (indices 201 ..), and the 512-band evaluation cell."""
    from paper_1709_10010_amd import learned
    import synth
    path = os.path.join(ROOT, "paper_1709_10010_amd", "weights", "precond_mlp.npz")
    if not os.path.exists(path):
        return {"note": "no trained weights in the tree"}
    net = learned.load(path)
    out = {"tol_Ry": 1e-6, "form": "fp32 mixed"}
    its, secs = {"tpa": [], "mlp": []}, {"tpa": [], "mlp": []}
    dth = 0.0
    for i in range(201, 201 + ncells):
        c = synth.make_cell(5, i)
        c.nbands = min(c.nbands, 256)
        r = learned.evaluate(c, net, tol=5e-7)
        for k in ("tpa", "mlp"):
            its[k].append(r[k]["iterations"])
            secs[k].append(r[k]["seconds"])
        dth = max(dth, r["max_theta_diff_Ha"])
    out["held_out_cells"] = {"cells": f"training family, indices 201..{200 + ncells} (never trained on or "
                                      f"used to pick the weights), at most 256 bands",
                             "mean_iterations": {k: round(float(np.mean(v)), 2) for k, v in its.items()},
                             "mean_seconds": {k: round(float(np.mean(v)), 4) for k, v in secs.items()},
                             "mlp_time_over_tpa": round(float(np.sum(secs["mlp"]) / np.sum(secs["tpa"])), 3),
                             "max_theta_diff_Ry": float(2 * dth)}
    cell = synth.make_cell(5, -1)
    r = learned.evaluate(cell, net, tol=5e-7)
    o = {"cell": f"{cell.name}: a={cell.A[0, 0]:.2f} bohr, {int(round(2 * cell.ecut_ha))} Ry, "
                 f"{cell.natom} atoms, {cell.nbands} bands, grid {cell.nr[0]}^3",
         "max_theta_diff_Ry": float(2 * r["max_theta_diff_Ha"])}
    for k in ("tpa", "mlp"):
        o[k] = {"iterations": r[k]["iterations"], "seconds": round(r[k]["seconds"], 4),
                "n_hpsi": r[k]["n_hpsi"], "converged": bool(r[k]["converged"])}
    o["mlp_time_over_tpa"] = round(r["mlp"]["seconds"] / r["tpa"]["seconds"], 3)
    out["evaluation_cell"] = o
    return out, net


def lanczos_section(steps: int):
    """Lanczos recursion on H (a second H*psi workload): 256 chains in
    lockstep on k-point 0 of the medium workload, `steps` steps after a
    warm-up.  Rate in chain-steps/s; the recursion kernel's HBM rate counts
    4 vectors of 16 npw bytes per chain-step (q_n, H q_n and q_{n-1} read,
    q_{n+1} written)."""
    import torch
    import synth
    from paper_1709_10010_amd import _lib
    from paper_1709_10010_amd.problems import band_block, build_problem
    cell = synth.make_cell(2)
    nch = cell.nbands
    p, _ = build_problem(cell, 0, max_bands=nch)
    fixed_tuning(p, "fp64")
    v = band_block(nch, p.npw)
    v[:, :p.npw] = torch.from_numpy(synth.psi_start(cell.seed, nch, p.npw, 0)).cuda()
    lz = _lib.Lanczos(p, nch, steps + 4)
    lz.start(v)
    lz.run(4)
    _lib.pw_profile_enable(p, True)
    _lib.pw_profile_read(p, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lz.run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = _lib.pw_profile_read(p, reset=True)
    _lib.pw_profile_enable(p, False)
    z = torch.tensor([0.1 + 0.05j, 0.5 + 0.05j], dtype=torch.complex128, device="cuda")
    g = lz.resolvent(z)
    torch.cuda.synchronize()
    vec_ms, vec_n = st.get("vec", (0.0, 1))
    out = {"workload": f"{nch} chains, k-point 0 of the medium workload (npw {p.npw}, 72^3, 576 projectors), "
                       f"{steps} steps",
           "chain_steps_per_s": round(nch * steps / dt, 1), "ms_per_step": round(dt * 1e3 / steps, 4),
           "recursion_kernel": {"avg_ms": round(vec_ms / max(vec_n, 1), 4),
                                "GB/s": round(4 * 16 * p.npw * nch / (vec_ms / max(vec_n, 1) * 1e-3) / 1e9, 1)},
           "share_of_step": {k: round(v[0] / max(sum(x[0] for x in st.values()), 1e-9), 3) for k, v in st.items()},
           "resolvent_finite": bool(torch.isfinite(torch.view_as_real(g)).all())}
    lz.close()
    p.close()
    return out


def _scf_golden(tag):
    out = {"energy": {}, "eig": {}, "n": []}
    with open(os.path.join(GOLDEN, f"config1_scf_{tag}.txt")) as f:
        for line in f:
            w = line.split()
            if not w or w[0].startswith("#"):
                continue
            if w[0] == "mu":
                out["mu"] = float(w[1])
            elif w[0] == "energy":
                out["energy"][w[1]] = float(w[2])
            elif w[0] == "eig":
                out["eig"][int(w[1])] = np.array([float(x) for x in w[2:]])
            elif w[0] == "exx_hist":
                out["exx_hist"] = [float(x) for x in w[1:]]
            elif w[0] == "n":
                out["n"].append((int(w[1]), int(w[2]), int(w[3]), float(w[4])))
    return out


def scf_section(steps: int, nstreams: int):
    """SCF loop around the solver.  Config-1 cell (12 electrons in 16 bands,
    Fermi width 0.02 Ha, linear mixing 0.5) at Gamma and at two k-points, to
    int |n_out - n_in| / N_el < 1e-9: time to convergence and errors against
    the oracle's converged loop (tests/golden).  Medium workload (5 k-points,
    256 bands, 320 electrons, width 0.02 Ha, Kerker mixing alpha 0.8, q0 1
    bohr^-1), the k-point solves side by side on streams, each step's
    Davidson target 1e-2 of the last density distance (between 5e-9 and
    1e-4 Ha): time to int |n_out - n_in| / N_el < 1e-6 (at most `steps`
    steps), seconds per step and the density distance, plus the density (256
    bands of one k-point) and Hartree/exchange kernels timed alone.  The
    hybrid double loop (ACE, exx_alpha 0.25) on the config-1 cell at Gamma:
    time to convergence and errors against the oracle's loop (tests/golden)."""
    import torch
    import synth
    from paper_1709_10010_amd import _lib
    from paper_1709_10010_amd.problems import band_block, build_problem
    out = {}
    kp = {"gamma": ([[0.0, 0.0, 0.0]], [1.0]), "2k": ([[0.0, 0.0, 0.0], [0.25, 0.1, -0.3]], [0.5, 0.5])}
    for tag, (kpts, kw) in kp.items():
        g = _scf_golden(tag)
        c = synth.make_cell(1)
        c.kpts = np.asarray(kpts)
        probs, davs = [], []
        for ik in range(len(kpts)):
            p, _ = build_problem(c, ik, max_bands=16)
            d = _lib.Davidson(p, 16, 0, 1e-10)
            x0 = band_block(16, p.npw)
            x0[:, :p.npw] = torch.from_numpy(synth.psi_start(c.seed, 16, p.npw, ik)).cuda()
            _lib.pw_davidson_init(d, x0)
            probs.append(p)
            davs.append(d)
        vion = torch.from_numpy(synth.vloc_on_grid(c)).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = _lib.Scf(probs, davs, kw, vion, 12.0, 0.02, 0.5)
        hist = []
        for _ in range(150):
            r = s.step(1e-10, 200, 1e-9)
            hist.append(r["drho"])
            if r["converged"]:
                break
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        n_in, _ = s.density()
        n = n_in.cpu().numpy()
        eig = max(float(np.abs(_lib.pw_davidson_query(d)["theta"] - g["eig"][ik]).max()) for ik, d in enumerate(davs))
        out[f"config1_{tag}"] = {
            "seconds": round(dt, 4), "steps": len(hist), "converged": r["converged"],
            "abs_mu_minus_oracle_Ha": abs(r["mu"] - g["mu"]),
            "abs_free_energy_minus_oracle_Ha": abs(r["free_energy"] - g["energy"]["free"]),
            "max_abs_eig_minus_oracle_Ha": eig,
            "max_density_sample_err_rel": max(abs(n[i, j, k] - v) for i, j, k, v in g["n"]) /
            max(v for *_, v in g["n"])}
        s.close()
        for d in davs:
            d.close()
        for p in probs:
            p.close()
    # the hybrid double loop (exx_alpha 0.25) on the config-1 cell at Gamma: through ACE,
    # and with the exchange operator applied directly (what ACE replaces)
    g = _scf_golden("gamma_hybrid")
    c = synth.make_cell(1)
    for key, direct in (("config1_gamma_hybrid", False), ("config1_gamma_hybrid_direct_exchange", True)):
        p, _ = build_problem(c, 0, max_bands=16)
        d = _lib.Davidson(p, 16, 0, 1e-10)
        x0 = band_block(16, p.npw)
        x0[:, :p.npw] = torch.from_numpy(synth.psi_start(c.seed, 16, p.npw, 0)).cuda()
        _lib.pw_davidson_init(d, x0)
        vion = torch.from_numpy(synth.vloc_on_grid(c)).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = _lib.Scf([p], [d], [1.0], vion, 12.0, 0.02, 0.5, exx_alpha=0.25, exx_tol=1e-10, exx_direct=direct)
        nstep = 0
        for nstep in range(1, 1001):
            r = s.step(1e-10, 200, 1e-10)
            if r["converged"]:
                break
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        n = s.density()[0].cpu().numpy()
        th = _lib.pw_davidson_query(d)["theta"]
        # states with an occupation (f/2 > 1e-8 at the oracle's mu): ACE equals V_x on them
        occ = g["eig"][0] < g["mu"] + 0.02 * np.log(1e8)
        out[key] = {
            "workload": "config-1 cell at Gamma, 12 electrons in 16 bands, exx_alpha 0.25 "
                        + ("with V_x applied directly (pair densities per band in every H*psi)" if direct
                           else "through ACE") + ", inner loops to int |n_out - n_in| / N_el < 1e-10, outer loop "
                        "until e_xx changes by < 1e-10 Ha",
            "seconds": round(dt, 4), "steps": nstep, "outer_steps": int(r["outer"]), "converged": r["converged"],
            "abs_mu_minus_oracle_Ha": abs(r["mu"] - g["mu"]),
            "abs_e_xx_minus_oracle_Ha": abs(r["e_xx"] - g["energy"]["exx"]),
            "abs_free_energy_minus_oracle_Ha": abs(r["free_energy"] - g["energy"]["free"]),
            "max_abs_eig_minus_oracle_Ha_occupied": float(np.abs(th - g["eig"][0])[occ].max()),
            "max_density_sample_err_rel": max(abs(n[i, j, k] - v) for i, j, k, v in g["n"]) /
            max(v for *_, v in g["n"])}
        if not direct:
            out[key]["max_abs_eig_minus_oracle_Ha"] = float(np.abs(th - g["eig"][0]).max())
        s.close()
        d.close()
        p.close()
    out["config1_gamma_hybrid_direct_exchange"]["ace_speedup"] = round(
        out["config1_gamma_hybrid_direct_exchange"]["seconds"] / out["config1_gamma_hybrid"]["seconds"], 2)
    # medium workload
    cell = synth.make_cell(2)
    nk, nb = len(cell.kpts), cell.nbands
    probs, davs = [], []
    for ik in range(nk):
        p, _ = build_problem(cell, ik, max_bands=nb)
        fixed_tuning(p, "fp64")
        d = _lib.Davidson(p, nb, 0, 5e-9)
        x0 = band_block(nb, p.npw)
        x0[:, :p.npw] = torch.from_numpy(synth.psi_start(cell.seed, nb, p.npw, ik)).cuda()
        _lib.pw_davidson_init(d, x0)
        probs.append(p)
        davs.append(d)
    streams = [torch.cuda.Stream() for _ in range(max(1, min(nstreams, nk)))]
    torch.cuda.synchronize()
    batch = _lib.BatchDavidson(davs, streams)
    vion = torch.from_numpy(synth.vloc_on_grid(cell)).cuda()
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    s = _lib.Scf(probs, davs, [1.0 / nk] * nk, vion, 320.0, 0.02, 0.8, batch=batch, kerker_q0=1.0)
    per_step, hist, dtol = [], [], 1e-4
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.step(dtol, 60, 1e-6)
        torch.cuda.synchronize()
        per_step.append(round(time.perf_counter() - t0, 4))
        hist.append(r["drho"])
        if r["converged"]:
            break
        if r["drho"] > 0:
            dtol = min(1e-4, max(5e-9, 1e-2 * r["drho"]))
    t_all = time.perf_counter() - t_all
    # the grid kernels alone: density of 256 bands of k-point 0, Hartree + exchange
    x = band_block(nb, probs[0].npw)
    _lib.pw_davidson_vectors(davs[0], x)
    n = torch.zeros(tuple(cell.nr), dtype=torch.float64, device="cuda")
    f = np.full(nb, 2.0 / nk)
    _lib.pw_density(probs[0], x, f, n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        _lib.pw_density(probs[0], x, f, n)
    torch.cuda.synchronize()
    t_rho = (time.perf_counter() - t0) / 3
    t0 = time.perf_counter()
    for _ in range(3):
        _lib.pw_hxc(probs[0], n)
    torch.cuda.synchronize()
    t_hxc = (time.perf_counter() - t0) / 3
    out["medium_workload"] = {
        "workload": f"a=20 bohr, 30 Ry, 72^3, 64 atoms, {nb} bands x {nk} k-points, 320 electrons, Fermi width "
                    f"0.02 Ha, Kerker mixing alpha 0.8 q0 1/bohr, k-point solves side by side on {len(streams)} "
                    f"streams, Davidson target 1e-2 of the last density distance (5e-9 .. 1e-4 Ha, at most 60 "
                    f"iterations) per SCF step",
        "seconds_to_1e-6": round(t_all, 3) if r["converged"] else None, "steps": len(hist),
        "converged": r["converged"],
        "seconds_per_step": per_step, "drho_per_step": hist, "mu_Ha": r["mu"], "free_energy_Ha": r["free_energy"],
        "density_256_bands_ms": round(t_rho * 1e3, 3), "hartree_exchange_ms": round(t_hxc * 1e3, 3)}
    s.close()
    batch.close()
    for d in davs:
        d.close()
    for p in probs:
        p.close()
    torch.cuda.empty_cache()
    return out


def exx_section(nocc: int, nphi: int):
    """Exact exchange at the medium workload's Gamma point (npw 22119, 72^3):
    nocc occupied states (the seeded start bands), the Fock operator applied
    directly to nphi bands (nocc pair densities and Poisson solves per band)
    against the ACE term of H*psi on all 256 bands (two GEMMs of a rank-nocc
    projector), and the ACE build itself (V_x on the occupied states, the
    Cholesky factor and the projector)."""
    import torch
    import synth
    from paper_1709_10010_amd import _lib
    from paper_1709_10010_amd.problems import band_block, build_problem
    cell = synth.make_cell(2)
    nb = cell.nbands
    p, _ = build_problem(cell, 0, max_bands=nb)
    fixed_tuning(p, "fp64")
    x = band_block(nb, p.npw)
    x[:, :p.npw] = torch.from_numpy(synth.psi_start(cell.seed, nb, p.npw, 0)).cuda()
    occ = x[:nocc].contiguous()
    w = np.ones(nocc)
    out = band_block(nphi, p.npw)
    _lib.pw_vx(p, occ, w, x[:2].contiguous(), out[:2].contiguous())       # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _lib.pw_vx(p, occ, w, x[:nphi].contiguous(), out)
    torch.cuda.synchronize()
    t_vx = time.perf_counter() - t0
    t0 = time.perf_counter()
    _lib.pw_ace_set(p, occ, w, 1.0)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    y = torch.zeros_like(x)
    for _ in range(2):
        _lib.pw_hpsi(p, x, y)
    _lib.pw_profile_enable(p, True)
    _lib.pw_profile_read(p, reset=True)
    for _ in range(5):
        _lib.pw_hpsi(p, x, y)
    torch.cuda.synchronize()
    st = _lib.pw_profile_read(p, reset=True)
    _lib.pw_profile_enable(p, False)
    ms_exx = st["exx"][0] / st["exx"][1]
    ms_hpsi = sum(v[0] for v in st.values()) / st["exx"][1]
    per_band_direct = t_vx / nphi * 1e3
    per_band_ace = ms_exx / nb
    out_d = {"workload": f"a=20 bohr, 30 Ry, Gamma, npw {p.npw}, 72^3 grid, {nocc} occupied states",
             "vx_direct_ms_per_band": round(per_band_direct, 4), "vx_direct_bands_timed": nphi,
             "pair_transforms_per_s": round(2 * nocc * nphi / t_vx, 1),
             "ace_term_ms_per_band": round(per_band_ace, 5),
             "ace_term_ms_256_bands": round(ms_exx, 4), "hpsi_with_ace_ms_256_bands": round(ms_hpsi, 4),
             "ace_apply_speedup_per_band": round(per_band_direct / per_band_ace, 1),
             "ace_build_s": round(t_build, 4)}
    _lib.pw_ace_clear(p)
    p.close()
    torch.cuda.empty_cache()
    return out_d


def davidson_cpu_baseline(dav):
    """Oracle FP64 Davidson on the config-1 cell (host cores)."""
    from oracle import davidson as odv
    from oracle import hamiltonian as ham
    import synth
    cell = synth.make_cell(1)
    po = ham.problem_from_cell(cell)
    t0 = time.perf_counter()
    r = odv.davidson(po, synth.psi_start(cell.seed, cell.nbands, po.npw), cell.nbands, 5e-9)
    dt = time.perf_counter() - t0
    dav["cpu_oracle_fp64_1e-8Ry"] = {"seconds": round(dt, 4), "iterations": r["iterations"], "kind": "oracle",
                                     "speedup_gpu_fp64": round(dt / dav["fp64_1e-8Ry"]["seconds"], 2)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the H*psi and Davidson path runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 8, "bytes_written": n * 8, "dispatches": 5}))
        return
    import synth
    from paper_1709_10010_amd import _lib
    from paper_1709_10010_amd.problems import band_block, build_problem

    if args.profile_davidson:
        cell = synth.make_cell(2)
        p, _ = build_problem(cell, 0, max_bands=cell.nbands)
        fixed_tuning(p, "fp64")
        x0 = band_block(cell.nbands, p.npw)
        x0[:, :p.npw] = torch.from_numpy(synth.psi_start(cell.seed, cell.nbands, p.npw, 0)).cuda()
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = _lib.davidson_solve(p, x0, tol=5e-9)
            torch.cuda.synchronize()
            note(f"Davidson k-point 0 solve {rep}: {time.perf_counter() - t0:.4f} s, {r['iterations']} iterations")
        print(json.dumps({"profile_davidson_seconds": round(time.perf_counter() - t0, 4),
                          "iterations": r["iterations"], "converged": bool(r["converged"])}))
        return

    prec = {"fp64": _lib.PW_FP64, "fp32": _lib.PW_MIXED_FP32, "bf16": _lib.PW_MIXED_BF16}[args.precision]
    cell = synth.make_cell(2)
    nk = max(1, min(args.kpoints, len(cell.kpts)))
    probs, psis, hpsis, infos = [], [], [], []
    for ik in range(nk):
        p, m = build_problem(cell, ik, precision=prec, max_bands=cell.nbands)
        inf = p.info()
        inf["n"] = cell.nr[0]
        inf["nx"] = int(len(np.unique(np.asarray(m)[:, 0] % cell.nr[0])))   # grid x rows holding sticks
        x = band_block(cell.nbands, inf["npw"])
        x[:, :inf["npw"]] = torch.from_numpy(synth.psi_start(cell.seed, cell.nbands, inf["npw"], ik)).cuda()
        probs.append(p)
        psis.append(x)
        hpsis.append(torch.zeros_like(x))
        infos.append(inf)
    for p in probs:
        if args.autotune:
            _lib.pw_problem_autotune(p, cell.nbands, reps=3)
        else:
            fixed_tuning(p, args.precision)
    tuning = _lib.pw_problem_tuning(probs[0])
    tuning["plane_kernel_id"] = tuning["plane_kernel"]
    tuning["plane_kernel"] = ("register", "wave", "lds")[tuning["plane_kernel"]]
    tuning["source"] = "autotuned" if args.autotune else "pinned"
    torch.cuda.synchronize()

    def step():
        for p, x, y in zip(probs, psis, hpsis):
            _lib.pw_hpsi(p, x, y)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nbands_step = nk * cell.nbands
    value = nbands_step * args.steps / dt

    # same steps again with the library's per-launch HIP events enabled
    for p in probs:
        _lib.pw_profile_enable(p, True)
        _lib.pw_profile_read(p, reset=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt_prof = time.perf_counter() - t1
    stages = {}
    for p in probs:
        for k, (ms, n) in _lib.pw_profile_read(p, reset=True).items():
            a = stages.setdefault(k, [0.0, 0])
            a[0] += ms
            a[1] += n
        _lib.pw_profile_enable(p, False)
    models = [stage_model(inf, cell.nbands, prec) for inf in infos]
    gemm_dtype = {0: "f64", 1: "f32", 2: "bf16"}[prec]
    vec_dtype = "f64" if prec == 0 else "f32"

    def rate(k):
        # modelled work of every profiled call / the stage's total time: the
        # algorithmic amount per launch over the average launch duration
        work = args.steps * sum(m[k][1] for m in models)
        return work / (stages[k][0] * 1e-3)

    dom = max(stages, key=lambda k: stages[k][0])
    kind = models[0][dom][0]
    if kind == "hbm":
        achieved = rate(dom) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None}
    else:
        achieved = rate(dom) / 1e12
        peak = PEAK_TFLOPS[gemm_dtype] if kind == "mfma" else PEAK_VALU_TFLOPS[vec_dtype]
        roof = {"bound": kind, "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": None}
    roof["kernel"] = dom
    roof["avg_launch_ms"] = round(stages[dom][0] / stages[dom][1], 4)
    roof["traffic"] = measured_traffic(dom, prec, tuning)     # HBM bytes per launch, counters
    if dom == "plane":
        # the plane pass's own HBM bytes for the bands of one launch: z-sticks
        # in and out, V(r) once
        inf, nbl = infos[0], tuning.get("band_chunk") or cell.nbands
        sz = 16 if prec == 0 else 8
        roof["hbm_bytes_algorithmic_per_launch"] = float(nbl * 2 * inf["nsticks"] * inf["n"] * sz
                                                          + inf["n"] ** 3 * sz // 2)
    stage_out = {}
    for k, (ms, n) in sorted(stages.items(), key=lambda kv: -kv[1][0]):
        kind_k = models[0].get(k, ("-", 0.0))[0]
        ent = {"avg_ms": round(ms / n, 4), "launches": n, "share": round(ms / sum(v[0] for v in stages.values()), 3)}
        if kind_k == "hbm":
            ent["GB/s"] = round(rate(k) / 1e9, 1)
        elif kind_k in ("mfma", "alu"):
            ent["TFLOP/s"] = round(rate(k) / 1e12, 2)
        if kind_k == "mfma":
            ent["mfma_TFLOP/s_executed"] = round(rate(k) * mfma_executed(prec) / 1e12, 2)
        stage_out[k] = ent

    # the three FFT stages together against both roofs: compulsory HBM bytes of
    # the stick/plane scheme (sphere in and out, the stick buffer written and
    # read in each direction, V once) and the nominal 5 m log2 m FFT flops
    fft_pipe = None
    if all(k in stages for k in ("zfft_inv", "plane", "zfft_fwd")):
        sz = 16 if prec == 0 else 8
        t_fft = sum(stages[k][0] for k in ("zfft_inv", "plane", "zfft_fwd")) * 1e-3
        b_fft = f_fft = 0.0
        for inf in infos:
            n = inf["n"]
            b_fft += cell.nbands * (32 * inf["npw"] + 4 * inf["nsticks"] * n * sz) + n ** 3 * sz / 2
            f_fft += cell.nbands * (n * (2 * inf["nx"] + 2 * n) * 5.0 * n * np.log2(n)
                                    + 2 * inf["nsticks"] * 5.0 * n * np.log2(n) + 2.0 * n ** 3)
        b_fft *= args.steps
        f_fft *= args.steps
        vpk = PEAK_VALU_TFLOPS["f64" if prec == 0 else "f32"]
        fft_pipe = {"ms_per_kpoint": round(t_fft / (args.steps * len(infos)) * 1e3, 4),
                    "hbm_GB/s_algorithmic": round(b_fft / t_fft / 1e9, 1),
                    "hbm_frac": round(b_fft / t_fft / 1e9 / PEAK_HBM_GBS, 4),
                    "TFLOP/s": round(f_fft / t_fft / 1e12, 2),
                    "valu_frac": round(f_fft / t_fft / 1e12 / vpk, 4),
                    "flop_per_byte": round(f_fft / b_fft, 2)}

    out = {
        "metric": "band-H*psi/s (plane-wave Hamiltonian applied to a band block)",
        "value": round(value, 1),
        "unit": "band-H*psi/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32 (FFT c64, GEMM fp32)", "bf16": "f32 (FFT c64, GEMM bf16)"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": f"a=20 bohr, 30 Ry, npw~22.1-22.2k, 72^3 grid, 64 atoms s+p+d (576 proj), "
                        f"{cell.nbands} bands x {nk} k-points per step, complex128 in/out",
            "global_batch": nbands_step,
            "precision_form": args.precision,
            "npw": [inf["npw"] for inf in infos],
            "nsticks": [inf["nsticks"] for inf in infos],
            "launch_choices_kpoint0": tuning,
        },
        "roofline": roof,
        "stages": stage_out,
        "fft_pipeline": fft_pipe,
        "ms_per_step_profiled": round(dt_prof / args.steps * 1e3, 4),
    }
    for p in probs:
        p.close()
    del psis, hpsis
    torch.cuda.empty_cache()
    note(f"H*psi step: {value:.1f} band-H*psi/s, dominant kernel {dom} at {roof['frac']} of its roof")
    net = None
    if not args.no_learned:
        lr = learned_section(args.learned_cells)
        if isinstance(lr, tuple):
            out["learned_preconditioner"], net = lr
        else:
            out["learned_preconditioner"] = lr
        note("learned preconditioner section done")
    if not args.no_lanczos:
        out["lanczos_recursion"] = lanczos_section(args.lanczos_steps)
        note("Lanczos section done")
    if not args.no_scf:
        out["scf"] = scf_section(args.scf_steps, args.streams + 1)
        note("SCF section done")
    if not args.no_exx:
        out["exact_exchange"] = exx_section(128, 16)
        note("exact-exchange section done")
    if not args.no_batched:
        out["batched_ragged_cells"] = batched_section(args.batched_cells, max(3, args.steps // 2), args.streams,
                                                      learned_net=net)
        note("batched section done")
    dav = None
    if not args.no_davidson:
        dav = davidson_small_section(args.davidson_reps)
        note("config-1 Davidson section done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cell, 0, args.cpu_seconds)
        if dav is not None:
            davidson_cpu_baseline(dav)
        note("CPU baseline done")
    if dav is not None:
        out["davidson_time_to_1e-8Ry"] = dav
        if not args.no_davidson_medium:
            out["davidson_medium_time_to_solution"] = davidson_medium_section(args.davidson_medium_kpoints)
            note("medium Davidson section done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
