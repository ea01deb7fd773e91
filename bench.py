#!/usr/bin/env python3
"""Benchmark: band-H*psi/s of the plane-wave Hamiltonian on one MI355X.

One step applies H to the whole band block of the medium workload: a cubic
cell a = 20 bohr, 30 Ry (npw ~ 22.1-22.2k), 72^3 grid, 64 atoms with s+p+d
projectors (576), 256 bands at Gamma + 4 k-points = 1280 band-H*psi per
step, inputs resident in HBM.  Prints one JSON line (rank 0, N = 1).

The dominant kernel's roofline figures come from HIP events the library
records around each of its launches on the launch stream over the timed
steps; the CPU baseline times the FP64 oracle on a bounded sample of the
same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--kpoints", type=int, default=5)
    ap.add_argument("--no-davidson", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-cells", type=int, default=64)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--davidson-reps", type=int, default=3)
    return ap.parse_args()


def stage_model(info, nb, prec, group):
    """Algorithmic bytes / flops per launch of each H*psi stage (one k-point, nb bands)."""
    npw, nst, nproj, n = info["npw"], info["nsticks"], info["nproj"], info["n"]
    s = 16 if prec == 0 else 8
    sv = 8 if prec == 0 else 4
    col = nst * n * s                       # one band's z-sticks
    return {
        "zfft_inv": ("hbm", nb * (16 * npw + col)),
        "plane": ("hbm", nb * (2 * col) + n ** 3 * sv * ((nb + group - 1) // group)),
        "zfft_fwd": ("hbm", nb * (col + 32 * npw)),
        "proj": ("mfma", 8.0 * npw * nproj * nb),
        "nlupd": ("mfma", 8.0 * npw * nproj * nb),
        "dmat": ("hbm", nb * nproj * 32),
    }


def cpu_baseline(cell, ik, budget_s):
    """FP64 oracle H*psi on the host: bands of one k-point until ~budget_s of work."""
    from oracle import hamiltonian as ham
    import synth
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        blas_threads = 1
    po = ham.problem_from_cell(cell, ik)
    psi = synth.psi_start(cell.seed, cell.nbands, po.npw, ik)
    ham.hpsi(po, psi[:2])                      # warm-up
    done, t0 = 0, time.perf_counter()
    chunk = 8
    while time.perf_counter() - t0 < budget_s and done + chunk <= cell.nbands:
        ham.hpsi(po, psi[done:done + chunk])
        done += chunk
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "band-H*psi/s", "cores": int(blas_threads),
            "kind": "oracle",
            "sample": f"{done} bands of k-point {ik} (npw={po.npw}, 72^3 grid, 576 projectors), "
                      f"{dt:.1f} s; numpy FFT single-threaded, BLAS threads={blas_threads}"}


def davidson_section(reps: int):
    """Config-1 time-to-solution (first H*psi to all residuals < 1e-8 Ry = 5e-9 Ha)."""
    import torch
    import synth
    from paper_1709_10010_amd import _lib
    from paper_1709_10010_amd.problems import band_block, build_problem

    cell = synth.make_cell(1)
    nb = cell.nbands
    p64, miller = build_problem(cell, 0, precision=_lib.PW_FP64, max_bands=nb)
    p32, _ = build_problem(cell, 0, precision=_lib.PW_MIXED_FP32, max_bands=nb, miller=miller)
    npw = p64.npw
    x0 = band_block(nb, npw)
    x0[:, :npw] = torch.from_numpy(synth.psi_start(cell.seed, nb, npw)).cuda()
    out = {"workload": "a=10 bohr, 15 Ry, npw 949, 24^3, 8 atoms s+p (32 proj), 16 bands, Gamma; "
                       "tol 1e-8 Ry (5e-9 Ha) on every band's residual 2-norm"}
    forms = {"fp64": dict(prob=p64), "fp32_then_fp64": dict(prob=p32, refine=p64, tol=1e-5)}
    for name, kw in forms.items():
        best = None
        for _ in range(reps + 1):          # first run warms up the kernels
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = _lib.davidson_solve(kw["prob"], x0, tol=kw.get("tol", 5e-9), refine=kw.get("refine"),
                                    refine_tol=5e-9)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if best is None or dt < best[0]:
                best = (dt, r)
        dt, r = best
        out[name] = {"seconds": round(dt, 5), "iterations": r["iterations"], "n_hpsi": r["n_hpsi"],
                     "converged": bool(r["converged"]), "max_residual_Ha": float(r["rho"].max())}
        if "iterations_first" in r:
            out[name]["iterations_reduced_precision"] = r["iterations_first"]
        out[name]["_theta"] = r["theta"]
    return out


def batched_section(ncells: int, steps: int):
    """64 ragged cells (a 10-18 bohr, 20-40 Ry, 8-48 atoms, 32-192 bands): one H*psi
    sweep per step, eager launches vs one HIP-graph launch per step."""
    import torch
    import synth
    from paper_1709_10010_amd import _lib
    from paper_1709_10010_amd.problems import band_block, build_problem

    probs, xs, ys, nbs, npws = [], [], [], [], []
    for i in range(ncells):
        c = synth.make_cell(4, i)
        p, _ = build_problem(c, 0, max_bands=c.nbands)
        x = band_block(c.nbands, p.npw)
        x[:, :p.npw] = torch.from_numpy(synth.psi_start(c.seed, c.nbands, p.npw)).cuda()
        probs.append(p)
        xs.append(x)
        ys.append(torch.zeros_like(x))
        nbs.append(c.nbands)
        npws.append(p.npw)
    b = _lib.Batch(probs, xs, ys)
    s = torch.cuda.Stream()
    out = {"cells": ncells, "bands_per_step": int(sum(nbs)), "npw_range": [min(npws), max(npws)]}
    with torch.cuda.stream(s):
        _lib.pw_batch_hpsi(b, s)
        s.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _lib.pw_batch_hpsi(b, s)
        s.synchronize()
        te = (time.perf_counter() - t0) / steps
        _lib.pw_batch_capture(b, s)
        _lib.pw_batch_launch(b, s)
        s.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _lib.pw_batch_launch(b, s)
        s.synchronize()
        tg = (time.perf_counter() - t0) / steps
    out["eager"] = {"ms_per_step": round(te * 1e3, 3), "band-H*psi/s": round(sum(nbs) / te, 1)}
    out["graph"] = {"ms_per_step": round(tg * 1e3, 3), "band-H*psi/s": round(sum(nbs) / tg, 1),
                    "launches_per_step": 1}
    b.close()
    return out


def learned_section():
    """TPA vs trained-MLP Davidson (FP32 form, 1e-6 Ry): a held-out cell of the
    training family and the 512-band evaluation cell."""
    from paper_1709_10010_amd import learned
    import synth
    path = os.path.join(ROOT, "paper_1709_10010_amd", "weights", "precond_mlp.npz")
    if not os.path.exists(path):
        return {"note": "no trained weights in the tree"}
    net = learned.load(path)
    out = {"tol_Ry": 1e-6, "form": "fp32 mixed"}
    val = synth.make_cell(5, 200)
    val.nbands = min(val.nbands, 256)
    for key, cell in (("held_out_training_family", val), ("evaluation_cell", synth.make_cell(5, -1))):
        r = learned.evaluate(cell, net, tol=5e-7)
        o = {"cell": f"{cell.name}: a={cell.A[0, 0]:.2f} bohr, {int(round(2 * cell.ecut_ha))} Ry, "
                     f"{cell.natom} atoms, {cell.nbands} bands, grid {cell.nr[0]}^3",
             "max_theta_diff_Ry": float(2 * r["max_theta_diff_Ha"])}
        for k in ("tpa", "mlp"):
            o[k] = {"iterations": r[k]["iterations"], "seconds": round(r[k]["seconds"], 4),
                    "n_hpsi": r[k]["n_hpsi"], "converged": bool(r[k]["converged"])}
        o["mlp_time_over_tpa"] = round(r["mlp"]["seconds"] / r["tpa"]["seconds"], 3)
        out[key] = o
    net.close()
    return out


def davidson_cpu_baseline(dav):
    """Oracle FP64 Davidson on config 1 (host cores) and eigenvalue agreement with the GPU."""
    from oracle import davidson as odv
    from oracle import hamiltonian as ham
    import synth
    cell = synth.make_cell(1)
    po = ham.problem_from_cell(cell)
    t0 = time.perf_counter()
    r = odv.davidson(po, synth.psi_start(cell.seed, cell.nbands, po.npw), cell.nbands, 5e-9)
    dt = time.perf_counter() - t0
    for k in ("fp64", "fp32_then_fp64"):
        if k in dav:
            dav[k]["max_abs_theta_minus_oracle_Ry"] = float(2.0 * np.abs(dav[k]["_theta"] - r["theta"]).max())
    dav["cpu_oracle"] = {"seconds": round(dt, 4), "iterations": r["iterations"], "kind": "oracle"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import synth
    from paper_1709_10010_amd import _lib
    from paper_1709_10010_amd.problems import band_block, build_problem

    prec = {"fp64": _lib.PW_FP64, "fp32": _lib.PW_MIXED_FP32, "bf16": _lib.PW_MIXED_BF16}[args.precision]
    cell = synth.make_cell(2)
    nk = max(1, min(args.kpoints, len(cell.kpts)))
    probs, psis, hpsis, infos = [], [], [], []
    for ik in range(nk):
        p, m = build_problem(cell, ik, precision=prec, max_bands=cell.nbands)
        inf = p.info()
        inf["n"] = cell.nr[0]
        x = band_block(cell.nbands, inf["npw"])
        x[:, :inf["npw"]] = torch.from_numpy(synth.psi_start(cell.seed, cell.nbands, inf["npw"], ik)).cuda()
        probs.append(p)
        psis.append(x)
        hpsis.append(torch.zeros_like(x))
        infos.append(inf)
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
    group = int(os.environ.get("PW_PLANE_GROUP", "8"))
    models = [stage_model(inf, cell.nbands, prec, group) for inf in infos]
    dom = max(stages, key=lambda k: stages[k][0])
    avg_ms = stages[dom][0] / stages[dom][1]
    kind, _ = models[0][dom]
    per_launch = float(np.mean([m[dom][1] for m in models]))
    gemm_dtype = {0: "f64", 1: "f32", 2: "bf16"}[prec]
    if kind == "hbm":
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None}
    else:
        achieved = per_launch / (avg_ms * 1e-3) / 1e12
        peak = PEAK_TFLOPS[gemm_dtype]
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": None}
    roof["kernel"] = dom
    stage_out = {}
    for k, (ms, n) in sorted(stages.items(), key=lambda kv: -kv[1][0]):
        kind_k, amt = models[0].get(k, ("-", 0.0))
        avg = ms / n
        ent = {"avg_ms": round(avg, 4), "launches": n, "share": round(ms / sum(v[0] for v in stages.values()), 3)}
        if kind_k == "hbm":
            ent["GB/s"] = round(float(np.mean([m[k][1] for m in models])) / (avg * 1e-3) / 1e9, 1)
        elif kind_k == "mfma":
            ent["TFLOP/s"] = round(float(np.mean([m[k][1] for m in models])) / (avg * 1e-3) / 1e12, 2)
        stage_out[k] = ent

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
        },
        "roofline": roof,
        "stages": stage_out,
        "ms_per_step_profiled": round(dt_prof / args.steps * 1e3, 4),
    }
    dav = None if args.no_davidson else davidson_section(args.davidson_reps)
    if not args.no_batched:
        out["batched_ragged_cells"] = batched_section(args.batched_cells, max(3, args.steps // 2))
    if not args.no_learned:
        out["learned_preconditioner"] = learned_section()
    if not args.no_cpu_baseline:
        cb = cpu_baseline(cell, 0, args.cpu_seconds)
        out["cpu_baseline"] = cb
        if dav is not None:
            davidson_cpu_baseline(dav)
    if dav is not None:
        for k in ("fp64", "fp32_then_fp64"):
            dav[k].pop("_theta", None)
        out["davidson_time_to_1e-8Ry"] = dav
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
