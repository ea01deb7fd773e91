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
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}       # dense MFMA
# vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz for FP64;
# FP32 counts the packed (two-wide) rate
PEAK_VALU_TFLOPS = {"f64": 78.6, "f32": 157.3}

# HBM bytes per launch measured with rocprofv3 (FETCH_SIZE x 2.0 + WRITE_SIZE
# x 1.0, factors from a plain device copy), valid only for the kernel source
# and launch choices they were taken with
MEASURED_TRAFFIC = {
    "plane": {"source": "paper_1709_10010_amd/csrc/fft.hip", "sha256_16": "08ada82ff90493df",
              "precision": 0, "band_chunk": 128, "plane_group": 2, "plane_kernel": 0,
              "bytes_per_launch": 589442585.9},
}


def measured_traffic(kernel, prec, tuning):
    """Counter-measured bytes per launch of `kernel`, or None once the kernel
    source or its launch choices differ from those of the measurement."""
    import hashlib
    m = MEASURED_TRAFFIC.get(kernel)
    if m is None or tuning is None or prec != m["precision"]:
        return None
    if (tuning.get("band_chunk"), tuning.get("plane_group"), tuning.get("plane_kernel_id")) != \
            (m["band_chunk"], m["plane_group"], m["plane_kernel"]):
        return None
    try:
        with open(os.path.join(ROOT, m["source"]), "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()[:16]
    except OSError:
        return None
    return m["bytes_per_launch"] if h == m["sha256_16"] else None


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
    ap.add_argument("--no-davidson-medium", action="store_true")
    ap.add_argument("--davidson-medium-kpoints", type=int, default=5)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch choices")
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


def davidson_medium_section(nk: int):
    """Config-2 time-to-solution, every k-point in turn (256 bands each): plain
    FP64 to 1e-8 Ry; the FP32 form to 1e-6 Ry alone; the FP32 form to 1e-5 Ha
    followed by FP64 iterations to 1e-8 Ry from the same subspace."""
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
    res = {k: {"seconds": 0.0, "iterations": 0, "n_hpsi": 0, "converged": True, "max_residual_Ha": 0.0,
               "theta": []} for k in forms}
    for ik in range(nk):
        p64, miller = build_problem(cell, ik, precision=_lib.PW_FP64, max_bands=nb)
        p32, _ = build_problem(cell, ik, precision=_lib.PW_MIXED_FP32, max_bands=nb, miller=miller)
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
            o["max_residual_Ha"] = max(o["max_residual_Ha"], float(r["rho"].max()))
            o["theta"].append(r["theta"])
        p64.close()
        p32.close()
    ref = np.concatenate(res["fp64_1e-8Ry"]["theta"])
    for name, o in res.items():
        th = np.concatenate(o.pop("theta"))
        o["seconds"] = round(o["seconds"], 3)
        o["max_abs_theta_minus_fp64_Ry"] = float(2.0 * np.abs(th - ref).max())
        out[name] = o
    base = res["fp64_1e-8Ry"]["seconds"]
    out["speedup_over_fp64_at_1e-8Ry"] = round(base / res["fp32_then_fp64_1e-8Ry"]["seconds"], 3)
    return out


def batched_section(ncells: int, steps: int, autotune: bool = True):
    """64 ragged cells (a 10-18 bohr, 20-40 Ry, 8-48 atoms, 32-192 bands): one H*psi
    sweep per step, eager launches vs one HIP-graph launch per step; each cell's
    launch choices autotuned first (outside the timed region)."""
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
    kinds = {}
    if autotune:
        for p, nb in zip(probs, nbs):
            _lib.pw_problem_autotune(p, nb, reps=2)
            k = _lib.pw_problem_tuning(p)["plane_kernel"]
            kinds[k] = kinds.get(k, 0) + 1
    b = _lib.Batch(probs, xs, ys)
    s = torch.cuda.Stream()
    out = {"cells": ncells, "bands_per_step": int(sum(nbs)), "npw_range": [min(npws), max(npws)],
           "autotuned": autotune, "plane_kernels": {("register", "wave", "lds")[k]: v for k, v in kinds.items()}}
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
    tuning = None
    if args.no_autotune:
        tuning = _lib.pw_problem_tuning(probs[0])
        tuning["plane_kernel_id"] = tuning["plane_kernel"]
        tuning["plane_kernel"] = ("register", "wave", "lds")[tuning["plane_kernel"]]
    else:
        # launch choices (plane kernel, bands per workgroup, sweep height,
        # split-K) searched once per problem, outside the timed region
        for p in probs:
            _lib.pw_problem_autotune(p, cell.nbands, reps=3)
        tuning = _lib.pw_problem_tuning(probs[0])
        tuning["plane_kernel_id"] = tuning["plane_kernel"]
        tuning["plane_kernel"] = ("register", "wave", "lds")[tuning["plane_kernel"]]
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
        inf, nbl = infos[0], (tuning or {}).get("band_chunk") or cell.nbands
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
    dav = None if args.no_davidson else davidson_section(args.davidson_reps)
    if not args.no_batched:
        out["batched_ragged_cells"] = batched_section(args.batched_cells, max(3, args.steps // 2),
                                                      autotune=not args.no_autotune)
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
        if not args.no_davidson_medium:
            out["davidson_medium_time_to_solution"] = davidson_medium_section(args.davidson_medium_kpoints)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
