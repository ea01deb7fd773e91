#!/usr/bin/env python3
"""Train the learned preconditioner on solver-generated pairs and save it.

    python -m paper_1709_10010_amd.train_precond --cells 200 --epochs 20

Training cells are the learned-preconditioner workload's training family
(seeded cells a = 16-24 bohr, 32-96 atoms s+p, 15 Ry, 4 bands per atom,
capped at --max-bands bands); each contributes snapshots of a TPA Davidson
solve (unconverged bands only) with targets from its own converged solve.
TPA is the reference: every --val-every epochs the network solves a held-out
validation cell (of the training family, or with --val-seed of the
evaluation family but another seed), and the parameters with the shortest
solve time relative to TPA on that cell are kept.  The weights (float32
params + feature scaler) go to weights/precond_mlp.npz; then the evaluation
cell (a = 24 bohr, 128 atoms, 30 Ry, 512 bands) is solved in the FP32
mixed form to 1e-6 Ry with TPA and with the network from the same start.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def _summary(r):
    return {"iterations": r["iterations"], "seconds": round(r["seconds"], 3), "n_hpsi": r["n_hpsi"],
            "converged": bool(r["converged"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cells", type=int, default=200)
    ap.add_argument("--first", type=int, default=0)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--bands-per-snap", type=int, default=12)
    ap.add_argument("--max-bands", type=int, default=128, help="cap on bands per training cell (0: 4 per atom)")
    ap.add_argument("--val-index", type=int, default=200)
    ap.add_argument("--val-seed", type=int, default=None,
                    help="validate on a cell of the evaluation family (a = 24, 128 atoms, 30 Ry, "
                         "512 bands) drawn from this seed instead of a training-family cell")
    ap.add_argument("--val-every", type=int, default=2)
    ap.add_argument("--no-eval", action="store_true", help="skip the evaluation-cell solves")
    ap.add_argument("--out", default=os.path.join(HERE, "weights", "precond_mlp.npz"))
    args = ap.parse_args()

    import synth
    from paper_1709_10010_amd import _lib, learned
    from paper_1709_10010_amd.problems import build_problem

    t0 = time.perf_counter()
    parts = []
    for i in range(args.first, args.first + args.cells):
        c = synth.make_cell(5, i)
        if args.max_bands:
            c.nbands = min(c.nbands, args.max_bands)
        tc = time.perf_counter()
        parts.append(learned.collect(c, bands_per_snap=args.bands_per_snap, seed=i))
        print(f"collected {c.name}: grid {c.nr[0]}^3, {c.nbands} bands, "
              f"{len(parts[-1][3])} band samples, {time.perf_counter() - tc:.1f} s", flush=True)
    ds = learned.build_dataset(parts)
    del parts
    print(f"dataset: {ds['nbands']} band samples, {ds['F'].shape[0]} (G, n) samples", flush=True)
    base = learned.baseline_loss(ds)
    print(f"plain TPA (s = 1) mean band loss on the training samples: {base:.4f}", flush=True)

    if args.val_seed is not None:
        vcell = synth.make_cell(5, -1, seed=args.val_seed)
        vcell.name = f"cfg5.eval_family.seed{args.val_seed}"
    else:
        vcell = synth.make_cell(5, args.val_index)
        if args.max_bands:
            vcell.nbands = min(vcell.nbands, args.max_bands)
    vprob, _ = build_problem(vcell, 0, precision=_lib.PW_MIXED_FP32, max_bands=vcell.nbands)
    learned.evaluate(vcell, None, prob=vprob, which=("tpa",))          # warm-up
    vt = learned.evaluate(vcell, None, prob=vprob, which=("tpa",))["tpa"]
    print(f"validation {vcell.name}: TPA {vt['iterations']} iterations, {vt['seconds']:.3f} s", flush=True)

    def validate(net):
        r = learned.evaluate(vcell, net, prob=vprob, which=("mlp",))["mlp"]
        return r["seconds"] / vt["seconds"] if r["converged"] else 1e9

    tt = time.perf_counter()
    net, hist = learned.train(ds, epochs=args.epochs, lr=args.lr, validate=validate,
                              val_every=args.val_every, log=lambda m: print(m, flush=True))
    train_s = time.perf_counter() - tt
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    learned.save(net, args.out)
    out = {"train_cells": args.cells, "band_samples": ds["nbands"], "samples": int(ds["F"].shape[0]),
           "epochs": args.epochs, "loss_tpa": round(base, 4), "loss_first": round(hist[0], 4),
           "loss_last": round(hist[-1], 4), "validation": {"cell": vcell.name, "tpa_seconds": round(vt["seconds"], 3),
                                                           "mlp_over_tpa": [(e, round(v, 3)) for e, v in net.val_history]},
           "train_seconds": round(train_s, 2)}
    del ds
    if not args.no_eval:
        cell = synth.make_cell(5, -1)
        r = learned.evaluate(cell, net, precision=_lib.PW_MIXED_FP32, tol=5e-7)
        out["eval"] = {"cell": cell.name, "nbands": cell.nbands, "precision": "fp32 mixed",
                       "tpa": _summary(r["tpa"]), "mlp": _summary(r["mlp"]),
                       "max_theta_diff_Ry": 2.0 * r["max_theta_diff_Ha"]}
    out["total_seconds"] = round(time.perf_counter() - t0, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
