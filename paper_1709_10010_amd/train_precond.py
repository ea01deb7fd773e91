#!/usr/bin/env python3
"""Train the learned preconditioner on solver-generated pairs and save it.

    python -m paper_1709_10010_amd.train_precond --cells 12 --epochs 40

Training cells are the learned-preconditioner workload's training family
(seeded cells a = 16-24 bohr, 32-96 atoms s+p, 15 Ry, 4 bands per atom);
each contributes snapshots of a TPA Davidson solve (unconverged bands only)
with targets from its own converged solve.  The weights (float32 params +
feature scaler) go to weights/precond_mlp.npz; a held-out cell is then
solved with TPA and with the network from the same start block.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cells", type=int, default=12)
    ap.add_argument("--first", type=int, default=0)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--bands-per-snap", type=int, default=48)
    ap.add_argument("--max-bands", type=int, default=0, help="cap on bands per training cell (0: 4 per atom)")
    ap.add_argument("--eval-index", type=int, default=199)
    ap.add_argument("--out", default=os.path.join(HERE, "weights", "precond_mlp.npz"))
    args = ap.parse_args()

    import synth
    from paper_1709_10010_amd import learned

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
    print(f"dataset: {ds['nbands']} band samples, {ds['F'].shape[0]} (G, n) samples", flush=True)
    base = learned.baseline_loss(ds)
    print(f"plain TPA (s = 1) mean band loss on the training samples: {base:.4f}", flush=True)
    tt = time.perf_counter()
    net, hist = learned.train(ds, epochs=args.epochs, lr=args.lr,
                              log=lambda m: print(m, flush=True))
    train_s = time.perf_counter() - tt
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    learned.save(net, args.out)
    cell = synth.make_cell(5, args.eval_index)
    r = learned.evaluate(cell, net, tol=5e-7)
    out = {"train_cells": args.cells, "band_samples": ds["nbands"], "samples": int(ds["F"].shape[0]),
           "epochs": args.epochs, "loss_tpa": base, "loss_first": hist[0], "loss_last": hist[-1],
           "train_seconds": round(train_s, 2), "total_seconds": round(time.perf_counter() - t0, 1),
           "eval_cell": cell.name, "eval": {k: {"iterations": r[k]["iterations"],
                                                "seconds": round(r[k]["seconds"], 3),
                                                "n_hpsi": r[k]["n_hpsi"]} for k in ("tpa", "mlp")},
           "max_theta_diff_Ha": r["max_theta_diff_Ha"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
