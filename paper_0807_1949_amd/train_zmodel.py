"""Train the learned impedance model on the 512^2 GRF diffusion workload and evaluate it.

    python -m paper_0807_1949_amd.train_zmodel [--train 4000:4200] [--eval 4200:4210]
        [--small] [--k-probe 50] [--epochs 40] [--out zmodel_c4.json] [--report report.json]

Labels come from probe sweeps of the method itself (see zmodel.py); the
network is trained on the GPU by libvtm's BF16 forward/backward kernels and
Adam.  Evaluation compares sweeps and time to relative residual 1e-8 against
the diagonal rule Z = 1/a_vv and against the best uniform multiplier
alpha/a_vv found by the same probe grid.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gen  # noqa: E402
from gen import configs as GC  # noqa: E402

from . import binding as B  # noqa: E402
from . import zmodel as Zm  # noqa: E402


def log(m):
    print(m, flush=True)


def _range(s):
    a, b = s.split(":")
    return list(range(int(a), int(b)))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", default="4000:4200")
    ap.add_argument("--eval", default="4200:4210")
    ap.add_argument("--small", action="store_true")
    ap.add_argument("--k-probe", type=int, default=50)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=Zm.DEFAULT_WEIGHTS)
    ap.add_argument("--report", default=None)
    ap.add_argument("--time-budget", type=float, default=1e9, help="stop labelling after this many seconds")
    args = ap.parse_args(argv)
    t_start = time.time()
    feats, labels, alphas = [], [], []
    used = []
    for seed in _range(args.train):
        if time.time() - t_start > args.time_budget:
            log(f"label budget reached after {len(used)} systems")
            break
        cfg = GC.c4(small=args.small, seed=seed)
        t0 = time.time()
        f, y, a = Zm.make_labels(cfg["A"], cfg["spec"], cfg["b"], k_probe=args.k_probe, log=log)
        feats.append(f)
        labels.append(y)
        alphas.append(a)
        used.append(seed)
        log(f"  system {seed}: {len(y)} VTLs, label mean {y.mean():.3f} sd {y.std():.3f}, {time.time() - t0:.1f}s")
    X = np.concatenate(feats)
    Y = np.concatenate(labels)
    log(f"training on {len(Y)} VTLs from {len(used)} systems")
    P, hist = Zm.fit(X, Y, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    Zm.save(P, args.out, meta=dict(train_seeds=used, k_probe=args.k_probe, epochs=args.epochs,
                                   loss=hist, label_mean=float(Y.mean()), label_sd=float(Y.std()),
                                   small=args.small))
    log(f"saved {args.out}")
    # evaluation on held-out systems
    a_glob = float(np.exp(np.median(np.log(alphas))))
    rows = []
    for seed in _range(args.eval):
        cfg = GC.c4(small=args.small, seed=seed)
        A, spec, b = cfg["A"], cfg["spec"], cfg["b"]
        hh = B.VTM(device=-1)
        hh.evs_partition(A, spec)
        z0 = hh.get_partition()["zdiag"]
        hh.close()
        r_diag = Zm.solve_iters(A, spec, b, 1e-8, B.VTM_Z_USER, z0)
        r_unif = Zm.solve_iters(A, spec, b, 1e-8, B.VTM_Z_USER, a_glob * z0)
        r_lrn = Zm.solve_iters(A, spec, b, 1e-8, B.VTM_Z_LEARNED, params=P)
        rows.append(dict(seed=seed, diag=r_diag, uniform=r_unif, learned=r_lrn))
        log(f"  eval {seed}: sweeps diag {r_diag['sweeps']}, uniform(alpha={a_glob:g}) {r_unif['sweeps']}, "
            f"learned {r_lrn['sweeps']}")
    summ = dict(
        uniform_alpha=a_glob,
        sweeps=dict(diag=float(np.mean([r["diag"]["sweeps"] for r in rows])),
                    uniform=float(np.mean([r["uniform"]["sweeps"] for r in rows])),
                    learned=float(np.mean([r["learned"]["sweeps"] for r in rows]))),
        time_s=dict(diag=float(np.mean([r["diag"]["time_s"] for r in rows])),
                    uniform=float(np.mean([r["uniform"]["time_s"] for r in rows])),
                    learned=float(np.mean([r["learned"]["time_s"] for r in rows]))),
    )
    log("summary " + json.dumps(summ))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(dict(summary=summ, rows=rows, train_seeds=used, loss=hist), f, indent=1)


if __name__ == "__main__":
    main()
