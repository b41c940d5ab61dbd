"""Learned performance model of the small-block kernels (paper, Sec. II: a
model learned from part of the tuning data predicts performance for every
shape).

Reads the tuner's full timing table, builds the feature vector of every
(shape, parameter set) with the library's own feature function, trains the
FP32 MLP on the GPU (library kernels) to predict the standardised log time,
and evaluates on held-out shapes: for each, the measured time of the
exhaustively best set divided by the measured time of the set the model
ranks first (1.0 = the model found the best).

    python -m paper_1910_04796_amd.learn --all ALL.csv.gz --holdout 100 --out WEIGHTS --report REPORT.json
"""
import argparse
import gzip
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "tune_db", "gfx950_mlp.txt")


def read_table(path):
    op = gzip.open if path.endswith(".gz") else open
    with op(path, "rt") as f:
        f.readline()
        rows = np.array([[float(x) for x in line.split(",")] for line in f if line.strip()])
    return rows


# Timing table columns: m, n, k, R (run length), tm, tn, kc, waves, us.
T_US = 8


def features(rows):
    from . import bsmm
    out = None
    for i, r in enumerate(rows):
        f = bsmm.bsmm_mlp_features(int(r[0]), int(r[1]), int(r[2]), r[4:8].astype(np.int32), int(r[3]))
        if out is None:
            out = np.zeros((len(rows), len(f)), np.float32)
        out[i] = f
    return out


def holdout_split(shapes, count, seed):
    """The held-out shapes: ``count`` (at most a fifth) drawn without
    replacement from the sorted shape list with the given seed."""
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(shapes), size=min(count, len(shapes) // 5), replace=False)
    return set(map(tuple, np.array(shapes)[pick].tolist()))


def read_plain(db_path):
    """Plain-rule timings (last column) of a tuning database, by (m, n, k, R)."""
    plain = {}
    for line in open(db_path):
        if line.strip() and not line.startswith("#"):
            f = line.split()
            if len(f) == 10:
                plain[(int(f[0]), int(f[1]), int(f[2]), int(f[3]))] = float(f[9])
    return plain


def evaluate(rows, held, pred, plain):
    """Per held-out shape and run length: exhaustive best / time of the
    model's first pick, and plain-rule time / time of the pick."""
    key = [(int(r[0]), int(r[1]), int(r[2]), int(r[3])) for r in rows]
    by_case = {}
    for i, k in enumerate(key):
        by_case.setdefault(k, []).append(i)
    ratios, speedups = [], []
    for c in sorted(by_case):
        if c[:3] not in held:
            continue
        idx = np.array(by_case[c])
        times = rows[idx, T_US]
        pick = times[int(np.argmin(pred[idx]))]
        ratios.append(times.min() / pick)
        if c in plain:
            speedups.append(plain[c] / pick)
    return np.array(ratios), np.array(speedups)


def init_params(F, seed):
    """He-uniform weights, zero biases (same layout as the library)."""
    H = 64
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-1, 1, H * F) * np.sqrt(6.0 / F), np.zeros(H),
             rng.uniform(-1, 1, H * H) * np.sqrt(6.0 / H), np.zeros(H),
             rng.uniform(-1, 1, H) * np.sqrt(6.0 / H), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def write_weights(path, mean, sd, P):
    with open(path, "w") as f:
        f.write(f"bsmm-mlp features {len(mean)}\n")
        f.write("mean " + " ".join(repr(float(x)) for x in mean) + "\n")
        f.write("std " + " ".join(repr(float(x)) for x in sd) + "\n")
        f.write(f"params {len(P)}\n" + " ".join(repr(float(x)) for x in P) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--all", required=True, help="tuner timing table (csv or csv.gz)")
    ap.add_argument("--holdout", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--report", default="")
    ap.add_argument("--db", default="", help="tuning database with plain-rule timings (last column)")
    args = ap.parse_args()
    from . import bsmm

    def log(s):
        print(f"[learn] {s}", file=sys.stderr, flush=True)

    rows = read_table(args.all)
    shapes = sorted({(int(r[0]), int(r[1]), int(r[2])) for r in rows})
    held = holdout_split(shapes, args.holdout, args.seed)
    is_held = np.array([(int(r[0]), int(r[1]), int(r[2])) in held for r in rows])
    X = features(rows)
    y = np.log(rows[:, T_US]).astype(np.float32)
    tr = ~is_held
    mean = X[tr].mean(axis=0)
    sd = X[tr].std(axis=0)
    sd[sd == 0] = 1.0
    ym, ys = float(y[tr].mean()), float(y[tr].std())
    Xn = ((X - mean) / sd).astype(np.float32)
    yn = ((y - ym) / ys).astype(np.float32)
    log(f"{len(rows)} timings, {len(shapes)} shapes, {len(held)} held out, {int(tr.sum())} train rows")
    t0 = time.time()
    P, loss = bsmm.bsmm_mlp_train(init_params(X.shape[1], args.seed), Xn[tr], yn[tr], epochs=args.epochs,
                                  batch=args.batch, lr=args.lr, seed=args.seed)
    train_s = time.time() - t0
    log(f"trained in {train_s:.1f} s, train MSE {loss:.4f} (standardised log time)")
    pred = bsmm.bsmm_mlp_forward(P, Xn)
    plain = read_plain(args.db) if args.db and os.path.exists(args.db) else {}
    ratios, speedups = evaluate(rows, held, pred, plain)
    write_weights(args.out, mean, sd, P)
    rep = {"shapes": len(shapes), "held_out": len(held), "train_rows": int(tr.sum()),
           "run_lengths": sorted({int(r[3]) for r in rows}), "heldout_cases": int(len(ratios)),
           "train_seconds": round(train_s, 2), "train_mse": round(float(loss), 5),
           "epochs": args.epochs, "batch": args.batch, "lr": args.lr, "seed": args.seed,
           "heldout_best_over_pick": {"mean": round(float(ratios.mean()), 4),
                                      "min": round(float(ratios.min()), 4),
                                      "share_ge_0.9": round(float((ratios >= 0.9).mean()), 4)}}
    if len(speedups):
        sp = np.array(speedups)
        rep["heldout_plain_over_pick"] = {"mean": round(float(sp.mean()), 4),
                                          "min": round(float(sp.min()), 4),
                                          "geomean": round(float(np.exp(np.log(sp).mean())), 4)}
    log(json.dumps(rep))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()
