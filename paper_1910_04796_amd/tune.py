"""Exhaustive autotuner of the small-block kernels (paper, Sec. II: every
requested (m, n, k) kernel is tuned over its parameter space).

For each shape the legal candidate parameter sets (register tile TM x TN,
k chunk, waves per workgroup, or the FP64 MFMA kernel) are timed by the
library on synthetic stacks of 30,000 products (the paper's batch size) in
runs of R products per C block, for R in {1, 8, 64} by default: short and
long runs favour different kernels, and real workloads span that range.  The best set per shape goes to the database read by the tuned
path (option ``tune_db``); every timing goes to a CSV that trains the learned
model.

    python -m paper_1910_04796_amd.tune --sizes 5,13,23,32 --db DB --all ALL
    python -m paper_1910_04796_amd.tune --random 600 --lo 4 --hi 64 --seed 0 --db DB --all ALL
"""
import argparse
import gzip
import itertools
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_DB = os.path.join(HERE, "tune_db", "gfx950.txt")


def shapes_from_sizes(sizes):
    return list(itertools.product(sizes, repeat=3))


def random_shapes(count, lo, hi, seed):
    rng = np.random.default_rng(seed)
    allv = np.array(list(itertools.product(range(lo, hi + 1), repeat=3)))
    idx = rng.choice(len(allv), size=count, replace=False)
    return [tuple(int(x) for x in allv[i]) for i in idx]


def tune(shapes, db_path, all_path, reps=5, run_lens=(1, 8, 32), products=30000, min_runs=3750,
         log=print):
    """Times every candidate of every shape at each run length R: a stack of
    max(products / R, min_runs) C blocks, each updated by a run of R
    products (the floor on C blocks keeps long-run stacks wide enough to fill
    the GPU, as a real multiply's stacks are).  A plain-text timing table is
    appended shape by shape, so an interrupted run keeps what it measured."""
    from . import bsmm
    rows = []
    best = {}
    t0 = time.time()
    stream = None
    if all_path and not all_path.endswith(".gz"):
        stream = open(all_path, "w")
        stream.write("m,n,k,R,tm,tn,kc,waves,us\n")
    for i, (m, n, k) in enumerate(shapes):
        cands = bsmm.bsmm_tune_candidates(m, n, k)
        for R in run_lens:
            plain = np.array([bsmm.bsmm_select_params(m, n, k, R)], np.int32)
            us_all = bsmm.bsmm_tune_shape(m, n, k, np.concatenate([cands, plain]),
                                          n_runs=max(products // R, min_runs), run_len=R, reps=reps)
            us, plain_us = us_all[:-1], float(us_all[-1])
            ok = us > 0
            new_rows = [(m, n, k, R, *[int(x) for x in c], float(u)) for c, u in zip(cands[ok], us[ok])]
            rows += new_rows
            if stream:
                stream.write("".join(",".join(str(x) for x in r[:8]) + f",{r[8]:.3f}\n" for r in new_rows))
                stream.flush()
            j = int(np.argmin(np.where(ok, us, np.inf)))
            best[(m, n, k, R)] = (tuple(int(x) for x in cands[j]), float(us[j]), plain_us)
        log(f"[tune] {i + 1}/{len(shapes)} ({m},{n},{k}): {len(cands)} candidates; "
            + "; ".join(f"R={R} best {best[(m, n, k, R)][0]} {best[(m, n, k, R)][1]:.1f} us "
                        f"plain {best[(m, n, k, R)][2]:.1f} us" for R in run_lens)
            + f" ({time.time() - t0:.0f} s)")
    if stream:
        stream.close()
    if db_path:
        os.makedirs(os.path.dirname(os.path.abspath(db_path)), exist_ok=True)
        with open(db_path, "w") as f:
            f.write("# m n k R tm tn kc waves best_us plain_us  (gfx950; max(%d / R, %d) C blocks, "
                    "each updated by a run of R products)\n" % (products, min_runs))
            for (m, n, k, R), (p, u, pu) in sorted(best.items()):
                f.write(f"{m} {n} {k} {R} {p[0]} {p[1]} {p[2]} {p[3]} {u:.2f} {pu:.2f}\n")
    if all_path and stream is None:
        with gzip.open(all_path, "wt") as f:
            f.write("m,n,k,R,tm,tn,kc,waves,us\n")
            for r in rows:
                f.write(",".join(str(x) for x in r[:8]) + f",{r[8]:.3f}\n")
    return best, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="")
    ap.add_argument("--random", type=int, default=0)
    ap.add_argument("--lo", type=int, default=4)
    ap.add_argument("--hi", type=int, default=64)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--skip", type=int, default=0, help="skip the first N random shapes")
    ap.add_argument("--count", type=int, default=0, help="tune at most N random shapes (0: all)")
    ap.add_argument("--db", default=DEFAULT_DB)
    ap.add_argument("--all", default="")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--run-lens", default="1,8,32", help="run lengths (products per C block) to time")
    args = ap.parse_args()
    if args.sizes:
        shapes = shapes_from_sizes([int(x) for x in args.sizes.split(",")])
    else:
        shapes = random_shapes(args.random, args.lo, args.hi, args.seed)[args.skip:]
        if args.count > 0:
            shapes = shapes[:args.count]
    from . import bsmm
    bsmm.bsmm_set_option("tune_db", "")  # the plain rule is the reference for every shape
    bsmm.bsmm_set_option("mlp_weights", "")
    tune(shapes, args.db, args.all, reps=args.reps, run_lens=[int(x) for x in args.run_lens.split(",")],
         log=lambda s: print(s, file=sys.stderr, flush=True))


if __name__ == "__main__":
    main()
