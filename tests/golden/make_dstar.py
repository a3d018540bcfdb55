"""Writes tests/golden/dstar_fp64.txt: the optimal dual objective D* of the
measured workloads, from the FP64 oracle's own L-BFGS solve (plain dense
evaluations, zero start), for time-to-tolerance targets and solver tests.

Calls only oracle/ (the solver and the cost) and synth/ (seeded inputs).
Every line: name, seed, n_src, n_tgt, classes, gamma, mu, D*, iterations,
oracle status (1 converged to gtol, 2 no further line-search step at FP64
resolution, 0 iteration limit), final ||grad||_inf, and D* minus the
objective 500 iterations before the end (how still the solve had become).

    python tests/golden/make_dstar.py [--jobs 7] [--only cfg1,cfg2,batch,held]
"""
import argparse
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "dstar_fp64.txt")
MAX_ITER = 30000
GTOL = 1e-13


def _instance(name, seed):
    if name == "cfg1":
        return synth.gaussian4_2d()
    if name.startswith("blobs4096_mu"):
        mu = float(name[len("blobs4096_mu"):])
        return synth.blobs(seed=2, n_src=4096, n_tgt=4096, d=64, n_groups=10, gamma=0.1, mu=mu)
    if name == "batch":
        return synth.instance_from_generator((4, seed))
    if name == "held":
        return synth.instance_from_generator((6, seed), n_hi=4096)
    raise ValueError(name)


def _solve(job):
    name, seed = job
    inst = _instance(name, seed)
    C, _ = oracle.cost_normalized(inst["xs"], inst["xt"])
    P = oracle.Problem(C, inst["labels"], inst["n_groups"], inst["gamma"], inst["mu"])
    t0 = time.time()
    r = oracle.solve(P, max_iter=MAX_ITER, gtol=GTOL)
    tr = r["trace"]
    still = r["obj"] - tr[max(0, len(tr) - 501)]
    return (name, seed, P.ns, P.nt, P.L, P.gamma, P.mu, r["obj"], r["iters"], r["status"],
            r["gnorm_inf"], still, time.time() - t0)


def jobs(only):
    out = []
    if "cfg2" in only:
        out += [(f"blobs4096_mu{mu:g}", 2) for mu in (1.0, 0.1, 0.01)]
    if "cfg1" in only:
        out.append(("cfg1", 1))
    if "held" in only:
        out += [("held", i) for i in range(1024)]
    if "batch" in only:
        out += [("batch", i) for i in range(256)]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=7)
    ap.add_argument("--only", default="cfg1,cfg2,batch,held")
    args = ap.parse_args()
    todo = jobs(set(args.only.split(",")))
    done = {}
    if os.path.exists(OUT):
        for ln in open(OUT):
            if ln.strip() and not ln.startswith("#"):
                f = ln.split()
                done[(f[0], int(f[1]))] = ln
    todo = [j for j in todo if j not in done]
    with Pool(args.jobs) as pool, open(OUT, "a") as fh:
        if not done:
            fh.write("# FP64 oracle D* (dense L-BFGS, history 10, strong Wolfe, zero start, "
                     f"max_iter {MAX_ITER}, gtol {GTOL:g}); cost = squared Euclidean / max, "
                     "uniform marginals\n")
            fh.write("# name seed n_src n_tgt classes gamma mu dstar iters status gnorm_inf "
                     "dstar_minus_obj_500_before\n")
        for r in pool.imap_unordered(_solve, todo):
            fh.write("%s %d %d %d %d %.17g %.17g %.17g %d %d %.3e %.3e\n" % r[:12])
            fh.flush()
            print("%s %d: D*=%.12g iters=%d status=%d g=%.2e still=%.2e (%.0f s)"
                  % (r[0], r[1], r[7], r[8], r[9], r[10], r[11], r[12]), flush=True)


if __name__ == "__main__":
    main()
