"""Benchmark: dual-gradient throughput and time to tolerance on one MI355X.

Workload: 4096 labelled source samples x 4096 target samples, d = 64, ten
Gaussian-blob classes (410 or 409 samples each), target = the blobs under a
random rotation plus a shift, cost = squared Euclidean distance built on the
GPU and normalised by its maximum, uniform marginals, gamma = 0.1, mu = 0.1
(--mu changes it).  Inputs are synthetic and seeded.

A "step" is one evaluation of the dual objective and its gradient over the
whole instance (dense: every (class, target) block), at the point an L-BFGS
run reaches after 200 iterations.  value = n_src * n_tgt * steps / time.
Also reported: the screened evaluation at the same point after a snapshot,
and time to 1e-6 relative objective of full dense and screened solves.

--gpus N > 1 exits with a message: this benchmark uses one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
# best plain read of a 1 GiB buffer measured on this MI355X (float4 grid-stride loads, HIP events);
# reported beside the roofline fraction as context (the fraction itself uses the published peak)
HBM_READ_CEILING_GBS = 6443.0
PROFILE_TRAFFIC = os.path.join(HERE, "profiles", "grad_tiles_blobs4096_traffic.json")
PROFILE_TRAFFIC_HBM = os.path.join(HERE, "profiles", "grad_tiles_blobs16384_traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--mu", type=float, default=0.1)
    ap.add_argument("--solve-iters", type=int, default=1500)
    ap.add_argument("--ref-iters", type=int, default=6000)
    ap.add_argument("--skip-cpu", action="store_true", help="omit the CPU oracle baseline")
    ap.add_argument("--skip-solve", action="store_true", help="omit the time-to-tolerance solves")
    ap.add_argument("--skip-mu-sweep", action="store_true", help="omit the mu in {0.01, 0.1, 1} sweep")
    ap.add_argument("--skip-onthefly", action="store_true",
                    help="omit the on-the-fly (matrix-core cost) workload")
    ap.add_argument("--otf-n", type=int, default=32768, help="on-the-fly workload: n_src = n_tgt")
    ap.add_argument("--otf-iters", type=int, default=500, help="on-the-fly workload: L-BFGS iterations")
    ap.add_argument("--skip-hbm", action="store_true", help="omit the 16384^2 (1 GiB cost) workload")
    ap.add_argument("--hbm-n", type=int, default=16384, help="HBM-scale workload: n_src = n_tgt")
    ap.add_argument("--skip-batched", action="store_true", help="omit the 256-instance batched workload")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--skip-batch-sequential", action="store_true",
                    help="batched workload: omit the one-after-another reference solves (no speedup)")
    ap.add_argument("--skip-warmstart", action="store_true", help="omit the learned warm-start workload")
    ap.add_argument("--skip-paper", action="store_true", help="omit the paper's synthetic experiments")
    ap.add_argument("--skip-agd", action="store_true", help="omit the accelerated-ascent solver workload")
    ap.add_argument("--skip-network", action="store_true", help="omit the warm-start network microbenchmark")
    ap.add_argument("--agd-n", type=int, nargs="*", default=[4096, 16384], help="accelerated ascent: n_src = n_tgt")
    ap.add_argument("--agd-iters", type=int, default=4000, help="accelerated ascent: iteration limit")
    ap.add_argument("--paper-iters", type=int, default=2000, help="paper synthetic: L-BFGS iteration limit")
    ap.add_argument("--paper-classes", type=int, nargs="*", default=[10, 20, 40, 80, 160, 320, 640, 1280])
    ap.add_argument("--ws-train", type=int, default=20000, help="training instances (cold solves)")
    ap.add_argument("--ws-held", type=int, default=1024, help="held-out instances")
    ap.add_argument("--ws-epochs", type=int, default=3)
    ap.add_argument("--ws-save", default=None, help="write the trained network parameters (.npy) here")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile configuration")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (traffic counter calibration)")
    return ap.parse_args()


def grad_source_hash():
    h = hashlib.sha256()
    for f in ("grad.hip", "otgs_internal.h"):
        with open(os.path.join(HERE, "paper_2303_07597_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(ns, nt, L, tj=32):
    """Bytes one dense gradient-tile launch must move at minimum: the cost
    once (4 B per entry), alpha and beta once, the row partials (one float per
    row and 32-column block), column sums and excess per (class, target)."""
    njb = -(-nt // tj)
    return 4 * ns * nt + 4 * (ns + nt) + 4 * ns * njb + 8 * L * nt


DSTAR_FILE = os.path.join(HERE, "tests", "golden", "dstar_fp64.txt")


def load_dstar():
    """FP64 optimal objectives written by tests/golden/make_dstar.py (the
    oracle's own L-BFGS, run to its float64 limit): {(name, seed): D*}."""
    out = {}
    if os.path.exists(DSTAR_FILE):
        with open(DSTAR_FILE) as fh:
            for ln in fh:
                if ln.strip() and not ln.startswith("#"):
                    f = ln.split()
                    out[(f[0], int(f[1]))] = float(f[7])
    return out


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline(inst, alpha, beta, dstar, budget_s=6.0):
    """The FP64 oracle on the host: the dense evaluation of the headline
    instance on one core and on every core (OpenMP over target columns, the
    same values), its L-BFGS time to 1e-6 of the FP64 D* on every core, and
    the paper's own comparison on one core - Algorithms 1-2 against the dense
    method, same iterations - on its synthetic set (40 classes of 10)."""
    import oracle
    import synth
    model, ncpu = cpu_info()
    C, _ = oracle.cost_normalized(inst["xs"], inst["xt"])
    P = oracle.Problem(C, inst["labels"], inst["n_groups"], inst["gamma"], inst["mu"])
    a64, b64 = alpha.astype(np.float64), beta.astype(np.float64)

    def rate(fn):
        fn()
        n, t0 = 0, time.perf_counter()
        while True:
            fn()
            n += 1
            el = time.perf_counter() - t0
            if el >= budget_s or n >= 400:
                return P.ns * P.nt * n / el, n, el
    v1, n1, e1 = rate(lambda: oracle.dual_grad(P, a64, b64))
    vall, nall, eall = rate(lambda: oracle.dual_grad_par(P, a64, b64, nthreads=ncpu))
    # time to 1e-6 relative objective, every core
    t0 = time.perf_counter()
    r = oracle.solve(P, max_iter=1500, nthreads=ncpu)
    t_solve = time.perf_counter() - t0
    rel = (dstar - r["trace"]) / abs(dstar) if dstar else None
    hit = int(np.nonzero(rel <= 1e-6)[0][0]) if rel is not None and np.any(rel <= 1e-6) else None
    ttt = t_solve * hit / max(r["iters"], 1) if hit is not None else None

    def cpu_ttt(inst_k, ds, max_iter):
        """Time to 1e-6 of the FP64 D* (every core): the solve's time up to the first iteration
        within 1e-6, by the share of its iterations."""
        Ck, _ = oracle.cost_normalized(inst_k["xs"], inst_k["xt"])
        Pk = oracle.Problem(Ck, inst_k["labels"], inst_k["n_groups"], inst_k["gamma"], inst_k["mu"])
        t0 = time.perf_counter()
        rk = oracle.solve(Pk, max_iter=max_iter, nthreads=ncpu)
        tk = time.perf_counter() - t0
        relk = (ds - rk["trace"]) / abs(ds)
        hk = np.nonzero(relk <= 1e-6)[0]
        return (tk * int(hk[0]) / max(rk["iters"], 1) if hk.size else None), (int(hk[0]) if hk.size else None)
    fix = load_dstar()
    t_cfg1, i_cfg1 = cpu_ttt(synth.gaussian4_2d(), fix[("cfg1", 1)], 3000)
    # a sample of the batched generator (instances 0..3 of the 256), each with its fixture
    sample = []
    for kk in range(4):
        tk, ik = cpu_ttt(synth.instance_from_generator((4, kk)), fix[("batch", kk)], 3000)
        sample.append(dict(k=kk, seconds=tk, iters=ik))
    # Algorithms 1-2 ("ours") against the dense method ("origin"), one core
    ps = synth.paper_synthetic(40, g=10)
    Cs, _ = oracle.cost_normalized(ps["xs"], ps["xt"])
    Ps = oracle.Problem(Cs, ps["labels"], 40, *oracle.rho_form(0.1, 0.8))
    t0 = time.perf_counter()
    ro = oracle.solve(Ps, max_iter=1000, use_screen=False)
    t_origin = time.perf_counter() - t0
    t0 = time.perf_counter()
    ru = oracle.solve(Ps, max_iter=1000, use_screen=True)
    t_ours = time.perf_counter() - t0
    return dict(value=v1, unit="entries/s", cores=1, kind="oracle", cpu_model=model, nproc=ncpu,
                sample=f"{n1} dense FP64 evaluations of the full {P.ns}x{P.nt} instance, single thread, {e1:.1f} s",
                all_cores=dict(value=vall, unit="entries/s", cores=ncpu,
                               sample=f"{nall} evaluations, OpenMP over target columns, {eall:.1f} s"),
                time_to_1e6=dict(seconds=ttt, iters=hit, cores=ncpu, solve_s=t_solve, solve_iters=r["iters"],
                                 d_star="FP64 oracle fixture"),
                time_to_1e6_cfg1=dict(workload="4 Gaussians in 2-D, 200 x 200, gamma=1, mu=0.1", seconds=t_cfg1,
                                      iters=i_cfg1, cores=ncpu),
                time_to_1e6_batch_sample=dict(workload="instances 0-3 of the 256-instance batched workload, "
                                                       "one after another", cores=ncpu,
                                              seconds_sum=sum(x["seconds"] or 0.0 for x in sample),
                                              all_reached=all(x["seconds"] is not None for x in sample),
                                              instances=sample),
                paper_synthetic_ours_vs_origin=dict(
                    workload="paper synthetic |L|=40, g=10, d=2, gamma=0.1, rho=0.8 (gamma'=0.02, mu'=4), "
                             "1000 L-BFGS iterations, one core",
                    origin_s=t_origin, ours_s=t_ours, speedup=t_origin / t_ours, iters=[ro["iters"], ru["iters"]],
                    same_objective=bool(abs(ro["obj"] - ru["obj"]) <= 1e-12 * abs(ro["obj"])),
                    paper_range="2-8.6x (one Xeon core)"))


FP32_MFMA_PEAK_TFLOPS = 157.3


def bench_onthefly(args, torch, synth, O):
    """Many-class workload with the cost recomputed from features on FP32
    matrix cores in every evaluation: n_src = n_tgt = 32768, d = 256, 100
    classes with Zipf(1.1) sizes, gamma = 0.05, mu = 0.5.  Reports the dense
    evaluation rate, the matrix-core utilisation of the tile kernels
    (2 d flop per entry over their summed launch time), and `otf_iters`
    L-BFGS iterations dense and screened (same trajectory)."""
    dev = torch.device("cuda")
    n, d = args.otf_n, 256
    inst = synth.zipf_blobs(seed=3, n_src=n, n_tgt=n, d=d, n_groups=100, gamma=0.05, mu=0.5)
    h = O.Handle([dict(labels=torch.from_numpy(inst["labels"]).to(dev), n_groups=100,
                       gamma=inst["gamma"], mu=inst["mu"],
                       x_src=torch.from_numpy(inst["xs"]).to(dev), x_tgt=torch.from_numpy(inst["xt"]).to(dev),
                       cost_mode=O.OT_GS_COST_ONTHEFLY, cost_scale=0.0)])
    a_pt, b_pt, _, _ = h.solve(max_iter=20, use_screen=0)
    if not args.no_autotune:
        h.autotune(repeats=3)
    tiles_cfg = {b: h.get_tile_config(b) for b in range(O.NBUCKET + 1) if h.get_tile_config(b)["n_tiles"] > 0}
    ga, gb = torch.empty_like(a_pt), torch.empty_like(b_pt)
    obj = torch.empty(1, dtype=torch.float64, device=dev)
    for _ in range(3):
        h.dual_grad(a_pt, b_pt, ga, gb, obj, mode=O.OT_GS_DENSE)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        h.dual_grad(a_pt, b_pt, ga, gb, obj, mode=O.OT_GS_DENSE)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    tiles_us = h.profile_tiles(reps)
    flops = 2.0 * d * n * n
    achieved = flops / (tiles_us * 1e-6) / 1e12
    out = dict(workload=f"zipf n_src=n_tgt={n} d={d} classes=100 gamma=0.05 mu=0.5, cost on the fly",
               point="after 20 dense L-BFGS iterations from zero",
               entries_per_s=n * n / el, ms_per_eval=1e3 * el,
               mfma=dict(bound="mfma", achieved=achieved, peak=FP32_MFMA_PEAK_TFLOPS, unit="TFLOP/s",
                         frac=achieved / FP32_MFMA_PEAK_TFLOPS, flop_per_launch=flops,
                         avg_launch_us=tiles_us, kernel="k_grad_tiles_otf (all buckets and passes)"),
               tile_config=tiles_cfg)
    if args.otf_iters > 0:
        K = args.otf_iters
        runs = {}
        for name, scr in (("dense", 0), ("screened", 1)):
            otr = torch.full((K + 1,), float("nan"), dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            h.stats(reset=True)
            t0 = time.perf_counter()
            _, _, inf, _ = h.solve(max_iter=K, use_screen=scr, obj_trace=otr)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            st = h.stats(reset=True)
            runs[name] = dict(wall_s=wall, iters=inf[0]["iters"], evals=inf[0]["evals"], obj=inf[0]["obj"],
                              tiles_computed_frac=st["tiles_computed"] / max(st["tiles_total"], 1),
                              pairs_skipped_frac=(1 - (st["pairs_unskipped"] + st["pairs_in_N"]) /
                                                  max(st["pairs_total"], 1)) if scr else 0.0)
        runs["speedup_screened"] = runs["dense"]["wall_s"] / runs["screened"]["wall_s"]
        out["solve"] = runs
    h.close()
    return out


def _trace_hits(tr, tt, dstar, tol=1e-6):
    """Per instance: first iteration within tol of D* and its device time (s)."""
    its, ts = [], []
    for k in range(tr.shape[0]):
        rel = (dstar[k] - tr[k]) / abs(dstar[k])
        hit = np.nonzero(rel <= tol)[0]
        if hit.size:
            its.append(int(hit[0]))
            ts.append((tt[k, hit[0]] - tt[k, 0]) / 100e6)
        else:
            its.append(None)
            ts.append(None)
    return its, ts


def _solve_traced(h, count, K, torch, **kw):
    dev = torch.device("cuda")
    tr = torch.full((count * (K + 1),), float("nan"), dtype=torch.float64, device=dev)
    tt = torch.zeros(count * (K + 1), dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a, b, info, _ = h.solve(max_iter=K, obj_trace=tr, time_trace=tt, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return (a, b, info, tr.cpu().numpy().reshape(count, K + 1), tt.cpu().numpy().reshape(count, K + 1), wall)


def _problems(insts, torch, O):
    dev = torch.device("cuda")
    return [dict(labels=torch.from_numpy(i["labels"]).to(dev), n_groups=i["n_groups"], gamma=i["gamma"],
                 mu=i["mu"], x_src=torch.from_numpy(i["xs"]).to(dev), x_tgt=torch.from_numpy(i["xt"]).to(dev),
                 cost_mode=O.OT_GS_COST_MATERIALIZE, cost_scale=0.0) for i in insts]


def bench_mu_sweep(args, torch, synth, O, n=4096, fix=None):
    """The blobs n x n workload at mu in {0.01, 0.1, 1}: time to 1e-6 relative
    objective of the dense and the screened solve (same trajectory), and the
    share of tiles and (group, target) pairs the screened solve skipped.
    D* is the FP64 oracle's (tests/golden) where it holds one for the
    instance, else the best value of the two runs (marked)."""
    dev = torch.device("cuda")
    out = {}
    for mu in (0.01, 0.1, 1.0):
        inst = synth.blobs(seed=2, n_src=n, n_tgt=n, d=64, n_groups=10, gamma=0.1, mu=mu)
        h = O.Handle([dict(labels=torch.from_numpy(inst["labels"]).to(dev), n_groups=10, gamma=0.1, mu=mu,
                           x_src=torch.from_numpy(inst["xs"]).to(dev), x_tgt=torch.from_numpy(inst["xt"]).to(dev),
                           cost_mode=O.OT_GS_COST_MATERIALIZE, cost_scale=0.0)])
        K = 10000   # mu = 1 needs about 4000 iterations to 1e-6
        res = {}
        st_tr = torch.zeros((K + 1) * 8, dtype=torch.int64, device=dev)
        for name, scr in (("dense", 0), ("screened", 1)):
            h.stats(reset=True)
            kw = dict(stats_trace=st_tr) if scr else {}
            _, _, inf, tr, tt, wall = _solve_traced(h, 1, K, torch, use_screen=scr, **kw)
            st = h.stats(reset=True)
            res[name] = (inf[0], tr, tt, wall, st)
        key = (f"blobs{n}_mu{mu:g}", 2)
        anchored = fix is not None and key in fix
        dstar = np.array([fix[key] if anchored else max(np.nanmax(res["dense"][1][0]),
                                                         np.nanmax(res["screened"][1][0]))])
        row = {"d_star": float(dstar[0]), "d_star_from": "FP64 oracle" if anchored else "best of the two runs"}
        for name in ("dense", "screened"):
            inf, tr, tt, wall, st = res[name]
            its, ts = _trace_hits(tr, tt, dstar)
            row[name] = dict(iters_to_1e6=its[0], time_to_1e6_s=ts[0], iters=inf["iters"], wall_s=wall,
                             final_rel_gap=float((dstar[0] - inf["obj"]) / abs(dstar[0])), status=inf["status"],
                             tiles_computed_frac=st["tiles_computed"] / max(st["tiles_total"], 1))
            if name == "screened":
                row[name]["pairs_skipped_frac"] = 1 - (st["pairs_unskipped"] + st["pairs_in_N"]) / max(
                    st["pairs_total"], 1)
        td, ts_ = row["dense"]["time_to_1e6_s"], row["screened"]["time_to_1e6_s"]
        row["speedup_time_to_1e6"] = (td / ts_) if (td and ts_) else None
        # per-iteration skipping of the screened solve (the handle's counters at every accepted
        # iteration): share of pairs skipped and of tiles computed between consecutive iterations,
        # at 20 iterations spread over the solve
        S = st_tr.cpu().numpy().reshape(K + 1, 8)[:res["screened"][0]["iters"] + 1].astype(np.float64)
        dS = np.diff(S, axis=0)
        curve = []
        for it in np.unique(np.linspace(1, len(dS), 20).astype(int)):
            d = dS[it - 1]
            curve.append([int(it), float(1 - (d[4] + d[2]) / max(d[1], 1)), float(d[7] / max(d[6], 1)), int(d[5])])
        # (refreshes: snapshot evaluations in the step, dense by construction; the pair counts
        # are those of the screen pass)
        row["screened"]["per_iteration"] = dict(columns=["iteration", "pairs_skipped_frac", "tiles_computed_frac",
                                                         "refreshes"], rows=curve)
        out[f"mu={mu:g}"] = row
        h.close()
    return out


def bench_hbm(args, torch, synth, O):
    """Blobs at n_src = n_tgt = 16384 (d = 64, 10 classes of ~1640 rows,
    whole-group tiles of 56 loads per lane; gamma = 0.1, mu = 0.1): the
    materialised cost is 1 GiB, four times the last-level cache, so each tile
    pass streams it from HBM.  Dense evaluation rate, the tile pass (every
    tile launch of one evaluation, HIP events) against 8 TB/s, and the mu
    sweep at this size."""
    dev = torch.device("cuda")
    n = args.hbm_n
    inst = synth.blobs(seed=2, n_src=n, n_tgt=n, d=64, n_groups=10, gamma=0.1, mu=args.mu)
    h = O.Handle(_problems([inst], torch, O))
    a_pt, b_pt, _, _ = h.solve(max_iter=200, use_screen=0)
    if not args.no_autotune:
        h.autotune(repeats=5)
    tiles_cfg = {b: h.get_tile_config(b) for b in range(O.NBUCKET + 1) if h.get_tile_config(b)["n_tiles"] > 0}
    ga, gb = torch.empty_like(a_pt), torch.empty_like(b_pt)
    obj = torch.empty(1, dtype=torch.float64, device=dev)
    dense = h.prepare_dual_grad(a_pt, b_pt, ga, gb, obj, mode=O.OT_GS_DENSE)
    for _ in range(5):
        dense()
    torch.cuda.synchronize()
    reps = 50
    t0 = time.perf_counter()
    for _ in range(reps):
        dense()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    tiles_us = h.profile_tiles(reps, alpha=a_pt, beta=b_pt)
    alg = algorithmic_bytes(n, n, 10)
    achieved = alg / (tiles_us * 1e-6) / 1e9
    h.close()
    traffic = None
    if n == 16384 and os.path.exists(PROFILE_TRAFFIC_HBM):
        with open(PROFILE_TRAFFIC_HBM) as fh:
            tr = json.load(fh)
        if tr.get("source_hash") == grad_source_hash():
            traffic = tr.get("bytes_per_launch")
    out = dict(workload=f"blobs n_src=n_tgt={n} d=64 classes=10 gamma=0.1 mu={args.mu:g}, cost 1 GiB",
               point="after 200 dense L-BFGS iterations from zero",
               entries_per_s=n * n / el, ms_per_eval=1e3 * el,
               roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                             frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                             measured_read_ceiling=HBM_READ_CEILING_GBS,
                             frac_of_read_ceiling=achieved / HBM_READ_CEILING_GBS, algorithmic_bytes_per_pass=alg,
                             avg_pass_us=tiles_us,
                             kernel="k_grad_tiles<56,0,false,1> (every tile launch of one evaluation)"),
               tile_config=tiles_cfg)
    if not args.skip_solve and not args.skip_mu_sweep:
        out["mu_sweep"] = bench_mu_sweep(args, torch, synth, O, n=n)
    return out


def bench_agd(args, torch, synth, O, fix):
    """The second solver (accelerated gradient ascent, OT_GS_SOLVER_AGD) under
    the same screening: blobs n x n (d = 64, 10 classes, gamma = 0.1) at
    mu = 0.1 and 1, dense and screened.  Time to 1e-6 relative objective
    against the FP64 optimum where the fixtures hold it (else the best of
    the two runs), whether the two trajectories agree bit for bit, and the
    share of tiles the screened solve computed."""
    out = {}
    for n in args.agd_n:
        for mu in (0.1, 1.0):
            inst = synth.blobs(seed=2, n_src=n, n_tgt=n, d=64, n_groups=10, gamma=0.1, mu=mu)
            h = O.Handle(_problems([inst], torch, O))
            K = args.agd_iters
            res = {}
            for name, scr in (("dense", 0), ("screened", 1)):
                h.stats(reset=True)
                _, _, inf, tr, tt, wall = _solve_traced(h, 1, K, torch, use_screen=scr, solver=O.OT_GS_SOLVER_AGD,
                                                       max_ls=60)
                res[name] = (inf[0], tr, tt, wall, h.stats(reset=True))
            h.close()
            key = (f"blobs{n}_mu{mu:g}", 2)
            anchored = key in fix
            dstar = np.array([fix[key] if anchored else max(np.nanmax(res["dense"][1][0]),
                                                             np.nanmax(res["screened"][1][0]))])
            row = dict(d_star=float(dstar[0]), d_star_from="FP64 oracle" if anchored else "best of the two runs",
                       same_trajectory=bool(np.array_equal(res["dense"][1], res["screened"][1], equal_nan=True)))
            for name in ("dense", "screened"):
                inf, tr, tt, wall, st = res[name]
                its, ts = _trace_hits(tr, tt, dstar)
                its4, ts4 = _trace_hits(tr, tt, dstar, tol=1e-4)
                row[name] = dict(iters_to_1e6=its[0], time_to_1e6_s=ts[0], iters_to_1e4=its4[0], time_to_1e4_s=ts4[0],
                                 iters=inf["iters"], evals=inf["evals"],
                                 wall_s=wall, status=inf["status"],
                                 final_rel_gap=float((dstar[0] - inf["obj"]) / abs(dstar[0])),
                                 tiles_computed_frac=st["tiles_computed"] / max(st["tiles_total"], 1))
            td, ts_ = row["dense"]["time_to_1e6_s"], row["screened"]["time_to_1e6_s"]
            row["speedup_time_to_1e6"] = (td / ts_) if (td and ts_) else None
            td4, ts4_ = row["dense"]["time_to_1e4_s"], row["screened"]["time_to_1e4_s"]
            row["speedup_time_to_1e4"] = (td4 / ts4_) if (td4 and ts4_) else None
            out[f"n={n} mu={mu:g}"] = row
    return out


def bench_network(args, torch, O):
    """The warm-start network (72-256-256-1, bf16 matrix-core products) on
    synthetic rows: Adam steps on 4096-row batches and inference over 65536
    rows.  Flop counts are the three products of each layer (forward, and
    for training the two backward products)."""
    dev = torch.device("cuda")
    g = torch.Generator(device="cpu").manual_seed(5)
    n, d_in, w, batch = 65536, 72, 256, 4096
    F = torch.randn(n, d_in, generator=g).to(dev)
    y = torch.randn(n, generator=g).to(dev)
    m = O.Mlp(d_in, width=w, max_rows=n)
    m.train(F, y, batch=batch, epochs=1, lr=1e-3)
    torch.cuda.synchronize()
    epochs = 4
    t0 = time.perf_counter()
    m.train(F, y, batch=batch, epochs=epochs, lr=1e-3)
    torch.cuda.synchronize()
    steps = epochs * (n // batch)
    t_step = (time.perf_counter() - t0) / steps
    out = m.forward(F)
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        m.forward(F, out=out)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / reps
    fwd_flop_row = 2.0 * (d_in * w + w * w + w)
    m.close()
    return dict(workload=f"network {d_in}-{w}-{w}-1, synthetic rows", train_batch=batch,
                ms_per_train_step=1e3 * t_step, train_tflops=3 * fwd_flop_row * batch / t_step / 1e12,
                ms_forward_65536_rows=1e3 * t_fwd, forward_tflops=fwd_flop_row * n / t_fwd / 1e12,
                bf16_peak_tflops=2500.0)


PAPER_GAMMAS = (1e3, 1e2, 1e1, 1.0, 1e-1, 1e-2, 1e-3)
PAPER_RHOS = (0.2, 0.4, 0.6, 0.8)


def _paper_grid_times(torch, synth, O, n_classes, g, max_iter, use_lower=1):
    """One size of the paper's synthetic set (Sec. 5.1): for every gamma of
    the grid, the four rho values as one batched handle (Sec. 5.2 sums the
    time over rho), solved densely ("origin") and with Algorithms 1-2
    ("ours"); both follow the same trajectory, so the ratio is pure cost."""
    dev = torch.device("cuda")
    rows = []
    for gam in PAPER_GAMMAS:
        insts = []
        for rho in PAPER_RHOS:
            g_, m_ = O.ot_gs_rho_to_mu(gam, rho)
            insts.append(synth.paper_synthetic(n_classes, g=g, gamma=g_, mu=m_))
        h = O.Handle(_problems(insts, torch, O))
        res = {}
        for name, scr in (("origin", 0), ("ours", 1)):
            h.stats(reset=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, info, _ = h.solve(max_iter=max_iter, use_screen=scr, use_lower=use_lower)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            st = h.stats(reset=True)
            res[name] = (wall, info, st)
        h.close()
        same = all(a["obj"] == b["obj"] and a["iters"] == b["iters"] for a, b in zip(res["origin"][1], res["ours"][1]))
        st = res["ours"][2]
        rows.append(dict(gamma=gam, origin_s=res["origin"][0], ours_s=res["ours"][0],
                         speedup=res["origin"][0] / res["ours"][0], same_trajectory=same,
                         iters=[x["iters"] for x in res["ours"][1]],
                         objs=[x["obj"] for x in res["ours"][1]],
                         pairs_computed_frac=(st["pairs_unskipped"] + st["pairs_in_N"]) / max(st["pairs_total"], 1),
                         pairs_in_N_frac=st["pairs_in_N"] / max(st["pairs_total"], 1)))
    return rows


def bench_paper_synthetic(args, torch, synth, O):
    """The paper's own synthetic experiments on the GPU: classes 10 -> 1280
    with 10 samples each (Fig. 2), samples per class 10 -> 160 with 10
    classes (Fig. A), the ablation without the set N at 10 classes
    (Fig. D), and Table 1's largest objective (gamma = 1e3, rho = 0.8).
    Times summed over rho per gamma as in Sec. 5.2; the paper's numbers are
    one Xeon core and are context, not targets."""
    K = args.paper_iters
    out = {"max_iter": K, "gammas": list(PAPER_GAMMAS), "rhos": list(PAPER_RHOS)}
    e1 = {}
    for L in args.paper_classes:
        rows = _paper_grid_times(torch, synth, O, L, 10, K)
        e1[str(L)] = dict(rows=rows, origin_s=sum(r["origin_s"] for r in rows), ours_s=sum(r["ours_s"] for r in rows),
                          max_speedup=max(r["speedup"] for r in rows),
                          table1_objective=rows[0]["objs"][-1])
        e1[str(L)]["speedup"] = e1[str(L)]["origin_s"] / e1[str(L)]["ours_s"]
        log(f"paper synthetic |L|={L}: ours/origin {e1[str(L)]['speedup']:.2f}x")
    out["classes_sweep"] = e1
    e7 = {}
    for g in (10, 20, 40, 80, 160):
        rows = _paper_grid_times(torch, synth, O, 10, g, K)
        e7[str(g)] = dict(origin_s=sum(r["origin_s"] for r in rows), ours_s=sum(r["ours_s"] for r in rows),
                          max_speedup=max(r["speedup"] for r in rows),
                          same_trajectory=all(r["same_trajectory"] for r in rows))
        e7[str(g)]["speedup"] = e7[str(g)]["origin_s"] / e7[str(g)]["ours_s"]
    out["samples_per_class_sweep"] = e7
    rows = _paper_grid_times(torch, synth, O, 10, 10, K, use_lower=0)
    out["without_N_10_classes"] = [dict(gamma=r["gamma"], speedup=r["speedup"]) for r in rows]
    return out


def bench_batched(args, torch, synth, O):
    """256 uneven instances (n, m ~ U[64, 2048], 2-31 classes with Dirichlet
    shares, d = 64, gamma, mu log-uniform) solved in one batched handle with
    screening, against the same instances solved one after another, cold,
    each in its own handle.  Time to 1e-6 relative objective for all."""
    K = 4000
    fix = load_dstar()
    insts = synth.batch_instances(seed=4, count=args.batch_count)
    probs = _problems(insts, torch, O)
    hb = O.Handle(probs)
    n = len(insts)
    _, _, info, tr, tt, wall = _solve_traced(hb, n, K, torch, use_screen=1)
    anchored = np.array([("batch", k) in fix for k in range(n)])
    dstar = np.array([fix[("batch", k)] if anchored[k] else np.nanmax(tr[k]) for k in range(n)])
    singles = []
    seq_total = 0.0
    if args.skip_batch_sequential:
        # the batched solve alone (for kernel traces of it): D* from its own trace
        its_b, ts_b = _trace_hits(tr, tt, dstar)
        hb.close()
        return dict(workload=f"{n} instances (batched solve only)", batched_wall_s=wall,
                    batched_all_reached_1e6=all(t is not None for t in ts_b),
                    batched_time_to_all_1e6_s=max((t for t in ts_b if t is not None), default=None))
    for k in range(n):
        h = O.Handle([probs[k]])
        _, _, inf1, tr1, tt1, w1 = _solve_traced(h, 1, K, torch, use_screen=1)
        h.close()
        if not anchored[k]:
            dstar[k] = max(dstar[k], np.nanmax(tr1[0]))
        singles.append((tr1[0], tt1[0], w1))
    its_b, ts_b = _trace_hits(tr, tt, dstar)
    its_s, ts_s = [], []
    for k, (t1, tt1, w1) in enumerate(singles):
        i1, s1 = _trace_hits(t1[None], tt1[None], dstar[k:k + 1])
        its_s.append(i1[0])
        ts_s.append(s1[0])
    ok_b = all(t is not None for t in ts_b)
    ok_s = all(t is not None for t in ts_s)
    t_b = max(t for t in ts_b if t is not None)
    t_s = float(sum(t for t in ts_s if t is not None))
    fin = np.array([x["obj"] for x in info])
    missed = [dict(k=k, n_src=int(insts[k]["xs"].shape[0]), n_tgt=int(insts[k]["xt"].shape[0]),
                   gamma=insts[k]["gamma"], mu=insts[k]["mu"], status=info[k]["status"], iters=info[k]["iters"],
                   rel_gap=float((dstar[k] - fin[k]) / abs(dstar[k])), single_reached=ts_s[k] is not None)
              for k in range(n) if ts_b[k] is None]
    hb.close()
    return dict(workload=f"{n} instances, n and m uniform in [64, 2048], d=64, 2-31 classes (Dirichlet shares), "
                         "gamma in [0.05, 1], mu in [0.01, 1] log-uniform, screened",
                d_star_from=f"FP64 oracle for {int(anchored.sum())} of {n} instances, else the best GPU run",
                reached_1e6_batched=int(sum(t is not None for t in ts_b)),
                reached_1e6_single=int(sum(t is not None for t in ts_s)),
                missed_1e6_batched=missed[:16],
                all_reached_1e6=ok_b and ok_s, batched_time_to_all_1e6_s=t_b, batched_wall_s=wall,
                sequential_time_to_1e6_sum_s=t_s, speedup=t_s / t_b,
                batched_iters_to_1e6_median=float(np.median([i for i in its_b if i is not None])),
                entries_per_instance_mean=float(np.mean([i["xs"].shape[0] * i["xt"].shape[0] for i in insts])))


def bench_warmstart(args, torch, synth, O):
    """Learned warm start: the network trained (on this GPU, by the library's
    kernels) on gauge-fixed converged duals of `ws_train` instances of the
    batched generator, evaluated on `ws_held` held-out instances with n, m up
    to 4096.  Iterations and time to 1e-6 relative objective from zero and
    from the prediction (inference included), and the final objectives."""
    import math
    dev = torch.device("cuda")
    d, w = 64, 256
    K = 4000
    # training data: batched cold solves
    feats, targets = [], []
    t_data = time.perf_counter()
    for c0 in range(0, args.ws_train, 256):
        insts = [synth.instance_from_generator((5, i)) for i in range(c0, min(args.ws_train, c0 + 256))]
        probs = _problems(insts, torch, O)
        h = O.Handle(probs)
        a, b, info, _ = h.solve(max_iter=K, use_screen=1)
        a, b = a.cpu().numpy(), b.cpu().numpy()
        tn = sum(i["xs"].shape[0] for i in insts)
        tm = sum(i["xt"].shape[0] for i in insts)
        F = torch.empty((tn + tm, d + 8), dtype=torch.float32, device=dev)
        O.features(probs, h.cost_scale(), F)
        ys, yt, os_, ot_ = [], [], 0, 0
        for i in insts:
            n, m = i["xs"].shape[0], i["xt"].shape[0]
            al, be = a[os_:os_ + n].astype(np.float64), b[ot_:ot_ + m].astype(np.float64)
            t = (al.mean() - be.mean()) / 2.0          # gauge: a.alpha = b.beta (uniform marginals)
            ys.append(al - t)
            yt.append(be + t)
            os_ += n
            ot_ += m
        feats.append(F)
        targets.append(torch.from_numpy(np.concatenate(ys + yt).astype(np.float32)).to(dev))
        h.close()
        if (c0 // 256) % 10 == 9:
            log(f"warm start: {c0 + 256} training instances solved")
    F = torch.cat(feats)
    y = torch.cat(targets)
    t_data = time.perf_counter() - t_data
    perm = torch.from_numpy(np.random.default_rng(5).permutation(y.numel())).to(dev)
    F, y = F[perm].contiguous(), y[perm].contiguous()
    batch = 4096
    M = O.Mlp(d + 8, w, max_rows=batch)
    r = np.random.default_rng(5)
    p0 = np.concatenate([r.standard_normal((d + 8) * w) * math.sqrt(2.0 / (d + 8)), np.zeros(w),
                         r.standard_normal(w * w) * math.sqrt(2.0 / w), np.zeros(w),
                         r.standard_normal(w) * math.sqrt(1.0 / w), [0.0]]).astype(np.float32)
    M.set_params(torch.from_numpy(p0).to(dev))
    steps = args.ws_epochs * ((y.numel() + batch - 1) // batch)
    ltr = torch.zeros(steps, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t_train = time.perf_counter()
    M.train(F, y, batch=batch, epochs=args.ws_epochs, lr=1e-3, loss_trace=ltr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t_train
    log(f"warm start: network trained ({steps} steps, {t_train:.1f} s)")
    lt = ltr.cpu().numpy()
    if args.ws_save:
        np.save(args.ws_save, M.get_params().cpu().numpy())
    del F, y
    # held-out instances
    held = [synth.instance_from_generator((6, i), n_hi=4096) for i in range(args.ws_held)]
    probs = _problems(held, torch, O)
    h = O.Handle(probs)
    n = len(held)
    K = 10000   # the slowest cold solves need more than 4000 iterations to reach 1e-6
    _, _, inf_c, tr_c, tt_c, wall_c = _solve_traced(h, n, K, torch, use_screen=1)
    torch.cuda.synchronize()
    log("warm start: held-out cold solves done")
    t0 = time.perf_counter()
    a0, b0 = h.warm_start(M, probs)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    tr_w = torch.full((n * (K + 1),), float("nan"), dtype=torch.float64, device=dev)
    tt_w = torch.zeros(n * (K + 1), dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, inf_w, _ = h.solve(a0, b0, max_iter=K, use_screen=1, init_user=1, obj_trace=tr_w, time_trace=tt_w)
    torch.cuda.synchronize()
    wall_w = time.perf_counter() - t0
    tr_w = tr_w.cpu().numpy().reshape(n, K + 1)
    tt_w = tt_w.cpu().numpy().reshape(n, K + 1)
    fix = load_dstar()
    anchored = np.array([("held", k) in fix for k in range(n)])
    dstar = np.array([fix[("held", k)] if anchored[k] else max(np.nanmax(tr_c[k]), np.nanmax(tr_w[k]))
                      for k in range(n)])
    its_c, ts_c = _trace_hits(tr_c, tt_c, dstar)
    its_w, ts_w = _trace_hits(tr_w, tt_w, dstar)
    fin_c = np.array([x["obj"] for x in inf_c])
    fin_w = np.array([x["obj"] for x in inf_w])
    ok = all(x is not None for x in its_c + its_w)
    ic = np.array([x if x is not None else K for x in its_c], dtype=float)
    iw = np.array([x if x is not None else K for x in its_w], dtype=float)
    tc = max(x for x in ts_c if x is not None)
    tw = max(x for x in ts_w if x is not None) + t_inf
    h.close()
    # the instances that miss 1e-6 of the better run in either run: status
    # (0 converged, 1 iteration limit, 2 no line-search step), iterations and
    # relative gap of each run
    missed = []
    for k in range(n):
        if its_c[k] is None or its_w[k] is None:
            gc = float((dstar[k] - fin_c[k]) / abs(dstar[k]))
            gw = float((dstar[k] - fin_w[k]) / abs(dstar[k]))
            missed.append(dict(k=k, n_src=int(held[k]["xs"].shape[0]), n_tgt=int(held[k]["xt"].shape[0]),
                               gamma=held[k]["gamma"], mu=held[k]["mu"],
                               cold=[inf_c[k]["status"], inf_c[k]["iters"], gc],
                               warm=[inf_w[k]["status"], inf_w[k]["iters"], gw]))
    return dict(workload=f"train {args.ws_train} / held-out {n} instances of the batched generator "
                         f"(held-out n, m up to 4096), network {d + 8}-{w}-{w}-1",
                train_rows=int(perm.numel()), train_data_s=t_data, train_s=t_train,
                train_steps=int(steps), loss_first=float(lt[:10].mean()), loss_last=float(lt[-10:].mean()),
                d_star_from=f"FP64 oracle for {int(anchored.sum())} of {n} instances, else the better GPU run",
                all_reached_1e6=ok,
                frac_reached_1e6_cold=float(np.mean([x is not None for x in its_c])),
                frac_reached_1e6_warm=float(np.mean([x is not None for x in its_w])),
                iters_to_1e6_cold_median=float(np.median(ic)), iters_to_1e6_warm_median=float(np.median(iw)),
                iters_to_1e6_cold_mean=float(ic.mean()), iters_to_1e6_warm_mean=float(iw.mean()),
                frac_instances_fewer_iters=float(np.mean(iw < ic)),
                # over the instances that reach 1e-6 in that run
                time_to_all_1e6_cold_s=tc, time_to_all_1e6_warm_s=tw, inference_s=t_inf,
                speedup_time=tc / tw,
                final_obj_max_rel_diff=float(np.max(np.abs(fin_w - fin_c) / np.abs(fin_c))),
                final_rel_gap_max_cold=float(np.max((dstar - fin_c) / np.abs(dstar))),
                final_rel_gap_max_warm=float(np.max((dstar - fin_w) / np.abs(dstar))),
                missed_1e6=missed[:16])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path runs on a "
              "single MI355X; sharding over several GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    import paper_2303_07597_amd.otgs as O

    dev = torch.device("cuda")
    inst = synth.blobs(seed=2, n_src=4096, n_tgt=4096, d=64, n_groups=10, gamma=0.1, mu=args.mu)
    ns, nt, L = inst["xs"].shape[0], inst["xt"].shape[0], inst["n_groups"]
    h = O.Handle([dict(labels=torch.from_numpy(inst["labels"]).to(dev), n_groups=L,
                       gamma=inst["gamma"], mu=inst["mu"],
                       x_src=torch.from_numpy(inst["xs"]).to(dev), x_tgt=torch.from_numpy(inst["xt"]).to(dev),
                       cost_mode=O.OT_GS_COST_MATERIALIZE, cost_scale=0.0)])

    log("dense workload created")
    # point of measurement: 200 L-BFGS iterations from zero (dense solve)
    a_pt, b_pt, info, _ = h.solve(max_iter=200, use_screen=0)
    torch.cuda.synchronize()
    if not args.no_autotune:
        h.autotune(repeats=20)
    tiles_cfg = {b: h.get_tile_config(b) for b in range(O.NBUCKET + 1) if h.get_tile_config(b)["n_tiles"] > 0}

    ga = torch.empty_like(a_pt)
    gb = torch.empty_like(b_pt)
    obj = torch.empty(1, dtype=torch.float64, device=dev)

    # one evaluation per call, arguments marshalled once
    dense = h.prepare_dual_grad(a_pt, b_pt, ga, gb, obj, mode=O.OT_GS_DENSE)

    for _ in range(args.warmup):
        dense()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dense()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # a separate pass with per-kernel events (they add host and launch
    # overhead, so the timed steps above run without them)
    h.kernel_timing(True)
    h.kernel_time(O.KERNEL_GRAD)          # clear
    for _ in range(args.steps):
        dense()
    torch.cuda.synchronize()
    h.kernel_timing(False)
    grad_ms, grad_n = h.kernel_time(O.KERNEL_GRAD)
    ms_step = 1e3 * el / args.steps
    value = ns * nt * args.steps / el
    # per-launch duration of the gradient-tile kernel: HIP events around
    # `steps` back-to-back launches on the stream the kernel runs on
    h.dual_grad(a_pt, b_pt, ga, gb, obj, mode=O.OT_GS_DENSE)
    grad_us = h.profile_tiles(args.steps, alpha=a_pt, beta=b_pt)
    grad_avg_s = grad_us * 1e-6
    alg_bytes = algorithmic_bytes(ns, nt, L)
    achieved = alg_bytes / grad_avg_s / 1e9
    traffic = None
    if os.path.exists(PROFILE_TRAFFIC):
        with open(PROFILE_TRAFFIC) as fh:
            tr = json.load(fh)
        if tr.get("source_hash") == grad_source_hash():
            traffic = tr.get("bytes_per_launch")

    log(f"dense evaluations: {ms_step:.4f} ms each, tiles {grad_us:.2f} us per launch")
    # screened evaluation at the same point after a snapshot there
    h.dual_grad(a_pt, b_pt, ga, gb, obj, mode=O.OT_GS_SNAPSHOT)
    h.stats(reset=True)
    screened = h.prepare_dual_grad(a_pt, b_pt, ga, gb, obj, mode=O.OT_GS_SCREENED)
    for _ in range(args.warmup):
        screened()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        screened()
    torch.cuda.synchronize()
    el_s = time.perf_counter() - t0
    st = h.stats(reset=True)
    screened = dict(entries_per_s=ns * nt * args.steps / el_s, ms_per_eval=1e3 * el_s / args.steps,
                    tiles_computed_frac=st["tiles_computed"] / max(st["tiles_total"], 1),
                    pairs_skipped_frac=1 - (st["pairs_unskipped"] + st["pairs_in_N"]) / max(st["pairs_total"], 1))

    log(f"screened evaluations: {screened['ms_per_eval']:.4f} ms each")
    solves = None
    fix = load_dstar()
    if not args.skip_solve:
        key = (f"blobs4096_mu{args.mu:g}", 2)
        if key in fix:
            dstar, dfrom = fix[key], "FP64 oracle"
        else:
            M = args.ref_iters
            tr = torch.full((M + 1,), float("nan"), dtype=torch.float64, device=dev)
            h.solve(max_iter=M, use_screen=0, obj_trace=tr)
            torch.cuda.synchronize()
            dstar, dfrom = float(np.nanmax(tr.cpu().numpy())), "best of a long run"
        out = {}
        for name, scr in (("dense", 0), ("screened", 1)):
            K = args.solve_iters
            otr = torch.full((K + 1,), float("nan"), dtype=torch.float64, device=dev)
            ttr = torch.zeros(K + 1, dtype=torch.int64, device=dev)
            torch.cuda.synchronize()
            h.stats(reset=True)
            t0 = time.perf_counter()
            _, _, inf, _ = h.solve(max_iter=K, use_screen=scr, obj_trace=otr, time_trace=ttr)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            s2 = h.stats(reset=True)
            o_ = otr.cpu().numpy()
            t_ = ttr.cpu().numpy().astype(np.float64) / 100e6     # device clock, 100 MHz
            rel = (dstar - o_) / abs(dstar)
            hit = np.nonzero(rel <= 1e-6)[0]
            # roofline of the whole solve: every evaluation's algorithmic bytes
            # (a screened one: the computed tiles' cost bytes plus the vectors
            # and pair arrays) at 8 TB/s against the measured wall time
            fr = s2["tiles_computed"] / max(s2["tiles_total"], 1)
            vec = alg_bytes - 4 * ns * nt
            ev_bytes = inf[0]["evals"] * (vec + fr * 4 * ns * nt)
            out[name] = dict(wall_s=wall, iters=inf[0]["iters"], evals=inf[0]["evals"], status=inf[0]["status"],
                             final_rel_gap=float(rel[inf[0]["iters"]]),
                             time_to_1e6_s=float(t_[hit[0]] - t_[0]) if hit.size else None,
                             iters_to_1e6=int(hit[0]) if hit.size else None,
                             tiles_computed_frac=fr,
                             solve_roofline=dict(algorithmic_bytes=ev_bytes,
                                                 frac=ev_bytes / (HBM_PEAK_GBS * 1e9) / wall))
        ttd, tts = out["dense"]["time_to_1e6_s"], out["screened"]["time_to_1e6_s"]
        solves = dict(d_star=dstar, d_star_from=dfrom, **out,
                      speedup_time_to_1e6=(ttd / tts) if (ttd and tts) else None)

    if args.copy_probe:
        x = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()

    log("solves done")
    sweep = None
    if not args.skip_solve and not args.skip_mu_sweep:
        sweep = bench_mu_sweep(args, torch, synth, O, fix=fix)
        log("mu sweep done")
    hbm = None
    if not args.skip_hbm:
        hbm = bench_hbm(args, torch, synth, O)
        log(f"HBM-scale workload: {hbm['ms_per_eval']:.3f} ms per dense evaluation")
    agd = None
    if not args.skip_solve and not args.skip_agd:
        agd = bench_agd(args, torch, synth, O, fix)
        log("accelerated-ascent solves done")
    otf = None
    if not args.skip_onthefly:
        otf = bench_onthefly(args, torch, synth, O)
        log(f"on-the-fly workload: {otf['ms_per_eval']:.3f} ms per dense evaluation")

    batched = None
    if not args.skip_batched:
        batched = bench_batched(args, torch, synth, O)
        if "speedup" in batched:
            log(f"batched workload: speedup {batched['speedup']:.2f} over sequential solves")
        else:
            log(f"batched workload: batched solve {batched['batched_wall_s']:.3f} s")
    warm = None
    if not args.skip_warmstart:
        warm = bench_warmstart(args, torch, synth, O)
        log(f"warm start: median iterations {warm['iters_to_1e6_cold_median']} -> "
            f"{warm['iters_to_1e6_warm_median']}")

    net = None
    if not args.skip_network:
        net = bench_network(args, torch, O)
        log(f"network: {net['ms_per_train_step']:.3f} ms per training step")
    paper = None
    if not args.skip_paper:
        paper = bench_paper_synthetic(args, torch, synth, O)
        log("paper synthetic experiments done")

    cpu = None
    if not args.skip_cpu:
        cpu = cpu_baseline(inst, a_pt.cpu().numpy(), b_pt.cpu().numpy(), fix.get((f"blobs4096_mu{args.mu:g}", 2)))

    line = dict(
        metric="dual-grad entries/s (dense, float32) + time-to-1e-6 rel obj (screened vs dense)",
        value=value, unit="entries/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=ms_step, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f32", data="synthetic",
        config=dict(workload="blobs n_src=n_tgt=4096 d=64 classes=10 gamma=0.1 mu=%g" % args.mu,
                    point="after 200 dense L-BFGS iterations from zero", parallelism="single GPU"),
        roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                      measured_read_ceiling=HBM_READ_CEILING_GBS,
                      kernel="k_grad_tiles<16,0,false>", algorithmic_bytes_per_launch=alg_bytes,
                      avg_launch_us=grad_avg_s * 1e6, launches=args.steps,
                      event_bracketed_us_per_call=1e3 * grad_ms / max(grad_n, 1), tile_config=tiles_cfg),
        cpu_baseline=cpu,
        screened_eval=screened,
        solves=solves,
        mu_sweep=sweep,
        hbm_scale=hbm,
        second_solver=agd,
        onthefly=otf,
        batched=batched,
        warm_start=warm,
        network=net,
        paper_synthetic=paper,
    )
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
