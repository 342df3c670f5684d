#!/usr/bin/env python3
"""Benchmark of the interior-point hot path on one MI355X.

Workload (default): the large block-angular LP — n = 2,000,000 columns,
m = 1,020,000 rows (200 diagonal blocks of 5,000 x 10,000 with 6 nnz per
column plus 20,000 linking rows of 20 nnz), 0 <= x <= 10, solved to 1e-6 with
the FP32 supernodal factorisation and FP64 refinement.  One step = one full
interior-point solve (every per-iteration stage: evaluation, assembly,
factorisation, triangular solves, refinement, step).  Inputs are generated
on the host, analysed once (ordering, supernodes) and resident in HBM before
the timed region.

Prints one JSON line (see the repository's contract): value = solves/s,
roofline of the dominant kernel (the MFMA Schur-update GEMM of the
factorisation) measured live with HIP events around each of its launches,
and a CPU baseline from the oracle timed on a bounded slice of the same
workload.
"""
import argparse
import json
import os
import sys
import time

T_START = time.time()
PEAK = {"fp32": 157.3, "fp64": 78.6}   # MI355X dense MFMA TFLOP/s
FORMS = {"primal": 0, "dual": 1, "augmented": 2, "auto": 3}          # PDIPM_KKT_*
FORM_NAMES = {0: "primal", 1: "dual", 2: "augmented"}
FORM_TEXT = {"primal": "primal condensed K (n x n)", "dual": "dual condensed M (m x m, normal equations)",
             "augmented": "augmented SQD system (n + m)"}


def make_problem(args):
    from paper_2508_16094_amd import workloads as w
    if args.workload == "lp_block":
        p = w.lp_block(nblocks=args.nblocks)
        name = f"lp_block n={p.n} m={p.m} ({args.nblocks} blocks 5000x10000, 6 nnz/col, 2% linking rows)"
    elif args.workload == "nlp_grid":
        p = w.nlp_grid()
        name = f"nlp_grid n={p.n} m={p.m} (700x700 grid, quadratic stencil constraints)"
    elif args.workload == "lp_small":
        p = w.lp_small()
        name = f"lp_small n={p.n} m={p.m}"
    else:
        raise SystemExit(f"unknown workload {args.workload}")
    return p, name


def bench_batch(args, log):
    """Batched form: many independent QPs (n log-uniform in [50, 2000],
    m = n/2) solved together; value = instances solved per second."""
    import numpy as np
    import torch
    from paper_2508_16094_amd import lib as L
    from paper_2508_16094_amd import workloads as w
    t = time.time()
    ps = w.qp_batch(args.count)
    sizes = np.array([p.n for p in ps])
    log(f"[bench] generated {len(ps)} QPs (sum n = {sizes.sum()}) in {time.time() - t:.1f}s")
    prec = {"fp32": L.PDIPM_FP32, "fp64": L.PDIPM_FP64, "auto": L.PDIPM_PRECISION_AUTO}[args.precision]
    t = time.time()
    b = L.BatchSolver(ps, precision=prec, print_level=1 if args.verbose else 0)
    st = b.stats()
    prec = st["precision"]   # the automatic choice resolved
    log(f"[bench] analysed in {time.time() - t:.1f}s: nnz(L)={st['nnz_L']:.4g} flops={st['flops']:.4g} "
        f"supernodes={st['n_super']} levels={st['n_levels']} workspace={b.workspace_bytes() / 1e9:.2f} GB")
    b.bind()
    chosen, ms = b.autotune(reps=2)
    log(f"[bench] autotune: blockings {b.blockings()} factor ms {np.round(ms, 2).tolist()} -> {chosen}")
    for i in range(args.warmup):
        res, info = b.solve()
        log(f"[bench] warmup {i}: {info}")
    torch.cuda.synchronize()
    t0 = time.time()
    for i in range(args.steps):
        res, info = b.solve()
        log(f"[bench] step {i}: {info}")
    torch.cuda.synchronize()
    elapsed = time.time() - t0
    ok = sum(r["status"] == 0 for r in res)
    iters = np.array([r["iterations"] for r in res])
    # the same instances one at a time through the FP64 single-instance path
    # (a sample spread over the sizes; the loop time is its mean times count)
    sample = list(range(0, len(ps), max(1, len(ps) // args.loop_sample)))[:args.loop_sample]
    loop_t = []
    for i in sample:
        s = L.IpmSolver(ps[i], precision=L.PDIPM_FP64).bind()
        s.solve()
        torch.cuda.synchronize()
        t1 = time.time()
        r = s.solve()
        torch.cuda.synchronize()
        loop_t.append(time.time() - t1)
    loop_est = float(np.mean(loop_t)) * len(ps)
    fac_tf = st["flops"] / (ms[chosen] * 1e-3) / 1e12
    peak = PEAK["fp32" if prec == L.PDIPM_FP32 else "fp64"]
    # the same batch with the other factor precision
    other = L.PDIPM_FP64 if prec == L.PDIPM_FP32 else L.PDIPM_FP32
    b2 = L.BatchSolver(ps, precision=other).bind()
    b2.autotune(reps=1)
    b2.solve()
    torch.cuda.synchronize()
    t2 = time.time()
    res2, info2 = b2.solve()
    torch.cuda.synchronize()
    t_other = time.time() - t2
    del b2
    log(f"[bench] other precision: {info2}")
    out = {
        "metric": "IPM solves/s + KKT factor TFLOP/s, GB/s; mixed/batched/warm vs FP64 at 1e-6 tol",
        "value": len(ps) * args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == L.PDIPM_FP32 else "f64", "data": "synthetic",
        "config": {"workload": f"qp_batch {len(ps)} QPs, n log-uniform [50, 2000], m = n/2, 4 nnz/col, "
                               f"diagonal Q; one batched solve per step",
                   "form": "batched, fp32 factor + fp64 refinement" if prec == L.PDIPM_FP32 else "batched, fp64",
                   "tol": 1e-6, "parallelism": "single GPU"},
        "solved": ok, "iterations_max": int(iters.max()), "iterations_mean": float(iters.mean()),
        "batch_info": info,
        "other_precision": {"dtype": "f64" if other == L.PDIPM_FP64 else "f32",
                            "solves_per_s": len(ps) / t_other,
                            "solved": sum(r["status"] == 0 for r in res2),
                            "iterations_max": int(max(r["iterations"] for r in res2)),
                            "fp64_from": info2["fp64_from"]},
        "loop_fp64_single_path": {"sample": len(sample), "mean_s": float(np.mean(loop_t)),
                                  "estimated_total_s": loop_est,
                                  "batched_speedup": loop_est / (elapsed / args.steps)},
        "roofline": {"bound": "mfma", "achieved": fac_tf, "peak": peak, "unit": "TFLOP/s",
                     "frac": fac_tf / peak, "traffic": None,
                     "kernel": "whole factorisation (sum c_j^2 / autotuned factor time)"},
    }
    if not args.no_cpu_baseline:
        from oracle import ipm as oipm
        from oracle import model
        from oracle import symbolic as osym
        import scipy.sparse as sp
        # the oracle on instances of up to 700 columns spread over the sizes,
        # scaled to the whole batch by factorisation work (sum c_j^2)
        cs = [i for i in sample if ps[i].n <= 700][:6]
        t = time.time()
        fl = 0.0
        for i in cs:
            p = ps[i]
            oipm.solve(p, tol=1e-6, dense_max=0)
            J = model.jacobian(p, np.zeros(p.n)).tocsr()
            H = sp.tril(model.hessian(p, np.zeros(p.n), np.ones(p.m))).tocsr()
            fl += float(osym.analyze(osym.kkt_pattern(p.n, J.indptr, J.indices, H.indptr, H.indices), p.n)["flops"])
        dt = time.time() - t
        est = dt * st["flops"] / fl
        out["cpu_baseline"] = {"value": len(ps) / est, "unit": "solves/s", "cores": 1, "kind": "oracle",
                               "sample": f"oracle IPM on {len(cs)} instances (n = {[int(ps[i].n) for i in cs]}): "
                                         f"{dt:.1f} s for sum c_j^2 = {fl:.3g}; scaled to the batch's "
                                         f"{st['flops']:.3g}"}
    print(json.dumps(out), flush=True)
    return 0


# stated sizes of the learned warm-start workload: training solves, fresh
# parameter vectors
WARM_TRAIN, WARM_TEST = 50000, 10000


def bench_warm(args, log):
    """Learned warm start on the parametric QP (100 x 200 grid, 64 parameters):
    training set solved by the batched solver, MLP 64-512-512-(n+m) trained
    on the GPU, fresh parameters solved cold and warm; value = warm solves/s
    on the test set, MLP inference included."""
    import numpy as np
    import torch
    from paper_2508_16094_amd import lib as L
    from paper_2508_16094_amd import warm
    from paper_2508_16094_amd import workloads as w
    pq = w.qp_param()
    n, m = pq.base.n, pq.base.m
    th_train = w.thetas(args.n_train, 0)
    th_test = w.thetas(args.n_test, 1)
    t = time.time()
    pb = warm.ParamBatch(pq, chunk=args.chunk)
    log(f"[bench] parametric QP n={n} m={m}: batch of {args.chunk} analysed and bound in {time.time() - t:.1f}s")
    res, X, Lm, t_train_solve = pb.solve(th_train, log=log)
    ok_train = sum(r["status"] == 0 for r in res)
    log(f"[bench] training set: {ok_train}/{len(res)} solved in {t_train_solve:.1f}s")
    keep = np.array([r["status"] == 0 for r in res])
    dims = [th_train.shape[1], 512, 512, n + m]
    model = L.MlpModel(dims, n_x=n, max_batch=args.mlp_batch, x_weight=args.mlp_xweight).bind()
    model.set_params(w.mlp_init(dims))
    torch.cuda.synchronize()
    t = time.time()
    losses = warm.train(model, th_train[keep], np.concatenate([X, Lm], axis=1)[keep], steps=args.mlp_steps,
                        batch=args.mlp_batch, lr=args.mlp_lr, log=log)
    torch.cuda.synchronize()
    t_train = time.time() - t
    train_tf = model.flops(args.mlp_batch, 1) * args.mlp_steps / t_train / 1e12
    cold, _, _, t_cold = pb.solve(th_test, log=log)
    torch.cuda.synchronize()
    t0 = time.time()
    xh, lh = warm.predict(model, th_test)
    torch.cuda.synchronize()
    t_inf = time.time() - t0
    wres, _, _, t_warm = pb.solve(th_test, starts=(xh, lh), log=log)
    ic = np.array([r["iterations"] for r in cold])
    iw = np.array([r["iterations"] for r in wres])
    fails = int(sum(r["status"] != 0 for r in wres))
    fallbacks = int(sum(1 for r in wres if r.get("fallback")))
    f_diff = max(abs(a["f"] - b["f"]) / max(1.0, abs(b["f"])) for a, b in zip(wres, cold))
    value = len(th_test) / (t_warm + t_inf)
    out = {
        "metric": "IPM solves/s + KKT factor TFLOP/s, GB/s; mixed/batched/warm vs FP64 at 1e-6 tol",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1e3 * (t_warm + t_inf), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"qp_param warm start: 100x200 grid QP (n={n}, m={m}), 64 parameters; "
                               f"MLP 64-512-512-{n + m} trained on {int(keep.sum())} solved instances, "
                               f"tested on {len(th_test)} fresh ones (batches of {args.chunk})",
                   "form": "warm start (bf16 MLP) + batched fp64 IPM", "tol": 1e-6,
                   "parallelism": "single GPU",
                   "scale": ("stated sizes" if args.n_train >= WARM_TRAIN and args.n_test >= WARM_TEST else
                             f"reduced: {args.n_train} of {WARM_TRAIN} training and {args.n_test} of "
                             f"{WARM_TEST} test instances (--n-train {WARM_TRAIN} --n-test {WARM_TEST} "
                             f"runs the stated sizes)")},
        "cold": {"solves_per_s": len(th_test) / t_cold, "iterations_mean": float(ic.mean()),
                 "iterations_p95": float(np.percentile(ic, 95))},
        "warm": {"solves_per_s": value, "iterations_mean": float(iw.mean()),
                 "iterations_p95": float(np.percentile(iw, 95)), "inference_s": t_inf,
                 "failures": fails, "cold_fallbacks": fallbacks, "max_rel_f_diff_vs_cold": f_diff},
        "training": {"instances": int(keep.sum()), "solve_s": t_train_solve, "mlp_steps": args.mlp_steps,
                     "mlp_batch": args.mlp_batch, "mlp_s": t_train, "loss_first": losses[0][1],
                     "loss_last": losses[-1][1]},
        "roofline": {"bound": "mfma", "achieved": train_tf, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": train_tf / 2500.0, "traffic": None,
                     "kernel": "MLP training step (k_gemm_bf16 products with epilogues, loss, Adam)"},
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_copy(args, log):
    """Plain device copy of a known size (calibration of the HBM byte
    counters): 1 GiB copied args.steps times."""
    import torch
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.time() - t0) / args.steps
    print(json.dumps({"workload": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n, "ms": 1e3 * dt,
                      "gbps": 8 * n / dt / 1e9}), flush=True)
    return 0


# the GEMM kernels with their tile mapping and load helpers, as hashed for
# the traffic records: [tile mapping .. solves)
GEMM_SOURCE_REGIONS = (("kernels.hip", "constexpr int TG = 8;",
                        "// --------------------------------------------------- triangular solves"),
                       ("host.cpp", "P.sld[k] =", "P.srow[k] = s.sn_rowptr[k];"),
                       ("host.cpp", "int64_t off = 0, uoff = 0, uvoff = 0;", "P.suv[k] = uvoff;"))


def gemm_source_digest():
    """sha256 over the source regions that decide the GEMMs' memory traffic:
    tile mapping and load helpers, the FP64 and FP32 kernels, the panel and
    update-matrix layout."""
    import hashlib
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2508_16094_amd", "csrc")
    parts = []
    for fn, a, b in GEMM_SOURCE_REGIONS:
        text = open(os.path.join(csrc, fn)).read()
        parts.append(text[text.index(a):text.index(b)])
    return hashlib.sha256("".join(parts).encode()).hexdigest()


def traffic_of(kernel, workload, alg_bytes_per_launch):
    """HBM bytes per launch of kernel on workload measured with hardware
    counters (profiles/traffic.json), or None when the GEMM source (tile
    mapping, load helpers, GEMM kernels, panel and update-matrix layout) changed since the
    counters were taken,
    or when the launch mix did (the algorithmic bytes per launch differ from
    the recorded ones by more than 0.5%)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic.json")
    try:
        rec = json.load(open(path)).get(f"{kernel}@{workload}")
        digest = gemm_source_digest()
    except (OSError, ValueError):
        return None
    if not rec or rec.get("gemm_source_sha256") != digest:
        return None
    ref = rec.get("algorithmic_bytes_per_launch")
    if not ref or abs(alg_bytes_per_launch - ref) > 0.005 * ref:
        return None
    return rec["bytes_per_launch"]


def host_cpu():
    """Host CPU model and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def sample_problem(workload):
    """The bounded sample the oracle solves for the CPU baseline: a smaller
    instance of the benchmarked workload's own generator."""
    from paper_2508_16094_amd import workloads as w
    if workload == "lp_block":
        return (w.lp_block(nblocks=1, block_rows=1000, block_cols=2000, n_link_rows=0),
                "one 1000 x 2000 block of the block-angular LP generator (no linking rows)")
    if workload == "nlp_grid":
        return w.nlp_grid(60, 60), "the 60 x 60 grid instance of the same generator"
    return w.lp_small(), "the same instance"


def cpu_baseline_sample(args, cap_s=40.0):
    """The oracle (plain FP64 CPU IPM, one thread) solving a bounded sample
    of the workload to the same tolerance, timed (at most about cap_s), with
    the condensed system the benchmark uses: the one the --form choice
    names, or for "auto" the one with fewer factorisation flops on the
    sample (the library's rule)."""
    import numpy as np
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits
    from oracle import ipm as oipm
    from oracle import model
    from oracle import symbolic as osym
    p, what = sample_problem(args.workload)
    J = model.jacobian(p, np.zeros(p.n)).tocsr()
    H = sp.tril(model.hessian(p, np.zeros(p.n), np.ones(p.m))).tocsr()
    flops = {"primal": float(osym.analyze(osym.kkt_pattern(p.n, J.indptr, J.indices, H.indptr, H.indices),
                                          p.n)["flops"])}
    if H.nnz == p.n and p.m > 0:
        flops["dual"] = float(osym.analyze(osym.dual_pattern(p.m, p.n, J.indptr, J.indices), p.m)["flops"])
    if args.form in flops:
        form = args.form
    else:
        form = min(flops, key=lambda f: (flops[f], f != "primal"))
    with threadpool_limits(limits=1):
        t0 = time.time()
        r = oipm.solve(p, tol=1e-6, dense_max=0, max_wall_time=cap_s, form=form)
        dt = time.time() - t0
    return {"what": what, "seconds": dt, "iterations": max(1, r["iterations"]), "flops": flops[form],
            "form": form, "status": oipm.STATUS_NAMES.get(r["status"], str(r["status"]))}


def cpu_baseline_scale(smp, flops_full, iters_full):
    """Scale the sample's time per iteration per factorisation flop to the
    full workload's sum_j (c_j^2 - 1) and iteration count (an estimate: the
    full instance would take the oracle hours)."""
    t_full = smp["seconds"] / (smp["iterations"] * smp["flops"]) * flops_full * iters_full
    return {"value": 1.0 / t_full, "unit": "solves/s", "cores": 1, "kind": "oracle", "estimate": True,
            "sample": f"oracle IPM solve ({smp.get('form', 'primal')} condensed system) of {smp['what']}: "
                      f"{smp['status']} after {smp['iterations']} "
                      f"iterations in {smp['seconds']:.1f} s (sum c_j^2 = {smp['flops']:.3g}); scaled to the "
                      f"benchmarked instance by factorisation flops ({flops_full:.3g}) and iterations "
                      f"({iters_full})",
            "host": host_cpu()}


def plan_steps(done, elapsed, t_step, reserve, budget):
    """Whether another timed step fits: the first always runs; later ones
    only while the elapsed time plus one more step (the slowest seen) plus
    the time reserved for what follows stays within the wall budget."""
    return done == 0 or (t_step is not None and elapsed + t_step + reserve <= budget)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lp_block")
    ap.add_argument("--nblocks", type=int, default=200)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "auto"],
                    help="factor precision; auto: the library keeps FP32 factors only where its cost model "
                         "predicts they pay")
    ap.add_argument("--form", default="auto", choices=["auto", "primal", "dual", "augmented"],
                    help="KKT system factored each iteration: auto (the condensed system with fewer "
                         "factorisation flops), the primal condensed K (n x n), the dual condensed "
                         "normal-equations matrix M (m x m; LP and diagonal QP) or the augmented SQD matrix")
    ap.add_argument("--no-compare-forms", action="store_true",
                    help="skip the solves with the other condensed system (reported next to the timed one)")
    ap.add_argument("--time-budget", type=float, default=450.0,
                    help="wall seconds from process start within which the JSON line is printed; "
                         "timed steps and warmups stop early to keep it")
    ap.add_argument("--no-fp64-compare", action="store_true",
                    help="skip the FP64 solve on the same handle (reported next to the FP32 form)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--print-level", type=int, default=None,
                    help="solver log on stderr (0 none, 1 per iteration, 2 per solve, 3 per refinement)")
    ap.add_argument("--count", type=int, default=4096, help="qp_batch: number of instances")
    ap.add_argument("--loop-sample", type=int, default=16, help="qp_batch: instances timed one at a time")
    ap.add_argument("--n-train", type=int, default=4096, help="warm: training instances")
    ap.add_argument("--n-test", type=int, default=256, help="warm: fresh test instances")
    ap.add_argument("--chunk", type=int, default=128, help="warm: instances per batched solve")
    ap.add_argument("--mlp-steps", type=int, default=3000)
    ap.add_argument("--mlp-batch", type=int, default=256)
    ap.add_argument("--mlp-lr", type=float, default=1e-3)
    ap.add_argument("--mlp-xweight", type=float, default=10000.0,
                    help="warm: weight of the x term of the loss (the log-lambda term dominates otherwise)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"--gpus {args.gpus}: the solver runs one instance on one GPU; multi-GPU sharding "
              "(etree subtrees per GPU) is not implemented, run with --gpus 1", file=sys.stderr)
        return 2

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    def since_start():
        return time.time() - T_START

    if args.workload in ("copy", "qp_batch", "warm"):
        import torch  # noqa: F401
        return {"copy": bench_copy, "qp_batch": bench_batch, "warm": bench_warm}[args.workload](args, log)

    # 1. the CPU baseline first, bounded, so that it never pushes the JSON
    #    line past the budget; it needs the plan's flops and the iteration
    #    count, so it is timed now and scaled once those are known
    cpu = None
    if not args.no_cpu_baseline:
        t = time.time()
        cpu = cpu_baseline_sample(args)
        log(f"[bench] cpu baseline sample in {time.time() - t:.1f}s")
    import torch
    from paper_2508_16094_amd import lib as L

    t = time.time()
    p, name = make_problem(args)
    log(f"[bench] generated {name} in {time.time() - t:.1f}s")
    prec = {"fp32": L.PDIPM_FP32, "fp64": L.PDIPM_FP64, "auto": L.PDIPM_PRECISION_AUTO}[args.precision]
    t = time.time()
    # FP32 form: FP64 factors take over for the rest of a solve once FP32
    # refinement cannot reach the accuracy the iteration needs; the FP64
    # space also serves the FP64 comparison solve on the same handle
    form = FORMS[args.form]
    s = L.IpmSolver(p, precision=prec, fp64_fallback=1, kkt_form=form,
                    print_level=args.print_level if args.print_level is not None else (1 if args.verbose else 0))
    st = s.stats()
    chosen = FORM_NAMES[st["kkt_form"]]
    prec = st["precision"]   # the automatic choice resolved
    t_setup = time.time() - t
    log(f"[bench] analysed in {t_setup:.1f}s: {chosen} system, order {st['n']}, nnz(L)={st['nnz_L']:.4g} "
        f"flops={st['flops']:.4g} "
        f"supernodes={st['n_super']} levels={st['n_levels']} workspace={s.workspace_bytes() / 1e9:.1f} GB")
    s.bind()
    torch.cuda.synchronize()
    # 2. warmup: at most one solve (each is a complete solve); its time sizes
    #    the timed loop
    t_step = None
    warm_done = 0
    for i in range(min(args.warmup, 1)):
        t = time.time()
        r = s.solve()
        torch.cuda.synchronize()
        t_step = time.time() - t
        warm_done += 1
        log(f"[bench] warmup {i}: status {r['status']} it {r['iterations']} {r['ms_total'] / 1e3:.2f}s")
    compare = prec == L.PDIPM_FP32 and not args.no_fp64_compare
    # the other condensed system, timed next to the chosen one where the dual
    # system applies (a diagonal Hessian: the LP workloads)
    dual_applies = args.workload in ("lp_block", "lp_small")
    others = [] if args.no_compare_forms or chosen == "augmented" or not dual_applies else \
        [{"primal": "dual", "dual": "primal"}[chosen]]
    # time kept for what follows the timed solves: the FP64 solve on the same
    # handle, and one FP32 and one FP64 solve of the other condensed system
    # (up to about 3x and 3x the timed step plus its setup)
    reserve = lambda: ((1.5 * t_step if compare else 0.0) + (7.0 * t_step + 15.0 if others else 0.0)  # noqa: E731
                       if t_step else 0.0)
    s.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.time()
    results = []
    while len(results) < max(1, args.steps) and plan_steps(len(results), since_start(), t_step, reserve(),
                                                         args.time_budget):
        t = time.time()
        r = s.solve()
        torch.cuda.synchronize()
        t_step = time.time() - t if t_step is None else max(t_step, time.time() - t)
        results.append(r)
        log(f"[bench] step {len(results) - 1}: status {r['status']} it {r['iterations']} {r['ms_total'] / 1e3:.2f}s "
            f"f {r['f']:.10e} P {r['P']:.1e} D {r['D']:.1e} C {r['C']:.1e}")
    torch.cuda.synchronize()
    elapsed = time.time() - t0
    prof = s.profile()
    last = results[-1]
    steps = len(results)

    def rate(flops, ms):
        return flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    # dominant kernel: the Schur-update GEMM with the larger summed launch
    # time (in the FP32 form of the block-angular LP the FP64 one: the
    # later iterations factor in FP64); the other precision's GEMM is
    # reported beside it
    key = "64" if prof["gemm64_ms"] >= prof["gemm32_ms"] else "32"
    other = "32" if key == "64" else "64"
    pkey = "fp" + key
    gemm_tf = rate(prof["gemm" + key + "_flops"], prof["gemm" + key + "_ms"])
    launches = prof["gemm" + key + "_launches"]
    nfac_key = prof["factorizations" + key]
    method_tf = rate(st["flops"] * nfac_key, prof["gemm" + key + "_ms"])
    factor_tf = rate(prof["factor_flops"], prof["factor_ms"])
    nfac = prof["factorizations32"] + prof["factorizations64"]

    def gemm_line(k):
        # rate and measured traffic of one precision's GEMM launches
        n_l = prof["gemm" + k + "_launches"]
        if n_l == 0:
            return None
        tf = rate(prof["gemm" + k + "_flops"], prof["gemm" + k + "_ms"])
        alg = prof["gemm" + k + "_bytes"] / n_l
        return {"kernel": "k_gemm_f" + k, "achieved": tf, "peak": PEAK["fp" + k], "unit": "TFLOP/s",
                "frac": tf / PEAK["fp" + k], "launches": n_l, "avg_launch_us": 1e3 * prof["gemm" + k + "_ms"] / n_l,
                "algorithmic_bytes_per_launch": alg,
                "traffic": traffic_of("k_gemm_f" + k, f"lp_block{args.nblocks}_{chosen}", alg)
                if args.workload == "lp_block" else None}
    out = {
        "metric": "IPM solves/s + KKT factor TFLOP/s, GB/s; mixed/batched/warm vs FP64 at 1e-6 tol",
        "value": steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm_done,
        "steps_requested": args.steps,
        "warmup_requested": args.warmup,
        "ms_per_step": 1e3 * elapsed / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == L.PDIPM_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": name, "form": "fp32 factor + fp64 refinement" if prec == L.PDIPM_FP32 else "fp64",
                   "kkt_system": FORM_TEXT[chosen], "kkt_choice": args.form, "precision_choice": args.precision,
                   "tol": 1e-6, "parallelism": "single GPU"},
        "status": last["status"], "iterations": last["iterations"], "f": last["f"],
        "fp64_refactors": last["fp64_refactors"], "refinement_steps": last["ir_steps"],
        "P": last["P"], "D": last["D"], "C": last["C"],
        "setup_s": t_setup,
        "factor_tflops": factor_tf,
        # per timed solve, and summed over the timed solves
        "factorizations": {"fp32": prof["factorizations32"] / steps, "fp64": prof["factorizations64"] / steps},
        "factorizations_timed_total": {"fp32": prof["factorizations32"], "fp64": prof["factorizations64"]},
        "factor_ms_per_iter": prof["factor_ms"] / max(1, nfac),
        "solve_gbps": prof["solve_bytes"] / (sum(r["ms_solve"] for r in results) * 1e-3) / 1e9
        if last["ms_solve"] > 0 else None,
        "roofline": {"bound": "mfma", "achieved": gemm_tf, "peak": PEAK[pkey], "unit": "TFLOP/s",
                     "frac": gemm_tf / PEAK[pkey],
                     "traffic": traffic_of("k_gemm_f32" if pkey == "fp32" else "k_gemm_f64",
                                           f"lp_block{args.nblocks}_{chosen}",
                                           prof["gemm" + key + "_bytes"] / max(1, launches))
                     if args.workload == "lp_block" else None,
                     "kernel": "k_gemm_f32" if pkey == "fp32" else "k_gemm_f64",
                     "launches": launches,
                     "algorithmic_bytes_per_launch": prof["gemm" + key + "_bytes"] / max(1, launches),
                     "avg_launch_us": 1e3 * prof["gemm" + key + "_ms"] / max(1, launches),
                     "method_rate": {"achieved": method_tf, "frac": method_tf / PEAK[pkey],
                                     "definition": "sum_j (c_j^2 - 1) per factorisation x factorisations in "
                                                   "this precision / summed time of its GEMM launches"},
                     "other_gemm": gemm_line(other)},
    }
    # 3. the plain FP64 GPU path on the same handle and instance
    if compare:
        if since_start() + 2.0 * t_step <= args.time_budget + 60.0:
            s.set_profiling(False)
            s.set_precision(L.PDIPM_FP64)
            t = time.time()
            r64 = s.solve()
            torch.cuda.synchronize()
            dt = time.time() - t
            s.set_precision(prec)
            log(f"[bench] fp64 path: status {r64['status']} it {r64['iterations']} {dt:.2f}s f {r64['f']:.10e}")
            out["fp64_path"] = {"solves_per_s": 1.0 / dt, "s_per_solve": dt, "status": r64["status"],
                                "iterations": r64["iterations"], "f": r64["f"], "P": r64["P"], "D": r64["D"],
                                "C": r64["C"], "fp32_form_speedup": (steps / elapsed) * dt,
                                "rel_f_diff_vs_fp32_form": abs(r64["f"] - last["f"]) / max(1.0, abs(r64["f"]))}
        else:
            out["fp64_path"] = {"skipped": "time budget"}
    # 4. the other condensed system(s) on the same instance, one solve each
    if others:
        out["forms"] = {chosen: {"fp32_solves_per_s": steps / elapsed if prec == L.PDIPM_FP32 else None,
                                 "fp64_solves_per_s": out.get("fp64_path", {}).get("solves_per_s"),
                                 "factor_flops": st["flops"], "nnz_L": st["nnz_L"], "order": st["n"]}}
        import gc
        del s
        gc.collect()
        torch.cuda.empty_cache()
        for other in others:
            rec = {}
            if since_start() + 3.0 * t_step + 15.0 > args.time_budget + 60.0:
                out["forms"][other] = {"skipped": "time budget"}
                continue
            t = time.time()
            so = L.IpmSolver(p, precision=L.PDIPM_FP32, fp64_fallback=1, kkt_form=FORMS[other])
            sto = so.stats()
            so.bind()
            rec.update(setup_s=time.time() - t, factor_flops=sto["flops"], nnz_L=sto["nnz_L"], order=sto["n"])
            for pr, key in ((L.PDIPM_FP32, "fp32"), (L.PDIPM_FP64, "fp64")):
                if since_start() + 3.0 * t_step > args.time_budget + 60.0:
                    rec[key + "_solves_per_s"] = None
                    continue
                so.set_precision(pr)
                t = time.time()
                ro = so.solve()
                torch.cuda.synchronize()
                dt = time.time() - t
                log(f"[bench] {other} system {key}: status {ro['status']} it {ro['iterations']} {dt:.2f}s "
                    f"f {ro['f']:.10e}")
                rec[key + "_solves_per_s"] = 1.0 / dt if ro["status"] == 0 else None
                rec[key + "_status"] = ro["status"]
                rec[key + "_rel_f_diff"] = abs(ro["f"] - last["f"]) / max(1.0, abs(last["f"]))
            out["forms"][other] = rec
            del so
            gc.collect()
            torch.cuda.empty_cache()
    if cpu is not None:
        out["cpu_baseline"] = cpu_baseline_scale(cpu, st["flops"], last["iterations"])
    out["wall_s"] = since_start()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
