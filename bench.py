"""Benchmark: Schur-complement PCG solves per second on the 2D unit square, n = 1024, rtol 1e-8.

One step is one complete solve x = A^{-1} b of -K Delta x + mu^{-1} (-Delta_Gamma)^{-1/2} x = b
(P1, 1024 x 1024 cells, Gamma the top edge): interior solve for the reduced right-hand side,
outer PCG on the interface Schur complement with the rational-approximation preconditioner
(FP64), multigrid-PCG interior solves in FP32 inside FP64 iterative refinement, and the
back-substitution.  Steps cycle through the (K, mu) grid K in {1, 1e-2, 1e-4} x
mu in {1e-6, 1e-3, 1, 1e3}; b ~ N(0, 1) per case (seeded).  Set-up (mesh plan, rational
tables, workspace) is outside the timed region; inputs are resident in HBM before timing.

Beside the headline figure the same JSON line carries the batched form: "batched_1024", a batch
of 32 instances at n = 1024 with K log-uniform in [1e-4, 1] and mu log-uniform in [1e-6, 1e2]
(every instance one complete solve, all advancing together through shared launches), and "c4",
256 instances with n uniform on {64, 96, ..., 512} and the same K, mu distributions
(preconditioner tables to 1e-8 with at most 20 poles).  Both report instance solves/s.

Prints one JSON line (rank 0, N = 1 only).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=24)
    ap.add_argument("--warmup", type=int, default=12)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--nu", type=int, default=2,
                    help="red-black sweep pairs per level (2: the autotuner's choice on MI355X for "
                         "this workload, see paper_2211_15308_amd.autotune.tune_solves)")
    ap.add_argument("--inner-rtol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--cases", default="all", help="'all' or 'K,mu'")
    ap.add_argument("--eager", action="store_true", help="launch kernels eagerly (no hipGraph replay)")
    ap.add_argument("--pmc-mode", action="store_true",
                    help="a few solves and a 256 MiB device copy, for rocprofv3 counter runs")
    ap.add_argument("--batched", choices=["all", "none", "1024", "c4"], default="all",
                    help="which batched workloads to run beside the headline figure")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched runs use --nu and the default per-step reduction instead of the autotuner")
    ap.add_argument("--weights", default=None,
                    help="warm-start network parameters (.npz); default: the package's trained weights")
    ap.add_argument("--learned", choices=["auto", "none", "only"], default="auto",
                    help="run the learned-warm-start comparison (auto: if weights exist)")
    ap.add_argument("--learned-steps", type=int, default=6)
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D cases")
    ap.add_argument("--cnn-only", action="store_true", help="only time the warm-start network kernels")
    ap.add_argument("--only-3d", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="the 2D parameter sweep: n in {128, ..., 2048} x K x mu, per-case counts, "
                         "solves/s and error against the oracle")
    ap.add_argument("--only-batched", action="store_true",
                    help="skip the headline single-problem run (for profiling the batched kernels)")
    return ap.parse_args()


def cases(args):
    if args.cases != "all":
        K, mu = (float(v) for v in args.cases.split(","))
        return [(K, mu)]
    return [(K, mu) for K in (1.0, 1e-2, 1e-4) for mu in (1e-6, 1e-3, 1.0, 1e3)]


def cpu_baseline(args, case_list):
    """The oracle's exact separable solver, timed on this host on a bounded sample of the cases.

    scipy.fft runs single-threaded by default and the banded solves are sequential, so the
    oracle uses one core.
    """
    import workloads
    from oracle import system
    n = args.n
    t0 = time.perf_counter()
    done = 0
    while time.perf_counter() - t0 < args.cpu_seconds:
        K, mu = case_list[done % len(case_list)]
        b = workloads.rhs(2, n, 1000 + done % len(case_list))
        system.solve_dst_2d(n, K, mu, b)
        done += 1
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} solves of the 2D n={n} problem by the oracle's separable sine-transform "
                      f"solver (FP64, numpy/scipy, one thread), cycling the same (K, mu) cases, {dt:.1f} s"}


# Algorithmic bytes of the finest-level down kernel per interior dof (FP32): it reads r and z,
# plus p' and x on iterations k >= 1, and writes r_new, p, x, the pre-smoothed u and a
# quarter-size coarse right-hand side (A p is a stencil in LDS, not a stored vector).
DOWN0_BYTES_K0 = 4 * 2 + 4 * 4 + 1
DOWN0_BYTES_K = DOWN0_BYTES_K0 + 4 * 2
HBM_PEAK_GBS = 8000.0


def traffic_from_profile(root, nu):
    """HBM bytes per launch from the committed PMC summary, if it matches the current kernel."""
    path = os.path.join(root, "profiles", "down0_traffic.json")
    try:
        rec = json.load(open(path))
        sha = kernel_source_sha(root)
    except (OSError, ValueError):
        return None
    kname = f"void fdd::k_mg_down<float, {nu}, true, 32, true>"
    if rec.get("kernel_sources_sha256") != sha or rec.get("kernel") != kname:
        return None
    return rec.get("traffic_bytes_per_launch")


def kernel_source_sha(root):
    """sha256 over the sources the multigrid kernels are compiled from."""
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels_mg.hip", "mg_device.h", "fdd_internal.h"):
        h.update(open(os.path.join(root, "paper_2211_15308_amd", "csrc", name), "rb").read())
    return h.hexdigest()


class OracleLeg:
    """The benchmark's use of the oracle, in one place after the GPU legs: the CPU baseline (timed
    by cpu_baseline) and the parity spot-checks of GPU solutions.  The GPU legs only copy the
    right-hand side and solution to the host and name the slot (a dict key or list index of the
    output) that receives the relative error; run() fills the slots."""

    def __init__(self):
        self.items = []

    def check(self, slot, key, n, K, mu, b, x):
        self.items.append((slot, key, n, K, mu, b.detach().cpu().numpy(), x.detach().cpu().numpy()))

    def run(self):
        import numpy as np
        from oracle import system
        for slot, key, n, K, mu, b, x in self.items:
            xr = system.solve_dst_2d(n, K, mu, b)
            slot[key] = float(np.linalg.norm(x - xr) / np.linalg.norm(xr))
        self.items = []


def setup_instances(F, cases, tol_p, max_p, tol_h, threads=8):
    """Problems and rational tables of a batch (host work, run on a thread pool), workspaces bound."""
    from concurrent.futures import ThreadPoolExecutor

    def one(c):
        P = F.setup_mesh(c["n"], c["K"], c["mu"])
        TP = P.build_rational_pc(F.FDD_RA_PRECOND, tol_p, max_p)
        TH = P.build_rational_pc(F.FDD_RA_OPERATOR, tol_h)
        return P, TP, TH

    with ThreadPoolExecutor(threads) as ex:
        out = list(ex.map(one, cases))
    for P, _, _ in out:
        P.bind_workspace()
    return out


def run_batched(F, args, label, cases, tol_p, max_p, leg):
    """Instance solves/s of one batch; roofline of the batched finest-level down kernel."""
    import numpy as np
    import torch

    import workloads
    import paper_2211_15308_amd.fdd as FF
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    inst = setup_instances(F, cases, tol_p, max_p, 1e-12)
    setup_s = time.perf_counter() - t0
    B = F.Batch([i[0] for i in inst], [i[1] for i in inst], [i[2] for i in inst])
    bs = [torch.as_tensor(workloads.rhs(2, c["n"], c["seed"]), dtype=torch.float64, device=dev)
          for c in cases]
    xs = [torch.zeros_like(b) for b in bs]
    opts = F.opts_default(outer_rtol=args.rtol, inner_rtol=args.inner_rtol, mg_nu=args.nu,
                          use_graph=0 if args.eager else 1)
    tune = None
    if not args.no_autotune:
        from paper_2211_15308_amd import autotune
        opts, tune = autotune.tune_batch(B, bs, xs, opts, reps=1)
    for _ in range(2):
        B.solve(bs, xs, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        st = B.solve(bs, xs, opts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    value = len(cases) * args.batch_steps / el
    # roofline pass: eager launches with an event pair on every batched down kernel
    B.set_kernel_timer(FF.FDD_KT_DOWN0)
    st_t = B.solve(bs, xs, opts)
    nl, ms, nlong, lms, _ = B.kernel_timer()
    B.set_kernel_timer(FF.FDD_KT_NONE)
    alg = 0.0
    for c, s_ in zip(cases, st_t):
        ni = (c["n"] - 1) ** 2
        its, runs = s_["inner_its_total"], s_["refine_steps"]
        # every PCG run updates on its counted iterations plus the one whose residual met the
        # run's tolerance; the first update of a run (k = 0) reads no p' and x
        alg += ni * (DOWN0_BYTES_K * its + DOWN0_BYTES_K0 * runs)
    achieved = alg / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    errs = [None] * min(3, len(cases))
    for i in range(len(errs)):
        c = cases[i]
        leg.check(errs, i, c["n"], c["K"], c["mu"], bs[i], xs[i])
    outer = [s_["outer_its"] for s_ in st]
    return {
        "label": label, "value": value, "unit": "instance solves/s", "instances": len(cases),
        "dofs": int(sum(c["n"] * (c["n"] - 1) for c in cases)), "ms_per_batch": 1e3 * el / args.batch_steps,
        "batches_timed": args.batch_steps, "setup_s": setup_s,
        "schedule": {"mg_nu": opts.mg_nu, "step_rtol": opts.step_rtol,
                     "autotune_ms_per_batch": tune["ms_per_batch"] if tune else None},
        "outer_its_min_mean_max": [min(outer), float(np.mean(outer)), max(outer)],
        "poles_P_min_max": [min(i[1].query()["m"] for i in inst), max(i[1].query()["m"] for i in inst)],
        "rel_err_vs_oracle_first3": errs,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": f"kb_mg_down<{opts.mg_nu},true,32> (finest level of every instance, "
                               "PCG update fused)",
                     "launches": nl, "avg_launch_us": 1e3 * ms / max(nl, 1),
                     "alg_bytes_per_batch_solve": alg},
    }


CNN_FWD_FLOP_PER_PX = 2 * 9 * (5 * 32 + 4 * 32 * 32 + 32 * 1)  # the six convolutions
# forward + data gradient (all layers but the first) + weight gradient
CNN_TRAIN_FLOP_PER_PX = 3 * CNN_FWD_FLOP_PER_PX - 2 * 9 * 5 * 32
MFMA_BF16_PEAK_TFLOPS = 2500.0


def cnn_timing(F, theta, reps=10):
    """Inference at n = 1024 and one training step at n = 256, batch 16: time and MFMA rate."""
    import torch
    out = {}
    for label, n, B, train in (("inference_n1024_b1", 1024, 1, False), ("train_step_n256_b16", 256, 16, True)):
        net = F.Cnn(B, n, train=train)
        net.set_params(theta)
        tr = torch.randn((B, n - 1), dtype=torch.float64, device="cuda")
        lk = torch.zeros(B, dtype=torch.float64, device="cuda")
        y = torch.empty((B, (n - 1) ** 2), dtype=torch.float32, device="cuda")
        tgt = torch.zeros_like(y)
        th = theta.clone()
        g, m, v = torch.zeros_like(th), torch.zeros_like(th), torch.zeros_like(th)

        def once(step):
            if train:
                net.set_params(th)
            net.forward(tr, lk, lk, y, n, rescale=not train)
            if train:
                net.loss(y, tgt, n)
                net.backward(B, n, g)
                net.adam_step(th, g, m, v, 1e-4, step)

        once(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(reps):
            once(k + 2)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        flop = (CNN_TRAIN_FLOP_PER_PX if train else CNN_FWD_FLOP_PER_PX) * B * (n - 1) ** 2
        tf = flop / (ms * 1e-3) / 1e12
        out[label] = {"ms": ms, "alg_tflops": tf, "frac_of_bf16_peak": tf / MFMA_BF16_PEAK_TFLOPS}
    return out


def run_learned(F, args, leg, sizes=(256, 512, 1024), mus=(1e-3, 1.0)):
    """Plain zero-guess vs learned-warm-start solves at K = 1 (same rtol): solves/s, inner its."""
    import torch

    import workloads
    from paper_2211_15308_amd import train_warmstart
    path = args.weights or train_warmstart.DEFAULT_OUT
    if not os.path.exists(path):
        return {"skipped": f"no trained weights at {os.path.relpath(path, ROOT)}"}
    theta_np, meta = train_warmstart.load_weights(path)
    theta = torch.as_tensor(theta_np, dtype=torch.float32, device="cuda")
    timing = cnn_timing(F, theta)
    res = {"weights": os.path.relpath(path, ROOT), "trained": {k: meta[k] for k in
                                                                ("n", "pairs", "steps", "val_loss", "train_seconds")},
           "network": timing, "cases": []}
    for n in sizes:
        net = F.Cnn(1, n)
        net.set_params(theta)
        for ci, mu in enumerate(mus):
            P = F.setup_mesh(n, 1.0, mu)
            P.bind_workspace()
            TP = P.build_rational_pc(F.FDD_RA_PRECOND, 1e-12)
            TH = P.build_rational_pc(F.FDD_RA_OPERATOR, 1e-12)
            b = torch.as_tensor(workloads.rhs(2, n, 5000 + 10 * ci + n), dtype=torch.float64, device="cuda")
            row = {"n": n, "K": 1.0, "mu": mu}
            for label, ws in (("plain", None), ("learned", net.h.value)):
                opts = F.opts_default(outer_rtol=args.rtol, inner_rtol=args.inner_rtol, mg_nu=args.nu)
                opts.warmstart = ws
                x = torch.zeros_like(b)
                for _ in range(2):
                    st = P.solve(TP, TH, b, x, opts)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.learned_steps):
                    st = P.solve(TP, TH, b, x, opts)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                row[label] = {"solves_per_s": args.learned_steps / el, "outer_its": st["outer_its"],
                              "inner_its": st["inner_its_total"], "warm_accepted": st["warm_accepted"],
                              "warm_starts": st["warm_starts"], "rel_err_vs_oracle": None}
                leg.check(row[label], "rel_err_vs_oracle", n, 1.0, mu, b, x)
            res["cases"].append(row)
    return res


def run_sweep(F, args, leg, sizes=(128, 256, 512, 1024, 2048)):
    """2D sweep n x K in {1, 1e-2, 1e-4} x mu in {1e-6, 1e-3, 1, 1e3} (seed 1000 + index): outer and
    inner iterations, solves/s (one warm-up and two timed solves) and the error of the solution."""
    import torch

    import workloads
    out = []
    idx = 0
    for n in sizes:
        for K in (1.0, 1e-2, 1e-4):
            for mu in (1e-6, 1e-3, 1.0, 1e3):
                P = F.setup_mesh(n, K, mu)
                P.bind_workspace()
                TP = P.build_rational_pc(F.FDD_RA_PRECOND, 1e-12)
                TH = P.build_rational_pc(F.FDD_RA_OPERATOR, 1e-12)
                b = torch.as_tensor(workloads.rhs(2, n, 1000 + idx), dtype=torch.float64, device="cuda")
                x = torch.zeros_like(b)
                opts = F.opts_default(outer_rtol=args.rtol, inner_rtol=args.inner_rtol, mg_nu=args.nu)
                P.solve(TP, TH, b, x, opts)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(2):
                    st = P.solve(TP, TH, b, x, opts)
                torch.cuda.synchronize()
                el = (time.perf_counter() - t0) / 2
                row = {"n": n, "K": K, "mu": mu, "solves_per_s": 1.0 / el, "outer_its": st["outer_its"],
                       "inner_its": st["inner_its_total"], "poles_P": TP.query()["m"],
                       "poles_H": TH.query()["m"], "rel_err_vs_oracle": None}
                leg.check(row, "rel_err_vs_oracle", n, K, mu, b, x)
                out.append(row)
                print(f"[sweep] n={n} K={K:g} mu={mu:g}: {row['solves_per_s']:.1f} solves/s, "
                      f"outer {row['outer_its']}, inner {row['inner_its']}", file=sys.stderr, flush=True)
                idx += 1
    return out


def run_3d(F, args, sizes=(32, 64, 128), mus=(1e-4, 1.0, 1e2), reps=2):
    """3D unit cube (Kuhn tetrahedra), Gamma = top face, K = 1: solves/s per (n, mu); FP64 outer
    PCG and face solves, FP32 multigrid-PCG inside FP64 refinement for the interior."""
    import torch

    import workloads
    out = []
    for n in sizes:
        for ci, mu in enumerate(mus):
            P = F.setup_mesh(n, 1.0, mu, dim=3)
            P.bind_workspace()
            TP = P.build_rational_pc(F.FDD_RA_PRECOND, 1e-12)
            TH = P.build_rational_pc(F.FDD_RA_OPERATOR, 1e-12)
            b = torch.as_tensor(workloads.rhs(3, n, 3000 + len(out)), dtype=torch.float64, device="cuda")
            x = torch.zeros_like(b)
            opts = F.opts_default(outer_rtol=args.rtol, inner_rtol=args.inner_rtol)
            st = P.solve(TP, TH, b, x, opts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                st = P.solve(TP, TH, b, x, opts)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / reps
            chk = P.solve(TP, TH, b, x, F.opts_default(outer_rtol=args.rtol, inner_rtol=args.inner_rtol,
                                                        check_true_residual=1))
            out.append({"n": n, "K": 1.0, "mu": mu, "dofs": P.N, "precision": "mixed",
                        "solves_per_s": 1.0 / el,
                        "outer_its": st["outer_its"], "inner_its": st["inner_its_total"],
                        "poles_P": TP.query()["m"], "poles_H": TH.query()["m"],
                        "true_rel_res": chk["true_rel_res"]})
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2211_15308_amd as F
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prec = F.FDD_MIXED if args.precision == "mixed" else F.FDD_FP64
    opts = F.opts_default(outer_rtol=args.rtol, inner_rtol=args.inner_rtol, precision=prec,
                          mg_nu=args.nu, use_graph=0 if args.eager else 1)
    case_list = cases(args)
    if args.cnn_only:
        from paper_2211_15308_amd import train_warmstart
        th, _ = train_warmstart.load_weights(args.weights or train_warmstart.DEFAULT_OUT)
        print(json.dumps({"network": cnn_timing(F, torch.as_tensor(th, device="cuda"))}))
        return
    if args.only_3d:
        print(json.dumps({"three_d": run_3d(F, args)}))
        return
    if args.sweep:
        leg = OracleLeg()
        res = run_sweep(F, args, leg)
        leg.run()
        print(json.dumps({"sweep": res}))
        return
    if args.learned == "only":
        leg = OracleLeg()
        res = run_learned(F, args, leg)
        leg.run()
        print(json.dumps({"learned": res}))
        return
    if args.only_batched:
        res = {}
        leg = OracleLeg()
        if args.batched in ("all", "1024"):
            res["batched_1024"] = run_batched(F, args, "32 instances, n=1024",
                                              workloads.batch_instances(count=32, seed=4, sizes=[1024]), 1e-12, 64,
                                              leg)
        if args.batched in ("all", "c4"):
            res["c4"] = run_batched(F, args, "256 instances, n in {64,...,512}",
                                    workloads.batch_instances(count=256, seed=4), 1e-8, 20, leg)
        leg.run()
        print(json.dumps(res))
        return
    if args.pmc_mode:
        # calibration copy of known size, then a short run of the benchmark workload
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        case_list = case_list[:2]
        args.steps, args.warmup = 2, 1
    probs = []
    for ci, (K, mu) in enumerate(case_list):
        P = F.setup_mesh(args.n, K, mu)
        P.bind_workspace()
        TP = P.build_rational_pc(F.FDD_RA_PRECOND, 1e-12)
        TH = P.build_rational_pc(F.FDD_RA_OPERATOR, 1e-12)
        b = torch.as_tensor(workloads.rhs(2, args.n, 1000 + ci), dtype=torch.float64, device=dev)
        x = torch.zeros_like(b)
        probs.append((P, TP, TH, b, x, K, mu))
    torch.cuda.synchronize()
    stats = []
    for s in range(args.warmup):
        P, TP, TH, b, x, K, mu = probs[s % len(probs)]
        P.solve(TP, TH, b, x, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        P, TP, TH, b, x, K, mu = probs[s % len(probs)]
        st = P.solve(TP, TH, b, x, opts)
        stats.append(dict(K=K, mu=mu, outer=st["outer_its"], inner=st["inner_its_total"],
                          refine=st["refine_steps"], ms=st["t_solve_ms"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = args.steps / elapsed
    if args.pmc_mode:
        print(json.dumps({"pmc_mode": True, "steps": args.steps}))
        return
    # roofline of the dominant kernel (the finest-level down kernel with the PCG update):
    # the same steps again, with a HIP event pair attached to every launch of it
    import paper_2211_15308_amd.fdd as FF
    for P, *_ in probs:
        P.set_kernel_timer(FF.FDD_KT_DOWN0)
    its = runs = 0
    for s in range(args.steps):
        P, TP, TH, b, x, K, mu = probs[s % len(probs)]
        st = P.solve(TP, TH, b, x, opts)
        its += st["inner_its_total"]
        runs += st["refine_steps"] if prec == F.FDD_MIXED else st["inner_solves"]
    launches = tot_ms = long_n = long_ms = 0
    for P, *_ in probs:
        nl, ms, nlong, lms, _ = P.kernel_timer()
        launches += nl
        tot_ms += ms
        long_n += nlong
        long_ms += lms
        P.set_kernel_timer(FF.FDD_KT_NONE)
    ni = (args.n - 1) ** 2
    elem = 4 if prec == F.FDD_MIXED else 8
    # working launches: those that did the update (the others returned at once after their PCG
    # run had converged): a run's counted iterations plus the one whose residual met the run's
    # tolerance, the first (k = 0) reading no p' and x; their algorithmic bytes over their own
    # time is the achieved rate
    alg_bytes = ni * elem / 4 * (DOWN0_BYTES_K * its + DOWN0_BYTES_K0 * runs)
    achieved = alg_bytes / (long_ms * 1e-3) / 1e9 if long_ms > 0 else 0.0
    traffic = traffic_from_profile(ROOT, args.nu) if prec == F.FDD_MIXED and args.n == 1024 else None
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": f"k_mg_down<float,{args.nu},true,32,true> (finest level, PCG update fused)",
                "launches": launches, "avg_launch_us": 1e3 * tot_ms / max(launches, 1),
                "working_launches": its + runs, "timed_long_launches": long_n,
                "avg_working_launch_us": 1e3 * long_ms / max(long_n, 1),
                "alg_bytes_per_working_launch": alg_bytes / max(its + runs, 1)}
    # parity spot-check of one solve of the first cases against the separable oracle
    leg = OracleLeg()
    errs = [None] * min(3, len(probs))
    for ci in range(len(errs)):
        P, TP, TH, b, x, K, mu = probs[ci]
        P.solve(TP, TH, b, x, opts)
        leg.check(errs, ci, args.n, K, mu, b, x)
    batched = {}
    if args.batched in ("all", "1024"):
        batched["batched_1024"] = run_batched(F, args, "32 instances, n=1024",
                                              workloads.batch_instances(count=32, seed=4, sizes=[1024]), 1e-12, 64,
                                              leg)
    if args.batched in ("all", "c4"):
        batched["c4"] = run_batched(F, args, "256 instances, n in {64,...,512}",
                                    workloads.batch_instances(count=256, seed=4), 1e-8, 20, leg)
    out = {
        "metric": "Schur-PCG solves/s, 2D 1024^2 P1 @1e-8 (plain)",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 outer / f32 inner" if prec == F.FDD_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": f"2D unit square P1, n={args.n} ({args.n * (args.n - 1)} dofs), Gamma = top edge, "
                               f"(K, mu) cycling {len(case_list)} cases of the sweep, b ~ N(0,1), "
                               f"outer rtol {args.rtol}, inner rtol {args.inner_rtol}",
                   "n": args.n, "cases": len(case_list), "precision": args.precision},
        "outer_its": [s["outer"] for s in stats[: len(case_list)]],
        "inner_its": [s["inner"] for s in stats[: len(case_list)]],
        "rel_err_vs_oracle": errs,
        "roofline": roofline,
        "cpu_baseline": None,
    }
    out.update(batched)
    if args.learned == "auto":
        out["learned"] = run_learned(F, args, leg)
    if not args.no_3d:
        out["three_d"] = run_3d(F, args)
    # the oracle leg, after every GPU measurement: parity spot-checks and the CPU baseline
    leg.run()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, case_list)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
