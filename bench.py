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
                    help="red-black sweep pairs per level for the legs beside the headline")
    ap.add_argument("--headline-nu", type=int, default=0,
                    help="smoother depth of the headline; 0: chosen with the step tolerance by the "
                         "autotuner (paper_2211_15308_amd.autotune.tune_solves) during set-up")
    ap.add_argument("--inner-rtol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--cpu-pf-n", type=int, default=256,
                    help="n of the paper-faithful CPU solver (sparse-LU Schur PCG) in the CPU baseline; 0: skip")
    ap.add_argument("--cpu-only", action="store_true",
                    help="only the CPU baselines (no GPU work): the DST and paper-faithful oracle solvers")
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
    ap.add_argument("--model", choices=["auto", "none", "only"], default="auto",
                    help="the paper's own model problem (Gamma = the whole boundary) beside the headline")
    ap.add_argument("--hdiv", choices=["auto", "none", "only"], default="auto",
                    help="the H(div) variant (eq. (graddiv), BDM1) beside the headline")
    ap.add_argument("--ds", choices=["auto", "none", "only"], default="auto",
                    help="the Darcy-Stokes outer solver (eq. (darcy_stokes), FGMRES) beside the headline")
    ap.add_argument("--ds-n", type=int, default=0,
                    help="Darcy-Stokes leg at this n only (the first (K, mu) case, no count sweep or "
                         "oracle checks): for profiling")
    ap.add_argument("--full-lazy", choices=["auto", "none", "only"], default="auto",
                    help="the full-system PCG with the lazy block preconditioner beside the headline")
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


SEEDS_PER_CASE = 3


def calibration_seed(ci):
    """Right-hand side of case ci solved during set-up only (never timed)."""
    return 1000 + ci


def timed_seed(ci, k):
    """The k-th timed right-hand side of case ci."""
    return 1100 + SEEDS_PER_CASE * ci + k


def host_info():
    """The host the CPU numbers were taken on: usable cores, CPU model, BLAS/FFT thread settings."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cores_available": len(os.sched_getaffinity(0)), "cpu_model": model,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def cpu_dst_rate(n, cases, seconds):
    """Solves/s of the oracle's separable sine-transform solver over a bounded sample of cases
    [(K, mu, seed)] (scipy.fft single-threaded by default; banded solves sequential: one core)."""
    import workloads
    from oracle import system
    t0 = time.perf_counter()
    done = 0
    while time.perf_counter() - t0 < seconds or done == 0:
        K, mu, seed = cases[done % len(cases)]
        system.solve_dst_2d(n, K, mu, workloads.rhs(2, n, seed))
        done += 1
    dt = time.perf_counter() - t0
    return done / dt, done, dt


def cpu_paper_faithful(n, K, mu, seed, rtol):
    """The paper's CPU solver shape: Schur-complement PCG (FP64, x0 = 0) with the interior block
    factorized once by sparse LU (SuperLU, one thread) and the rational preconditioner of eq. (RA)
    (the oracle's own AAA table to 1e-12 on the exact spectrum) applied by banded solves.
    Assembly and factorization are reported apart from the solve."""
    import numpy as np

    import workloads
    from oracle import aaa, ra, spectral, system
    t0 = time.perf_counter()
    R = system.Riesz(2, n, K, mu)
    lam = spectral.interface_eigs_1d(n)
    c0, c, p = aaa.ra_table(spectral.f_precond(K, 1.0 / mu), lam[0], lam[-1], tol=1e-12, extra=lam)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    R.interior_lu()
    t_fact = time.perf_counter() - t0
    L, M = R.P.A_G, R.P.M_G
    b = workloads.rhs(2, n, seed)
    t0 = time.perf_counter()
    x, its, _ = R.schur_pcg(b, precond=lambda r: ra.apply_tridiagonal(L, M, c0, c, p, r), rtol=rtol)
    t_solve = time.perf_counter() - t0
    err = float(np.linalg.norm(x - system.solve_dst_2d(n, K, mu, b)) / np.linalg.norm(x))
    return {"n": n, "K": K, "mu": mu, "solves_per_s": 1.0 / t_solve, "solve_s": t_solve,
            "factorization_s": t_fact, "assembly_gevp_and_table_s": t_setup, "outer_its": its,
            "poles": len(p), "rel_err_vs_separable": err, "threads": 1}


def cpu_baseline(args, dst_cases, pf_case):
    """The oracle timed on this host on bounded samples of the headline workload.

    value: the oracle's separable sine-transform solver (exact, O(n^2 log n)) at the headline n,
    one core.  Beside it the paper-faithful solver (sparse-LU Schur PCG with the same RA poles)
    on one case at n = args.cpu_pf_n (its element-by-element assembly and factorization at
    n = 1024 take minutes, so the default run uses a smaller n; the n = 1024 figure is recorded
    separately by --cpu-only --cpu-pf-n 1024).
    """
    rate, done, dt = cpu_dst_rate(args.n, dst_cases, args.cpu_seconds)
    out = {"value": rate, "unit": "solves/s", "cores": 1, "kind": "oracle",
           "sample": f"{done} solves of the 2D n={args.n} problem by the oracle's separable "
                     f"sine-transform solver (FP64, numpy/scipy, one thread), cycling the timed "
                     f"(K, mu, seed) cases, {dt:.1f} s",
           "host": host_info()}
    if args.cpu_pf_n:
        K, mu, seed = pf_case
        out["paper_faithful"] = cpu_paper_faithful(args.cpu_pf_n, K, mu, seed, args.rtol)
    return out


def cpu_instances(cases, seconds):
    """Instance solves/s of the oracle's separable solver over a bounded sample of batch instances."""
    import workloads
    from oracle import system
    t0 = time.perf_counter()
    done = 0
    while time.perf_counter() - t0 < seconds or done == 0:
        c = cases[done % len(cases)]
        system.solve_dst_2d(c["n"], c["K"], c["mu"], workloads.rhs(2, c["n"], c["seed"]))
        done += 1
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "instance solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} instance solves by the oracle's separable sine-transform solver "
                      f"(one thread), cycling the batch's instances, {dt:.1f} s"}


def cpu_3d(n, K, mu, seed):
    """One 3D solve by the oracle's sparse LU of the full system (SuperLU, one thread)."""
    import workloads
    from oracle import system
    t0 = time.perf_counter()
    R = system.Riesz(3, n, K, mu)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    R.solve_splu(workloads.rhs(3, n, seed))
    dt = time.perf_counter() - t0
    return {"n": n, "K": K, "mu": mu, "solves_per_s": 1.0 / dt, "kind": "oracle sparse LU of the full system",
            "assembly_and_gevp_s": t_setup, "cores": 1}


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


def batched_traffic_from_profile(root, nu):
    """HBM bytes per working launch of the batched finest down kernel (32 x 1024^2 batch) from the
    committed PMC record, if it matches the current kernel sources."""
    path = os.path.join(root, "profiles", "kb_down0_traffic.json")
    try:
        rec = json.load(open(path))
        sha = kernel_source_sha(root, ("kernels_batch.hip", "mg_device.h", "fdd_internal.h"))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sources_sha256") != sha or rec.get("kernel") != f"void fdd::kb_mg_down<{nu}, true, 32>":
        return None
    return rec


def kernel_source_sha(root, names=("kernels_mg.hip", "mg_device.h", "fdd_internal.h")):
    """sha256 over the sources a kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for name in names:
        h.update(open(os.path.join(root, "paper_2211_15308_amd", "csrc", name), "rb").read())
    return h.hexdigest()


class OracleLeg:
    """The benchmark's use of the oracle, in one place after the GPU legs: the CPU baseline (timed
    by cpu_baseline) and the parity spot-checks of GPU solutions.  The GPU legs only copy the
    right-hand side and solution to the host and name the slot (a dict key or list index of the
    output) that receives the relative error; run() fills the slots."""

    def __init__(self):
        self.items = []
        self.jobs = []

    def check(self, slot, key, n, K, mu, b, x):
        self.items.append((slot, key, n, K, mu, b.detach().cpu().numpy(), x.detach().cpu().numpy()))

    def defer(self, slot, key, fn):
        """slot[key] = fn() when the leg runs (CPU timings of the oracle beside a GPU leg)."""
        self.jobs.append((slot, key, fn))

    def run(self):
        import numpy as np
        from oracle import system
        for slot, key, n, K, mu, b, x in self.items:
            xr = system.solve_dst_2d(n, K, mu, b)
            slot[key] = float(np.linalg.norm(x - xr) / np.linalg.norm(xr))
        self.items = []
        for slot, key, fn in self.jobs:
            slot[key] = fn()
        self.jobs = []


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
    res = {
        "label": label, "value": value, "unit": "instance solves/s", "instances": len(cases),
        "dofs": int(sum(c["n"] * (c["n"] - 1) for c in cases)), "ms_per_batch": 1e3 * el / args.batch_steps,
        "batches_timed": args.batch_steps, "setup_s": setup_s,
        "schedule": {"mg_nu": opts.mg_nu, "step_rtol": opts.step_rtol,
                     "mid_tile": tune["mid_tile"] if tune else 0, "tile_edges": B.tile_edges(),
                     "autotune_ms_per_batch": tune["ms_per_batch"] if tune else None},
        "outer_its_min_mean_max": [min(outer), float(np.mean(outer)), max(outer)],
        "poles_P_min_max": [min(i[1].query()["m"] for i in inst), max(i[1].query()["m"] for i in inst)],
        "rel_err_vs_oracle_first3": errs,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": f"kb_mg_down<{opts.mg_nu},true,32> (finest level of every instance, "
                               "PCG update fused)",
                     "alg_bytes_per_working_launch": alg / max(nlong, 1),
                     "launches": nl, "avg_launch_us": 1e3 * ms / max(nl, 1),
                     "alg_bytes_per_batch_solve": alg,
                     "working_set_MB": sum(i[0].workspace_bytes() + 16 * i[0].N for i in inst) / 1e6},
        "cpu_baseline": None,
    }
    tr = batched_traffic_from_profile(ROOT, opts.mg_nu) if label.startswith("32 instances") else None
    if tr:
        # measured HBM bytes of a working launch (FETCH_SIZE and WRITE_SIZE, scaled by a copy)
        res["roofline"]["traffic"] = tr["traffic_bytes_per_launch"]
    leg.defer(res, "cpu_baseline", lambda: cpu_instances(cases, args.cpu_seconds / 4))
    return res


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
                opts = F.opts_default(outer_rtol=args.rtol, inner_rtol=args.inner_rtol, mg_nu=args.nu,
                                      check_true_residual=1)
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
            row["cpu_oracle_solves_per_s"] = None
            seed = 5000 + 10 * ci + n
            leg.defer(row, "cpu_oracle_solves_per_s",
                      lambda n=n, mu=mu, seed=seed: cpu_dst_rate(n, [(1.0, mu, seed)], 1.0)[0])
            res["cases"].append(row)
    # batched form: 8 instances of one n (K = 1, mu alternating), plain vs one batched forward
    # pass per outer iteration
    res["batched"] = []
    for n in sizes:
        count = 8
        net = F.Cnn(count, n)
        net.set_params(theta)
        probs, TPs, THs, bs = [], [], [], []
        for i in range(count):
            mu = mus[i % len(mus)]
            P = F.setup_mesh(n, 1.0, mu)
            P.bind_workspace()
            probs.append(P)
            TPs.append(P.build_rational_pc(F.FDD_RA_PRECOND, 1e-12))
            THs.append(P.build_rational_pc(F.FDD_RA_OPERATOR, 1e-12))
            bs.append(torch.as_tensor(workloads.rhs(2, n, 5500 + 10 * i + n), dtype=torch.float64, device="cuda"))
        B = F.Batch(probs, TPs, THs)
        row = {"n": n, "instances": count, "K": 1.0, "mu": list(mus)}
        for label, ws in (("plain", None), ("learned", net.h.value)):
            opts = F.opts_default(outer_rtol=args.rtol, inner_rtol=args.inner_rtol, mg_nu=args.nu)
            opts.warmstart = ws
            xs = [torch.zeros_like(b) for b in bs]
            for _ in range(2):
                st = B.solve(bs, xs, opts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.batch_steps):
                st = B.solve(bs, xs, opts)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            row[label] = {"instance_solves_per_s": count * args.batch_steps / el,
                          "inner_its_mean": sum(s_["inner_its_total"] for s_ in st) / count,
                          "outer_its_mean": sum(s_["outer_its"] for s_ in st) / count,
                          "warm_accepted": sum(s_["warm_accepted"] for s_ in st),
                          "warm_starts": sum(s_["warm_starts"] for s_ in st),
                          "rel_err_vs_oracle_first": None}
            leg.check(row[label], "rel_err_vs_oracle_first", n, 1.0, mus[0], bs[0], xs[0])
        res["batched"].append(row)
    return res


def run_full_lazy(F, args, leg, n=1024, reps=2):
    """Full-system PCG with the lazy block preconditioner (one V-cycle for the leading block, H and
    S_Gamma^{-1} by RA) on the headline's 12 (K, mu) cases: solves/s, PCG counts and parity
    against the separable oracle, FP32 and FP64 V-cycles, same outer rtol.  Each case is solved
    once untimed, then `reps` times on timed right-hand sides."""
    import torch

    import workloads
    res = {"n": n, "rtol": args.rtol, "mg_nu": args.nu, "variants": {}}
    case_list = cases(args)
    probs = []
    for ci, (K, mu) in enumerate(case_list):
        P = F.setup_mesh(n, K, mu)
        P.bind_workspace()
        TP = P.build_rational_pc(F.FDD_RA_PRECOND, 1e-12)
        TH = P.build_rational_pc(F.FDD_RA_OPERATOR, 1e-12)
        bs = [torch.as_tensor(workloads.rhs(2, n, timed_seed(ci, k)), dtype=torch.float64, device="cuda")
              for k in range(reps)]
        b_cal = torch.as_tensor(workloads.rhs(2, n, calibration_seed(ci)), dtype=torch.float64, device="cuda")
        probs.append((P, TP, TH, b_cal, bs, K, mu))
    for label, prec in (("fp32_vcycles", F.FDD_MIXED), ("fp64_vcycles", F.FDD_FP64)):
        opts = F.opts_default(outer_rtol=args.rtol, precision=prec, mg_nu=args.nu, outer_maxit=200,
                              check_true_residual=1)
        for P, TP, TH, b_cal, bs, K, mu in probs:
            P.solve_full(TP, TH, b_cal, torch.zeros_like(b_cal), opts)
        torch.cuda.synchronize()
        rows = []
        t0 = time.perf_counter()
        for k in range(reps):
            for P, TP, TH, b_cal, bs, K, mu in probs:
                x = torch.zeros_like(bs[k])
                st = P.solve_full(TP, TH, bs[k], x, opts)
                rows.append({"K": K, "mu": mu, "its": st["outer_its"], "true_rel_res": st["true_rel_res"], "x": x,
                             "b": bs[k]})
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        v = {"solves_per_s": len(rows) / el, "ms_per_solve": 1e3 * el / len(rows),
             "its_min_mean_max": [min(r["its"] for r in rows), sum(r["its"] for r in rows) / len(rows),
                                  max(r["its"] for r in rows)],
             "true_rel_res_max": max(r["true_rel_res"] for r in rows),
             "rel_err_vs_oracle_first3": [None] * 3}
        for q in range(3):
            r = rows[q]
            leg.check(v["rel_err_vs_oracle_first3"], q, n, r["K"], r["mu"], r["b"], r["x"])
        res["variants"][label] = v
    return res


def run_model(F, args, leg, n=1024, reps=2, ts=(-0.5, 0.5), gammas=(1.0, 1e3)):
    """The paper's own model problem (Gamma = the whole boundary, K(-Delta + I) + gamma
    (-Delta_Gamma + I)^t), K = 1: solves/s, outer and inner counts and true residuals at n, rtol
    1e-8 (FP32 V-cycles inside FP64 PCG); parity spot-checks at n = 128 against the oracle's
    sparse solve, and the oracle's Schur PCG (sparse LU interior solves) timed at n = 128."""
    import numpy as np
    import torch

    res = {"n": n, "K": 1.0, "rtol": args.rtol, "cases": []}
    for t in ts:
        for g in gammas:
            P = F.setup_model(n, 1.0, g, t)
            P.bind_workspace()
            TP = P.build_rational_pc(F.FDD_RA_PRECOND, 1e-12)
            TH = P.build_rational_pc(F.FDD_RA_OPERATOR, 1e-12)
            opts = F.opts_default(outer_rtol=args.rtol, inner_rtol=args.inner_rtol, mg_nu=args.nu,
                                  check_true_residual=1)
            bs = [torch.as_tensor(np.random.default_rng(7000 + k).standard_normal(P.N), dtype=torch.float64,
                                  device="cuda") for k in range(reps + 1)]
            x = torch.zeros_like(bs[0])
            P.solve(TP, TH, bs[reps], x, opts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sts = [P.solve(TP, TH, bs[k], x, opts) for k in range(reps)]
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            row = {"t": t, "gamma": g, "solves_per_s": reps / el, "outer_its": sts[-1]["outer_its"],
                   "inner_its": sts[-1]["inner_its_total"],
                   "true_rel_res_max": max(s_["true_rel_res"] for s_ in sts)}
            # parity spot-check at n = 128 (the oracle assembles and factors that size in seconds)
            Q = F.setup_model(128, 1.0, g, t)
            Q.bind_workspace()
            QP = Q.build_rational_pc(F.FDD_RA_PRECOND, 1e-12)
            QH = Q.build_rational_pc(F.FDD_RA_OPERATOR, 1e-12)
            bq = torch.as_tensor(np.random.default_rng(7100).standard_normal(Q.N), dtype=torch.float64, device="cuda")
            xq = torch.zeros_like(bq)
            stq = Q.solve(QP, QH, bq, xq, F.opts_default(outer_rtol=1e-10, inner_rtol=1e-12))
            row["n128_outer_its"] = stq["outer_its"]
            row["n128_rel_err_vs_oracle"] = None
            bh, xh = bq.cpu().numpy(), xq.cpu().numpy()

            def parity(t=t, g=g, bh=bh, xh=xh):
                from oracle import model
                M = model.ModelProblem(128, 1.0, g, t)
                xr = M.solve_splu(bh)
                return float(np.linalg.norm(xh - xr) / np.linalg.norm(xr))
            leg.defer(row, "n128_rel_err_vs_oracle", parity)
            res["cases"].append(row)

    def cpu_rate():
        from oracle import model
        M = model.ModelProblem(128, 1.0, 1.0, -0.5)
        b = np.random.default_rng(7200).standard_normal(M.N)
        t0 = time.perf_counter()
        M.interior_lu()
        t_fact = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, its = M.schur_pcg(b, rtol=args.rtol)
        return {"n": 128, "t": -0.5, "gamma": 1.0, "solves_per_s": 1.0 / (time.perf_counter() - t0),
                "factorization_s": t_fact, "outer_its": its, "kind": "oracle Schur PCG, sparse LU interior, exact S_Gamma",
                "cores": 1}
    res["cpu_baseline"] = None
    leg.defer(res, "cpu_baseline", cpu_rate)
    return res


def run_hdiv(F, args, leg, n=512, reps=2, gammas=(1e-3, 1.0, 1e3), robust_sizes=(64, 128, 256, 512)):
    """The H(div) variant (Sec. 3 remark, eq. (graddiv); BDM1, Gamma = the whole boundary), K = 1,
    outer rtol 1e-10, inner 1e-12:
    solves/s at n (6n^2 + 4n dofs) per gamma with outer/inner counts and true residuals, the outer
    counts over n (the robustness of Fig. 4, right), parity spot-checks at n = 64 against the
    oracle's sparse LU, and the oracle's Schur PCG (sparse LU interior, exact S_Gamma) timed at
    n = 32.  FP64 throughout."""
    import numpy as np
    import torch

    # the paper's stop rule of Sec. 3: the preconditioned residual norm reduced by 1e10
    rtol, inner_rtol = 1e-10, 1e-12
    res = {"n": n, "K": 1.0, "rtol": rtol, "inner_rtol": inner_rtol, "cases": [], "outer_its_over_n": {}}
    for g in gammas:
        P = F.setup_hdiv(n, 1.0, g)
        P.bind_workspace()
        TP = P.build_rational_pc(F.FDD_RA_PRECOND, 1e-12)
        opts = F.opts_default(outer_rtol=rtol, inner_rtol=inner_rtol, check_true_residual=1)
        bs = [torch.as_tensor(np.random.default_rng(8000 + k).standard_normal(P.N), dtype=torch.float64,
                              device="cuda") for k in range(reps + 1)]
        x = torch.zeros_like(bs[0])
        P.solve(TP, None, bs[reps], x, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = [P.solve(TP, None, bs[k], x, opts) for k in range(reps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        row = {"gamma": g, "dofs": P.N, "solves_per_s": reps / el, "outer_its": sts[-1]["outer_its"],
               "inner_its": sts[-1]["inner_its_total"], "poles_P": TP.query()["m"],
               "true_rel_res_max": max(s_["true_rel_res"] for s_ in sts)}
        # parity spot-check at n = 64
        Q = F.setup_hdiv(64, 1.0, g)
        Q.bind_workspace()
        QP = Q.build_rational_pc(F.FDD_RA_PRECOND, 1e-12)
        bq = torch.as_tensor(np.random.default_rng(8100).standard_normal(Q.N), dtype=torch.float64, device="cuda")
        xq = torch.zeros_like(bq)
        Q.solve(QP, None, bq, xq, F.opts_default(outer_rtol=1e-10, inner_rtol=1e-12))
        row["n64_rel_err_vs_oracle"] = None
        bh, xh = bq.cpu().numpy(), xq.cpu().numpy()

        def parity(g=g, bh=bh, xh=xh):
            from oracle import hdiv
            xr = hdiv.HdivProblem(64, 1.0, g).solve_splu(bh)
            return float(np.linalg.norm(xh - xr) / np.linalg.norm(xr))
        leg.defer(row, "n64_rel_err_vs_oracle", parity)
        res["cases"].append(row)
        progress(f"H(div) n={n} gamma={g:g}: {row['solves_per_s']:.1f} solves/s, outer {row['outer_its']}")
        counts = []
        for m in robust_sizes:
            R = F.setup_hdiv(m, 1.0, g)
            R.bind_workspace()
            RP = R.build_rational_pc(F.FDD_RA_PRECOND, 1e-12)
            br = torch.as_tensor(np.random.default_rng(8200 + m).standard_normal(R.N), dtype=torch.float64,
                                 device="cuda")
            counts.append(R.solve(RP, None, br, torch.zeros_like(br), opts)["outer_its"])
        res["outer_its_over_n"][f"gamma={g:g}"] = dict(zip([str(m) for m in robust_sizes], counts))

    def cpu_rate():
        from oracle import hdiv
        M = hdiv.HdivProblem(32, 1.0, 1.0)
        b = np.random.default_rng(8300).standard_normal(M.N)
        t0 = time.perf_counter()
        M.interior_lu()
        t_fact = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, its = M.schur_pcg(b, rtol=rtol)
        return {"n": 32, "gamma": 1.0, "solves_per_s": 1.0 / (time.perf_counter() - t0),
                "factorization_s": t_fact, "outer_its": its,
                "kind": "oracle Schur PCG, sparse LU interior, exact S_Gamma", "cores": 1}
    res["cpu_baseline"] = None
    leg.defer(res, "cpu_baseline", cpu_rate)
    return res


def run_darcy_stokes(F, args, leg, sizes=(256, 512), reps=2, params=((1e-2, 1e-4), (1.0, 1.0)),
                     alpha=3.0, robust_sizes=(64, 128, 256)):
    """The Darcy-Stokes outer solver (Sec. 4 eq. (darcy_stokes), eq. (darcy_stokes_precond);
    Appendix): FGMRES to rtol 1e-10 with the block-diagonal preconditioner.  Appendix setting:
    velocity and pressure blocks to 1e-12 (velocity PCG with a nu = 1 V-cycle, pressure mass by
    Chebyshev), the Darcy block by the lazy PCG to 1e-5; Sec. 4 setting: one V-cycle for the Stokes
    blocks (one nu = 2 velocity V-cycle, the pressure mass to 1e-3, eight Chebyshev steps), Darcy
    PCG to 1e-4 with FP32 V-cycles; alpha = 3.  Solves/s per size and (K, mu) with FGMRES and inner counts and true
    residuals, FGMRES counts over n (Fig. 6), a parity spot-check at n = 32 against the oracle's
    sparse LU, and the oracle's FGMRES (sparse LU for the Stokes blocks and the Riesz map) timed at
    n = 32.  FP64 throughout."""
    import numpy as np
    import torch

    rtol = 1e-10
    res = {"alpha": alpha, "rtol": rtol, "cases": [], "its_over_n": {}}
    if args.ds_n:
        sizes, params, robust_sizes = (args.ds_n,), params[:1], ()

    def problem(n, K, mu):
        P = F.setup_darcy_stokes(n, K, mu, alpha, krylov=200)
        P.bind_workspace()
        return P, P.build_rational_pc(F.FDD_RA_PRECOND, 1e-12), P.build_rational_pc(F.FDD_RA_OPERATOR, 1e-12)

    settings = (("appendix", F.ds_opts_default(rtol=rtol)),
                ("sec4", F.ds_opts_default(rtol=rtol, velocity_rtol=0.0, darcy_rtol=1e-4, mg_nu=2,
                                           pressure_rtol=1e-3, darcy_precision=F.FDD_MIXED)))
    for n in sizes:
        for K, mu in (params if n == sizes[0] else params[:1]):
            P, TP, TH = problem(n, K, mu)
            bs = [torch.as_tensor(np.random.default_rng(9000 + k).standard_normal(P.N), dtype=torch.float64,
                                  device="cuda") for k in range(reps + 1)]
            x = torch.zeros_like(bs[0])
            for name, o in settings:
                P.solve(TP, TH, bs[reps], x, o)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sts = [P.solve(TP, TH, bs[k], x, o) for k in range(reps)]
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                row = {"n": n, "K": K, "mu": mu, "setting": name, "dofs": P.N, "solves_per_s": reps / el,
                       "ms_per_solve": 1e3 * el / reps, "fgmres_its": sts[-1]["its"],
                       "velocity_its_total": sts[-1]["velocity_its_total"],
                       "pressure_its_total": sts[-1]["pressure_its_total"],
                       "darcy_its_total": sts[-1]["darcy_its_total"],
                       "true_rel_res_max": max(s_["true_rel_res"] for s_ in sts)}
                res["cases"].append(row)
                progress(f"Darcy-Stokes n={n} K={K:g} mu={mu:g} {name}: {row['solves_per_s']:.2f} solves/s, "
                         f"FGMRES {row['fgmres_its']}")
            del P
    for K, mu in params:
        counts = []
        for m in robust_sizes:
            P, TP, TH = problem(m, K, mu)
            b = torch.as_tensor(np.random.default_rng(9100 + m).standard_normal(P.N), dtype=torch.float64,
                                device="cuda")
            counts.append(P.solve(TP, TH, b, torch.zeros_like(b), settings[0][1])["its"])
        res["its_over_n"][f"K={K:g},mu={mu:g}"] = dict(zip([str(m) for m in robust_sizes], counts))
    if args.ds_n:
        return res
    # parity spot-check at n = 32
    K, mu = params[0]
    Q, QP, QH = problem(32, K, mu)
    bq = torch.as_tensor(np.random.default_rng(9200).standard_normal(Q.N), dtype=torch.float64, device="cuda")
    xq = torch.zeros_like(bq)
    Q.solve(QP, QH, bq, xq, settings[0][1])
    res["n32_rel_err_vs_oracle"] = None
    bh, xh = bq.cpu().numpy(), xq.cpu().numpy()

    def parity(bh=bh, xh=xh):
        from oracle import darcy_stokes
        xr = darcy_stokes.DarcyStokes(32, K, mu, alpha).solve_splu(bh)
        return float(np.linalg.norm(xh - xr) / np.linalg.norm(xr))
    leg.defer(res, "n32_rel_err_vs_oracle", parity)

    def cpu_rate():
        from oracle import darcy_stokes
        O = darcy_stokes.DarcyStokes(32, K, mu, alpha)
        b = np.random.default_rng(9300).standard_normal(O.N)
        t0 = time.perf_counter()
        B = O.precond_exact()
        t_fact = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, its, _ = darcy_stokes.fgmres(lambda v: O.A @ v, b, B, rtol=rtol, maxit=300)
        return {"n": 32, "K": K, "mu": mu, "solves_per_s": 1.0 / (time.perf_counter() - t0),
                "factorization_s": t_fact, "fgmres_its": its,
                "kind": "oracle FGMRES, sparse LU Stokes blocks and Riesz map", "cores": 1}
    res["cpu_baseline"] = None
    leg.defer(res, "cpu_baseline", cpu_rate)
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


def run_3d(F, args, leg, sizes=(32, 64, 128), mus=(1e-4, 1.0, 1e2), reps=2):
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
            if n == sizes[0] and ci == 0:
                out[-1]["cpu_baseline"] = None
                leg.defer(out[-1], "cpu_baseline", lambda n=n, mu=mu, seed=3000 + len(out) - 1: cpu_3d(n, 1.0, mu, seed))
            else:
                out[-1]["cpu_baseline"] = "not run: the oracle's sparse LU takes minutes beyond n = 32"
    return out


def progress(msg):
    """One line per finished step on stderr (the JSON result alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver and this benchmark run on one GPU only; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.cpu_only:
        case_list = cases(args)
        dst_cases = [(K, mu, timed_seed(ci, k)) for k in range(SEEDS_PER_CASE) for ci, (K, mu) in enumerate(case_list)]
        print(json.dumps({"cpu_baseline": cpu_baseline(args, dst_cases, (case_list[0][0], case_list[0][1],
                                                                         timed_seed(0, 0)))}))
        return
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
        leg = OracleLeg()
        res = run_3d(F, args, leg)
        if not args.no_cpu_baseline:
            leg.run()
        print(json.dumps({"three_d": res}))
        return
    if args.sweep:
        leg = OracleLeg()
        res = run_sweep(F, args, leg)
        leg.run()
        print(json.dumps({"sweep": res}))
        return
    if args.model == "only":
        leg = OracleLeg()
        res = run_model(F, args, leg)
        leg.run()
        print(json.dumps({"model_problem": res}))
        return
    if args.hdiv == "only":
        leg = OracleLeg()
        res = run_hdiv(F, args, leg)
        leg.run()
        print(json.dumps({"hdiv": res}))
        return
    if args.ds == "only":
        leg = OracleLeg()
        res = run_darcy_stokes(F, args, leg)
        leg.run()
        print(json.dumps({"darcy_stokes": res}))
        return
    if args.full_lazy == "only":
        leg = OracleLeg()
        res = run_full_lazy(F, args, leg)
        leg.run()
        print(json.dumps({"full_lazy": res}))
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
        if args.pmc_mode:
            # calibration copy of known size (256 MiB), then the 1024^2 batch once, untuned
            src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
            torch.empty_like(src).copy_(src)
            torch.cuda.synchronize()
            args.batch_steps, args.no_autotune, args.batched = 1, True, "1024"
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
    # set-up (not timed as solves, reported as setup_s): mesh plans, rational tables, workspaces,
    # and for every case two solves of a right-hand side that is never timed (the first measures
    # the launch schedule, the second captures the outer-iteration graphs)
    t_setup = time.perf_counter()
    probs = []
    for ci, (K, mu) in enumerate(case_list):
        P = F.setup_mesh(args.n, K, mu)
        P.bind_workspace()
        TP = P.build_rational_pc(F.FDD_RA_PRECOND, 1e-12)
        TH = P.build_rational_pc(F.FDD_RA_OPERATOR, 1e-12)
        b_cal = torch.as_tensor(workloads.rhs(2, args.n, calibration_seed(ci)), dtype=torch.float64, device=dev)
        bs = [torch.as_tensor(workloads.rhs(2, args.n, timed_seed(ci, k)), dtype=torch.float64, device=dev)
              for k in range(SEEDS_PER_CASE)]
        x = torch.zeros_like(b_cal)
        probs.append((P, TP, TH, bs, x, K, mu, b_cal))
    tune = None
    if args.headline_nu == 0 and not args.pmc_mode:
        # the smoother depth and per-step reduction: timed on the calibration right-hand sides
        from paper_2211_15308_amd import autotune
        opts, tune = autotune.tune_solves([(P, TP, TH, b_cal, x) for P, TP, TH, bs, x, K, mu, b_cal in probs],
                                          opts, reps=1)
    elif args.headline_nu:
        opts.mg_nu = args.headline_nu
    for P, TP, TH, bs, x, K, mu, b_cal in probs:
        for _ in range(2):
            P.solve(TP, TH, b_cal, x, opts)
    probs = [q[:7] for q in probs]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    progress(f"headline set-up done ({setup_s:.1f} s, mg_nu {opts.mg_nu}, step_rtol {opts.step_rtol:g})")

    def step_case(s):
        ci = s % len(probs)
        k = (s // len(probs)) % SEEDS_PER_CASE
        return ci, k

    # one step = one complete solve: rhs reduction, outer PCG, back-substitution and the true
    # residual ||b - A x|| / ||b|| (check_true_residual = 1)
    opts.check_true_residual = 1
    stats = []
    for s in range(args.warmup):
        ci, k = step_case(s)
        P, TP, TH, bs, x, K, mu = probs[ci]
        P.solve(TP, TH, bs[k], x, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.warmup, args.warmup + args.steps):
        ci, k = step_case(s)
        P, TP, TH, bs, x, K, mu = probs[ci]
        st = P.solve(TP, TH, bs[k], x, opts)
        stats.append(dict(K=K, mu=mu, seed=timed_seed(ci, k), outer=st["outer_its"], inner=st["inner_its_total"],
                          refine=st["refine_steps"], res=st["true_rel_res"], ms=st["t_solve_ms"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = args.steps / elapsed
    progress(f"headline timed: {value:.1f} solves/s")
    if args.pmc_mode:
        print(json.dumps({"pmc_mode": True, "steps": args.steps}))
        return
    # roofline of the dominant kernel (the finest-level down kernel with the PCG update):
    # the same steps again, with a HIP event pair attached to every launch of it
    import paper_2211_15308_amd.fdd as FF
    for P, *_ in probs:
        P.set_kernel_timer(FF.FDD_KT_DOWN0)
    its = runs = 0
    for s in range(args.warmup, args.warmup + args.steps):
        ci, k = step_case(s)
        P, TP, TH, bs, x, K, mu = probs[ci]
        st = P.solve(TP, TH, bs[k], x, opts)
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
    traffic = traffic_from_profile(ROOT, opts.mg_nu) if prec == F.FDD_MIXED and args.n == 1024 else None
    ws_mb = (probs[0][0].workspace_bytes() + 2 * 8 * probs[0][0].N) / 1e6
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": f"k_mg_down<float,{opts.mg_nu},true,32,true> (finest level, PCG update fused)",
                "launches": launches, "avg_launch_us": 1e3 * tot_ms / max(launches, 1),
                "working_launches": its + runs, "timed_long_launches": long_n,
                "avg_working_launch_us": 1e3 * long_ms / max(long_n, 1),
                "alg_bytes_per_working_launch": alg_bytes / max(its + runs, 1),
                "working_set_MB": ws_mb,
                "cache_note": (f"one instance's working set ({ws_mb:.0f} MB) fits the 256 MB Infinity Cache, so "
                               "part of this kernel's traffic may be served from it; the batched roofline "
                               "(batched_1024, ~32x larger working set) is the one measured beyond it")}
    # parity spot-check of one solve of the first cases against the separable oracle
    leg = OracleLeg()
    errs = [None] * min(3, len(probs))
    for ci in range(len(errs)):
        P, TP, TH, bs, x, K, mu = probs[ci]
        P.solve(TP, TH, bs[0], x, opts)
        leg.check(errs, ci, args.n, K, mu, bs[0], x)
    batched = {}
    if args.batched in ("all", "1024"):
        progress("batched 32 x 1024^2")
        batched["batched_1024"] = run_batched(F, args, "32 instances, n=1024",
                                              workloads.batch_instances(count=32, seed=4, sizes=[1024]), 1e-12, 64,
                                              leg)
    if args.batched in ("all", "c4"):
        progress("batched 256 instances n <= 512")
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
        "setup_s": setup_s,
        "schedule": {"mg_nu": opts.mg_nu, "step_rtol": opts.step_rtol,
                     "autotune_ms_per_solve": tune["ms_per_solve"] if tune else None},
        "timed_solves": [dict(K=s_["K"], mu=s_["mu"], seed=s_["seed"], outer_its=s_["outer"],
                              inner_its=s_["inner"], true_rel_res=s_["res"]) for s_ in stats],
        "true_rel_res_max": max(s_["res"] for s_ in stats),
        "rel_err_vs_oracle": errs,
        "roofline": roofline,
        "cpu_baseline": None,
    }
    out.update(batched)
    if args.full_lazy == "auto":
        progress("full-system lazy PCG")
        out["full_lazy"] = run_full_lazy(F, args, leg)
    if args.model == "auto":
        progress("model problem")
        out["model_problem"] = run_model(F, args, leg)
    if args.hdiv == "auto":
        progress("H(div) variant")
        out["hdiv"] = run_hdiv(F, args, leg)
    if args.ds == "auto":
        progress("Darcy-Stokes")
        out["darcy_stokes"] = run_darcy_stokes(F, args, leg)
    if args.learned == "auto":
        progress("learned warm start")
        out["learned"] = run_learned(F, args, leg)
    if not args.no_3d:
        progress("3D")
        out["three_d"] = run_3d(F, args, leg)
    progress("oracle leg (parity spot-checks, CPU baselines)")
    # the oracle leg, after every GPU measurement: parity spot-checks and the CPU baseline
    leg.run()
    if not args.no_cpu_baseline:
        dst_cases = [(s_["K"], s_["mu"], s_["seed"]) for s_ in stats]
        out["cpu_baseline"] = cpu_baseline(args, dst_cases, (case_list[0][0], case_list[0][1], timed_seed(0, 0)))
    progress("done")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
