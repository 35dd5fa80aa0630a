"""Trains the warm-start network on the GPU with the library's own kernels.

Training pairs: interface traces t = sum_{k <= 64} a_k sin(k pi x), a_k ~ N(0, 1/k^2), scaled to
unit root-mean-square, and their discrete harmonic extensions E t (the interior solution of
A_II u = lift(t)) computed by the library's plain interior solver at n = 256.  Each pair gets
log10 K and log10 mu labels drawn log-uniformly (E does not depend on them; the channels only
label the trace distribution).  Loss: mean squared error over interior pixels; Adam.  The last
1/20 of the pairs is held out for validation.

Usage:
  python -m paper_2211_15308_amd.train_warmstart --pairs 20000 --epochs 4 --out weights.npz

Writes the FP32 parameter vector (library layout) and the loss history to an .npz file.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_OUT = os.path.join(HERE, "weights", "warmstart_n256.npz")


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--epochs", type=float, default=4.0)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--init-seed", type=int, default=6)
    ap.add_argument("--max-seconds", type=float, default=600.0, help="stop training after this long")
    ap.add_argument("--out", default=DEFAULT_OUT)
    return ap.parse_args(argv)


def make_pairs(F, n, count, seed, log=print):
    """(traces (count, n-1) float64, targets (count, (n-1)^2) float32, labels) on the device."""
    import torch

    import workloads
    _, tr = workloads.sine_series_traces(count, n, kmax=64, seed=seed)
    tr = tr / np.sqrt(np.mean(tr * tr, axis=1))[:, None]
    rng = np.random.default_rng(seed + 1)
    lk = rng.uniform(-4.0, 0.0, count)
    lmu = rng.uniform(-6.0, 2.0, count)
    P = F.setup_mesh(n, 1.0, 1.0)
    P.bind_workspace()
    opts = F.opts_default(inner_rtol=1e-10)
    T = torch.as_tensor(tr, dtype=torch.float64, device="cuda")
    Y = torch.empty((count, (n - 1) ** 2), dtype=torch.float32, device="cuda")
    f = torch.zeros((n - 1) ** 2, dtype=torch.float64, device="cuda")
    u = torch.empty_like(f)
    t0 = time.perf_counter()
    for k in range(count):
        f[(n - 2) * (n - 1):] = T[k]
        P.interior_solve(f, u, opts)
        Y[k] = u.float()
        if (k + 1) % 2000 == 0:
            log(f"  targets {k + 1}/{count} ({time.perf_counter() - t0:.1f} s)")
    return T, Y, torch.as_tensor(lk, device="cuda"), torch.as_tensor(lmu, device="cuda")


def train(args, log=print):
    import torch

    import paper_2211_15308_amd as F
    import workloads
    n, B = args.n, args.batch
    t0 = time.perf_counter()
    T, Y, LK, LMU = make_pairs(F, n, args.pairs, args.seed, log)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    log(f"[train] {args.pairs} pairs at n={n} in {t_data:.1f} s")
    nval = max(args.pairs // 20, B)
    ntr = args.pairs - nval
    theta = torch.as_tensor(F.pack_params(workloads.cnn_init(seed=args.init_seed)), dtype=torch.float32,
                            device="cuda")
    net = F.Cnn(B, n, train=True)
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    grad = torch.zeros_like(theta)
    out = torch.empty((B, (n - 1) ** 2), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(args.seed)
    steps = int(args.epochs * ntr / B)
    hist = []

    def validate():
        tot = 0.0
        for s in range(0, nval - B + 1, B):
            idx = torch.arange(ntr + s, ntr + s + B, device="cuda")
            net.forward(T[idx], LK[idx], LMU[idx], out, n, rescale=False)
            net.loss(out, Y[idx], n, loss)
            tot += loss.item()
        return tot / (nval // B)

    t1 = time.perf_counter()
    perm = torch.randperm(ntr, generator=gen, device="cuda")
    pos = 0
    done = 0
    run = 0.0
    for step in range(1, steps + 1):
        if pos + B > ntr:
            perm = torch.randperm(ntr, generator=gen, device="cuda")
            pos = 0
        idx = perm[pos:pos + B]
        pos += B
        lr = args.lr * 0.5 * (1.0 + np.cos(np.pi * (step - 1) / steps))  # cosine decay
        net.set_params(theta)
        net.forward(T[idx].contiguous(), LK[idx].contiguous(), LMU[idx].contiguous(), out, n, rescale=False)
        net.loss(out, Y[idx].contiguous(), n, loss)
        net.backward(B, n, grad)
        net.adam_step(theta, grad, m, v, float(lr), step)
        done = step
        if step % 250 == 0 or step == steps:
            run = loss.item()
            el = time.perf_counter() - t1
            hist.append((step, run, el))
            log(f"  step {step}/{steps} loss {run:.4e} ({el:.1f} s, {1e3 * el / step:.2f} ms/step)")
            if el > args.max_seconds:
                log("  time limit reached")
                break
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    net.set_params(theta)
    val = validate()
    log(f"[train] {done} steps in {t_train:.1f} s; validation loss {val:.4e}")
    meta = {"n": n, "pairs": args.pairs, "batch": B, "steps": done, "lr": args.lr, "seed": args.seed,
            "init_seed": args.init_seed, "train_seconds": t_train, "data_seconds": t_data,
            "ms_per_step": 1e3 * t_train / max(done, 1), "val_loss": val,
            "history": hist, "device": torch.cuda.get_device_name(0)}
    return theta.cpu().numpy(), meta


def main(argv=None):
    args = parse(argv)
    theta, meta = train(args, log=lambda s: print(s, flush=True))
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.savez(args.out, theta=theta, meta=json.dumps(meta))
    print(json.dumps({k: v for k, v in meta.items() if k != "history"}), flush=True)


def load_weights(path=DEFAULT_OUT):
    """(theta float32 numpy, meta dict) of a saved training run."""
    with np.load(path, allow_pickle=False) as z:
        return z["theta"], json.loads(str(z["meta"]))


if __name__ == "__main__":
    main()
