"""GPU parity of the warm-start network (fdd_cnn_*) against the oracle's FP64 network.

The GPU computes in BF16 (weights, activations, gradients between layers) with FP32
accumulation, the oracle in FP64 on the same BF16-rounded parameters: the tolerances (a few
percent, relative, over whole tensors) are those of BF16 rounding through six layers.  Inputs
are seeded (workloads.py); expected values come from oracle/cnn.py only.
"""
import numpy as np
import pytest

import workloads
from oracle import cnn

torch = pytest.importorskip("torch")
F = pytest.importorskip("paper_2211_15308_amd")

pytestmark = pytest.mark.gpu


def bf16_round(a):
    return torch.as_tensor(np.asarray(a), dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def setup(n, B, seed=0, train=True):
    params = workloads.cnn_init(seed=6)
    params = [(bf16_round(W), bf16_round(b)) for W, b in params]
    theta = torch.as_tensor(F.pack_params(params), dtype=torch.float32, device="cuda")
    net = F.Cnn(B, n, train=train)
    net.set_params(theta)
    rng = np.random.default_rng(seed)
    traces = rng.standard_normal((B, n - 1))
    lk = rng.uniform(-4, 0, B)
    lmu = rng.uniform(-6, 2, B)
    return params, theta, net, traces, lk, lmu


def oracle_inputs(traces, n, lk, lmu):
    s = np.sqrt(np.mean(traces ** 2, axis=1))
    X = cnn.features(traces / s[:, None], n, 10.0 ** lk, 10.0 ** lmu)
    return bf16_round(X), s


@pytest.mark.parametrize("n,B", [(40, 3), (70, 2)])
def test_forward_matches_oracle(n, B):
    # n - 1 = 39 and 69: ragged column tiles (32 + 7, 64 + 5) and a partial last row tile
    print(f"[cnn forward] n={n} B={B}", flush=True)
    params, theta, net, traces, lk, lmu = setup(n, B)
    out = torch.empty((B, (n - 1) ** 2), dtype=torch.float32, device="cuda")
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
    net.forward(d(traces), d(lk), d(lmu), out, n, rescale=True)
    got = out.cpu().numpy().astype(np.float64).reshape(B, n - 1, n - 1)
    X, s = oracle_inputs(traces, n, lk, lmu)
    ref, _ = cnn.forward(params, X)
    ref = ref * s[:, None, None]
    err = rel(got, ref)
    emax = float(np.abs(got - ref).max() / np.abs(ref).max())
    per = [rel(got[b], ref[b]) for b in range(B)]
    print(f"  rel err {err:.2e}  element max {emax:.2e}  per image {max(per):.2e}", flush=True)
    # about 3x the measured BF16 error through six layers (8.8e-3 relative, 1.0e-2 element-wise
    # against the largest output): a wrong tap or channel block shows in the element-wise bound
    assert err <= 2.5e-2 and emax <= 3e-2
    # per image, and the rescaling by the trace norm
    for b in range(B):
        assert per[b] <= 3e-2


def test_backward_matches_oracle_and_is_deterministic():
    n, B = 40, 3
    print("[cnn backward]", flush=True)
    params, theta, net, traces, lk, lmu = setup(n, B, seed=1)
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
    rng = np.random.default_rng(7)
    target = rng.standard_normal((B, n - 1, n - 1)) * 0.3
    out = torch.empty((B, (n - 1) ** 2), dtype=torch.float32, device="cuda")
    tgt = torch.as_tensor(target.reshape(B, -1), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    grads = []
    for rep in range(2):
        grad = torch.zeros(net.param_count, dtype=torch.float32, device="cuda")
        net.forward(d(traces), d(lk), d(lmu), out, n, rescale=False)
        net.loss(out, tgt, n, loss)
        net.backward(B, n, grad)
        torch.cuda.synchronize()
        grads.append(grad.cpu().numpy().astype(np.float64))
    assert np.array_equal(grads[0], grads[1])
    X, s = oracle_inputs(traces, n, lk, lmu)
    o_ref, cache = cnn.forward(params, X)
    l_ref, dout = cnn.mse(o_ref, target)
    g_ref = cnn.backward(params, cache, dout)
    print(f"  loss gpu {loss.item():.6e} oracle {l_ref:.6e}", flush=True)
    assert abs(loss.item() - l_ref) <= 2e-2 * l_ref
    got = F.unpack_params(grads[0])
    for k, ((gW, gb), (rW, rb)) in enumerate(zip(got, g_ref)):
        eW, eb = rel(gW, rW), rel(gb, rb)
        mW = float(np.abs(gW - rW).max() / np.abs(rW).max())
        print(f"  layer {k + 1}: dW rel err {eW:.2e} (element max {mW:.2e})  db rel err {eb:.2e}",
              flush=True)
        # about 3x the measured (at most 9.5e-4 relative, 1.3e-3 element-wise)
        assert eW <= 3e-3 and mW <= 4e-3 and eb <= 3e-3


def test_adam_matches_oracle_step():
    n, B = 16, 1
    params, theta, net, traces, lk, lmu = setup(n, B, train=True)
    rng = np.random.default_rng(3)
    g = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in params]
    gt = torch.as_tensor(F.pack_params(g), dtype=torch.float32, device="cuda")
    m = torch.zeros_like(gt)
    v = torch.zeros_like(gt)
    th = theta.clone()
    st = {}
    ref = params
    for step in (1, 2):
        net.adam_step(th, gt, m, v, 1e-3, step)
        ref = cnn.adam_step(ref, [(a.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for a, b in g], st, lr=1e-3)
    torch.cuda.synchronize()
    got = th.cpu().numpy().astype(np.float64)
    assert np.allclose(got, F.pack_params(ref), rtol=0, atol=1e-6)


def _lift(n, t):
    f = torch.zeros((n - 1) ** 2, dtype=torch.float64, device="cuda")
    f[(n - 2) * (n - 1):] = t
    return f


def test_training_on_device_lowers_the_loss():
    # a short run of the training loop on sine-series traces; targets from the plain solver
    n, B, steps = 32, 8, 150
    print("[cnn train]", flush=True)
    _, traces = workloads.sine_series_traces(32, n, kmax=16, seed=5)
    traces = traces / np.sqrt(np.mean(traces ** 2, axis=1))[:, None]
    P = F.setup_mesh(n, 1.0, 1.0)
    P.bind_workspace()
    opts = F.opts_default(inner_rtol=1e-10)
    T = torch.as_tensor(traces, dtype=torch.float64, device="cuda")
    Y = torch.zeros((len(traces), (n - 1) ** 2), dtype=torch.float64, device="cuda")
    for k in range(len(traces)):
        P.interior_solve(_lift(n, T[k]), Y[k], opts)
    Y32 = Y.float()
    params = workloads.cnn_init(seed=6)
    theta = torch.as_tensor(F.pack_params(params), dtype=torch.float32, device="cuda")
    net = F.Cnn(B, n, train=True)
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    grad = torch.zeros_like(theta)
    out = torch.empty((B, (n - 1) ** 2), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    lk = torch.zeros(B, dtype=torch.float64, device="cuda")
    losses = []
    for step in range(1, steps + 1):
        idx = torch.arange((step - 1) * B, step * B, device="cuda") % len(traces)
        net.set_params(theta)
        net.forward(T[idx].contiguous(), lk, lk, out, n, rescale=False)
        net.loss(out, Y32[idx].contiguous(), n, loss)
        net.backward(B, n, grad)
        net.adam_step(theta, grad, m, v, 2e-3, step)
        if step % 10 == 0 or step == 1:
            losses.append(loss.item())
    print(f"  loss {losses[0]:.3e} -> {losses[-1]:.3e}", flush=True)
    assert losses[-1] < 0.25 * losses[0]


def test_warm_started_solve_stays_exact():
    # whatever the network predicts, the solve converges to the same solution: the guess enters
    # scaled by its Galerkin factor (dropped unless that lowers the energy error), and the inner
    # tolerance judges the result
    from oracle import system
    n = 64
    print("[warm solve]", flush=True)
    P = F.setup_mesh(n, 1.0, 1e-3)
    P.bind_workspace()
    TP = P.build_rational_pc(F.FDD_RA_PRECOND, 1e-12)
    TH = P.build_rational_pc(F.FDD_RA_OPERATOR, 1e-12)
    b = workloads.rhs(2, n, 5000)
    bd = torch.as_tensor(b, device="cuda")
    x_ref = system.solve_dst_2d(n, 1.0, 1e-3, b)
    params = workloads.cnn_init(seed=6)
    for scale in (1.0, 0.0):  # an untrained network, and one that predicts zero
        theta = torch.as_tensor(F.pack_params(params) * scale, dtype=torch.float32, device="cuda")
        net = F.Cnn(1, n)
        net.set_params(theta)
        for use_graph in (0, 1):
            x = torch.zeros_like(bd)
            opts = F.opts_default(outer_rtol=1e-10, inner_rtol=1e-12, use_graph=use_graph)
            opts.warmstart = net.h.value
            st = P.solve(TP, TH, bd, x, opts)
            err = rel(x.cpu().numpy(), x_ref)
            print(f"  scale {scale:g} graph {use_graph}: err {err:.2e} outer {st['outer_its']} "
                  f"warm {st['warm_starts']} kept {st['warm_accepted']}", flush=True)
            assert err <= 1e-8
            assert st["warm_starts"] == st["outer_its"]
            if scale == 0.0:
                assert st["warm_accepted"] == 0
