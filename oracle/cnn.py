"""FP64 reference of the warm-start network (oracle; test infrastructure only).

The learned initial guess for the interior Dirichlet solves: a plain convolutional network
maps an interface trace t (values at the n - 1 free Gamma nodes) to an approximation of the
discrete harmonic extension E t on the (n - 1) x (n - 1) interior grid, i.e. of the solution of
A_II u = lift(t) (the interior block of the paper's eq. (block_op); E = -A_II^{-1} A_IG).  The
paper itself has no network; everything here is the plain definition of the network written
out, and the hand-derived backpropagation through it.

Layout: images are NHWC float64 arrays (batch, rows j, columns i, channels); row j - 1 and
column i - 1 hold interior node (i, j), so an image reshapes to the free-dof order of the
interior, index (j - 1)(n - 1) + (i - 1).

Network: six 3x3 convolutions with zero ('same') padding and a bias, channel widths
5 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, the exact (erf) GELU after the first five, none after
the last.  A weight tensor has shape (3, 3, C_in, C_out) and is applied as a correlation:
out[y, x, o] = b[o] + sum_{dy, dx, c} in[y + dy - 1, x + dx - 1, c] W[dy, dx, c, o].

Input channels (the trace must reach every pixel; a 3x3 stack of six layers sees only 13 x 13):
  0: t_i broadcast down column i      1: y = j / n      2: y t_i
  3: log10 K                          4: log10 mu
Loss: mean squared error over all interior pixels.  Optimizer: Adam (Kingma and Ba 2015).

Parity: pinned in tests/test_oracle_cnn.py -- the convolution against scipy.signal.correlate2d
and a delta kernel, GELU against known values of the normal distribution and its odd-part
identity, the backward pass against central finite differences, Adam against its closed-form
first steps.
"""
import numpy as np
from scipy.special import erf

WIDTHS = (5, 32, 32, 32, 32, 32, 1)


def features(traces, n, K, mu):
    """Input channels (B, n-1, n-1, 5) for traces (B, n-1); K, mu scalars or length-B arrays."""
    t = np.asarray(traces, dtype=np.float64)
    B, m = t.shape
    assert m == n - 1
    K = np.broadcast_to(np.asarray(K, dtype=np.float64), (B,))
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), (B,))
    y = np.arange(1, n) / n                      # node j = 1..n-1 on row j-1
    X = np.zeros((B, m, m, 5))
    X[..., 0] = t[:, None, :]
    X[..., 1] = y[None, :, None]
    X[..., 2] = y[None, :, None] * t[:, None, :]
    X[..., 3] = np.log10(K)[:, None, None]
    X[..., 4] = np.log10(mu)[:, None, None]
    return X


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    phi = np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * phi


def conv3x3(X, W, b):
    """'same' 3x3 correlation with zero padding plus bias."""
    B, H, Wd, C = X.shape
    Xp = np.zeros((B, H + 2, Wd + 2, C))
    Xp[:, 1:-1, 1:-1, :] = X
    out = np.broadcast_to(b, (B, H, Wd, W.shape[3])).copy()
    for dy in range(3):
        for dx in range(3):
            out += Xp[:, dy:dy + H, dx:dx + Wd, :] @ W[dy, dx]
    return out


def conv3x3_backward(X, W, dZ):
    """Gradients of conv3x3(X, W, b) against X, W and b for the output gradient dZ."""
    B, H, Wd, C = X.shape
    Xp = np.zeros((B, H + 2, Wd + 2, C))
    Xp[:, 1:-1, 1:-1, :] = X
    dW = np.zeros_like(W)
    dXp = np.zeros_like(Xp)
    for dy in range(3):
        for dx in range(3):
            win = Xp[:, dy:dy + H, dx:dx + Wd, :]
            dW[dy, dx] = np.einsum("bhwc,bhwo->co", win, dZ)
            dXp[:, dy:dy + H, dx:dx + Wd, :] += dZ @ W[dy, dx].T
    db = dZ.sum(axis=(0, 1, 2))
    return dXp[:, 1:-1, 1:-1, :], dW, db


def forward(params, X):
    """Network output (B, H, W) and the per-layer cache (input, pre-activation)."""
    cache = []
    a = X
    L = len(params)
    for k, (W, b) in enumerate(params):
        z = conv3x3(a, W, b)
        cache.append((a, z))
        a = gelu(z) if k < L - 1 else z
    return a[..., 0], cache


def mse(out, target):
    """Mean squared error and its gradient against out."""
    d = out - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params, cache, dout):
    """Gradients [(dW, db)] of a scalar loss with gradient dout (B, H, W) against out."""
    grads = [None] * len(params)
    g = dout[..., None]
    L = len(params)
    for k in range(L - 1, -1, -1):
        a, z = cache[k]
        dz = g if k == L - 1 else g * gelu_grad(z)
        da, dW, db = conv3x3_backward(a, params[k][0], dz)
        grads[k] = (dW, db)
        g = da
    return grads


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (in place on copies); state = {'t': int, 'm': [...], 'v': [...]}."""
    t = state.get("t", 0) + 1
    if "m" not in state:
        state["m"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        state["v"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    new = []
    for k, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        upd = []
        for idx, (p, g) in enumerate(((W, gW), (b, gb))):
            m = b1 * state["m"][k][idx] + (1.0 - b1) * g
            v = b2 * state["v"][k][idx] + (1.0 - b2) * g * g
            state["m"][k] = tuple(m if q == idx else state["m"][k][q] for q in range(2))
            state["v"][k] = tuple(v if q == idx else state["v"][k][q] for q in range(2))
            mh = m / (1.0 - b1 ** t)
            vh = v / (1.0 - b2 ** t)
            upd.append(p - lr * mh / (np.sqrt(vh) + eps))
        new.append(tuple(upd))
    state["t"] = t
    return new


def warm_start(params, trace, n, K, mu):
    """The learned initial guess for A_II u = lift(trace), interior free-dof order.

    E is linear, so the trace is scaled to unit root-mean-square before the network and the
    output scaled back; a zero trace gives a zero guess.
    """
    t = np.asarray(trace, dtype=np.float64)
    s = np.sqrt(np.mean(t * t))
    if s == 0.0:
        return np.zeros((n - 1) ** 2)
    out, _ = forward(params, features((t / s)[None, :], n, K, mu))
    return s * out[0].ravel()
