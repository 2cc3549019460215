"""FP64 CPU oracle of the wrench-surrogate MLP and its training step.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library.

What it computes (plain numpy, binary64):
  * standardisation x' = (x - mu_x)/sd_x, y' = (y - mu_y)/sd_y with the
    column mean and population standard deviation (sd = 1 where < 1e-12);
  * optionally a residual output: y = x[res_col .. res_col + n_out) + the
    de-standardised network output, so the targets, their statistics and
    the loss refer to y - x[res_col ..];
  * the network z_l = a_{l-1} W_l^T + b_l, a_l = GELU(z_l) for the hidden
    layers (GELU in its exact form 0.5 z (1 + erf(z / sqrt 2))), a linear
    output layer; inputs zero-padded to 128 columns (256 for more than 128
    inputs), outputs padded to 16;
  * the loss L = 1/(m n_out) sum (out' - y')^2 over the first n_out outputs and
    its gradient by the chain rule (backpropagation written out per layer);
  * Adam (Kingma and Ba 2015, Algorithm 1: moment estimates with bias
    correction);
  * the plain-SPH fallback of the haptic loop: a row whose input leaves the
    training range (column minimum and maximum, widened by margin times the
    range on each side) returns the residual base, the simulator's own last
    wrench, instead of the network's output (the decision in FP32, as the
    library takes it).
With quant=True the values that the GPU path feeds to its BF16 matrix
products (weights, standardised inputs, hidden activations, output and
hidden-layer gradients) are rounded to BF16 at the same points; everything
else stays binary64.  quant=False is the pure FP64 network that the
finite-difference pins check.
"""
from __future__ import annotations

import math

import numpy as np

K_IN = 128      # padded input width for up to 128 inputs (256 above)
N_OUT_PAD = 16  # padded output width


def k_in(n_in=K_IN):
    """Padded input width of a network with n_in inputs."""
    return K_IN if n_in <= K_IN else 2 * K_IN


def bf16(a):
    """Round to BF16: first to binary32 (round to nearest even), then to the
    nearest value with 8 significant bits (ties to even)."""
    f = np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(a))


def _erf(x):
    return np.vectorize(math.erf, otypes=[np.float64])(x)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d/dz of 0.5 z (1 + erf(z/sqrt2)) = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def shapes(hidden, layers, n_in=K_IN):
    """(N_l, K_l) of every layer, output layer last."""
    out = [(hidden, k_in(n_in))]
    out += [(hidden, hidden)] * (layers - 1)
    out.append((N_OUT_PAD, hidden))
    return out


def param_count(hidden, layers, n_in=K_IN):
    return sum(n * k + n for n, k in shapes(hidden, layers, n_in))


def unpack(params, hidden, layers, n_in=K_IN):
    """Flat FP32/FP64 vector -> list of (W [N][K], b [N]) as float64 views."""
    p = np.asarray(params, np.float64)
    out, o = [], 0
    for n, k in shapes(hidden, layers, n_in):
        W = p[o:o + n * k].reshape(n, k)
        o += n * k
        b = p[o:o + n]
        o += n
        out.append((W, b))
    assert o == p.size
    return out


def pack(layers_wb):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers_wb])


def _res(X, n_out, res_col):
    X = np.asarray(X, np.float64)
    if res_col is None:
        return np.zeros((X.shape[0], n_out))
    return X[:, res_col:res_col + n_out]


def fit_normalizer(X, Y, res_col=None):
    X, Y = np.asarray(X, np.float64), np.asarray(Y, np.float64)
    Y = Y - _res(X, Y.shape[1], res_col)
    mx, my = X.mean(0), Y.mean(0)
    sx, sy = X.std(0), Y.std(0)
    sx = np.where(sx < 1e-12, 1.0, sx)
    sy = np.where(sy < 1e-12, 1.0, sy)
    return mx, sx, my, sy


def input_range(X):
    """Column minimum and maximum of the training inputs."""
    X = np.asarray(X, np.float32)
    return X.min(0), X.max(0)


def guard_bounds(lo, hi, margin):
    """a = lo - margin (hi - lo), b = hi + margin (hi - lo), each operation
    rounded to FP32."""
    lo, hi = np.asarray(lo, np.float32), np.asarray(hi, np.float32)
    mw = np.float32(margin) * (hi - lo)
    return lo - mw, hi + mw


def guard_rows(X, lo, hi, margin):
    """True for rows with a column outside [a, b] (NaN counts as outside)."""
    a, b = guard_bounds(lo, hi, margin)
    X = np.asarray(X, np.float32)
    inside = (X >= a) & (X <= b)
    return ~inside.all(1)


def guarded(out, X, lo, hi, margin, n_out, res_col):
    """The haptic loop's output: the network's where the row is inside the
    range, the residual base (input columns res_col ..) where it is not."""
    fall = guard_rows(X, lo, hi, margin)
    base = np.asarray(X, np.float64)[:, res_col:res_col + n_out]
    return np.where(fall[:, None], base, out), fall


def _q(a, quant):
    return bf16(a) if quant else a


def forward(params, X, norm, hidden, layers, n_out, quant=True, res_col=None):
    """Returns (out in raw units [m][n_out], cache for backward)."""
    mx, sx, my, sy = (np.asarray(v, np.float64) for v in norm)
    X = np.asarray(X, np.float64)
    m, n_in = X.shape
    xs = np.zeros((m, k_in(n_in)))
    xs[:, :n_in] = (X - mx) / sx
    a = _q(xs, quant)
    wb = unpack(params, hidden, layers, n_in)
    acts, zs = [a], []
    for l, (W, b) in enumerate(wb):
        z = a @ _q(W, quant).T + b
        zs.append(z)
        if l < len(wb) - 1:
            a = _q(gelu(z), quant)
            acts.append(a)
    out_s = zs[-1][:, :n_out]
    return out_s * sy + my + _res(X, n_out, res_col), {"acts": acts, "zs": zs, "out_s": out_s}


def loss_and_grad(params, X, Y, norm, hidden, layers, n_out, quant=True, res_col=None):
    """Loss on standardised outputs and its gradient (parameter layout)."""
    mx, sx, my, sy = (np.asarray(v, np.float64) for v in norm)
    Y = np.asarray(Y, np.float64)
    m = Y.shape[0]
    _, c = forward(params, X, norm, hidden, layers, n_out, quant, res_col)
    ys = (Y - _res(X, n_out, res_col) - my) / sy
    d = c["out_s"] - ys
    loss = float(np.sum(d * d) / (m * n_out))
    wb = unpack(params, hidden, layers, np.shape(X)[1])
    dz = np.zeros((m, N_OUT_PAD))
    dz[:, :n_out] = 2.0 * d / (m * n_out)
    dz = _q(dz, quant)
    grads = [None] * len(wb)
    for l in range(len(wb) - 1, -1, -1):
        W, _ = wb[l]
        a_prev = c["acts"][l]
        gW = dz.T @ a_prev
        gb = dz.sum(0)
        if l == len(wb) - 1:
            gW[n_out:] = 0.0
            gb[n_out:] = 0.0
        grads[l] = (gW, gb)
        if l > 0:
            da = dz @ _q(W, quant)
            dz = _q(da * gelu_grad(c["zs"][l - 1]), quant)
    return loss, pack(grads)


def adam(params, m1, m2, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t = 1 for the first); returns new (params, m1, m2)."""
    g = np.asarray(grad, np.float64)
    m1 = beta1 * np.asarray(m1, np.float64) + (1.0 - beta1) * g
    m2 = beta2 * np.asarray(m2, np.float64) + (1.0 - beta2) * g * g
    mh = m1 / (1.0 - beta1 ** t)
    vh = m2 / (1.0 - beta2 ** t)
    return np.asarray(params, np.float64) - lr * mh / (np.sqrt(vh) + eps), m1, m2
