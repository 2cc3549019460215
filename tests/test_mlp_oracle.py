"""Pins of the FP64 MLP oracle (wrench surrogate): each test checks the oracle
against something other than itself: central finite differences of the
loss, textbook values of the normal CDF, closed forms of Adam (Kingma and Ba,
Algorithm 1) and torch's own BF16 rounding."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M


def _rand_params(seed, hidden, layers, scale=0.3):
    rng = np.random.default_rng(seed)
    wb = []
    for n, k in M.shapes(hidden, layers):
        wb.append((rng.standard_normal((n, k)) * scale / math.sqrt(k), rng.standard_normal(n) * 0.1))
    W, b = wb[-1]
    W[6:] = 0.0
    b[6:] = 0.0
    return M.pack(wb)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-8, 8, 5000),
                        [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0, 65504.0]])
    t = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(x), t)
    # ties to even: 1 + 2^-8 -> 1; 1 + 3 2^-8 -> 1 + 2^-6
    assert M.bf16(1 + 2 ** -8) == 1.0 and M.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6


def test_gelu_textbook_values():
    # GELU(z) = z Phi(z): Phi(1) = 0.8413447460685429, Phi(-1) = 0.15865525393145707
    assert M.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-15)
    assert M.gelu(np.array([-1.0]))[0] == pytest.approx(-0.15865525393145707, rel=1e-14)
    assert M.gelu(np.array([0.0]))[0] == 0.0
    z = np.linspace(-6, 6, 241)
    fd = (M.gelu(z + 1e-6) - M.gelu(z - 1e-6)) / 2e-6
    assert np.allclose(M.gelu_grad(z), fd, atol=1e-8)
    assert M.gelu_grad(np.array([0.0]))[0] == 0.5


@pytest.mark.parametrize("hidden,layers", [(64, 1), (64, 3)])
def test_gradient_matches_finite_differences(hidden, layers):
    """Backpropagation of the pure FP64 network against central differences
    of the loss on a sample of parameters of every layer and both kinds."""
    rng = np.random.default_rng(7)
    n_in, n_out, m = 20, 6, 9
    X = rng.standard_normal((m, n_in))
    Y = rng.standard_normal((m, n_out))
    norm = M.fit_normalizer(X, Y)
    p = _rand_params(3, hidden, layers)
    L0, g = M.loss_and_grad(p, X, Y, norm, hidden, layers, n_out, quant=False)
    # parameters of every layer: weights on real inputs, biases, output rows
    idx, o = [], 0
    for n, k in M.shapes(hidden, layers):
        idx += list(o + rng.integers(0, min(n, 6 if n == 16 else n)) * k + rng.integers(0, min(k, n_in), 4))
        o += n * k
        idx += list(o + rng.integers(0, min(n, 6 if n == 16 else n), 2))
        o += n
    for i in idx:
        e = 1e-5
        pp, pm = p.copy(), p.copy()
        pp[i] += e
        pm[i] -= e
        fd = (M.loss_and_grad(pp, X, Y, norm, hidden, layers, n_out, False)[0] -
              M.loss_and_grad(pm, X, Y, norm, hidden, layers, n_out, False)[0]) / (2 * e)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-10), i
    # padded output rows and padded input columns receive no gradient from the loss
    wb = M.unpack(g, hidden, layers)
    assert np.all(wb[-1][0][n_out:] == 0) and np.all(wb[-1][1][n_out:] == 0)
    assert np.all(wb[0][0][:, n_in:] == 0)


def test_zero_hidden_weights_closed_form():
    """With every weight zero the output is the output bias b; the loss is
    mean (b - y')^2 and its bias gradient 2 mean_rows (b - y') / n_out."""
    hidden, layers, n_out = 64, 2, 6
    rng = np.random.default_rng(2)
    X = rng.standard_normal((11, 30))
    Y = rng.standard_normal((11, n_out)) * 3 + 1
    norm = M.fit_normalizer(X, Y)
    p = np.zeros(M.param_count(hidden, layers))
    b = rng.standard_normal(n_out)
    p[-16:-16 + n_out] = b
    ys = (Y - norm[2]) / norm[3]
    L, g = M.loss_and_grad(p, X, Y, norm, hidden, layers, n_out, quant=False)
    assert L == pytest.approx(np.mean((b - ys) ** 2), rel=1e-14)
    assert np.allclose(g[-16:-16 + n_out], 2 * np.mean(b - ys, axis=0) / n_out, rtol=1e-13)
    out, _ = M.forward(p, X, norm, hidden, layers, n_out, quant=False)
    assert np.allclose(out, b * norm[3] + norm[2], rtol=1e-14)


def test_residual_output_closed_form():
    """With every weight zero and a residual block of inputs, the output is
    those inputs plus the de-standardised output bias; the target statistics
    are those of y minus the residual inputs, and a target equal to the
    residual inputs plus mu_y costs b^2."""
    hidden, layers, n_out, rc = 64, 2, 6, 4
    rng = np.random.default_rng(12)
    X = rng.standard_normal((13, 20))
    Y = X[:, rc:rc + n_out] + rng.standard_normal((13, n_out)) * 0.5
    norm = M.fit_normalizer(X, Y, res_col=rc)
    d = Y - X[:, rc:rc + n_out]
    assert np.allclose(norm[2], d.mean(0), rtol=1e-14) and np.allclose(norm[3], d.std(0), rtol=1e-14)
    p = np.zeros(M.param_count(hidden, layers))
    b = rng.standard_normal(n_out)
    p[-16:-16 + n_out] = b
    out, _ = M.forward(p, X, norm, hidden, layers, n_out, quant=False, res_col=rc)
    assert np.allclose(out, X[:, rc:rc + n_out] + b * norm[3] + norm[2], rtol=1e-14)
    Yc = X[:, rc:rc + n_out] + norm[2]
    L, g = M.loss_and_grad(p, X, Yc, norm, hidden, layers, n_out, quant=False, res_col=rc)
    assert L == pytest.approx(np.mean(b ** 2), rel=1e-13)
    assert np.allclose(g[-16:-16 + n_out], 2 * b / n_out, rtol=1e-13)


def test_guard_closed_forms():
    """The plain-SPH fallback decision at hand-picked values: lo = 0, hi = 2,
    margin 0.5 give the exact bounds [-1, 3]; the bounds themselves are
    inside, the next float beyond them and NaN are outside; margin 0 is the
    training range itself; a column that was constant in training admits
    only its value."""
    lo = np.array([0.0, -4.0, 7.0], np.float32)
    hi = np.array([2.0, 4.0, 7.0], np.float32)
    a, b = M.guard_bounds(lo, hi, 0.5)
    assert a.tolist() == [-1.0, -8.0, 7.0] and b.tolist() == [3.0, 8.0, 7.0]
    a0, b0 = M.guard_bounds(lo, hi, 0.0)
    assert a0.tolist() == lo.tolist() and b0.tolist() == hi.tolist()
    up = np.nextafter(np.float32(3.0), np.float32(4.0))
    dn = np.nextafter(np.float32(7.0), np.float32(0.0))
    X = np.array([[3.0, 0.0, 7.0],        # on the upper bound
                  [-1.0, -8.0, 7.0],      # on the lower bounds
                  [up, 0.0, 7.0],         # one ulp above
                  [0.0, 0.0, dn],         # the constant column moved
                  [np.nan, 0.0, 7.0],     # not a number
                  [1.0, 1.0, 7.0]], np.float32)
    assert M.guard_rows(X, lo, hi, 0.5).tolist() == [False, False, True, True, True, False]
    assert M.guard_rows(X[[5]], lo, hi, 0.0).tolist() == [False]
    assert M.guard_rows(X[[0]], lo, hi, 0.0).tolist() == [True]


def test_guarded_output_is_the_residual_base():
    """Rows that fall back carry exactly the residual input columns, the
    others the network's output unchanged; the range is the columns' min/max."""
    rng = np.random.default_rng(21)
    X = rng.standard_normal((40, 10)).astype(np.float32)
    lo, hi = M.input_range(X)
    assert np.array_equal(lo, X.min(0)) and np.array_equal(hi, X.max(0))
    Xt = X[:6].copy()
    Xt[1, 4] = hi[4] + 10.0
    Xt[3, 0] = np.nan
    out = rng.standard_normal((6, 3))
    g, fall = M.guarded(out, Xt, lo, hi, 0.0, 3, res_col=2)
    assert fall.tolist() == [False, True, False, True, False, False]
    assert np.array_equal(g[[1, 3]], Xt[[1, 3], 2:5].astype(np.float64))
    assert np.array_equal(g[[0, 2, 4, 5]], out[[0, 2, 4, 5]])


def test_adam_closed_forms():
    """Step 1 from zero moments moves every weight by lr g/(|g| + eps); a
    constant gradient keeps the bias-corrected moments at g and g^2 exactly,
    so t steps move by t lr g/(|g| + eps)."""
    rng = np.random.default_rng(4)
    g = rng.standard_normal(50) * 10.0 ** rng.integers(-3, 3, 50)
    w0 = rng.standard_normal(50)
    lr, eps = 1e-3, 1e-8
    w, m1, m2 = M.adam(w0, np.zeros(50), np.zeros(50), g, 1, lr, eps=eps)
    assert np.allclose(w, w0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    w, m1, m2 = w0, np.zeros(50), np.zeros(50)
    for t in range(1, 8):
        w, m1, m2 = M.adam(w, m1, m2, g, t, lr, eps=eps)
    assert np.allclose(w, w0 - 7 * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-13)


def test_quantised_forward_close_to_fp64():
    """BF16 rounding at the product inputs changes outputs by about 2^-8
    relative per rounding, far below the signal."""
    hidden, layers, n_out = 128, 3, 6
    rng = np.random.default_rng(5)
    X = rng.standard_normal((40, 100))
    Y = rng.standard_normal((40, n_out))
    norm = M.fit_normalizer(X, Y)
    p = _rand_params(6, hidden, layers, scale=1.0)
    a, _ = M.forward(p, X, norm, hidden, layers, n_out, quant=True)
    b, _ = M.forward(p, X, norm, hidden, layers, n_out, quant=False)
    rel = np.abs(a - b).max() / np.abs(b).max()
    assert 1e-5 < rel < 3e-2
