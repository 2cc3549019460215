"""Surrogate-MLP kernels through the C ABI against the FP64 oracle: the BF16
MFMA product in every operand layout (ragged sizes, empty contraction), the
column normaliser, the forward pass (batched and the one-sample haptic
chain), the gradient of the loss, Adam, and a short training run."""
import numpy as np
import pytest

from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu

H, LAYERS, N_IN, N_OUT = 256, 3, 126, 6


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2511_15908_amd import mlp
    mlp.lib()
    return torch


def _bits(a):
    """float64 array -> BF16 bit patterns (int16) after oracle rounding."""
    f = M.bf16(a).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def _data(seed, m, n_in=N_IN, n_out=N_OUT):
    from paper_2511_15908_amd import scenes
    rng = scenes.SplitMix64(seed, 51)
    X = rng.normal(m * n_in).reshape(m, n_in) * (1.0 + np.arange(n_in) % 7) + np.arange(n_in) * 0.1
    A = rng.normal(n_in * n_out).reshape(n_in, n_out) / np.sqrt(n_in)
    Y = np.tanh(((X - X.mean(0)) / X.std(0)) @ A) * 3.0 + 1.0 + 0.1 * rng.normal(m * n_out).reshape(m, n_out)
    return X.astype(np.float32), Y.astype(np.float32)


@pytest.mark.parametrize("al,bl", [(0, 0), (0, 1), (1, 1), (1, 0)])
@pytest.mark.parametrize("M_,N_,K_", [(100, 72, 70), (64, 64, 32), (1, 16, 256), (130, 200, 1000)])
def test_gemm_layouts(torch, al, bl, M_, N_, K_):
    from paper_2511_15908_amd import mlp, scenes
    rng = scenes.SplitMix64(M_ * 7 + N_ + K_, 52)
    A = rng.normal(M_ * K_).reshape(M_, K_)
    B = rng.normal(K_ * N_).reshape(K_, N_)
    lda = K_ if al == 0 else (M_ + 7) // 8 * 8
    ldb = K_ if bl == 0 else (N_ + 7) // 8 * 8
    lda = (lda + 7) // 8 * 8
    ldb = (ldb + 7) // 8 * 8
    Ab = np.zeros((M_, lda) if al == 0 else (K_, lda), np.int16)
    Bb = np.zeros((N_, ldb) if bl == 0 else (K_, ldb), np.int16)
    if al == 0:
        Ab[:, :K_] = _bits(A)
    else:
        Ab[:, :M_] = _bits(A.T)
    if bl == 0:
        Bb[:, :K_] = _bits(B.T)
    else:
        Bb[:, :N_] = _bits(B)
    dA = torch.tensor(Ab, device="cuda")
    dB = torch.tensor(Bb, device="cuda")
    Cg = mlp.gemm_bf16(dA, dB, M_, N_, K_, al, bl, lda, ldb).cpu().numpy().astype(np.float64)
    ref = M.bf16(A) @ M.bf16(B)
    scale = np.abs(M.bf16(A)) @ np.abs(M.bf16(B))
    err = np.abs(Cg - ref) / np.maximum(scale, 1e-30)
    assert err.max() < 2e-6, err.max()


def test_gemm_empty_contraction(torch):
    from paper_2511_15908_amd import mlp
    A = torch.zeros((64, 8), dtype=torch.int16, device="cuda")
    Cg = mlp.gemm_bf16(A, A, 64, 64, 0, 0, 0, 8, 8)
    assert float(Cg.abs().max()) == 0.0


def _net(torch, seed=9, max_batch=4096, hidden=H, layers=LAYERS, n_in=N_IN):
    from paper_2511_15908_amd import mlp, surrogate
    net = mlp.Mlp(n_in, N_OUT, hidden=hidden, layers=layers, max_batch=max_batch)
    p = surrogate.init_params(seed, hidden, layers, n_in, N_OUT)
    net.set_params(p)
    return net, p


def test_normalizer_and_forward(torch):
    X, Y = _data(1, 333)
    net, p = _net(torch)
    dX, dY = torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda")
    net.fit_normalizer(dX, dY)
    norm_g = net.get_normalizer()
    norm_o = M.fit_normalizer(X, Y)
    for a, b in zip(norm_g, norm_o):
        assert np.allclose(a, b, rtol=2e-6, atol=1e-6)
    # both sides use the same (FP32) statistics from here on
    norm = [np.asarray(v, np.float64) for v in norm_g]
    out_g = net.forward(dX).cpu().numpy().astype(np.float64)
    out_o, _ = M.forward(p.astype(np.float64), X, norm, H, LAYERS, N_OUT, quant=True)
    scale = np.abs(out_o).max()
    err = np.abs(out_g - out_o).max() / scale
    print(f"forward: max |diff| / max |out| = {err:.2e}")
    assert err < 5e-3
    # the one-sample haptic chain (host in, host out)
    for r in (0, 17, 332):
        y1 = net.predict_one(X[r]).astype(np.float64)
        assert np.abs(y1 - out_o[r]).max() / scale < 5e-3
        assert np.abs(y1 - out_g[r]).max() / scale < 1e-3


def test_gradients_match_oracle(torch):
    X, Y = _data(2, 700)
    net, p = _net(torch, seed=10)
    dX, dY = torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda")
    net.fit_normalizer(dX, dY)
    norm = [np.asarray(v, np.float64) for v in net.get_normalizer()]
    g_gpu, loss_gpu = net.gradients(dX, dY)
    loss_o, g_o = M.loss_and_grad(p.astype(np.float64), X, Y, norm, H, LAYERS, N_OUT, quant=True)
    assert loss_gpu == pytest.approx(loss_o, rel=2e-3)
    o = 0
    for li, (n, k) in enumerate(M.shapes(H, LAYERS)):
        for name, size in (("W", n * k), ("b", n)):
            a = g_gpu[o:o + size].astype(np.float64)
            b = g_o[o:o + size]
            o += size
            rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            cos = a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30)
            print(f"layer {li} {name}: rel L2 {rel:.2e} cos {cos:.6f}")
            assert rel < 2e-3 and cos > 0.99999
    # the loss is the oracle's; gradient pass leaves parameters unchanged
    assert np.array_equal(net.get_params(), p)


def test_wide_inputs_match_oracle(torch):
    """More than 128 inputs: the first layer pads to 256 columns; forward
    (batched and the one-sample chain) and gradients against the oracle."""
    n_in = 198
    X, Y = _data(12, 900, n_in=n_in)
    net, p = _net(torch, seed=13, n_in=n_in)
    assert p.size == M.param_count(H, LAYERS, n_in) == net.n_params
    dX, dY = torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda")
    net.fit_normalizer(dX, dY)
    norm = [np.asarray(v, np.float64) for v in net.get_normalizer()]
    out_g = net.forward(dX).cpu().numpy().astype(np.float64)
    out_o, _ = M.forward(p.astype(np.float64), X, norm, H, LAYERS, N_OUT, quant=True)
    scale = np.abs(out_o).max()
    err = np.abs(out_g - out_o).max() / scale
    print(f"wide forward: max |diff| / max |out| = {err:.2e}")
    assert err < 5e-3
    for r in (0, 450, 899):
        y1 = net.predict_one(X[r]).astype(np.float64)
        assert np.abs(y1 - out_g[r]).max() / scale < 1e-3
    g_gpu, loss_gpu = net.gradients(dX, dY)
    loss_o, g_o = M.loss_and_grad(p.astype(np.float64), X, Y, norm, H, LAYERS, N_OUT, quant=True)
    assert loss_gpu == pytest.approx(loss_o, rel=2e-3)
    o = 0
    for li, (n, k) in enumerate(M.shapes(H, LAYERS, n_in)):
        for name, size in (("W", n * k), ("b", n)):
            a = g_gpu[o:o + size].astype(np.float64)
            b = g_o[o:o + size]
            o += size
            rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            print(f"wide layer {li} {name}: rel L2 {rel:.2e}")
            assert rel < 2e-3
    # padded input columns keep zero weights and zero gradients
    W0 = g_gpu[:H * 256].reshape(H, 256)
    assert not W0[:, n_in:].any()


def test_adam_matches_oracle(torch):
    from paper_2511_15908_amd import scenes
    net, p = _net(torch, seed=11, max_batch=64)
    rng = scenes.SplitMix64(12, 53)
    w, m1, m2 = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    mask = np.ones(p.size)
    mask[-16 * H - 16:][np.r_[np.arange(N_OUT * H, 16 * H), 16 * H + np.arange(N_OUT, 16)]] = 0
    for t in range(1, 4):
        g = (rng.normal(p.size) * 10.0 ** (rng.uniform(p.size) * 4 - 3)).astype(np.float32) * mask
        net.adam_step(g, 1e-3)
        w, m1, m2 = M.adam(w, m1, m2, g.astype(np.float64), t, 1e-3)
        got = net.get_params().astype(np.float64)
        assert np.abs(got - w).max() < 1e-6 * (1 + np.abs(w).max())


def test_train_step_is_gradient_then_adam(torch):
    X, Y = _data(3, 512)
    a, p = _net(torch, seed=13)
    b, _ = _net(torch, seed=13)
    dX, dY = torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda")
    for n in (a, b):
        n.fit_normalizer(dX, dY)
    for _ in range(3):
        a.train_step(dX, dY, 1e-3)
        g, _ = b.gradients(dX, dY)
        b.adam_step(g, 1e-3)
    assert np.array_equal(a.get_params(), b.get_params())


def test_training_reduces_loss(torch):
    from paper_2511_15908_amd import scenes
    X, Y = _data(4, 8192)
    net, _ = _net(torch, seed=14)
    dX, dY = torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda")
    net.fit_normalizer(dX, dY)
    rng = scenes.SplitMix64(15, 54)
    _, l0 = net.gradients(dX[:4096], dY[:4096])
    for it in range(300):
        idx = torch.tensor((rng.uniform(1024) * 8192).astype(np.int64), device="cuda")
        net.train_step(dX[idx].contiguous(), dY[idx].contiguous(), 1e-3)
    _, l1 = net.gradients(dX[:4096], dY[:4096])
    print(f"loss {l0:.4f} -> {l1:.4f}")
    assert l1 < 0.1 * l0


def test_residual_output_matches_oracle(torch):
    """Residual mode (the outputs add raw input columns 13..18): normaliser,
    forward (batched and one-sample) and gradient against the oracle."""
    from paper_2511_15908_amd import mlp, surrogate
    rc = 13
    X, Y = _data(5, 500)
    Y = (Y + X[:, rc:rc + N_OUT]).astype(np.float32)
    net = mlp.Mlp(N_IN, N_OUT, hidden=H, layers=LAYERS, max_batch=1024, residual_col=rc)
    p = surrogate.init_params(16, H, LAYERS, N_IN, N_OUT)
    net.set_params(p)
    dX, dY = torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda")
    net.fit_normalizer(dX, dY)
    norm_g = [np.asarray(v, np.float64) for v in net.get_normalizer()]
    for a, b in zip(norm_g, M.fit_normalizer(X, Y, res_col=rc)):
        assert np.allclose(a, b, rtol=2e-6, atol=1e-6)
    out_g = net.forward(dX).cpu().numpy().astype(np.float64)
    out_o, _ = M.forward(p.astype(np.float64), X, norm_g, H, LAYERS, N_OUT, quant=True, res_col=rc)
    scale = np.abs(out_o).max()
    assert np.abs(out_g - out_o).max() / scale < 5e-3
    y1 = net.predict_one(X[7]).astype(np.float64)
    assert np.abs(y1 - out_o[7]).max() / scale < 5e-3
    g_gpu, loss_gpu = net.gradients(dX, dY)
    loss_o, g_o = M.loss_and_grad(p.astype(np.float64), X, Y, norm_g, H, LAYERS, N_OUT, quant=True, res_col=rc)
    assert loss_gpu == pytest.approx(loss_o, rel=2e-3)
    rel = np.linalg.norm(g_gpu - g_o) / np.linalg.norm(g_o)
    assert rel < 2e-3


def test_guard_falls_back_to_residual_base(torch):
    """Plain-SPH fallback: the fitted range equals the columns' min/max; rows
    outside it (margin 0.25; one column beyond a bound, NaN) return exactly the
    residual input columns, rows inside the unguarded output bit for bit,
    batched and one-sample, and the counters count them; margin < 0 turns
    the guard off."""
    from paper_2511_15908_amd import mlp, surrogate
    rc, margin = 13, 0.25
    X, Y = _data(8, 700)
    Y = (Y + X[:, rc:rc + N_OUT]).astype(np.float32)
    net = mlp.Mlp(N_IN, N_OUT, hidden=H, layers=LAYERS, max_batch=1024, residual_col=rc)
    net.set_params(surrogate.init_params(18, H, LAYERS, N_IN, N_OUT))
    with pytest.raises(mlp.MlpError):
        net.set_guard(margin)                       # no range yet
    dX, dY = torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda")
    net.fit_normalizer(dX, dY)
    lo, hi = net.get_input_range()
    lo_o, hi_o = M.input_range(X)
    assert np.array_equal(lo, lo_o) and np.array_equal(hi, hi_o)
    # test rows: the first ones inside, then single columns pushed past the bounds
    a, b = M.guard_bounds(lo, hi, margin)
    Xt = X[:64].copy()
    Xt[3, 0] = np.nextafter(b[0], np.float32(np.inf))
    Xt[9, 100] = np.nextafter(a[100], np.float32(-np.inf))
    Xt[20, 50] = b[50]                              # on the bound: inside
    Xt[21, 60] = a[60]
    Xt[30, rc + 2] = hi[rc + 2] + 5.0 * (hi[rc + 2] - lo[rc + 2])
    Xt[40, 7] = np.nan
    fall_o = M.guard_rows(Xt, lo, hi, margin)
    assert fall_o.tolist().count(True) == 4 and not fall_o[20] and not fall_o[21]
    dXt = torch.tensor(Xt, device="cuda")
    plain = net.forward(dXt).cpu().numpy()
    net.set_guard(margin)
    got = net.forward(dXt).cpu().numpy()
    exp, _ = M.guarded(plain.astype(np.float64), Xt, lo, hi, margin, N_OUT, rc)
    assert np.array_equal(got[fall_o], Xt[fall_o, rc:rc + N_OUT])
    ok = ~fall_o
    ok[40] = False                                  # NaN row: the plain output is NaN there
    assert np.array_equal(got[ok], plain[ok]) and np.array_equal(got[~fall_o & ok], exp[~fall_o & ok].astype(np.float32))
    assert net.guard_count() == (64, 4)
    # the one-sample haptic chain
    for r in (0, 3, 9, 20, 30, 40):
        y = net.predict_one(Xt[r])
        if fall_o[r]:
            assert np.array_equal(y, Xt[r, rc:rc + N_OUT]), r
        else:
            net.set_guard(-1.0)
            y_plain = net.predict_one(Xt[r])
            net.set_guard(margin)
            assert np.array_equal(y, y_plain), r
    assert net.guard_count() == (64 + 6, 4 + 4)
    net.set_guard(-1.0)
    assert np.array_equal(net.forward(dXt).cpu().numpy()[ok], plain[ok])
    assert net.guard_count() == (70, 8)


# ---------------------------------------------------------------- element-wise bounds
#
# Element-wise error bounds derived from the arithmetic and propagated layer
# by layer through the oracle's cached activations (standardised units).
#
# Against the BF16-mirroring oracle (quant=True) both sides round the same
# values to BF16 at the same points, so an operand differs only where the
# GPU's FP32 value and the oracle's FP64 value can fall on different sides of
# a BF16 rounding midpoint: there by one BF16 step, elsewhere not at all.
# Whether that can happen is decided per element from the bound on the
# pre-rounding value.  Products accumulate in FP32 (K 2^-24 of sum |a||w|).
#
# Against the pure FP64 network (quant=False) every GEMM operand is rounded to
# BF16 on the GPU (2^-9 relative, weights and activations), a worst-case sum.
#
# GELU is 1.129-Lipschitz and its derivative 0.798-Lipschitz; the FP32 GELU
# and its derivative are taken as accurate to 2^-21 relative plus 2^-23 |z|.

U8, U9, U21, U22, U23, U24 = (2.0 ** -e for e in (8, 9, 21, 22, 23, 24))
LIP_GELU, LIP_DGELU = 1.129, 0.798


def _bf16_step(v):
    """One BF16 step at |v| (8 significant bits)."""
    r = np.abs(M.bf16(v))
    e = np.floor(np.log2(np.maximum(r, 2.0 ** -126)))
    return 2.0 ** (e - 7)


def _flip(v, err):
    """Largest change of bf16(v) when v moves by at most err: 0 unless a
    rounding midpoint lies within err (+ the FP32 rounding of v) of v."""
    step = _bf16_step(v)
    gap = 0.5 * step - np.abs(v - M.bf16(v))
    return np.where(gap <= err + U23 * np.abs(v), 2.0 * step, 0.0)


def _fwd_bounds(p, c, quant, xs_err):
    """Bounds on |d a_l| (GEMM inputs) and |d z_l| for every layer."""
    wb = M.unpack(p, H, LAYERS)
    A, E = [], []
    da = _flip(c["pre"][0], xs_err) if quant else U9 * np.abs(c["acts"][0]) + xs_err
    for l, (W, _) in enumerate(wb):
        A.append(da)
        a = np.abs(c["acts"][l])
        Wq = np.abs(M.bf16(W))
        aw = a @ Wq.T
        e = da @ Wq.T + (0.0 if quant else U9) * aw + W.shape[1] * U24 * aw + U24 * np.abs(c["zs"][l])
        E.append(e)
        if l + 1 < len(wb):
            z = c["zs"][l]
            v_err = LIP_GELU * e + U21 * np.abs(c["pre"][l + 1]) + U23 * np.abs(z)
            da = _flip(c["pre"][l + 1], v_err) if quant else U9 * np.abs(c["acts"][l + 1]) + v_err
    return A, E


def _grad_bounds(p, c, A, E, ddz, m, quant):
    """Bounds on the gradient elements (parameter layout), from the bound
    ddz on the output-layer gradient dz_L."""
    wb = M.unpack(p, H, LAYERS)
    L = len(wb)
    cur = c["dz_L"]
    out = [None] * L
    for l in range(L - 1, -1, -1):
        W, _ = wb[l]
        a = np.abs(c["acts"][l])
        ac = np.abs(cur)
        gW = ddz.T @ a + ac.T @ A[l] + m * U24 * (ac.T @ a)
        gb = ddz.sum(0) + m * U24 * ac.sum(0)
        if l == L - 1:
            gW[N_OUT:] = 0.0
            gb[N_OUT:] = 0.0
        out[l] = (gW, gb)
        if l > 0:
            Wb = M.bf16(W) if quant else W
            Wq = np.abs(M.bf16(W))
            da = cur @ Wb
            g1 = M.gelu_grad(c["zs"][l - 1])
            dda = ddz @ Wq + (0.0 if quant else U9) * (ac @ Wq) + W.shape[0] * U24 * (ac @ Wq)
            pre = da * g1
            err = dda * np.abs(g1) + np.abs(da) * LIP_DGELU * E[l - 1] + U21 * np.abs(pre)
            if quant:
                cur = M.bf16(pre)
                ddz = _flip(pre, err)
            else:
                cur = pre
                ddz = err + U9 * np.abs(pre)
    return M.pack(out)


def _forward_with_pre(p, X, norm, quant):
    """The oracle's forward pass plus the pre-rounding values of every GEMM
    input (standardised inputs, GELU outputs)."""
    out, c = M.forward(p, X, norm, H, LAYERS, N_OUT, quant=quant)
    mx, sx = norm[0], norm[1]
    xs = np.zeros((X.shape[0], M.K_IN))
    xs[:, :N_IN] = (X.astype(np.float64) - mx) / sx
    c["pre"] = [xs] + [M.gelu(z) for z in c["zs"][:-1]]
    return out, c, xs


@pytest.mark.parametrize("quant", [True, False])
def test_elementwise_forward_and_gradients(torch, quant):
    """Batch 4096 (16 split-K slices in the weight gradients): every output
    and every gradient element within its derived bound, against the
    BF16-mirroring oracle and against the pure FP64 network."""
    m = 4096
    X, Y = _data(6, m)
    net, p = _net(torch, seed=19)
    dX, dY = torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda")
    net.fit_normalizer(dX, dY)
    norm = [np.asarray(v, np.float64) for v in net.get_normalizer()]
    p64 = p.astype(np.float64)
    out_o, c, xs = _forward_with_pre(p64, X, norm, quant)
    A, E = _fwd_bounds(p64, c, quant, U22 * np.abs(xs))
    sy = norm[3]
    out_g = net.forward(dX).cpu().numpy().astype(np.float64)
    bound_out = E[-1][:, :N_OUT] * sy + U22 * np.abs(out_o)
    diff = np.abs(out_g - out_o)
    print(f"quant={quant}: forward max |diff|/bound {np.max(diff / bound_out):.3f}, "
          f"max |diff| {diff.max():.2e}, elements at zero bound {int(np.sum(bound_out == 0))}")
    assert np.all(diff <= bound_out)
    g_gpu, loss_gpu = net.gradients(dX, dY)
    loss_o, g_o = M.loss_and_grad(p64, X, Y, norm, H, LAYERS, N_OUT, quant=quant)
    ys = (Y.astype(np.float64) - norm[2]) / sy
    dz_L = np.zeros((m, 16))
    dz_L[:, :N_OUT] = 2.0 * (c["out_s"] - ys) / (m * N_OUT)
    c["dz_L"] = M.bf16(dz_L) if quant else dz_L
    err = np.zeros((m, 16))
    err[:, :N_OUT] = 2.0 * (E[-1][:, :N_OUT] + U22 * np.abs(ys)) / (m * N_OUT) + U22 * np.abs(dz_L[:, :N_OUT])
    ddz = _flip(dz_L, err) if quant else err + U9 * np.abs(dz_L)
    bound_g = _grad_bounds(p64, c, A, E, ddz, m, quant)
    diff = np.abs(g_gpu.astype(np.float64) - g_o)
    worst = float(np.max(diff / np.maximum(bound_g, 1e-300)))
    print(f"quant={quant}: gradient max |diff|/bound {worst:.3f} over {g_o.size} elements "
          f"(max |diff| {diff.max():.2e})")
    assert np.all(diff <= bound_g), np.flatnonzero(diff > bound_g)[:10]
    assert loss_gpu == pytest.approx(loss_o, rel=2e-3 if quant else 2e-2)
