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


def _net(torch, seed=9, max_batch=4096, hidden=H, layers=LAYERS):
    from paper_2511_15908_amd import mlp, surrogate
    net = mlp.Mlp(N_IN, N_OUT, hidden=hidden, layers=layers, max_batch=max_batch)
    p = surrogate.init_params(seed, hidden, layers, N_IN, N_OUT)
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
