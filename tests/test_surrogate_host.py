"""Host-side logic of the wrench-surrogate pipeline (no GPU): the haptic
rolling mean carried across walks, the feature-row layout whose residual
columns are the last SPH wrench (the plain-SPH fallback returns exactly
those), the two hold baselines, the error floor and the force spectrum."""
import math

import numpy as np

from paper_2511_15908_amd import surrogate as S


def _brute_means(samples, per_tick, K):
    out = []
    for t in range(1, samples.shape[0] // per_tick + 1):
        e = t * per_tick
        out.append(samples[max(e - K, 0):e].mean(0))
    return np.array(out)


def test_tick_means_carry_the_window_across_calls():
    rng = np.random.default_rng(3)
    per_tick, K = 4, 10
    steps = rng.standard_normal((4 * 23, 6))
    whole, _ = S.tick_means(np.zeros((0, 6)), steps, per_tick, K)
    assert np.allclose(whole, _brute_means(steps, per_tick, K), rtol=1e-13, atol=1e-13)
    # the same samples in three calls of uneven length
    tail = np.zeros((0, 6))
    parts = []
    for a, b in ((0, 4 * 2), (4 * 2, 4 * 15), (4 * 15, 4 * 23)):
        m, tail = S.tick_means(tail, steps[a:b], per_tick, K)
        parts.append(m)
        assert tail.shape[0] <= K - 1
    assert np.allclose(np.concatenate(parts), whole, rtol=1e-13, atol=1e-13)
    # a window of one sample is the last step of each tick (prefix-sum differences)
    m1, t1 = S.tick_means(np.zeros((0, 6)), steps, per_tick, 1)
    assert np.allclose(m1, steps[per_tick - 1::per_tick], rtol=1e-12, atol=1e-12) and t1.shape[0] == 0


def _log(n, rng):
    W = rng.standard_normal((n, 6))
    return {"c": rng.standard_normal((n, 3)), "q": rng.standard_normal((n, 4)),
            "v": rng.standard_normal((n, 3)), "w": rng.standard_normal((n, 3)),
            "wrench": W, "probes": rng.standard_normal((n, S.N_PROBES))}


def test_feature_row_layout():
    rng = np.random.default_rng(4)
    lg = _log(400, rng)
    t, d = np.array([150, 233]), np.array([0, 7])
    X, Y = S.feature_rows(lg, t, d)
    assert X.shape == (2, S.N_FEATURES) and S.N_FEATURES == 186
    for r in range(2):
        t0 = t[r] - d[r]
        W0 = lg["wrench"][t0]
        lags = []
        for j in (1, 2, 3, 5, 7, 10, 14, 20, 28, 40):
            lags += [lg["v"][t[r] - j] - lg["v"][t[r]], lg["w"][t[r] - j] - lg["w"][t[r]]]
        exp = np.concatenate([lg["c"][t[r]], lg["q"][t[r]], lg["v"][t[r]], lg["w"][t[r]], W0] +
                             [lg["wrench"][t0 - S.SPH_EVERY * k] - W0 for k in range(1, S.N_HIST)] +
                             [lg["probes"][t0], [d[r] / S.SPH_EVERY]] + lags)
        assert np.allclose(X[r], exp.astype(np.float32))
        # the residual columns are the last SPH wrench: the fallback's output
        assert np.array_equal(X[r, S.RES_COL:S.RES_COL + 6], W0.astype(np.float32))
        assert np.array_equal(Y[r], lg["wrench"][t[r]].astype(np.float32))


def test_hold_baselines():
    rng = np.random.default_rng(5)
    lg = _log(300, rng)
    t, d = np.arange(100, 300), (np.arange(100, 300) - 3) % S.SPH_EVERY
    zoh, avg = S.baselines(lg, t, d)
    W = lg["wrench"]
    assert np.array_equal(zoh, W[t - d])
    for i in (0, 57, 199):
        held = [W[(t[i] - j) - ((d[i] - j) % S.SPH_EVERY)] for j in range(S.SPH_EVERY)]
        assert np.allclose(avg[i], np.mean(held, 0), rtol=1e-13)
    # a constant wrench is held exactly
    lg["wrench"] = np.tile(np.arange(6.0), (300, 1))
    z2, a2 = S.baselines(lg, t, d)
    assert np.array_equal(z2, lg["wrench"][t]) and np.allclose(a2, lg["wrench"][t], rtol=1e-15)


class _Scene:
    info = {"radius": 0.05}
    params = {"rho0": 1000.0}


def test_wrench_error_floor():
    V = 4.0 / 3.0 * math.pi * 0.05 ** 3
    fF = 1000.0 * 9.81 * V
    truth = np.zeros((2, 6))
    pred = np.array([[0.1 * fF, 0, 0, 0, 0, 0], [0, 0, 0, 0, 0, 0.2 * fF * 0.1]])
    e = S.wrench_errors(pred, truth, _Scene())
    assert np.allclose(e, [0.1, 0.2], rtol=1e-12)
    big = np.array([[10 * fF, 0, 0, 0, 0, 0]])
    assert np.allclose(S.wrench_errors(big * 1.01, big, _Scene()), [0.01], rtol=1e-9)


def test_force_spectrum_bands():
    t = np.arange(3000) * 1e-3
    for f, band in ((5.0, "2-10 Hz"), (30.0, "25-50 Hz"), (70.0, "50-100 Hz")):
        W = np.zeros((3000, 6))
        W[:, 1] = 2.0 + np.sin(2 * math.pi * f * t)
        share = S.force_spectrum({"wrench": W})
        assert share[band] > 0.999, (f, share)
        assert abs(sum(share.values()) - 1.0) < 1e-9


def test_second_stage_is_a_rolling_mean_of_the_haptic_wrench():
    rng = np.random.default_rng(6)
    lg = _log(300, rng)
    out = S.second_stage(lg, n=40)
    W = lg["wrench"]
    for t in (0, 5, 39, 40, 299):
        assert np.allclose(out["wrench"][t], W[max(0, t - 39):t + 1].mean(0), rtol=1e-12, atol=1e-12)
    assert out["c"] is lg["c"] and np.array_equal(lg["wrench"], W)     # the input log is not changed


def test_walks_continue_where_the_previous_one_ended():
    """A segment's pose stream starts from the state one tick after the
    previous segment (position, orientation and velocities carried over)."""
    import types
    sc = types.SimpleNamespace(info={"c0": np.array([0.3, 0.25, 0.25]), "walk_lo": (0.12, 0.12, 0.12),
                                     "walk_hi": (0.43, 0.38, 0.40)})
    for kind in ("haptic", "coupled"):
        st0 = S.start_state(sc)
        (C, Q, V, W), st1 = S.walk(kind, sc, 7, 50, st0)
        assert C.shape == (50, 3) and np.array_equal(C[0], st0[0]) and np.array_equal(Q[0], st0[1])
        (C2, Q2, V2, W2), _ = S.walk(kind, sc, 8, 20, st1)
        for a, b in zip((C2[0], Q2[0], V2[0], W2[0]), st1):
            assert np.array_equal(a, b)
        # one tick after the last sample of the first walk: a small step, not a jump
        assert np.linalg.norm(C2[0] - C[-1]) < 1e-3 * 5.0 and abs(abs(Q2[0] @ Q[-1]) - 1.0) < 1e-4


def test_merge_logs_pools_training_walks(tmp_path):
    rng = np.random.default_rng(9)
    a = [_log(120, rng) for _ in range(5)]     # 3 training, 1 held out, 1 evaluated
    b = [_log(120, rng) for _ in range(4)]     # 2 training, then 2 evaluated
    S.write_logs(tmp_path / "a.npz", a, 3)
    S.write_logs(tmp_path / "b.npz", b, 2)
    nt, ne = S.merge_logs(tmp_path / "m.npz", [tmp_path / "a.npz", tmp_path / "b.npz"])
    assert (nt, ne) == (5, 3)
    logs, n_train = S.load_logs(tmp_path / "m.npz")
    assert n_train == 5 and len(logs) == 9
    order = a[:3] + b[:2] + [a[3]] + [a[4]] + b[2:]
    for got, want in zip(logs, order):
        for k in want:
            assert np.array_equal(got[k], want[k].astype(np.float32).astype(np.float64))

