"""Learned haptic-rate wrench surrogate around the SPH step (arXiv 2511.15908
Sec. 3.3): data collection through the SPH C ABI, feature rows, training and
haptic-tick inference through the MLP C ABI.  Argument marshalling and
bookkeeping only: the physics and the network run in libsph.so."""
from __future__ import annotations

import copy
import math
import sys

import numpy as np

from . import scenes

P_INIT = 40    # SplitMix64 purpose ids of the surrogate's random draws
P_BATCH = 41


def init_params(seed, hidden, layers, n_in, n_out):
    """LeCun-uniform initial weights (variance 1/fan_in over the real inputs),
    zero biases, padded rows and columns zero; flat parameter layout of
    include/sph_mlp.h."""
    rng = scenes.SplitMix64(seed, P_INIT)
    parts = []
    k0 = 128 if n_in <= 128 else 256          # padded input width of the parameter layout
    shapes = [(hidden, k0, n_in)] + [(hidden, hidden, hidden)] * (layers - 1) + [(16, hidden, hidden)]
    for li, (n, k, fan) in enumerate(shapes):
        a = math.sqrt(3.0 / fan)
        W = (2.0 * rng.uniform(n * k) - 1.0).reshape(n, k) * a
        W[:, fan:] = 0.0
        if li == len(shapes) - 1:
            W[n_out:] = 0.0
        parts += [W.ravel(), np.zeros(n)]
    return np.concatenate(parts).astype(np.float32)


# --------------------------------------------------------------------------
# haptic loop bookkeeping
# --------------------------------------------------------------------------
# Per 1 kHz tick t the haptic loop knows: the device pose and velocities at t
# (13 inputs), the last N_HIST wrenches that SPH delivered at its slower rate,
# every SPH_EVERY ticks (the newest, W(t0), as is; the older ones as
# differences from it: 48), the probe densities of the SPH state at t0 (64
# body-frame points at probe_radius), t - t0 in units of SPH_EVERY (1), and
# the device's recent velocities, which it samples every tick: v and w at
# t - j for the lags V_LAGS, as differences from v(t), w(t) (60) -- 186
# inputs.  The body's recent accelerations drive the fluid's reaction
# (added mass, pressure waves), and the rolling mean spans the last 40
# ticks; without them the network cannot tell how the body moved since t0.
# The network predicts the change W(t) - W(t0) (residual output over input
# columns RES_COL..RES_COL+5).

N_HIST = 8
SPH_EVERY = 10
GUARD_MARGIN = 0.5     # plain-SPH fallback outside the training range widened by half of it per side
N_PROBES = 64
V_LAGS = (1, 2, 3, 5, 7, 10, 14, 20, 28, 40)
N_FEATURES = 13 + 6 * N_HIST + N_PROBES + 1 + 6 * len(V_LAGS)
RES_COL = 13


def probe_points(scene):
    """Body-frame probe points: a Fibonacci sphere of N_PROBES points one
    lattice spacing outside the grabbed sphere."""
    return scenes.fibonacci_sphere(N_PROBES, scene.info["probe_radius"], (0.0, 0.0, 0.0))


def make_sim(scene, device="cuda", max_ticks=4000, per_tick=4, batch=1):
    """`batch` copies of the haptic scene stepped together in one context (one
    walk each), each with the body-frame probes on its own grabbed sphere and
    a per-step body and probe log long enough for a walk of max_ticks ticks."""
    from ._binding import Sim
    k = int(batch)
    if k < 1:
        raise ValueError("batch must be >= 1")
    sim = Sim([scene] * k, device=device, max_probes=N_PROBES * k, log_steps=per_tick * max_ticks)
    sim.bodies = [int(sim.obj0[i]) + scene.info["body"] for i in range(k)]
    sim.set_probes(np.tile(probe_points(scene), (k, 1)), np.repeat(np.asarray(sim.bodies, np.int32), N_PROBES))
    sim.per_tick = per_tick
    sim.wrench_tail = [np.zeros((0, 6)) for _ in range(k)]   # last per-step wrenches, for the rolling mean
    return sim


def make_net(max_batch=4096, device="cuda", seed=1, hidden=256, layers=3):
    from .mlp import Mlp
    net = Mlp(N_FEATURES, 6, hidden=hidden, layers=layers, max_batch=max_batch, device=device, residual_col=RES_COL)
    net.set_params(init_params(seed, hidden, layers, N_FEATURES, 6))
    return net


def tick_means(tail, steps, per_tick, K):
    """The haptic wrench at the end of every tick: the mean of the last
    min(K, available) per-step wrenches, where `tail` holds the (at most
    K - 1) per-step wrenches before `steps` ([per_tick * ticks][6]).  Returns
    the [ticks][6] means and the tail for the next call."""
    allw = np.concatenate([tail, steps])
    cs = np.concatenate([np.zeros((1, steps.shape[1])), np.cumsum(allw, 0)])
    end = tail.shape[0] + per_tick * np.arange(1, steps.shape[0] // per_tick + 1)   # samples up to each tick's end
    start = np.maximum(end - K, 0)
    means = (cs[end] - cs[start]) / (end - start)[:, None]
    return means, (allw[-(K - 1):] if K > 1 else allw[:0])


def collect(sim, scene, walks):
    """Drive the grabbed sphere of each scene copy with its walk (c, q, v, w
    per tick; `walks` holds one walk per copy, or is one walk for a context
    of one), sim.per_tick SPH steps per tick; log per tick the pose, the
    haptic wrench (the rolling mean of the per-step wrenches over the scene's
    smoothing window, as sph_get_body_wrench returns it at the end of the
    tick) and the probe densities.  The device logs every step, so the loop
    only enqueues work and the host reads the logs once per walk.  Returns
    one log per walk (a single log for a single walk)."""
    single = isinstance(walks[0], np.ndarray)
    if single:
        walks = [walks]
    k = len(sim.bodies)
    if len(walks) != k:
        raise ValueError(f"{len(walks)} walks for {k} scene copies")
    n = walks[0][0].shape[0]
    if any(w[0].shape[0] != n for w in walks):
        raise ValueError("the walks of one batch must have the same length")
    per_tick = sim.per_tick
    K = int(scene.params["smoothing_window"])
    if n * per_tick > sim.log_steps:
        raise ValueError(f"walk of {n} ticks exceeds the log ({sim.log_steps} steps)")
    sim.read_log()                                   # start from an empty log
    for t in range(n):
        for b, (C, Q, V, W) in zip(sim.bodies, walks):
            sim.set_body_pose(b, C[t], Q[t], V[t], W[t])
        sim.step(per_tick)
    probes = sim.read_probe_log()                    # [steps][copies * N_PROBES]
    rec = sim.read_log()                             # [steps][bodies][20]
    if rec.shape[0] != n * per_tick or probes.shape[0] != n * per_tick:
        raise RuntimeError("step log shorter than the walk")
    end_rows = per_tick * np.arange(1, n + 1) - 1
    logs = []
    for i, (b, (C, Q, V, W)) in enumerate(zip(sim.bodies, walks)):
        kb = sim.kinematic.index(b)
        wr, sim.wrench_tail[i] = tick_means(sim.wrench_tail[i], rec[:, kb, 13:19], per_tick, K)
        pr = probes[end_rows, i * N_PROBES:(i + 1) * N_PROBES]
        q = np.where(Q[:, :1] < 0, -Q, Q)
        logs.append({"c": C.copy(), "q": q, "v": V.copy(), "w": W.copy(), "wrench": wr, "probes": pr})
    return logs[0] if single else logs


def feature_rows(log, ticks, lags):
    """Input rows and targets W(t) for ticks t whose last SPH update came
    d = lags ticks earlier."""
    t = np.asarray(ticks, np.int64)
    d = np.asarray(lags, np.int64)
    t0 = t - d
    W = log["wrench"]
    w0 = W[t0]
    hist = [w0] + [W[t0 - SPH_EVERY * k] - w0 for k in range(1, N_HIST)]
    lags = []
    for j in V_LAGS:
        lags += [log["v"][t - j] - log["v"][t], log["w"][t - j] - log["w"][t]]
    X = np.concatenate([log["c"][t], log["q"][t], log["v"][t], log["w"][t]] + hist +
                       [log["probes"][t0], (d / SPH_EVERY)[:, None]] + lags, 1)
    return X.astype(np.float32), W[t].astype(np.float32)


def first_tick():
    return max(SPH_EVERY * (N_HIST - 1) + SPH_EVERY - 1, max(V_LAGS))


def training_rows(log):
    """Every tick with every phase of the SPH update grid."""
    n = log["c"].shape[0]
    t = np.arange(first_tick(), n)
    tt = np.repeat(t, SPH_EVERY)
    dd = np.tile(np.arange(SPH_EVERY), t.size)
    return feature_rows(log, tt, dd)


def eval_rows(log, phase=0):
    """Ticks t >= first_tick() with SPH updates at ticks = phase mod SPH_EVERY."""
    n = log["c"].shape[0]
    t = np.arange(first_tick(), n)
    d = (t - phase) % SPH_EVERY
    return t, d, feature_rows(log, t, d)


def baselines(log, t, d, k_avg=SPH_EVERY):
    """The haptic loop without the network: zero-order hold of the last SPH
    wrench, and the hold followed by a rolling mean over the last k_avg ticks
    (Sec. 3.3)."""
    W = log["wrench"]
    zoh = W[t - d]
    acc = np.zeros_like(zoh)
    for j in range(k_avg):
        tj = t - j
        dj = (d - j) % SPH_EVERY
        acc += W[tj - dj]
    return zoh, acc / k_avg


def predict(net, X, chunk=None):
    """Batched network outputs for the rows X (numpy), through mlp_forward."""
    import torch
    chunk = chunk or net.cfg.max_batch
    out = []
    for s in range(0, X.shape[0], chunk):
        xt = torch.from_numpy(np.ascontiguousarray(X[s:s + chunk])).to(net.device)
        out.append(net.forward(xt).cpu().numpy())
    return np.concatenate(out, 0).astype(np.float64)


def wrench_errors(pred, truth, scene):
    """Relative wrench error per tick with the floors of the parity norms:
    |dF| / max(|F|, rho0 g V), |dT| / max(|T|, rho0 g V L) (V the body volume,
    L its diameter); returns the larger of the two per tick."""
    R = scene.info["radius"]
    V = 4.0 / 3.0 * math.pi * R ** 3
    fF = scene.params["rho0"] * 9.81 * V
    fT = fF * 2 * R
    eF = np.linalg.norm(pred[:, :3] - truth[:, :3], axis=1) / np.maximum(np.linalg.norm(truth[:, :3], axis=1), fF)
    eT = np.linalg.norm(pred[:, 3:] - truth[:, 3:], axis=1) / np.maximum(np.linalg.norm(truth[:, 3:], axis=1), fT)
    return np.maximum(eF, eT)


def train(net, X, Y, steps, batch=4096, lr0=1e-3, lr1=1e-5, seed=1, holdout=None, every=250):
    """Adam on random minibatches (the library's kernels) with a cosine
    learning-rate decay; X, Y float32 device tensors.  With holdout =
    (log, scene) the parameters with the smallest held-out wrench error
    (checked every `every` steps) are kept.  Returns [(step, loss,
    held-out error)]."""
    import torch
    rng = scenes.SplitMix64(seed, P_BATCH)
    n = X.shape[0]
    net.fit_normalizer(X, Y)
    if holdout is not None:
        hlog, hscene = holdout
        th, dh, (Xh, Yh) = eval_rows(hlog)
    hist, best = [], (float("inf"), None)
    for it in range(steps):
        idx = torch.from_numpy((rng.uniform(batch) * n).astype(np.int64)).to(X.device)
        lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * it / max(steps - 1, 1)))
        net.train_step(X.index_select(0, idx), Y.index_select(0, idx), lr)
        if (it + 1) % every == 0 or it == steps - 1:
            e = float("nan")
            if holdout is not None:
                e = float(wrench_errors(predict(net, Xh), Yh.astype(np.float64), hscene)[dh > 0].mean())
                if e < best[0]:
                    best = (e, net.get_params())
            hist.append((it + 1, net.last_loss(), e))
    if best[1] is not None:
        net.set_params(best[1])
    return hist


def evaluate(net, logs, scene):
    """Errors of the surrogate and of the two baselines on the ticks between
    SPH updates (d > 0), against the plain-SPH haptic wrench at every tick;
    `logs` is one log or a list, whose ticks are pooled.  With the network's
    guard on, "surrogate" is the haptic loop with its plain-SPH fallback and
    "network_only" the network's own outputs; surrogate.fallback_frac is the
    share of evaluated rows (every tick) that fell back."""
    if isinstance(logs, dict):
        logs = [logs]
    margin = getattr(net, "guard_margin", -1.0)
    names = ("surrogate", "network_only", "zero_order_hold", "hold_rolling_mean")
    errs = {k: [] for k in names}
    n0 = net.guard_count() if margin >= 0 else (0, 0)
    for log in logs:
        t, d, (X, Y) = eval_rows(log)
        truth = Y.astype(np.float64)
        zoh, avg = baselines(log, t, d)
        p = predict(net, X)
        if margin >= 0:
            net.set_guard(-1.0)
            p_net = predict(net, X)
            net.set_guard(margin)
        else:
            p_net = p
        for name, q in zip(names, (p, p_net, zoh, avg)):
            errs[name].append(wrench_errors(q, truth, scene)[d > 0])
    out = {}
    for name, parts in errs.items():
        e = np.concatenate(parts)
        out[name] = {"mean": float(e.mean()), "p50": float(np.median(e)), "p95": float(np.percentile(e, 95)),
                     "max": float(e.max()), "walk_means": [float(x.mean()) for x in parts]}
    if margin >= 0:
        n1 = net.guard_count()
        out["surrogate"]["fallback_frac"] = (n1[1] - n0[1]) / max(n1[0] - n0[0], 1)
    return out


def force_spectrum(log, bands=((0, 2), (2, 10), (10, 25), (25, 50), (50, 100), (100, 500))):
    """Share of the haptic force's variance (sum over the three components,
    mean removed, 1 kHz samples) in each frequency band (a, b] in Hz."""
    F = log["wrench"][:, :3]
    P = (np.abs(np.fft.rfft(F - F.mean(0), axis=0)) ** 2).sum(1)
    f = np.fft.rfftfreq(F.shape[0], 1e-3)
    tot = P[1:].sum()
    return {f"{a}-{b} Hz": float(P[(f > a) & (f <= b)].sum() / tot) for a, b in bands}


# haptic output of the experiment scenes: rolling mean over 160 SPH steps =
# 40 ticks of 1 ms (Sec. 3.3, tens of haptic cycles)
HAPTIC_WINDOW = 160
SCENE_KINDS = ("haptic", "coupled")


def experiment_scene(kind, n_fluid, base=None):
    """The surrogate's scene: "haptic" (the sphere in a tank sized for
    n_fluid, a hand-like smooth walk) or "coupled" (the coupled fluid + soft +
    rigid scene with its Ornstein-Uhlenbeck random walk), both with the 40 ms
    haptic rolling mean.  base: an already built scene of that kind, used
    with its own parameters copied (it is not changed)."""
    if kind not in SCENE_KINDS:
        raise ValueError(f"scene kind must be one of {SCENE_KINDS}")
    if base is not None:
        sc = copy.copy(base)
        sc.params = dict(base.params)
    elif kind == "haptic":
        return scenes.haptic_scene(n_fluid=n_fluid)
    else:
        sc = scenes.coupled_1m(n_fluid=n_fluid)
    sc.params["smoothing_window"] = HAPTIC_WINDOW
    return sc


def start_state(scene):
    """Pose stream state (c, q, v, w) at the scene's initial pose, at rest."""
    return (np.asarray(scene.info["c0"], np.float64), np.array([1.0, 0, 0, 0]), np.zeros(3), np.zeros(3))


def walk(kind, scene, seed, n, state):
    """n ticks of the scene kind's pose stream from `state` (c, q, v, w);
    returns the walk (c, q, v, w arrays) and the state one tick after it, where
    the next walk continues."""
    c, q, v, w = state
    lo, hi = scene.info["walk_lo"], scene.info["walk_hi"]
    if kind == "haptic":
        C, Q, V, W = scenes.smooth_walk(seed, n + 1, c, lo, hi, q0=q, v0=v, w0=w)
    else:
        C, Q, V, W = scenes.random_walk(seed, n + 1, c, box_lo=lo, box_hi=hi, q0=q, v0=v, w0=w)
    return (C[:n], Q[:n], V[:n], W[:n]), (C[n], Q[n], V[n], W[n])


def spectrum_run(n_fluid, ticks=3000, warmup_ticks=300, kind="haptic"):
    """Band shares of the haptic force over one walk (seed 101) after a
    warm-up walk (seed 11), one context."""
    sc = experiment_scene(kind, n_fluid)
    sim = make_sim(sc, max_ticks=max(ticks, warmup_ticks))
    st = start_state(sc)
    for n, sd in ((warmup_ticks, 11), (ticks, 101)):
        wk, st = walk(kind, sc, sd, n, st)
        lg = collect(sim, sc, wk)
    return force_spectrum(lg)


def haptic_rate(net, X, n=500):
    """Haptic ticks per second of the one-workgroup chain: host round trip
    (features in, wrench out, synchronised) and device-only back to back."""
    import time
    import torch
    for k in range(10):
        net.predict_one(X[k % X.shape[0]])
    t0 = time.perf_counter()
    for k in range(n):
        net.predict_one(X[k % X.shape[0]])
    host = n / (time.perf_counter() - t0)
    xd = torch.from_numpy(np.ascontiguousarray(X[:n])).to(net.device)
    yd = torch.zeros((xd.shape[0], 6), device=net.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(xd.shape[0]):
        net.predict_one_device(xd[k], yd[k])
    e1.record()
    torch.cuda.synchronize()
    dev = xd.shape[0] / (e0.elapsed_time(e1) * 1e-3)
    return {"host_round_trip_hz": host, "device_chain_hz": dev}


def load_logs(path):
    """Logs kept by run_experiment(save_logs=...): (logs, number of training walks)."""
    z = np.load(path)
    logs, i = [], 0
    while f"{i}_c" in z:
        logs.append({k: z[f"{i}_{k}"].astype(np.float64) for k in ("c", "q", "v", "w", "wrench", "probes")})
        i += 1
    return logs, int(z["n_train"])


def write_logs(path, logs, n_train):
    np.savez_compressed(path, n_train=n_train, **{f"{i}_{key}": a.astype(np.float32)
                                                 for i, lg in enumerate(logs) for key, a in lg.items()})


def merge_logs(out, paths):
    """Pool the logs of several runs (made with different walk_seed0): every
    run's training walks train, the first run's held-out walk stays the
    held-out walk, and every other walk (the other runs' held-out walks
    included) is evaluated."""
    train, hold, ev = [], None, []
    for p in paths:
        lg, nt = load_logs(p)
        train += lg[:nt]
        if hold is None:
            hold, ev = lg[nt], ev + lg[nt + 1:]
        else:
            ev += lg[nt:]
    write_logs(out, train + [hold] + ev, len(train))
    return len(train), len(ev)


def second_stage(log, n=HAPTIC_WINDOW // 4):
    """A copy of the log whose haptic wrench passes a second rolling mean over
    the last n ticks (partial at the walk's start): the two boxcars make a
    triangular window twice as long, which damps the band the 100 Hz updates
    cannot follow far more than one boxcar does."""
    W = log["wrench"]
    c = np.concatenate([np.zeros((1, W.shape[1])), np.cumsum(W, 0)])
    t = np.arange(W.shape[0])
    lo = np.maximum(t + 1 - n, 0)
    out = dict(log)
    out["wrench"] = (c[t + 1] - c[lo]) / (t + 1 - lo)[:, None]
    return out


def train_and_evaluate(logs, n_train, sc, steps, seed=1, guard_margin=GUARD_MARGIN, stages=1):
    """Train on logs[:n_train] with early stopping on logs[n_train], evaluate on
    the rest (with stages = 2 the haptic wrench of every log passes a second
    rolling mean first); returns (net, summary dict)."""
    import time
    import torch
    if stages == 2:
        logs = [second_stage(lg) for lg in logs]
    elif stages != 1:
        raise ValueError("stages must be 1 or 2")
    rows = [training_rows(lg) for lg in logs[:n_train]]
    X = torch.from_numpy(np.concatenate([r[0] for r in rows])).to("cuda")
    Y = torch.from_numpy(np.concatenate([r[1] for r in rows])).to("cuda")
    del rows
    net = make_net(seed=seed)
    t0 = time.perf_counter()
    hist = train(net, X, Y, steps, seed=seed, holdout=(logs[n_train], sc))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    if guard_margin is not None and guard_margin >= 0:
        net.set_guard(guard_margin)
    errs = evaluate(net, logs[n_train + 1:], sc)
    return net, {"training_rows": int(X.shape[0]), "train_s": t_train, "train_steps": steps,
                 "best_holdout_error": min(h[2] for h in hist), "errors": errs}


def haptic_under_load(kind="haptic", n_fluid=100_000, seconds=2.0, scene=None, seed=1, log=print):
    """The 1 kHz haptic chain and plain SPH on one GPU at the same time, on two
    streams of default priority: a host thread keeps SPH steps of the scene
    queued on one stream (4 per tick, at most ~40 steps ahead) while the
    haptic loop, paced by the wall clock at 1 ms, runs the one-workgroup
    network chain on the other (features in, wrench out, its own stream
    synchronised) with the plain-SPH fallback off, so every tick runs the
    whole network.  Reports the chain's latency alone and under load, the
    ticks whose latency exceeded the 1 ms period, and the SPH step rate alone
    and under the haptic load."""
    import threading
    import time
    import torch
    from ._binding import Sim
    sc = experiment_scene(kind, n_fluid, base=scene)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    sim = Sim(sc, stream=sa)
    with torch.cuda.stream(sb):
        net = make_net(seed=seed, max_batch=256)
        rng = scenes.SplitMix64(seed, P_BATCH + 1)
        X = torch.from_numpy(rng.normal(256 * N_FEATURES).reshape(256, N_FEATURES).astype(np.float32)).cuda()
        Y = torch.from_numpy(rng.normal(256 * 6).reshape(256, 6).astype(np.float32)).cuda()
        net.fit_normalizer(X, Y)
        net.set_guard(-1.0)
    xs = X.cpu().numpy()

    def chain_latency(n):
        lat = np.empty(n)
        for k in range(n):
            t0 = time.perf_counter()
            net.predict_one(xs[k % xs.shape[0]])
            lat[k] = time.perf_counter() - t0
        return lat

    chain_latency(50)
    idle = chain_latency(500)
    # SPH alone
    sim.step(40)
    sa.synchronize()
    t0 = time.perf_counter()
    sim.step(200)
    sa.synchronize()
    sph_alone = 200 / (time.perf_counter() - t0)
    # both at once
    stop = threading.Event()
    done = [0]

    def sph_worker():
        evs = []
        while not stop.is_set():
            sim.step(4)
            e = torch.cuda.Event()
            e.record(sa)
            evs.append(e)
            done[0] += 4
            if len(evs) > 10:                 # keep about 40 steps queued
                evs.pop(0).synchronize()
        sa.synchronize()

    # the SPH thread hands the interpreter lock back within 0.2 ms (the
    # default switch interval, 5 ms, would hold a tick back for that long)
    switch = sys.getswitchinterval()
    sys.setswitchinterval(2e-4)
    th = threading.Thread(target=sph_worker)
    th.start()
    time.sleep(0.2)                           # let the SPH queue fill
    n_ticks = int(seconds * 1000)
    lat = np.empty(n_ticks)
    delay = np.empty(n_ticks)
    late = 0
    steps0, t_start = done[0], time.perf_counter()
    for k in range(n_ticks):
        due = t_start + 1e-3 * k
        rest = due - time.perf_counter()
        if rest > 3e-4:
            time.sleep(rest - 3e-4)               # sleeping lets the SPH thread run
        while time.perf_counter() < due:
            pass
        t0 = time.perf_counter()
        net.predict_one(xs[k % xs.shape[0]])
        lat[k] = time.perf_counter() - t0
        delay[k] = t0 - due
        late += int(t0 + lat[k] > due + 1e-3)
    wall = time.perf_counter() - t_start
    steps = done[0] - steps0
    stop.set()
    th.join()
    sys.setswitchinterval(switch)
    us = lambda a, q: round(float(np.percentile(a, q)) * 1e6, 1)   # noqa: E731
    r = {"scene": sc.name, "n_particles": int(sc.n), "ticks": n_ticks,
         "chain_latency_us_alone": {"p50": us(idle, 50), "p99": us(idle, 99), "max": round(float(idle.max()) * 1e6, 1)},
         "chain_latency_us_under_sph": {"p50": us(lat, 50), "p99": us(lat, 99),
                                        "max": round(float(lat.max()) * 1e6, 1)},
         "tick_start_delay_us": {"p99": us(delay, 99), "max": round(float(delay.max()) * 1e6, 1)},
         "ticks_past_their_1ms_period": late, "haptic_hz_achieved": round(n_ticks / wall, 1),
         "sph_steps_per_s_alone": round(sph_alone, 1), "sph_steps_per_s_with_haptic": round(steps / wall, 1)}
    log(f"  haptic chain under SPH load: {r}")
    sim.close()
    net.close()
    return r


def run_experiment(n_fluid=100_000, train_segments=4, ticks=3000, eval_ticks=1500, steps=1500, seed=1,
                   warmup_ticks=300, eval_segments=3, batch=1, guard_margin=GUARD_MARGIN, log=print,
                   kind="haptic", save_logs=None, scene=None, walk_seed0=0, two_stages=False):
    """Collect plain-SPH haptic logs (a 1 kHz smooth walk per segment, 4 SPH
    steps per tick), train on the first segments with early stopping on a
    held-out segment, evaluate on the last ones (pooled: a single walk's
    smoothness swings the hold baseline's error several-fold).

    `batch` copies of the scene are stepped together, one walk each: every
    copy first takes a warm-up walk, then the copies walk in rounds; the
    training walks are train_segments rounded up to a multiple of the batch,
    the first walk after them is the held-out one and the rest, at least
    eval_segments, are evaluated.  A copy's walk starts where its previous one
    ended.  After training the network's plain-SPH fallback is set with
    guard_margin (None: no fallback).  `kind` picks the scene and its pose
    stream (experiment_scene); save_logs, a path, keeps the logs (float32,
    npz) for study away from the GPU; scene, an already built scene of that
    kind, saves building it again; walk_seed0 shifts every walk seed (runs
    whose logs are pooled); two_stages also trains and evaluates a second
    network on the same logs with the haptic wrench passed through a second
    rolling mean (summary under "two_stages").  Returns a summary dict."""
    import time
    import torch
    k = int(batch)
    sc = experiment_scene(kind, n_fluid, base=scene)
    sim = make_sim(sc, max_ticks=max(warmup_ticks, ticks, eval_ticks), batch=k)
    sts = [start_state(sc)] * k
    n_train = -(-train_segments // k) * k
    n_eval = -(-(1 + eval_segments) // k) * k
    w0 = int(walk_seed0)
    rounds = [(warmup_ticks, [w0 + 11 + i for i in range(k)])]
    rounds += [(ticks, [w0 + 101 + j for j in range(r, r + k)]) for r in range(0, n_train, k)]
    ev = [w0 + 801] + [w0 + 901 + j for j in range(n_eval - 1)]
    rounds += [(eval_ticks, ev[r:r + k]) for r in range(0, n_eval, k)]
    logs = []
    t0 = time.perf_counter()
    for n, seeds in rounds:
        ws = [walk(kind, sc, sd, n, st) for sd, st in zip(seeds, sts)]
        logs += collect(sim, sc, [w for w, _ in ws])
        sts = [st for _, st in ws]
        log(f"  collected {n} ticks x {k} (walk seeds {seeds[0]}..{seeds[-1]})")
    t_collect = time.perf_counter() - t0
    logs = logs[k:]                                  # warm-up walks
    if save_logs:
        write_logs(save_logs, logs, n_train)
    net, res = train_and_evaluate(logs, n_train, sc, steps, seed=seed, guard_margin=guard_margin)
    rate = haptic_rate(net, eval_rows(logs[-1])[2][0])
    out = {"scene": sc.name, "n_particles": int(sc.n), "batch": k, "training_walks": n_train,
           "eval_walks": n_eval - 1, "ticks_collected": int(sum(n * len(sd) for n, sd in rounds)),
           "collect_s": t_collect, **res, **rate}
    if two_stages:
        out["two_stages"] = train_and_evaluate(logs, n_train, sc, steps, seed=seed, guard_margin=guard_margin,
                                               stages=2)[1]
    return out


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="plain-SPH haptic logs -> surrogate training -> evaluation")
    ap.add_argument("--n-fluid", type=int, default=100_000)
    ap.add_argument("--segments", type=int, default=4)
    ap.add_argument("--ticks", type=int, default=3000)
    ap.add_argument("--eval-ticks", type=int, default=1500)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--eval-segments", type=int, default=3)
    ap.add_argument("--batch", type=int, default=1, help="scene copies stepped together, one walk each")
    ap.add_argument("--scene", choices=SCENE_KINDS, default="haptic",
                    help="haptic: sphere in a tank sized for n_fluid, smooth walk; coupled: the coupled "
                         "fluid + soft + rigid scene with its random walk")
    ap.add_argument("--save-logs", default=None, help="keep the collected logs in this .npz file")
    ap.add_argument("--walk-seed0", type=int, default=0, help="shift of every walk seed (runs pooled later)")
    ap.add_argument("--haptic-stages", type=int, default=1, choices=(1, 2),
                    help="2: the haptic wrench passes a second rolling mean over 40 ticks (with --load-logs)")
    ap.add_argument("--under-load", action="store_true",
                    help="only time the 1 kHz haptic chain while plain SPH runs on the same GPU")
    ap.add_argument("--merge-logs", nargs="+", default=None, metavar="PATH",
                    help="OUT IN1 IN2 ...: pool the logs of several runs into OUT (no GPU work)")
    ap.add_argument("--load-logs", default=None,
                    help="train and evaluate on logs kept by --save-logs (scene from --scene, --n-fluid)")
    ap.add_argument("--spectrum", action="store_true",
                    help="only the band shares of the haptic force over one walk (no training)")
    a = ap.parse_args()
    if a.spectrum:
        print(json.dumps({"n_fluid": a.n_fluid, "scene": a.scene,
                          "band_share": spectrum_run(a.n_fluid, kind=a.scene)}), flush=True)
        raise SystemExit(0)
    if a.under_load:
        print(json.dumps(haptic_under_load(a.scene, a.n_fluid, log=lambda m: print(m, flush=True))), flush=True)
        raise SystemExit(0)
    if a.merge_logs:
        nt, ne = merge_logs(a.merge_logs[0], a.merge_logs[1:])
        print(json.dumps({"merged": a.merge_logs[0], "training_walks": nt, "eval_walks": ne}), flush=True)
        raise SystemExit(0)
    if a.load_logs:
        lg, nt = load_logs(a.load_logs)
        sc = experiment_scene(a.scene, a.n_fluid)
        _, r = train_and_evaluate(lg, nt, sc, a.steps, stages=a.haptic_stages)
        print(json.dumps({"scene": sc.name, "logs": a.load_logs, "haptic_stages": a.haptic_stages,
                          "training_walks": nt,
                          "eval_walks": len(lg) - nt - 1, **r}), flush=True)
        raise SystemExit(0)
    r = run_experiment(a.n_fluid, a.segments, a.ticks, a.eval_ticks, a.steps, eval_segments=a.eval_segments,
                       batch=a.batch, log=lambda m: print(m, flush=True), kind=a.scene, save_logs=a.save_logs,
                       walk_seed0=a.walk_seed0)
    print(json.dumps(r), flush=True)
