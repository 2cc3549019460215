"""Benchmark of the SPH hot path on one MI355X.

Workload: the coupled fluid + soft + rigid scene at 1M fluid particles
(1,000,000 fluid, 8,000 soft with 66,120 springs, a 3,079-particle grabbed
sphere driven by a seeded 1 kHz random-walk pose, 59,569 tank particles;
FP32, dt = 2.5e-4 s).  One step = one sph_step (placement, neighbour search,
springs, density, forces, FP64 body wrench, integration); the sphere's pose
is set every 4 steps (1 kHz).  Inputs are resident in HBM before timing.

    python bench.py [--gpus 1] [--steps 100] [--warmup 10]

Prints one JSON line.  value = (fluid + soft) particle updates per second.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
# Plain (non-packed) VALU lane operations per second: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz (the published FP32 figure counts an FMA as 2 and packed
# FP32 as 2 more: 157.3 / 4).
PEAK_LANE_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# Algorithmic work of the neighbour sums in VALU lane operations (add, mul,
# fma, compare = 1; sqrt, reciprocal = 4): a candidate test costs 7 (three
# differences, r^2, compare); the method needs 1000 candidate tests per
# particle (5^3 stencil of cells of size h around each particle) and
# 14 lane-ops per neighbour for the density term and 45 for the force term.
LANE_OPS_CANDIDATE = 7
CANDIDATES_PER_PARTICLE = 1000
LANE_OPS_DENSITY_PAIR = 14
LANE_OPS_FORCE_PAIR = 45
# The same in FLOPs (FMA = 2) as written in the oracle, for reference.
FLOP_DENSITY_PAIR = 17
FLOP_FORCE_PAIR = 49
# Compulsory HBM bytes per particle of the memory-bound phases (FP32 SoA,
# unfused): keys 12 + type word 4 (the key launch also places the kinematic
# bodies' particles) + key 4 + arrival rank 4; counting sort: scatter 8 + 4
# (the slot scan adds 16 B per slot, under 1 B per particle at 1M);
# reorder arrived 4 + key 4 + 32 + 32 + inverse 4 + cell bounds 6;
# integrate 40 + 24.  The whole step, neighbour sums included (their
# compulsory traffic: 24 and 48), is 254 bytes per particle.
HBM_BYTES_PER_PARTICLE = {"keys": 24, "sort": 12, "reorder": 82, "integrate": 64}
HBM_BYTES_STEP_PER_PARTICLE = 254
# Kernel times come from HIP events on every PROFILE_EVERY-th timed step
# (the event records cost a few microseconds each, two per phase).
PROFILE_EVERY = 4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="coupled_1m")
    ap.add_argument("--n-fluid", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 256-scene batch leg (graph-replayed steps of independent stirring tanks)")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the haptic-rate surrogate legs (16 copies of the 100k haptic scene: logs, training, "
                         "evaluation, about 2 minutes; then a short run on the coupled 1M scene, about 1.5 minutes)")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the 256-scene batch leg and print its record (for profiling it alone)")
    ap.add_argument("--mlp-train-only", action="store_true",
                    help="run only surrogate training steps (batch 4096, 186-256-256-256-6) and print their "
                         "rate in matrix-core FLOP/s (for profiling the MFMA kernels)")
    return ap.parse_args()


def log(msg, quiet=False):
    if not quiet:
        print(msg, file=sys.stderr, flush=True)


def _omp(threads):
    """Set the OpenMP team size of the oracle's parallel loops (libgomp)."""
    import ctypes
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(threads))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time_oracle(scene, steps):
    import oracle
    o = oracle.Oracle(scene, scene.precision)
    nmov = int((scene.type != 2).sum())
    t0 = time.perf_counter()
    for _ in range(steps):
        o.step()
    dt = time.perf_counter() - t0
    return {"particle_updates_per_s": nmov * steps / dt, "s_per_step": dt / steps, "steps": steps,
            "n_particles": int(scene.n), "n_fluid_soft": nmov}


def cpu_baseline(scene, log_fn=None):
    """The oracle as it stands, timed on the host cores: whole FP64 oracle
    steps (neighbour lists, density, forces, springs, wrench, integration).
    value: 3 steps of the benchmark scene on all cores; beside it one step on
    one core, the FP64 dam break in full (100 steps) on all cores and for
    10 steps on one core, and 3 steps of the 250k stirring tank on all cores."""
    import oracle
    from paper_2511_15908_amd import scenes
    oracle.build(force=False)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    say = log_fn or (lambda m: None)
    _omp(cores)
    say(f"cpu baseline: benchmark scene, 3 steps on {cores} threads")
    allc = _time_oracle(scene, 3)
    _omp(1)
    say("cpu baseline: benchmark scene, 1 step on 1 thread")
    one = _time_oracle(scene, 1)
    dam = scenes.dam_break()
    say("cpu baseline: dam break (FP64, 100 steps) on all threads, 10 steps on 1 thread")
    _omp(cores)
    dam_all = _time_oracle(dam, 100)
    _omp(1)
    dam_one = _time_oracle(dam, 10)
    _omp(cores)
    say("cpu baseline: stirring tank (250k fluid, FP32 state), 3 steps on all threads")
    stir = _time_oracle(scenes.stirring_tank(), 3)
    return {"value": allc["particle_updates_per_s"], "unit": "particle-updates/s", "cores": cores,
            "kind": "oracle", "cpu_model": _cpu_model(),
            "sample": f"3 full FP64 oracle steps of the same {scene.n:,}-particle scene "
                      f"({allc['n_fluid_soft']:,} fluid+soft) on {cores} threads, "
                      f"{3 * allc['s_per_step']:.1f} s wall",
            "one_thread": {"value": one["particle_updates_per_s"], "sample": "1 step of the same scene",
                           "s_per_step": round(one["s_per_step"], 2)},
            "dam_break_fp64": {"n_particles": dam_all["n_particles"],
                               "all_threads": {"value": dam_all["particle_updates_per_s"], "steps": 100,
                                               "s_per_step": round(dam_all["s_per_step"], 4)},
                               "one_thread": {"value": dam_one["particle_updates_per_s"], "steps": 10,
                                              "s_per_step": round(dam_one["s_per_step"], 4)}},
            "stirring_250k": {"n_particles": stir["n_particles"],
                              "all_threads": {"value": stir["particle_updates_per_s"], "steps": 3,
                                              "s_per_step": round(stir["s_per_step"], 3)}}}


def profiled_traffic(kernel, n_particles):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 summary,
    only for the workload it was taken on (the 1M coupled scene, by its
    particle count) and while the profiled kernel source is unchanged."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_sums_coupled_1m_traffic.json")
    src = os.path.join(ROOT, "paper_2511_15908_amd", "csrc", "k_sums.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    if rec.get("source_sha256_k_sums") != sha or kernel not in rec.get("kernels", {}):
        return None
    if rec.get("n_particles") != n_particles:
        return None
    return rec["kernels"][kernel]["bytes"]


def batch_leg(dev, n_scenes=256, steps=64):
    """The batched data-generation workload: independent stirring tanks in one
    context (one launch per kernel for all scenes), paddles on device pose
    tracks, two-step graph replays, per-step body log."""
    import torch
    import paper_2511_15908_amd as P
    from paper_2511_15908_amd import scenes
    scs = scenes.stirring_batch(seed=4, n_scenes=n_scenes)
    st = torch.cuda.Stream(device=dev)
    sim = P.Sim(scs, device=dev, stream=st, log_steps=steps + 2, track_steps=steps + 2)
    sim.set_graph(True)
    dt = scs[0].params["dt"]
    for i, sc in enumerate(scs):
        tr = np.array([np.concatenate(scenes.batch_pose(sc, k * dt)) for k in range(steps + 2)])
        sim.set_body_track(int(sim.obj0[i]) + 1, tr)
    sim.step(2)
    sim.synchronize()
    s0 = sim.stats()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    el = time.perf_counter() - t0
    s1 = sim.stats()
    log = sim.read_log()
    nf = sum(sc.counts()["fluid"] for sc in scs)
    d = {k: (s1[k] - s0[k]) / steps for k in s0}
    n_all = sum(sc.n for sc in scs)
    return {"workload": f"{n_scenes} independent stirring tanks, 2k-30k fluid each (log-uniform), "
                        f"{n_all:,} particles, dt = 5e-4 s",
            "steps": steps, "ms_per_step": 1e3 * el / steps, "fluid_updates_per_s": nf * steps / el,
            "particle_updates_per_s": n_all * steps / el,
            "log_records": int(log.shape[0] * log.shape[1]),
            "per_particle": {"density_pairs": d["pairs_density"] / n_all, "force_pairs": d["pairs_force"] / n_all,
                             "candidate_tests": d["candidates"] / n_all},
            "lane_efficiency_density": d["pairs_density"] / max(64 * d["iter_density"], 1),
            "lane_efficiency_force": d["pairs_force"] / max(64 * d["iter_force"], 1),
            "particles_per_wavefront": n_all / max(d["waves"], 1)}


# Dense products of one surrogate training step per sample (186 inputs padded
# to 256, three hidden layers of 256, 6 outputs padded to 16): forward
# X W^T of every layer, weight gradients dZ^T A of every layer, and the data
# gradients dZ W of every layer but the first; 2 FLOP per multiply-add.
MLP_SHAPES = [(256, 256), (256, 256), (256, 256), (16, 256)]
MLP_FLOP_PER_SAMPLE = 2 * (2 * sum(n * k for n, k in MLP_SHAPES) + sum(n * k for n, k in MLP_SHAPES[1:]))
PEAK_BF16_TFLOPS = 2500.0


def mlp_train_leg(dev, steps=200, warmup=20, batch=4096):
    """Training steps of the wrench surrogate on synthetic rows (the
    library's BF16-MFMA kernels), timed with HIP events on the network's
    stream."""
    import torch
    from paper_2511_15908_amd import mlp, scenes, surrogate
    rng = scenes.SplitMix64(77, 9)
    n_in, n_out = surrogate.N_FEATURES, 6
    X = torch.tensor(rng.normal(batch * n_in).reshape(batch, n_in).astype(np.float32), device=dev)
    Y = torch.tensor(rng.normal(batch * n_out).reshape(batch, n_out).astype(np.float32), device=dev)
    net = mlp.Mlp(n_in, n_out, hidden=256, layers=3, max_batch=batch, device=dev)
    net.set_params(surrogate.init_params(7, 256, 3, n_in, n_out))
    net.fit_normalizer(X, Y)
    for _ in range(warmup):
        net.train_step(X, Y, 1e-4)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(steps):
        net.train_step(X, Y, 1e-4)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    tflops = MLP_FLOP_PER_SAMPLE * batch / (ms * 1e-3) / 1e12
    return {"batch": batch, "steps": steps, "ms_per_train_step": round(ms, 4),
            "flop_per_step": MLP_FLOP_PER_SAMPLE * batch, "achieved_tflops": round(tflops, 3),
            "peak_bf16_tflops": PEAK_BF16_TFLOPS, "frac": round(tflops / PEAK_BF16_TFLOPS, 5),
            "loss": net.last_loss()}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported (single-GPU build)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2511_15908_amd as P
    from paper_2511_15908_amd import scenes

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.calibrate_copy:
        nbytes = 1 << 30
        src = torch.ones(nbytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "copies": 3}))
        return
    if a.batch_only:
        print(json.dumps({"batch": batch_leg(dev)}), flush=True)
        return
    if a.mlp_train_only:
        print(json.dumps({"mlp_train": mlp_train_leg(dev)}), flush=True)
        return
    t0 = time.perf_counter()
    sc = scenes.coupled_1m(n_fluid=a.n_fluid)
    log(f"scene {sc.name}: {sc.counts()} built in {time.perf_counter() - t0:.1f} s", a.quiet)
    sim = P.Sim(sc, device=dev)
    info = sim.info()
    dt = sc.params["dt"]
    body = 1
    per_tick = 4                                     # 1 kHz pose updates at dt = 2.5e-4
    n_ticks = (a.warmup + a.steps) // per_tick + 2
    C_, Q_, V_, W_ = scenes.random_walk(3, n_ticks, sc.info["c0"])
    nmov = info["n_fluid"] + info["n_soft"]

    def run(k0, k):
        for s in range(k0, k0 + k):
            if s % per_tick == 0:
                t = s // per_tick
                sim.set_body_pose(body, C_[t], Q_[t], V_[t], W_[t])
            sim.step(1)

    run(0, a.warmup)
    sim.synchronize()
    torch.cuda.synchronize()
    s0 = sim.stats()
    sim.profile_begin(a.steps, every=PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(a.warmup, a.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    phases = sim.profile_read()
    s1 = sim.stats()
    F, T = sim.wrench(body)                          # also reports instability
    ms_step = 1e3 * el / a.steps
    value = nmov * a.steps / el
    # roofline of the dominant kernel
    pairs_d = (s1["pairs_density"] - s0["pairs_density"]) / a.steps
    pairs_f = (s1["pairs_force"] - s0["pairs_force"]) / a.steps
    cand = (s1["candidates"] - s0["candidates"]) / a.steps
    ms = {k: v[0] / max(v[1], 1) for k, v in phases.items()}
    dom = "forces" if ms["forces"] >= ms["density"] else "density"
    lane_ops = {"density": nmov * CANDIDATES_PER_PARTICLE * LANE_OPS_CANDIDATE + pairs_d * LANE_OPS_DENSITY_PAIR,
                "forces": pairs_f * LANE_OPS_FORCE_PAIR}
    flops = {"density": pairs_d * FLOP_DENSITY_PAIR, "forces": pairs_f * FLOP_FORCE_PAIR}
    achieved = lane_ops[dom] / (ms[dom] * 1e-3) / 1e12
    roof = {"bound": "alu", "kernel": f"k_{dom}", "achieved": round(achieved, 3),
            "peak": round(PEAK_LANE_TOPS, 2), "unit": "Tlane-op/s", "frac": round(achieved / PEAK_LANE_TOPS, 4),
            "traffic": profiled_traffic(f"k_{dom}", int(info["n"])), "avg_launch_ms": round(ms[dom], 4),
            "launches_timed": phases[dom][1], "timed_every_nth_step": PROFILE_EVERY,
            "algorithmic_lane_ops_per_launch": int(lane_ops[dom]),
            "other_kernel": {k: {"avg_launch_ms": round(ms[k], 4),
                                 "frac": round(lane_ops[k] / (ms[k] * 1e-3) / 1e12 / PEAK_LANE_TOPS, 4)}
                             for k in ("density", "forces") if k != dom},
            "pair_flops": {k: {"tflops": round(flops[k] / (ms[k] * 1e-3) / 1e12, 3),
                               "frac_of_157.3": round(flops[k] / (ms[k] * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4)}
                           for k in ("density", "forces")}}
    out = {
        "metric": "SPH particle-updates/s @1M + haptic wrench Hz: surrogate vs plain, <=5% err",
        "value": value, "unit": "particle-updates/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"coupled fluid+soft+rigid, {info['n_fluid']:,} fluid + {info['n_soft']:,} soft "
                               f"+ {info['n_body_particles']:,} grabbed sphere + tank, {info['n']:,} particles, "
                               f"h=0.01 m, dt=2.5e-4 s, 1 kHz pose; readings: negative pressure clamped to 0, "
                               f"nu = {sc.params['nu']:g} m^2/s (nu proportional to h)",
                   "n_particles": info["n"], "precision": "fp32 particles, fp64 wrench",
                   "parallelism": "single GPU"},
        "wrench_hz_plain": a.steps / el,
        "realtime_factor": a.steps * dt / el,
        "pairs_per_step": {"density": pairs_d, "force": pairs_f, "candidates_tested": cand,
                           "lane_efficiency_density": pairs_d / max(64 * (s1["iter_density"] - s0["iter_density"]) / a.steps, 1),
                           "lane_efficiency_force": pairs_f / max(64 * (s1["iter_force"] - s0["iter_force"]) / a.steps, 1)},
        "phase_ms": {k: round(v, 4) for k, v in ms.items()},
        "roofline": roof,
        # the memory-bound phases against HBM (algorithmic bytes / HIP-event phase time)
        "hbm": {"peak_gbs": PEAK_HBM_GBS,
                "whole_step": {"bytes_per_particle": HBM_BYTES_STEP_PER_PARTICLE,
                               "achieved_gbs": round(HBM_BYTES_STEP_PER_PARTICLE * info["n"] / (ms_step * 1e-3) / 1e9, 1),
                               "frac": round(HBM_BYTES_STEP_PER_PARTICLE * info["n"] / (ms_step * 1e-3) / 1e9
                                             / PEAK_HBM_GBS, 4)},
                "phases": {k: {"bytes_per_particle": b_, "ms": round(ms[k], 4),
                               "achieved_gbs": round(b_ * info["n"] / (ms[k] * 1e-3) / 1e9, 1),
                               "frac": round(b_ * info["n"] / (ms[k] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
                           for k, b_ in HBM_BYTES_PER_PARTICLE.items() if ms.get(k, 0) > 0}},
    }
    # measured device copy bandwidth (read + write bytes of a 1 GiB torch copy)
    src = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    out["hbm"]["copy_gbs"] = round(5 * 2 * (1 << 30) / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del src, dst
    # cell occupancy of the last step (targets beyond 64 need a second wavefront pass)
    keys = sim.read("key")
    cnt = np.bincount(keys)
    cnt = cnt[cnt > 0]
    out["cells"] = {"occupied": int(cnt.size), "mean": float(cnt.mean()), "max": int(cnt.max()),
                    "over64": int((cnt > 64).sum()),
                    "passes_per_target": float(np.ceil(cnt / 64).sum() * 64 / cnt.sum())}
    del sim
    if not a.no_batch:
        log("batch leg: 256 stirring tanks (2k-30k fluid each), pose tracks, graph replay ...", a.quiet)
        out["batch"] = batch_leg(dev)
    if not a.no_surrogate:
        from paper_2511_15908_amd import surrogate as S
        log("surrogate leg: plain-SPH haptic logs of 16 copies of the 100k haptic scene (one walk each), "
            "training, evaluation ...", a.quiet)
        r = S.run_experiment(batch=16, train_segments=32, ticks=3000, eval_ticks=1500, eval_segments=15,
                             steps=3000, log=lambda m: log(m, a.quiet))
        e = r["errors"]
        out["surrogate"] = {
            "scene": r["scene"], "n_particles": r["n_particles"], "sph_update_hz": 100, "haptic_hz": 1000,
            "error_vs_plain_sph": {k: round(v["mean"], 4) for k, v in e.items()},
            "error_p95": {k: round(v["p95"], 4) for k, v in e.items()},
            "tick_rate_hz": {"host_round_trip": round(r["host_round_trip_hz"], 1),
                             "device_chain": round(r["device_chain_hz"], 1)},
            "eval_walks": r["eval_walks"],
            # "surrogate": the haptic loop with its plain-SPH fallback (rows outside the
            # training range keep the last SPH wrench); "network_only": the network alone
            "fallback": {"margin": S.GUARD_MARGIN, "rows_frac": round(e["surrogate"].get("fallback_frac", 0.0), 4)},
            "training": {"walks": r["training_walks"], "rows": r["training_rows"], "steps": r["train_steps"],
                         "seconds": round(r["train_s"], 2), "scene_copies_stepped_together": r["batch"],
                         "ticks_simulated": r["ticks_collected"], "collect_seconds": round(r["collect_s"], 1)}}
        log("haptic chain at 1 kHz while plain SPH runs on the same GPU (100k haptic scene) ...", a.quiet)
        out["surrogate"]["haptic_under_sph_load"] = S.haptic_under_load("haptic", 100_000, seconds=2.0,
                                                                        log=lambda m: log(m, a.quiet))
        log("surrogate leg: the coupled scene itself (1M fluid, soft cube, sphere on its random walk), "
            "a short run: 4 training walks ...", a.quiet)
        r = S.run_experiment(kind="coupled", scene=sc, train_segments=4, ticks=2000, eval_ticks=1000,
                             eval_segments=2, steps=2000, warmup_ticks=200, log=lambda m: log(m, a.quiet),
                             two_stages=True)
        e = r["errors"]
        e2 = r["two_stages"]["errors"]
        out["surrogate_coupled_1m"] = {
            "scene": r["scene"], "n_particles": r["n_particles"], "walk": "Ornstein-Uhlenbeck, 1 kHz",
            "sph_update_hz": 100, "haptic_hz": 1000,
            "error_vs_plain_sph": {k: round(v["mean"], 4) for k, v in e.items()},
            "error_p95": {k: round(v["p95"], 4) for k, v in e.items()},
            "eval_walks": r["eval_walks"],
            "fallback": {"margin": S.GUARD_MARGIN, "rows_frac": round(e["surrogate"].get("fallback_frac", 0.0), 4)},
            # the same logs with a second 40-tick rolling mean in the haptic loop
            "two_rolling_means": {"error_vs_plain_sph": {k: round(v["mean"], 4) for k, v in e2.items()},
                                  "error_p95": {k: round(v["p95"], 4) for k, v in e2.items()}},
            "training": {"walks": r["training_walks"], "rows": r["training_rows"], "steps": r["train_steps"],
                         "ticks_simulated": r["ticks_collected"], "collect_seconds": round(r["collect_s"], 1)},
            "haptic_under_sph_load": S.haptic_under_load("coupled", a.n_fluid, seconds=2.0, scene=sc,
                                                         log=lambda m: log(m, a.quiet))}
    log(json.dumps(out, indent=1), a.quiet)
    if not a.no_cpu_baseline:
        log("timing the CPU oracle (same scene, all threads and one thread; FP64 dam break) ...", a.quiet)
        out["cpu_baseline"] = cpu_baseline(sc, lambda m: log(m, a.quiet))
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
