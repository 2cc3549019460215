"""Batches of independent scenes in one context (one launch per kernel for
all scenes): bitwise equality with one context per scene, parity with the
oracle scene by scene, graph replay against eager stepping, the per-step
body log, and the 256-scene stirring batch."""
import numpy as np
import pytest

from tests import _cmp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2511_15908_amd as P
    P.load_library()
    return P


def _mixed(prec):
    """Scenes of different spacing (hence h and grid) and size."""
    from paper_2511_15908_amd import scenes
    out = [scenes.small_scene(seed=21, precision=prec, spacing=0.01),
           scenes.small_scene(seed=22, precision=prec, nf=(10, 7, 6), spacing=0.013, with_soft=False),
           scenes.small_scene(seed=23, precision=prec, nf=(16, 8, 9), spacing=0.02)]
    out += scenes.stirring_batch(seed=9, n_scenes=2, n_min=2000, n_max=4000, precision=prec)
    for sc in out:                  # a batch shares dt
        sc.params["dt"] = 2.5e-4
    return out


def _poses(scs, k):
    from paper_2511_15908_amd import scenes
    return [scenes.random_pose_velocity(100 * k + i, sc.object_pose0[1, :3], vmax=0.2, wmax=1.0)
            for i, sc in enumerate(scs)]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_equals_one_context_per_scene(gpu, prec):
    scs = _mixed(prec)
    batch = gpu.Sim(scs, precision=prec)
    singles = [gpu.Sim(sc, precision=prec) for sc in scs]
    for k in range(3):
        for i, (sc, p) in enumerate(zip(scs, _poses(scs, k))):
            batch.set_body_pose(int(batch.obj0[i]) + 1, *p)
            singles[i].set_body_pose(1, *p)
        batch.step(1)
        for s in singles:
            s.step(1)
    for field in ("x", "v", "rho", "f", "psi"):
        whole = batch.read(field)
        for i, s in enumerate(singles):
            part = whole[batch.part0[i]:batch.part0[i + 1]]
            assert np.array_equal(part, s.read(field)), (field, i)
    for i, s in enumerate(singles):
        F, T = batch.wrench(int(batch.obj0[i]) + 1)
        F1, T1 = s.wrench(1)
        assert np.array_equal(F, F1) and np.array_equal(T, T1)


def test_batch_mixed_readings(gpu):
    """Scenes of one batch with their own readings and pressure constants:
    every field, density and pressure included, equals one context per
    scene bit for bit."""
    scs = _mixed("f64")
    for sc, fl, kf in zip(scs, [8, 0, 9, 12, 1], [1.0, 1.5, 0.8, 1.0, 2.0]):
        sc.params["flags"] = fl
        sc.params["k_pressure"] = kf * float(sc.params["k_pressure"])
    batch = gpu.Sim(scs, precision="f64")
    singles = [gpu.Sim(sc, precision="f64") for sc in scs]
    for k in range(2):
        for i, (sc, p) in enumerate(zip(scs, _poses(scs, k))):
            batch.set_body_pose(int(batch.obj0[i]) + 1, *p)
            singles[i].set_body_pose(1, *p)
        batch.step(1)
        for s in singles:
            s.step(1)
    for field in ("x", "v", "rho", "p", "f", "psi"):
        whole = batch.read(field)
        for i, s in enumerate(singles):
            part = whole[batch.part0[i]:batch.part0[i + 1]]
            assert np.array_equal(part, s.read(field)), (field, i)
    bnd = scs[0].type == 2
    assert (batch.read("rho")[:batch.part0[1]][bnd] > 0).all()     # unified: own boundary density


def test_batch_parity_with_oracle(gpu, orc):
    """One FP32 step of a 5-scene batch against the oracle scene by scene:
    cell keys (minus the scene's key offset) and neighbour sets bit-exact,
    density 1e-5, force 1e-4."""
    scs = _mixed("f32")
    batch = gpu.Sim(scs)
    poses = _poses(scs, 7)
    for i, p in enumerate(poses):
        batch.set_body_pose(int(batch.obj0[i]) + 1, *p)
    batch.step(1)
    keys = batch.read("key").astype(np.int64)
    rho, f = batch.read("rho"), batch.read("f")
    cg, og, ig = batch.neighbors()
    slot0 = 0
    for i, sc in enumerate(scs):
        o = orc.Oracle(sc, "f32")
        o.set_pose(1, *poses[i])
        r = o.step(keep_neighbors=True)
        a, b = batch.part0[i], batch.part0[i + 1]
        assert np.array_equal(keys[a:b] - slot0, r["keys"].astype(np.int64)), i
        slot0 += 1 << (3 * orc.grid_info(sc.params, "f32")["bits"])
        co, oo, io = r["nbr"]
        fs = np.nonzero(sc.type != 2)[0]
        for t in fs[::7]:
            got = ig[og[a + t]:og[a + t] + cg[a + t]] - a
            assert np.array_equal(got, io[oo[t]:oo[t] + co[t]]), (i, t)
        assert _cmp.rel_density(rho[a:b][fs], r["rho"][fs]) <= 1e-5
        mref = float(np.median(sc.mass[fs]))
        assert _cmp.rel_force(f[a:b][fs], r["f"][fs], mref * 9.81) <= 1e-4


def test_graph_replay_matches_eager(gpu):
    """The same batch stepped eagerly and by two-step graph replays on a
    non-default stream, with pose updates, odd step counts and host reads
    between replays: bitwise equal after every call."""
    import torch
    scs = _mixed("f32")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    eager = gpu.Sim(scs, stream=s1)
    graph = gpu.Sim(scs, stream=s2)
    graph.set_graph(True)
    for k, n in enumerate((2, 2, 3, 1, 4, 2)):
        for i, p in enumerate(_poses(scs, 20 + k)):
            o = int(eager.obj0[i]) + 1
            eager.set_body_pose(o, *p)
            graph.set_body_pose(o, *p)
        eager.step(n)
        graph.step(n)
        for field in ("x", "v", "f"):
            assert np.array_equal(eager.read(field), graph.read(field)), (k, field)
    assert eager.info()["steps"] == graph.info()["steps"] == 14


def test_body_log(gpu):
    from paper_2511_15908_amd import scenes
    scs = scenes.stirring_batch(seed=5, n_scenes=3, n_min=2000, n_max=3000)
    sim = gpu.Sim(scs, log_steps=8)
    bodies = sim.kinematic
    want = []
    for k in range(5):
        sim.step(1)
        want.append([np.concatenate(sim.wrench(b)) for b in bodies])
    log = sim.read_log()
    assert log.shape == (5, len(bodies), 20)
    assert np.array_equal(log[:, :, 13:19], np.asarray(want))
    assert np.array_equal(log[:, 0, 19], np.arange(5))
    sim.step(12)
    log = sim.read_log()
    assert log.shape == (8, len(bodies), 20)
    assert np.array_equal(log[:, 0, 19], np.arange(9, 17) - 5)
    assert sim.read_log().shape[0] == 0


def _track(sc, n, dt):
    from paper_2511_15908_amd import scenes
    return np.array([np.concatenate(scenes.batch_pose(sc, k * dt)) for k in range(n)])


def test_body_track_equals_per_step_poses(gpu):
    """A pose track taken on the device equals the same poses set before
    every step from the host, bitwise; after the track the pose
    extrapolates."""
    from paper_2511_15908_amd import scenes
    sc = scenes.stirring_batch(seed=6, n_scenes=1, n_min=3000, n_max=3000)[0]
    dt = sc.params["dt"]
    tr = _track(sc, 6, dt)
    a = gpu.Sim(sc)
    b = gpu.Sim(sc, track_steps=8)
    b.set_body_track(1, tr)
    for k in range(6):
        a.set_body_pose(1, tr[k, :3], tr[k, 3:7], tr[k, 7:10], tr[k, 10:13])
        a.step(1)
    b.step(6)
    assert np.array_equal(a.read("x"), b.read("x")) and np.array_equal(a.read("f"), b.read("f"))
    a.step(3)
    b.step(3)
    assert np.array_equal(a.read("x"), b.read("x"))
    with pytest.raises(gpu.SphError):
        b.set_body_track(1, np.zeros((9, 13)))       # above the capacity
    with pytest.raises(gpu.SphError):
        b.set_body_track(0, tr[:2])                  # static tank


def test_stirring_batch_256(gpu):
    """The 256-scene batch (log-uniform 2k-30k fluid each, 3.4M particles):
    paddle paths as device pose tracks, graph replays with no host work per
    step, the body log; two of its scenes checked bitwise against their own
    contexts."""
    import time
    import torch
    from paper_2511_15908_amd import scenes
    scs = scenes.stirring_batch(seed=4, n_scenes=256)
    st = torch.cuda.Stream()
    n = 64
    sim = gpu.Sim(scs, stream=st, log_steps=n, track_steps=n)
    sim.set_graph(True)
    dt = scs[0].params["dt"]
    pick = [3, 200]
    singles = {i: gpu.Sim(scs[i], stream=st, track_steps=n) for i in pick}
    for i, sc in enumerate(scs):
        sim.set_body_track(int(sim.obj0[i]) + 1, _track(sc, n, dt))
    for i in pick:
        singles[i].set_body_track(1, _track(scs[i], n, dt))
        singles[i].step(n)
    sim.step(2)
    sim.synchronize()
    t0 = time.perf_counter()
    sim.step(n - 2)
    sim.synchronize()
    el = time.perf_counter() - t0
    n_upd = sum(sc.counts()["fluid"] for sc in scs) * (n - 2)
    print(f"256 scenes, {sum(sc.n for sc in scs)} particles: {n - 2} graph-replayed steps in {el:.3f} s "
          f"({el / (n - 2) * 1e3:.2f} ms/step, {n_upd / el / 1e6:.0f} M fluid particle-updates/s)")
    log = sim.read_log()
    assert log.shape == (n, 256, 20) and np.all(np.isfinite(log))
    x = sim.read("x")
    for i in pick:
        assert np.array_equal(x[sim.part0[i]:sim.part0[i + 1]], singles[i].read("x"))


def test_batch_probes_equal_one_context_per_scene(gpu):
    """Density probes in a batch: points in a body's frame sample that body's
    scene, world points scene 0; every value (and the per-step probe log)
    bitwise equal to one context per scene."""
    from paper_2511_15908_amd import scenes
    scs = _mixed("f32")[:3]
    rng = scenes.SplitMix64(5, 33)
    body_pts = (rng.uniform(48).reshape(-1, 3) - 0.5) * 0.12
    world_pts = np.asarray(scs[0].params["domain_lo"]) + 0.05 + rng.uniform(12).reshape(-1, 3) * 0.1
    batch = gpu.Sim(scs, max_probes=64, log_steps=4)
    pts = np.concatenate([body_pts] * 3 + [world_pts])
    frame = np.concatenate([np.full(16, int(batch.obj0[i]) + 1) for i in range(3)] + [np.full(4, -1)])
    batch.set_probes(pts, frame.astype(np.int32))
    singles = []
    for i, sc in enumerate(scs):
        s = gpu.Sim(sc, max_probes=64, log_steps=4)
        p, f = (np.concatenate([body_pts, world_pts]), np.r_[np.full(16, 1), np.full(4, -1)]) if i == 0 \
            else (body_pts, np.full(16, 1))
        s.set_probes(p, f.astype(np.int32))
        singles.append(s)
    for k in range(3):
        for i, p in enumerate(_poses(scs, k)):
            batch.set_body_pose(int(batch.obj0[i]) + 1, *p)
            singles[i].set_body_pose(1, *p)
        batch.step(1)
        for s in singles:
            s.step(1)
    g = batch.read_probes()
    ref = [s.read_probes() for s in singles]
    for i in range(3):
        assert np.array_equal(g[16 * i:16 * i + 16], ref[i][:16]), i
    assert np.array_equal(g[48:], ref[0][16:])
    assert np.count_nonzero(g[:48]) > 10
    lg = batch.read_probe_log()
    assert lg.shape == (3, 52) and np.array_equal(lg[-1], g)
