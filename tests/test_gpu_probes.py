"""Density probes (Eq. density evaluated at free points, Sec. 3.4) through the
C ABI against the oracle's brute-force probe sum: world and body-frame
points, points in empty space and outside the grid, both precisions, the
full-size coupled scene, and the argument checks."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2511_15908_amd as P
    P.load_library()
    return P


def _probe_points(sc, seed, n_world=48, n_body=64):
    from paper_2511_15908_amd import scenes
    rng = scenes.SplitMix64(seed, 31)
    lo = np.asarray(sc.params["domain_lo"], np.float64)
    hi = np.asarray(sc.params["domain_hi"], np.float64)
    world = lo + (hi - lo) * rng.uniform(3 * n_world).reshape(-1, 3)
    world = np.concatenate([world, [lo - 0.3, hi + 0.05, (lo + hi) / 2]])   # outside, centre
    body = np.nonzero(sc.object == 1)[0]
    rad = float(np.linalg.norm(sc.x[body] - sc.x[body].mean(0), axis=1).max())
    d = rng.uniform(3 * n_body).reshape(-1, 3) - 0.5
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rad * (1.0 + 0.8 * rng.uniform(n_body))
    bf = d * r[:, None]
    pts = np.concatenate([world, bf])
    frame = np.concatenate([np.full(world.shape[0], -1), np.full(n_body, 1)]).astype(np.int32)
    return pts, frame


@pytest.mark.parametrize("prec,tol", [("f32", 1e-6), ("f64", 1e-13)])
def test_probes_small_scene(gpu, orc, prec, tol):
    from paper_2511_15908_amd import scenes
    sc = scenes.small_scene(seed=93, precision=prec)
    pts, frame = _probe_points(sc, 93)
    sim = gpu.Sim(sc, precision=prec, max_probes=256)
    sim.set_probes(pts, frame)
    o = orc.Oracle(sc, prec)
    for k in range(3):
        pose = scenes.random_pose_velocity(93 + k, sc.object_pose0[1, :3])
        sim.set_body_pose(1, *pose)
        o.set_pose(1, *pose)
        sim.step(1)
        r = o.step(probes=(pts, frame))
        g = sim.read_probes()
        err = np.abs(g - r["probe"]).max() / 1000.0
        print(f"{prec} step {k}: probe max |diff|/rho0 = {err:.2e}, nonzero {np.count_nonzero(r['probe'])}")
        assert err <= tol
        assert np.count_nonzero(r["probe"]) > 20
        assert np.array_equal(g == 0, r["probe"] == 0)


def test_probes_coupled_1m(gpu, orc):
    from paper_2511_15908_amd import scenes
    sc = scenes.coupled_1m()
    pts, frame = _probe_points(sc, 5)
    sim = gpu.Sim(sc, max_probes=pts.shape[0])
    C, Q, V, W = scenes.random_walk(3, 40, sc.info["c0"])
    pose = (C[21], Q[21], V[21], W[21])
    sim.set_body_pose(1, *pose)
    sim.set_probes(pts, frame)
    sim.step(1)
    g = sim.read_probes()
    o = orc.Oracle(sc, "f32")
    o.set_pose(1, *pose)
    o.place()
    ref = orc.probe_density(sc.params, "f32", o.x, sc.mass, sc.type, o.probe_points_world(pts, frame))
    err = np.abs(g - ref).max() / 1000.0
    print(f"coupled_1m probes: max |diff|/rho0 = {err:.2e}, nonzero {np.count_nonzero(ref)}")
    assert err <= 1e-6
    assert np.array_equal(g == 0, ref == 0)


def test_probe_argument_errors(gpu):
    from paper_2511_15908_amd import scenes
    sc = scenes.small_scene(seed=94)
    sim = gpu.Sim(sc, max_probes=4)
    with pytest.raises(gpu.SphError):
        sim.set_probes(np.zeros((5, 3)))                    # above max_probes
    with pytest.raises(gpu.SphError):
        sim.set_probes(np.zeros((1, 3)), [0])               # static tank has no moving frame
    with pytest.raises(gpu.SphError):
        sim.set_probes(np.zeros((1, 3)), [7])               # no such object
    with pytest.raises(gpu.SphError):
        sim.set_probes(np.full((1, 3), np.nan))
    sim.set_probes(np.zeros((2, 3)), [-1, 1])
    sim.step(1)
    assert sim.read_probes().shape == (2,)
    sim.set_probes(np.zeros((0, 3)))
    sim.step(1)
    assert sim.read_probes().shape == (0,)


def test_probe_log_matches_per_step_reads(gpu):
    """The per-step probe log holds, bitwise, what read_probes returns after
    each step, for the steps the body log returns, oldest first (ring
    wrap-around included); read_log empties both logs; graph replays log as
    eager steps do."""
    import torch
    from paper_2511_15908_amd import scenes
    sc = scenes.small_scene(seed=94, precision="f32")
    pts, frame = _probe_points(sc, 94)
    st = torch.cuda.Stream()
    for graph in (False, True):
        sim = gpu.Sim(sc, max_probes=256, log_steps=5, stream=st)
        sim.set_probes(pts, frame)
        if graph:
            sim.set_graph(True)
        per = []
        for k in range(8):
            sim.set_body_pose(1, *scenes.random_pose_velocity(94 + k, sc.object_pose0[1, :3]))
            sim.step(1)
            per.append(sim.read_probes())
        lg = sim.read_probe_log()
        assert lg.shape == (5, pts.shape[0])
        assert np.array_equal(lg, np.array(per[-5:]))
        body = sim.read_log()
        assert body.shape[0] == 5
        assert sim.read_probe_log().shape[0] == 0
        # two more steps (one graph replay when enabled), read without per-step reads
        sim.step(2)
        lg2 = sim.read_probe_log()
        assert lg2.shape == (2, pts.shape[0])
        assert np.array_equal(lg2[-1], sim.read_probes())
