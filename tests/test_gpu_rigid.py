"""Free rigid bodies (object_kinematic 2) through the C ABI: closed-form fall
and spin of a body alone, FP64 parity with the oracle for a body in fluid
over free / grabbed / released phases, argument errors, and the sign of the
buoyant motion of a light and a heavy sphere (Archimedes)."""
import math

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


def _lone_cube():
    from paper_2511_15908_amd import scenes
    s = 0.01
    cube = scenes.block_surface_sites(0, 3, 0, 3, 0, 3).astype(float) * s + 0.1
    n = cube.shape[0]
    params = scenes._params(2 * s, 1e-3, (-0.1,) * 3, (0.4,) * 3, "f64")
    return scenes.Scene(name="cube", precision="f64", params=params, x=cube, v=np.zeros_like(cube),
                        mass=np.full(n, 0.01), type=np.full(n, 2, np.uint8), object=np.zeros(n, np.int32),
                        object_kinematic=np.array([2], np.uint8),
                        object_pose0=np.array([[0.0, 0, 0, 1, 0, 0, 0]]), spacing=s)


def test_free_fall_and_spin_closed_form(gpu):
    sc = _lone_cube()
    sim = gpu.Sim(sc, precision="f64")
    c0, q0, v0, w0 = sim.body_state(0)
    assert np.allclose(c0, 0.1 + 1.5 * sc.spacing, atol=1e-15)
    sim.set_body_pose(0, c0, q0, [0, 0, 0], [0, 0, 2.0])
    N, dt, g = 30, 1e-3, 9.81
    sim.step(N)
    c, q, v, w = sim.body_state(0)
    assert v[2] == pytest.approx(-N * g * dt, rel=1e-12)
    assert c[2] == pytest.approx(c0[2] - g * dt * dt * N * (N + 1) / 2, rel=1e-12)
    assert np.allclose(w, [0, 0, 2.0], atol=1e-12)
    # the particles follow the body: placed at the start of the last step,
    # i.e. at the pose before its final advance
    x = sim.read("x")
    assert x.mean(0)[2] == pytest.approx(c0[2] - g * dt * dt * (N - 1) * N / 2, abs=1e-12)


def _fluid_with_free_cube(seed=41):
    from paper_2511_15908_amd import scenes
    sc = scenes.small_scene(seed=seed, precision="f64", with_soft=False)
    body = sc.object == 1
    sc.object_kinematic = np.asarray(sc.object_kinematic).copy()
    sc.object_kinematic[1] = 2
    sc.mass = sc.mass.copy()
    sc.mass[body] = 700.0 * sc.spacing ** 3 * 2.0        # a light body (mass elements of its surface sites)
    return sc


def test_free_body_parity_with_oracle(gpu, orc):
    """FP64, 12 steps: 4 free, 4 grabbed (pose from the device), 4 released;
    body state and all particle positions against the oracle."""
    from paper_2511_15908_amd import scenes
    sc = _fluid_with_free_cube()
    sim = gpu.Sim(sc, precision="f64")
    o = orc.Oracle(sc, "f64")
    cg, qg, vg, wg = sim.body_state(1)
    assert np.allclose(cg, o.pose[1][0], rtol=0, atol=1e-14)
    pose = scenes.random_pose_velocity(41, cg, vmax=0.2, wmax=1.0)
    for k in range(12):
        if k == 4:
            sim.grab(1)
            o.grab(1)
            sim.set_body_pose(1, *pose)
            o.set_pose(1, *pose)
        if k == 8:
            sim.release(1)
            o.release(1)
        sim.step(1)
        o.step()
    c, q, v, w = sim.body_state(1)
    co, qo, vo, wo = o.pose[1]
    errs = [np.abs(c - co).max(), np.abs(q - qo).max(), np.abs(v - vo).max(), np.abs(w - wo).max(),
            np.abs(sim.read("x") - o.x).max()]
    print("free body FP64 parity: c %.2e q %.2e v %.2e w %.2e x %.2e" % tuple(errs))
    assert errs[0] < 1e-12 and errs[1] < 1e-12 and errs[2] < 1e-10 and errs[3] < 1e-9 and errs[4] < 1e-12
    F, T = sim.wrench(1)
    Fo, To = o.samples[1][-1][:3], o.samples[1][-1][3:]
    assert np.abs(F - Fo).max() <= 1e-9 * max(1.0, np.abs(Fo).max())


def test_grab_release_errors(gpu):
    from paper_2511_15908_amd import scenes
    sc = scenes.small_scene(seed=42)
    sim = gpu.Sim(sc)
    with pytest.raises(gpu.SphError):
        sim.grab(1)              # kinematic, not a free body
    with pytest.raises(gpu.SphError):
        sim.release(0)           # static tank
    with pytest.raises(gpu.SphError):
        sim.body_state(0)
    sc2 = _lone_cube()
    sc2.mass[:] = 0.0
    with pytest.raises(gpu.SphError):
        gpu.Sim(sc2, precision="f64")   # a free body needs positive masses


@pytest.mark.parametrize("density,sign", [(500.0, 1.0), (2000.0, -1.0)])
def test_buoyancy_sign(gpu, density, sign):
    """A free sphere in the 100k haptic scene: lighter than water it starts
    rising, heavier it starts sinking (FP32, 0.05 s)."""
    from paper_2511_15908_amd import scenes
    sc = scenes.haptic_scene()
    body = sc.object == 1
    sc.object_kinematic = np.asarray(sc.object_kinematic).copy()
    sc.object_kinematic[1] = 2
    sc.mass = sc.mass.copy()
    V = 4.0 / 3.0 * math.pi * sc.info["radius"] ** 3
    sc.mass[body] = density * V / body.sum()
    sim = gpu.Sim(sc)
    sim.step(200)
    c, q, v, w = sim.body_state(1)
    print(f"density {density}: v_z after 0.05 s = {v[2]:.4f} m/s")
    assert sign * v[2] > 0.02


def test_kinematic_body_without_particles(gpu, orc):
    """A kinematic object that owns no particles still gets its step: a zero
    wrench sample and the pose advanced by its velocities (the oracle's pose
    advance, step by step), next to a scene whose other bodies interact."""
    from paper_2511_15908_amd import scenes
    sc = scenes.small_scene(seed=21)
    empty = int(sc.object_kinematic.shape[0])
    sc.object_kinematic = np.append(sc.object_kinematic, np.uint8(1))
    sc.object_pose0 = np.vstack([sc.object_pose0, [0.1, 0.2, 0.05, 1.0, 0.0, 0.0, 0.0]])
    sim = gpu.Sim(sc)
    c, q = np.array([0.1, 0.2, 0.05]), np.array([0.9, 0.1, -0.2, 0.3])
    v, w = np.array([0.3, -0.1, 0.2]), np.array([1.5, -0.5, 2.0])
    sim.set_body_pose(empty, c, q, v, w)
    q = q / np.linalg.norm(q)
    dt = sc.params["dt"]
    for _ in range(10):
        sim.step(1)
        c, q = orc.pose_advance(c, q, v, w, dt)
    F, T = sim.wrench(empty)
    assert np.all(np.asarray(F) == 0.0) and np.all(np.asarray(T) == 0.0)
    cg, qg, vg, wg = sim.body_state(empty)
    assert np.allclose(cg, c, rtol=0, atol=1e-14)
    assert np.allclose(qg, q, rtol=0, atol=1e-14)
    assert np.array_equal(vg, v) and np.array_equal(wg, w)
