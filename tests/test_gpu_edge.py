"""Edge cases of the HIP path through the C ABI: empty and tiny scenes,
closed-form free fall, cells far above 64 particles (and above the
reorder's LDS staging), a sparse grid of 2^24 key slots, particles outside the
grid, neighbourhood capacity overflow, the instability flag, the
alternative-reading flags, a non-default stream, argument errors."""
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


def _scene(x, v=None, types=None, mass=1e-3, h=0.02, precision="f32", lo=(-0.2,) * 3, hi=(0.2,) * 3,
           gravity=(0.0, 0.0, -9.81), objects=None, kinematic=False):
    from paper_2511_15908_amd import scenes
    x = np.asarray(x, np.float64).reshape(-1, 3)
    n = x.shape[0]
    types = np.zeros(n, np.uint8) if types is None else np.asarray(types, np.uint8)
    obj = np.full(n, -1, np.int32)
    kin, poses = [], []
    if objects is not None:
        obj = np.asarray(objects, np.int32)
        no = int(obj.max()) + 1 if n else 0
        kin = [1 if kinematic else 0] * no
        poses = [[0, 0, 0, 1, 0, 0, 0]] * no
    params = scenes._params(h, 1e-4, lo, hi, precision)
    params["gravity"] = gravity
    sc = scenes.Scene(name="edge", precision=precision, params=params, x=x,
                      v=np.zeros_like(x) if v is None else np.asarray(v, np.float64),
                      mass=np.full(n, mass), type=types, object=obj,
                      object_kinematic=np.asarray(kin, np.uint8),
                      object_pose0=np.asarray(poses, np.float64).reshape(-1, 7), spacing=h / 2)
    return sc


def _compare_one_step(gpu, orc, sc, prec, tol_rho, tol_f):
    sim = gpu.Sim(sc, precision=prec)
    sim.step(1)
    o = orc.Oracle(sc, prec)
    r = o.step(keep_neighbors=True)
    fs = np.nonzero(sc.type != 2)[0]
    assert np.array_equal(sim.read("key"), r["keys"])
    cg, og, ig = sim.neighbors()
    co, oo, io = r["nbr"]
    for t in fs:
        assert np.array_equal(ig[og[t]:og[t] + cg[t]], io[oo[t]:oo[t] + co[t]])
    assert _cmp.rel_density(sim.read("rho")[fs], r["rho"][fs]) <= tol_rho
    mref = float(np.median(sc.mass[fs]))
    assert _cmp.rel_force(sim.read("f")[fs], r["f"][fs], mref * 9.81) <= tol_f
    return sim


def test_empty_scene(gpu):
    sc = _scene(np.zeros((0, 3)))
    sim = gpu.Sim(sc)
    sim.step(3)
    sim.synchronize()
    assert sim.read("x").shape == (0, 3)
    assert sim.info()["steps"] == 3


def test_single_particle_free_fall_closed_form(gpu):
    """One isolated fluid particle: only gravity acts (its self pair gives no
    force), so symplectic Euler gives v_n = -n g dt and
    z_n = z0 - g dt^2 n(n+1)/2 (Eq. euler)."""
    sc = _scene([[0.01, 0.02, 0.05]], precision="f64")
    sim = gpu.Sim(sc, precision="f64")
    n = 50
    sim.step(n)
    dt, g = sc.params["dt"], 9.81
    x = sim.read("x")[0]
    v = sim.read("v")[0]
    assert v[2] == pytest.approx(-n * g * dt, rel=1e-12)
    assert x[2] == pytest.approx(0.05 - g * dt * dt * n * (n + 1) / 2, rel=1e-12)
    assert x[0] == 0.01 and x[1] == 0.02


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_overfull_cell(gpu, orc, prec):
    """200 particles inside one grid cell (4 target chunks of a wavefront,
    many super-chunks), with random velocities."""
    from paper_2511_15908_amd import scenes
    rng = scenes.SplitMix64(5, 9)
    x = (rng.uniform(600).reshape(200, 3) - 0.5) * 0.03 - 0.02     # inside the cell [-0.04, 0.0002)^3
    v = (rng.uniform(600).reshape(200, 3) - 0.5) * 0.2
    sc = _scene(x, v, precision=prec)
    tol = (1e-5, 1e-4) if prec == "f32" else (1e-13, 1e-12)
    _compare_one_step(gpu, orc, sc, prec, *tol)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("n", [64, 65, 72, 73, 128, 136, 137])
def test_cell_pass_structure(gpu, orc, n, prec):
    """One grid cell of n particles, every fifth a static boundary particle:
    whole passes of 64 (64, 128), a remainder of up to 8 served in transposed
    mode inside the last pass (65, 72, 136), one past that (73, 137: a second,
    split pass).  Neighbour sets bit-exact, density and forces against the
    oracle."""
    from paper_2511_15908_amd import scenes
    rng = scenes.SplitMix64(31 + n, 9)
    x = (rng.uniform(3 * n).reshape(n, 3) - 0.5) * 0.03 - 0.02     # inside the cell [-0.04, 0.0002)^3
    v = (rng.uniform(3 * n).reshape(n, 3) - 0.5) * 0.2
    types = np.where(np.arange(n) % 5 == 4, 2, 0).astype(np.uint8)
    v[types == 2] = 0.0
    sc = _scene(x, v, types=types, objects=np.where(types == 2, 0, -1), precision=prec)
    tol = (1e-5, 1e-4) if prec == "f32" else (1e-13, 1e-12)
    _compare_one_step(gpu, orc, sc, prec, *tol)


@pytest.mark.parametrize("n", [72, 73, 136])
def test_cell_pass_structure_kinematic(gpu, orc, n):
    """As above with every fifth particle a kinematic body particle (a target
    of the force pass, also among the leftovers): the body particles'
    reactions and the body wrench against the oracle."""
    from paper_2511_15908_amd import scenes
    rng = scenes.SplitMix64(41 + n, 9)
    x = (rng.uniform(3 * n).reshape(n, 3) - 0.5) * 0.03 - 0.02
    types = np.where(np.arange(n) % 5 == 4, 2, 0).astype(np.uint8)
    sc = _scene(x, types=types, objects=np.where(types == 2, 0, -1), kinematic=True)
    sim = _compare_one_step(gpu, orc, sc, "f32", 1e-5, 1e-4)
    o = orc.Oracle(sc, "f32")
    r = o.step()
    b = np.nonzero(types == 2)[0]
    mref = float(np.median(sc.mass[types != 2]))
    assert _cmp.rel_force(sim.read("f")[b], r["f"][b], mref * 9.81) <= 1e-4
    F, T = sim.wrench(0)
    assert _cmp.rel_vec(F, r["wrench"][0][0], mref * 9.81 * b.size) <= 1e-4


@pytest.mark.parametrize("n", [72, 73])
def test_cell_pass_structure_unified(gpu, orc, n):
    """The unified boundary reading (flag 8) in a cell whose boundary particles
    are density targets too: the density pass then serves more targets per
    pass than the force pass.  Boundary densities against the oracle."""
    from paper_2511_15908_amd import scenes
    rng = scenes.SplitMix64(51 + n, 9)
    x = (rng.uniform(3 * n).reshape(n, 3) - 0.5) * 0.03 - 0.02
    types = np.where(np.arange(n) % 3 == 2, 2, 0).astype(np.uint8)
    sc = _scene(x, types=types, objects=np.where(types == 2, 0, -1))
    sc.params["flags"] = 8
    _compare_one_step(gpu, orc, sc, "f32", 1e-5, 1e-4)
    sim = gpu.Sim(sc)
    sim.step(1)
    r = orc.Oracle(sc, "f32").step()
    b = np.nonzero(types == 2)[0]
    assert _cmp.rel_density(sim.read("rho")[b], r["rho"][b]) <= 1e-5


def test_crowded_cell_beyond_reorder_staging(gpu, orc):
    """2,500 particles in one grid cell: the reorder ranks them against their
    cell slice in global memory (the slice does not fit its LDS staging) and
    the neighbourhood still fits the candidate capacity; FP64, one step."""
    from paper_2511_15908_amd import scenes
    rng = scenes.SplitMix64(8, 9)
    x = (rng.uniform(7500).reshape(2500, 3) - 0.5) * 0.035 - 0.02    # inside the cell [-0.04, 0.0002)^3
    sc = _scene(x, precision="f64", mass=1e-5)
    _compare_one_step(gpu, orc, sc, "f64", 1e-13, 1e-12)


def test_huge_sparse_grid(gpu, orc):
    """A domain of 220 cells per axis (2^24 key slots, 16,384 scan tiles: the
    slot scan takes its three-kernel path) holding a few hundred particles,
    some of them alone in far cells."""
    from paper_2511_15908_amd import scenes
    rng = scenes.SplitMix64(9, 9)
    near = (rng.uniform(900).reshape(300, 3) - 0.5) * 0.2
    far = np.array([[4.0, -4.0, 3.9], [4.01, -4.0, 3.9], [-4.3, 4.2, -4.35], [2.0, 2.0, -3.0]])
    sc = _scene(np.concatenate([near, far]), lo=(-4.4,) * 3, hi=(4.4,) * 3)
    sim = _compare_one_step(gpu, orc, sc, "f32", 1e-5, 1e-4)
    assert sim.info()["cell_slots"] == 1 << 24


def test_particles_outside_grid(gpu, orc):
    """Particles beyond the grid bounds use the edge cells; neighbour sets
    and sums are unchanged."""
    from paper_2511_15908_amd import scenes
    rng = scenes.SplitMix64(6, 9)
    inside = (rng.uniform(900).reshape(300, 3) - 0.5) * 0.3
    outside = np.array([[0.25, 0.0, 0.0], [0.26, 0.005, 0.0], [-0.3, -0.3, 0.31], [-0.305, -0.3, 0.31],
                        [0.0, 0.5, -0.4]])
    sc = _scene(np.concatenate([inside, outside]), precision="f32")
    _compare_one_step(gpu, orc, sc, "f32", 1e-5, 1e-4)


def test_capacity_overflow_is_reported(gpu):
    """5,000 particles in one cell exceed the 64-word neighbourhood capacity:
    the step reports SPH_ERR_CAPACITY, and since the overflowing cells kept
    stale values the context refuses every later step (the error is sticky)."""
    from paper_2511_15908_amd import scenes
    rng = scenes.SplitMix64(7, 9)
    x = (rng.uniform(15000).reshape(5000, 3) - 0.5) * 0.03 - 0.02
    sc = _scene(x)
    sim = gpu.Sim(sc)
    sim.step(1)
    with pytest.raises(gpu.SphError) as e:
        sim.synchronize()
    assert e.value.status == 7
    steps = sim.info()["steps"]
    with pytest.raises(gpu.SphError) as e:
        sim.step(1)            # refused, nothing enqueued
    assert e.value.status == 7
    assert sim.info()["steps"] == steps
    with pytest.raises(gpu.SphError) as e:
        sim.synchronize()      # reported again
    assert e.value.status == 7
    x = sim.read("x", check=False)   # reads still copy the (undefined) state for diagnosis
    assert x.shape == (sc.n, 3)
    sim.close()


def test_instability_flag(gpu):
    sc = _scene([[0.0, 0.0, 0.0], [0.05, 0.0, 0.0]])
    sim = gpu.Sim(sc, v_max=1e-3)
    sim.step(1)            # |v| = g dt = 9.81e-4 <= 1e-3
    sim.synchronize()
    sim.step(1)            # 1.96e-3 > 1e-3
    with pytest.raises(gpu.SphError) as e:
        sim.synchronize()
    assert e.value.status == 5


@pytest.mark.parametrize("flag", [1, 2, 4, 7, 8, 9, 12, 15])
def test_reading_flags(gpu, orc, flag):
    """The alternative readings (clamped pressure, single boundary pressure
    term, no boundary viscosity, boundary particles with a density and
    pressure of their own) match the oracle too; with the last, the boundary
    particles' density and pressure as well."""
    from paper_2511_15908_amd import scenes
    sc = scenes.small_scene(seed=51, precision="f64")
    sc.params["flags"] = flag
    sim = gpu.Sim(sc, precision="f64")
    pose = scenes.random_pose_velocity(51, sc.object_pose0[1, :3])
    sim.set_body_pose(1, *pose)
    sim.step(1)
    o = orc.Oracle(sc, "f64")
    o.set_pose(1, *pose)
    r = o.step()
    fs = np.nonzero(sc.type != 2)[0]
    dn = np.arange(sc.n) if flag & 8 else fs
    assert _cmp.rel_density(sim.read("rho")[dn], r["rho"][dn]) <= 1e-13
    assert np.allclose(sim.read("p")[dn], r["p"][dn], rtol=1e-9, atol=1e-9)
    if not flag & 8:
        assert not sim.read("rho")[sc.type == 2].any()
    mref = float(np.median(sc.mass[fs]))
    assert _cmp.rel_force(sim.read("f")[fs], r["f"][fs], mref * 9.81) <= 1e-12
    F, T = sim.wrench(1)
    assert _cmp.rel_vec(F, r["wrench"][1][0], 1000 * 9.81 * 27 * sc.spacing ** 3) <= 1e-12


def test_non_default_stream(gpu):
    import torch
    from paper_2511_15908_amd import scenes
    sc = scenes.small_scene(seed=61)
    a = gpu.Sim(sc)
    a.step(3)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = gpu.Sim(sc)
        b.step(3)
    assert np.array_equal(a.read("x"), b.read("x"))
    assert np.array_equal(a.read("f"), b.read("f"))


def test_argument_errors(gpu):
    from paper_2511_15908_amd import scenes
    sc = scenes.small_scene(seed=71)
    sim = gpu.Sim(sc)
    with pytest.raises(gpu.SphError) as e:
        sim.set_body_pose(0, [0, 0, 0], [1, 0, 0, 0])      # static tank
    assert e.value.status == 1
    with pytest.raises(gpu.SphError):
        sim.set_body_pose(5, [0, 0, 0], [1, 0, 0, 0])      # no such object
    with pytest.raises(gpu.SphError):
        sim.set_body_pose(1, [0, 0, 0], [0, 0, 0, 0])      # zero quaternion
    with pytest.raises(gpu.SphError):
        sim.wrench(0)
    sim.step(1)
    sim.synchronize()


def test_fluid_only_no_boundary(gpu, orc):
    from paper_2511_15908_amd import scenes
    sc = scenes.small_scene(seed=81, with_soft=False, with_body=False)
    keep = sc.type != 2
    for name in ["x", "v", "mass", "type", "object"]:
        setattr(sc, name, getattr(sc, name)[keep])
    sc.object_kinematic = np.zeros(0, np.uint8)
    sc.object_pose0 = np.zeros((0, 7))
    _compare_one_step(gpu, orc, sc, "f32", 1e-5, 1e-4)


def test_static_boundary_fields_stay_zero(gpu):
    """Each step's sort moves sorted slots between particles, and a pass with
    at most 32 targets serves none of the cell's static boundary particles;
    these must still read rho = 0 and force = 0 (the field contract) after
    many steps of a collapsing column."""
    from paper_2511_15908_amd import scenes
    sc = scenes.dam_break(precision="f32")
    sim = gpu.Sim(sc)
    sim.step(60)
    kin = np.nonzero(sc.object_kinematic)[0]
    static = np.nonzero((sc.type == 2) & ~np.isin(sc.object, kin))[0]
    assert static.size
    assert np.all(sim.read("rho")[static] == 0)
    assert np.all(sim.read("f")[static] == 0)


def test_profile_sampling(gpu):
    """Event timing on every step, and on every k-th armed step: launch counts
    per phase, positive times, the steps past the armed ones unrecorded, and
    k = 0 refused."""
    from paper_2511_15908_amd import scenes
    sc = scenes.small_scene(seed=5)
    sim = gpu.Sim(sc)
    for every, want in [(1, 10), (3, 4), (4, 3), (20, 1)]:
        sim.profile_begin(10, every=every)
        sim.step(12)
        ph = sim.profile_read()
        for name in ["keys", "density", "forces", "integrate"]:
            ms, launches = ph[name]
            assert launches == want, (every, name, launches)
            assert ms > 0.0
    with pytest.raises(gpu.SphError):
        sim.profile_begin(10, every=0)
    sim.step(2)
    sim.synchronize()
