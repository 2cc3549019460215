"""sph_init_static (the entry point for callers that cannot allocate device
memory) against sph_init with a caller workspace: the same scene stepped
through both gives bitwise-identical fields, neighbour sets and wrenches, on
two contexts in a row (the second on a smaller scene, which finds the
previous context's contents in the array)."""
import ctypes as C

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


def _compare(P, sc, steps=3):
    from paper_2511_15908_amd import scenes
    pose = scenes.random_pose_velocity(int(sc.n) % 97, sc.object_pose0[1, :3])
    ref = P.Sim(sc)
    sta = P.Sim(sc, static_workspace=True)
    assert sta.ws is None
    for s in (ref, sta):
        s.set_body_pose(1, *pose)
    for _ in range(steps):
        ref.step(1)
        sta.step(1)
        for f in ("x", "v", "rho", "p", "f", "key", "psi", "fspring"):
            a, b = ref.read(f), sta.read(f)
            assert np.array_equal(a, b), f
        for smoothed in (False, True):
            Fa, Ta = ref.wrench(1, smoothed)
            Fb, Tb = sta.wrench(1, smoothed)
            assert np.array_equal(Fa, Fb) and np.array_equal(Ta, Tb)
    na, nb = ref.neighbors(), sta.neighbors()
    assert all(np.array_equal(u, w) for u, w in zip(na, nb))
    assert ref.stats() == sta.stats()
    ref.close()
    return sta


def test_static_workspace_matches_caller_workspace(gpu):
    from paper_2511_15908_amd import scenes
    big = scenes.small_scene(seed=31)
    small = scenes.small_scene(seed=32, nf=(6, 5, 4), n_tank=(12, 8, 8))
    assert small.n < big.n
    print(f"no-alloc: scene n={big.n}, then n={small.n}", flush=True)
    first = _compare(gpu, big)
    # the array is held: a second static context on this device is refused
    from paper_2511_15908_amd import _binding as B
    with pytest.raises(B.SphError) as ei:
        gpu.Sim(small, static_workspace=True)
    assert ei.value.status == 4
    first.close()
    second = _compare(gpu, small)
    second.close()


def test_static_workspace_rejects_oversized_scene(gpu):
    from paper_2511_15908_amd import _binding as B
    from paper_2511_15908_amd import scenes
    sc = scenes.haptic_scene(n_fluid=400_000)
    assert B.workspace_size(sc) > B.SPH_STATIC_WORKSPACE_BYTES
    with pytest.raises(B.SphError) as ei:
        gpu.Sim(sc, static_workspace=True)
    assert ei.value.status == 2
    # the refusal holds nothing: a static context still opens afterwards
    s = gpu.Sim(scenes.small_scene(seed=33, nf=(5, 5, 5), n_tank=(10, 8, 8)), static_workspace=True)
    s.step(1)
    s.synchronize()
    s.close()
