"""Seeded synthetic scenes for the SPH hot path.

This module only builds inputs: particle positions and velocities on lattices,
boundary samplings of tanks and bodies, soft-body spring tables and the pose
trajectories that drive kinematic bodies.  It holds none of the method's
arithmetic (no kernel, no density, no force, no neighbour search), so both the
HIP library and the CPU oracle can consume the same arrays.

Geometry follows the paper's scenario types (Sec. 3.2 unified particles, Sec.
3.3 grabbed rigid body, Table 1 scenes): a static boundary tank, fluid filled
on a lattice, a kinematic rigid body sampled as boundary particles, and a
mass-spring soft cube (Sec. 3.2, Alg. 2 spring kernel).

Randomness: SplitMix64 (Steele, Lea and Flood 2014; Vigna's reference
constants), u = (z >> 11) * 2^-53, one stream per (scene seed, purpose).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FLUID, SOFT, BOUNDARY = 0, 1, 2

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# purpose ids for independent streams
P_JITTER, P_PHASE, P_WALK, P_PERTURB, P_BATCH = 1, 2, 3, 4, 5


class SplitMix64:
    """Counter-based SplitMix64 stream: value k is mix(seed + (k+1)*gamma)."""

    def __init__(self, seed: int, purpose: int = 0):
        s = (int(seed) * 1000003 + int(purpose) * 7919 + 0x5EED) & 0xFFFFFFFFFFFFFFFF
        self.state = np.uint64(s)
        self.count = 0

    def next_u64(self, n: int) -> np.ndarray:
        k = np.arange(self.count + 1, self.count + 1 + n, dtype=np.uint64)
        self.count += n
        with np.errstate(over="ignore"):
            z = self.state + k * _GAMMA
            z = (z ^ (z >> np.uint64(30))) * _M1
            z = (z ^ (z >> np.uint64(27))) * _M2
            z = z ^ (z >> np.uint64(31))
        return z

    def uniform(self, n: int) -> np.ndarray:
        return (self.next_u64(n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def normal(self, n: int) -> np.ndarray:
        u1 = self.uniform(n)
        u2 = self.uniform(n)
        return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2)


@dataclass
class Scene:
    name: str
    precision: str                 # "f32" | "f64"
    params: dict                   # h, rho0, k_pressure, nu, gravity, dt, domain_lo/hi, flags, smoothing_window
    x: np.ndarray                  # (n,3) float64
    v: np.ndarray                  # (n,3) float64
    mass: np.ndarray               # (n,) float64 (fluid/soft; ignored for boundary)
    type: np.ndarray               # (n,) uint8
    object: np.ndarray             # (n,) int32, -1 for fluid/soft
    object_kinematic: np.ndarray   # (n_objects,) uint8
    object_pose0: np.ndarray       # (n_objects,7) float64: c[3], q[4] (w,x,y,z)
    spring_ij: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.uint32))
    spring_L0: np.ndarray = field(default_factory=lambda: np.zeros(0))
    spring_k: np.ndarray = field(default_factory=lambda: np.zeros(0))
    spring_c: np.ndarray = field(default_factory=lambda: np.zeros(0))
    spacing: float = 0.0
    info: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def counts(self) -> dict:
        return {
            "fluid": int((self.type == FLUID).sum()),
            "soft": int((self.type == SOFT).sum()),
            "boundary": int((self.type == BOUNDARY).sum()),
            "all": self.n,
        }


# --------------------------------------------------------------------------
# lattice samplers
# --------------------------------------------------------------------------

def _grid(i0, i1, j0, j1, k0, k1):
    i, j, k = np.meshgrid(np.arange(i0, i1 + 1), np.arange(j0, j1 + 1),
                          np.arange(k0, k1 + 1), indexing="ij")
    ijk = np.stack([i.ravel(), j.ravel(), k.ravel()], 1)
    # lexicographic (k, j, i): k slowest
    order = np.lexsort((ijk[:, 0], ijk[:, 1], ijk[:, 2]))
    return ijk[order]


def tank_sites(nx: int, ny: int, nz: int) -> np.ndarray:
    """Open-top single-layer tank on lattice sites: floor k=0 over
    i in 0..nx, j in 0..ny; walls k in 1..nz on the perimeter."""
    floor = _grid(0, nx, 0, ny, 0, 0)
    walls = _grid(0, nx, 0, ny, 1, nz)
    per = (walls[:, 0] == 0) | (walls[:, 0] == nx) | (walls[:, 1] == 0) | (walls[:, 1] == ny)
    return np.concatenate([floor, walls[per]], 0)


# Initial fluid placement near boundaries.  With boundary volumes psi_b from
# the boundary particles' own neighbourhoods, a single-layer wall one spacing
# from the first fluid layer reads about 1.37 rho0 there (its psi_b stands in
# for the missing half space but sits closer than it); a gap of 1.7 spacings
# reads about rho0 and starts the fluid near rest.  Obstacles keep fluid
# sites at least OBSTACLE_CLEARANCE spacings from their particles.
WALL_GAP = 1.7
OBSTACLE_CLEARANCE = 1.5


def open_tank(Wx: float, Wy: float, nz: int, s: float) -> np.ndarray:
    """Open-top single-layer tank: floor z = 0 over [0, Wx] x [0, Wy], walls at
    x = 0, Wx and y = 0, Wy for z = s .. nz s; each side sampled at the
    spacing nearest s that divides it."""
    xs = np.linspace(0.0, Wx, int(round(Wx / s)) + 1)
    ys = np.linspace(0.0, Wy, int(round(Wy / s)) + 1)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    floor = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], 1)
    ring = np.concatenate([np.stack([xs, np.zeros_like(xs)], 1), np.stack([xs, np.full_like(xs, Wy)], 1),
                           np.stack([np.zeros(ys.size - 2), ys[1:-1]], 1),
                           np.stack([np.full(ys.size - 2, Wx), ys[1:-1]], 1)])
    walls = [np.concatenate([ring, np.full((ring.shape[0], 1), k * s)], 1) for k in range(1, nz + 1)]
    return np.concatenate([floor] + walls, 0)


def tank_width(n_columns: int, s: float) -> float:
    """Inner width of a tank holding n_columns fluid columns WALL_GAP spacings
    from both walls."""
    return (n_columns - 1 + 2.0 * WALL_GAP) * s


def clearance(points: np.ndarray, dmin: float):
    """exclude_fn: true for positions closer than dmin to any of points."""
    from scipy.spatial import cKDTree
    tree = cKDTree(np.asarray(points, np.float64))

    def fn(xyz):
        d, _ = tree.query(xyz, k=1)
        return d < dmin
    return fn


def block_surface_sites(i0, i1, j0, j1, k0, k1) -> np.ndarray:
    g = _grid(i0, i1, j0, j1, k0, k1)
    surf = ((g[:, 0] == i0) | (g[:, 0] == i1) | (g[:, 1] == j0) | (g[:, 1] == j1)
            | (g[:, 2] == k0) | (g[:, 2] == k1))
    return g[surf]


def fibonacci_sphere(n: int, r: float, c) -> np.ndarray:
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    return np.asarray(c, np.float64) + r * np.stack([rho * np.cos(phi), rho * np.sin(phi), z], 1)


def fill_to_count(n_fluid, i_range, j_range, s, occupied: set, exclude_fn=None, k_start=1, gap=1.0):
    """Take tank-interior lattice sites in (k, j, i) order, skipping occupied
    sites and sites for which exclude_fn(xyz) is true, until n_fluid are placed.
    Site index a maps to position (a + gap - 1) s (gap = 1: on the lattice of
    the tank); returns the integer sites."""
    out = []
    need = n_fluid
    k = k_start
    ii, jj = np.meshgrid(np.arange(i_range[0], i_range[1] + 1),
                         np.arange(j_range[0], j_range[1] + 1), indexing="xy")
    layer_ij = np.stack([ii.ravel(), jj.ravel()], 1)      # j slowest, i fastest
    while need > 0:
        ijk = np.concatenate([layer_ij, np.full((layer_ij.shape[0], 1), k)], 1)
        if occupied:
            keep = np.array([tuple(t) not in occupied for t in ijk.tolist()], bool)
            ijk = ijk[keep]
        if exclude_fn is not None and ijk.shape[0]:
            ijk = ijk[~exclude_fn((ijk.astype(np.float64) + (gap - 1.0)) * s)]
        take = ijk[:need]
        out.append(take)
        need -= take.shape[0]
        k += 1
        if k > 100000:
            raise RuntimeError("fill_to_count did not converge")
    return np.concatenate(out, 0)


def soft_cube_springs(ijk: np.ndarray):
    """Springs between lattice neighbours of a solid block: the 6 axis and 12
    face-diagonal neighbours (each unordered pair once).  Returns (m,2) index
    pairs into ijk."""
    index = {tuple(t): n for n, t in enumerate(ijk.tolist())}
    offs = []
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        offs.append(tuple(e))
    for a in range(3):
        for b in range(a + 1, 3):
            for sb in (1, -1):
                e = [0, 0, 0]
                e[a] = 1
                e[b] = sb
                offs.append(tuple(e))
    pairs = []
    for n, t in enumerate(ijk.tolist()):
        for o in offs:
            m = index.get((t[0] + o[0], t[1] + o[1], t[2] + o[2]))
            if m is not None:
                pairs.append((n, m))
    return np.asarray(pairs, np.int64).reshape(-1, 2)


def viscosity_for(h: float) -> float:
    """Kinematic viscosity proportional to the smoothing length, 1e-3 m^2/s at
    h = 1 cm: c h / nu stays about 158 (c = sqrt(250) m/s) at every
    resolution, i.e. the same damping per particle spacing (an artificial
    viscosity alpha = 8 nu / (c h) of about 0.05)."""
    return 1e-3 * h / 0.01


def _params(h, dt, lo, hi, precision, k_pressure=250.0, nu=1e-3, rho0=1000.0,
            flags=0, smoothing_window=20):
    return {
        "h": float(h), "rho0": float(rho0), "k_pressure": float(k_pressure),
        "nu": float(nu), "gravity": (0.0, 0.0, -9.81), "dt": float(dt),
        "domain_lo": tuple(float(a) for a in lo), "domain_hi": tuple(float(a) for a in hi),
        "flags": int(flags), "smoothing_window": int(smoothing_window),
        "precision": precision,
    }


def _assemble(name, precision, params, s, parts, kin, poses, springs=None, info=None):
    """parts: list of (xyz (m,3), type, object, mass)"""
    xs, ts, os_, ms = [], [], [], []
    for xyz, ty, ob, m in parts:
        xs.append(np.asarray(xyz, np.float64))
        ts.append(np.full(len(xyz), ty, np.uint8))
        os_.append(np.full(len(xyz), ob, np.int32))
        ms.append(np.full(len(xyz), m, np.float64))
    x = np.concatenate(xs, 0)
    sc = Scene(name=name, precision=precision, params=params, x=x,
               v=np.zeros_like(x), mass=np.concatenate(ms), type=np.concatenate(ts),
               object=np.concatenate(os_), object_kinematic=np.asarray(kin, np.uint8),
               object_pose0=np.asarray(poses, np.float64).reshape(-1, 7), spacing=s,
               info=dict(info or {}))
    if springs is not None:
        ij, L0, ks, cs = springs
        sc.spring_ij = np.asarray(ij, np.uint32).reshape(-1, 2)
        sc.spring_L0 = np.asarray(L0, np.float64)
        sc.spring_k = np.asarray(ks, np.float64)
        sc.spring_c = np.asarray(cs, np.float64)
    return sc


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------

def dam_break(seed: int = 1, precision: str = "f64") -> Scene:
    """Dam break, 8,000 fluid particles (20^3 lattice, spacing 0.02 m, h = 2
    spacing, +-1e-4 m seeded jitter) in the corner of an open 1.0 m long
    tank as wide as the column, a fixed 0.1 m cube (single-layer surface)
    1.7 spacings beyond the column, dt = 1e-3 s."""
    s, h, dt = 0.02, 0.04, 1e-3
    g = WALL_GAP
    fl = (_grid(1, 20, 1, 20, 1, 20).astype(np.float64) + (g - 1.0)) * s
    rng = SplitMix64(seed, P_JITTER)
    fl = fl + (2.0 * rng.uniform(fl.size).reshape(fl.shape) - 1.0) * 1e-4
    Wx, Wy = 50 * s, tank_width(20, s)
    tank = open_tank(Wx, Wy, 33, s)
    x0 = (g + 19 + g) * s
    y0 = 0.5 * (Wy - 5 * s)
    cube = block_surface_sites(0, 5, 0, 5, 1, 6).astype(np.float64) * s + np.array([x0, y0, 0.0])
    c_cube = np.array([x0 + 2.5 * s, y0 + 2.5 * s, 3.5 * s])
    m = 1000.0 * s ** 3
    lo = (-0.5 * s, -0.5 * s, -0.5 * s)
    hi = (Wx + 0.5 * s, Wy + 0.5 * s, 40.5 * s)
    params = _params(h, dt, lo, hi, precision, nu=viscosity_for(h), flags=1)
    poses = [[0, 0, 0, 1, 0, 0, 0], list(c_cube) + [1, 0, 0, 0]]
    return _assemble("dam_break_8k", precision, params, s,
                     [(fl, FLUID, -1, m), (tank, BOUNDARY, 0, 0.0), (cube, BOUNDARY, 1, 0.0)],
                     kin=[0, 1], poses=poses, info={"steps": 100, "body": 1})


def stirring_tank(seed: int = 2, n_fluid: int = 250_000, precision: str = "f32") -> Scene:
    """Stirring tank: 100 x 50 fluid columns at spacing 0.01 m in an open tank
    of about 1.02 x 0.52 x 0.6 m, a solid 4 x 25 x 40 lattice paddle (4,000
    kinematic boundary particles) on a seeded 1 Hz, 0.1 m sinusoid, n_fluid
    fluid particles filled layer by layer, dt = 5e-4 s."""
    s, h, dt = 0.01, 0.02, 5e-4
    g = WALL_GAP
    Wx, Wy = tank_width(100, s), tank_width(50, s)
    tank = open_tank(Wx, Wy, 60, s)
    pad = (_grid(49, 52, 13, 37, 6, 45).astype(np.float64) + (g - 1.0)) * s
    fl = (fill_to_count(n_fluid, (1, 100), (1, 50), s, set(), clearance(pad, OBSTACLE_CLEARANCE * s), gap=g)
          .astype(np.float64) + (g - 1.0)) * s
    c0 = pad.mean(0)
    m = 1000.0 * s ** 3
    phase = 2.0 * math.pi * float(SplitMix64(seed, P_PHASE).uniform(1)[0])
    lo = (-0.5 * s, -0.5 * s, -0.5 * s)
    hi = (Wx + 1.5 * s, Wy + 1.5 * s, 70.5 * s)
    params = _params(h, dt, lo, hi, precision, nu=viscosity_for(h), flags=1)
    poses = [[0, 0, 0, 1, 0, 0, 0], list(c0) + [1, 0, 0, 0]]
    return _assemble(f"stirring_tank_{n_fluid}", precision, params, s,
                     [(fl, FLUID, -1, m), (tank, BOUNDARY, 0, 0.0), (pad, BOUNDARY, 1, 0.0)],
                     kin=[0, 1], poses=poses,
                     info={"body": 1, "phase": phase, "amplitude": 0.1, "freq": 1.0, "c0": c0})


# Soft cube material: a Young's modulus of 5e4 Pa.  Equal central springs on
# the 6 axis and 12 face-diagonal lattice neighbours give an isotropic solid
# with lambda = mu = k_s / s (Cauchy relation), i.e. E = 2.5 k_s / s and a
# Poisson ratio of exactly 1/4 (a ratio of 0.3 cannot be reached with central
# springs); matching E gives k_s = 0.4 E s = 100 N/m at s = 5 mm.
SOFT_E = 5e4


def coupled_soft_cube(s: float, g: float = 1.0):
    """The coupled scene's 20^3 soft cube at lattice spacing s: its lattice
    indices, positions, spring pairs (indices into the cube) and per-spring
    rest length, stiffness and damping (damping ratio about 0.1 at mass
    rho0 s^3)."""
    ijk = _grid(11, 30, 41, 60, 1, 20)
    pos = (ijk.astype(np.float64) + (g - 1.0)) * s
    m = 1000.0 * s ** 3
    ij = soft_cube_springs(ijk)
    L0 = np.linalg.norm(pos[ij[:, 0]] - pos[ij[:, 1]], axis=1)
    ks = 0.4 * SOFT_E * s                  # 100 N/m at s = 5 mm
    cs = 0.1 * 2.0 * math.sqrt(ks * m)
    return ijk, pos, ij, L0, np.full(len(L0), ks), np.full(len(L0), cs)


# the coupled scene's random walk: the box its centre is reflected at
WALK_BOX = ((0.12, 0.12, 0.12), (0.43, 0.38, 0.40))


def coupled_1m(seed: int = 3, n_fluid: int = 1_000_000, precision: str = "f32") -> Scene:
    """Coupled fluid + soft + rigid: 100 x 100 fluid columns at spacing 5 mm in
    an open tank of about 0.51 x 0.51 x 0.6 m, a 20^3 soft cube on the fluid
    lattice (66,120 springs, k_s = 100 N/m), a grabbed sphere of radius
    0.05 m as three Fibonacci shells (3,079 particles), n_fluid fluid
    particles, h = 1 cm, dt = 2.5e-4 s."""
    s, h, dt = 0.005, 0.01, 2.5e-4
    g = WALL_GAP
    W = tank_width(100, s)
    tank = open_tank(W, W, 120, s)
    soft_ijk, soft, ij, L0, ks, cs = coupled_soft_cube(s, g)
    occ = set(map(tuple, soft_ijk.tolist()))
    c0 = np.array([0.30, 0.25, 0.25])
    R = 0.05
    shells = [fibonacci_sphere(int(round(4 * math.pi * r * r / (s * s))), r, c0)
              for r in (R, R - s, R - 2 * s)]
    sph = np.concatenate(shells, 0)
    fl = (fill_to_count(n_fluid, (1, 100), (1, 100), s, occ, clearance(sph, OBSTACLE_CLEARANCE * s), gap=g)
          .astype(np.float64) + (g - 1.0)) * s
    m = 1000.0 * s ** 3
    nf = fl.shape[0]
    ij_glob = ij + nf                       # soft particles follow the fluid
    lo = (-0.5 * s, -0.5 * s, -0.5 * s)
    hi = (W + 1.5 * s, W + 1.5 * s, 125.0 * s)          # at most 32 cells of 2h (1 + 2^-10) per axis
    params = _params(h, dt, lo, hi, precision, nu=viscosity_for(h), flags=1)
    poses = [[0, 0, 0, 1, 0, 0, 0], list(c0) + [1, 0, 0, 0]]
    return _assemble(f"coupled_{n_fluid}", precision, params, s,
                     [(fl, FLUID, -1, m), (soft, SOFT, -1, m), (tank, BOUNDARY, 0, 0.0),
                      (sph, BOUNDARY, 1, 0.0)],
                     kin=[0, 1], poses=poses,
                     springs=(ij_glob, L0, ks, cs),
                     info={"body": 1, "radius": R, "c0": c0, "walk_lo": WALK_BOX[0], "walk_hi": WALK_BOX[1],
                           "probe_radius": R + s})


def haptic_scene(seed: int = 5, n_fluid: int = 100_000, precision: str = "f32") -> Scene:
    """The coupled scene's resolution and grabbed sphere (spacing 5 mm,
    h = 1 cm, dt = 2.5e-4 s, radius 0.05 m as three Fibonacci shells) in a
    tank whose square footprint holds n_fluid particles about 0.3 m deep,
    for the haptic-rate surrogate's training and validation runs.  The
    sphere starts submerged at the footprint centre; walk box and probe
    radius in info."""
    s, h, dt = 0.005, 0.01, 2.5e-4
    g = WALL_GAP
    nin = max(8, int(round(math.sqrt(n_fluid / 60.0))))       # fluid columns per side
    depth = n_fluid / (nin * nin) * s
    nz = int(math.ceil(depth / s * 1.35)) + 2
    W = tank_width(nin, s)
    tank = open_tank(W, W, nz, s)
    R = 0.05
    c0 = np.array([0.5 * W, 0.5 * W, min(0.17, 0.55 * depth)])
    shells = [fibonacci_sphere(int(round(4 * math.pi * r * r / (s * s))), r, c0)
              for r in (R, R - s, R - 2 * s)]
    sph = np.concatenate(shells, 0)
    fl = (fill_to_count(n_fluid, (1, nin), (1, nin), s, set(), clearance(sph, OBSTACLE_CLEARANCE * s), gap=g)
          .astype(np.float64) + (g - 1.0)) * s
    m = 1000.0 * s ** 3
    lo = (-0.5 * s, -0.5 * s, -0.5 * s)
    hi = (W + 1.5 * s, W + 1.5 * s, (nz + 3) * s)
    # haptic output: rolling mean over 160 steps = 40 ticks of 1 ms
    params = _params(h, dt, lo, hi, precision, nu=viscosity_for(h), flags=1, smoothing_window=160)
    poses = [[0, 0, 0, 1, 0, 0, 0], list(c0) + [1, 0, 0, 0]]
    margin = R + 5 * s
    info = {"body": 1, "radius": R, "c0": c0, "fluid_depth": depth,
            "walk_lo": (margin, margin, R + 6 * s), "walk_hi": (W - margin, W - margin, depth),
            "probe_radius": R + s}
    return _assemble(f"haptic_{n_fluid}", precision, params, s,
                     [(fl, FLUID, -1, m), (tank, BOUNDARY, 0, 0.0), (sph, BOUNDARY, 1, 0.0)],
                     kin=[0, 1], poses=poses, info=info)


def stirring_batch(seed: int = 4, n_scenes: int = 256, n_min: int = 2000, n_max: int = 30000,
                   precision: str = "f32"):
    """Independent stirring tanks for batched data generation: fluid counts
    N_k = floor(exp(U(ln n_min, ln n_max))); scene k is the stirring tank
    (1 x 0.5 m footprint, fluid ~0.5 m deep, 0.6 m walls) at spacing
    s_k = 0.5 / n_y, n_y = round((N_k / 2)^(1/3)), h_k = 2 s_k, with a paddle
    of the same physical size (0.04 x 0.25 x 0.40 m) as a solid lattice block
    at s_k; dt = 5e-4 s.  Each paddle follows its own band-limited path
    (batch_pose): four sinusoids, frequencies U(0.2, 3] Hz, amplitudes
    summing to 0.075 m, so the excursion stays within 0.15 m."""
    rng = SplitMix64(seed, P_BATCH)
    u = rng.uniform(n_scenes)
    counts = np.floor(np.exp(math.log(n_min) + u * (math.log(n_max) - math.log(n_min)))).astype(int)
    out = []
    for k, nf in enumerate(counts):
        ny = max(4, int(round((nf / 2.0) ** (1.0 / 3.0))))
        s = 0.5 / ny
        h, dt = 2.0 * s, 5e-4
        g = WALL_GAP
        nx = 2 * ny
        Wx, Wy = tank_width(nx, s), tank_width(ny, s)
        nz = int(math.ceil(0.6 / s))
        tank = open_tank(Wx, Wy, nz, s)
        pi = max(1, int(round(0.04 / s)))
        pj = max(1, int(round(0.25 / s)))
        pk = max(1, int(round(0.40 / s)))
        i0 = nx // 2 - pi // 2
        j0 = (ny - pj) // 2 + 1
        k0 = max(1, int(round(0.06 / s)))
        pad = (_grid(i0, i0 + pi - 1, j0, j0 + pj - 1, k0, k0 + pk - 1).astype(np.float64) + (g - 1.0)) * s
        fl = (fill_to_count(int(nf), (1, nx), (1, ny), s, set(), clearance(pad, OBSTACLE_CLEARANCE * s), gap=g)
              .astype(np.float64) + (g - 1.0)) * s
        c0 = pad.mean(0)
        lo = (-0.5 * s, -0.5 * s, -0.5 * s)
        hi = (Wx + 1.5 * s, Wy + 1.5 * s, (nz + 5) * s)
        params = _params(h, dt, lo, hi, precision, nu=viscosity_for(h), flags=1)
        r = SplitMix64(seed * 7919 + k, P_PHASE).uniform(12)
        freqs = 0.2 + 2.8 * r[0:4]
        w = r[4:8] + 0.05
        amps = 0.075 * w / w.sum()
        phases = 2.0 * math.pi * r[8:12]
        poses = [[0, 0, 0, 1, 0, 0, 0], list(c0) + [1, 0, 0, 0]]
        m = 1000.0 * s ** 3
        out.append(_assemble(f"batch_{k}_{int(nf)}", precision, params, s,
                             [(fl, FLUID, -1, m), (tank, BOUNDARY, 0, 0.0), (pad, BOUNDARY, 1, 0.0)],
                             kin=[0, 1], poses=poses,
                             info={"body": 1, "c0": c0, "freqs": freqs, "amps": amps, "phases": phases}))
    return out


def batch_pose(scene: Scene, t: float):
    """Pose of a batch scene's paddle at time t: x = x0 + sum_m a_m
    [sin(2 pi f_m t + phi_m) - sin phi_m], no rotation."""
    f, a, ph = scene.info["freqs"], scene.info["amps"], scene.info["phases"]
    c = np.asarray(scene.info["c0"], np.float64).copy()
    c[0] += float(np.sum(a * (np.sin(2 * math.pi * f * t + ph) - np.sin(ph))))
    v = np.zeros(3)
    v[0] = float(np.sum(a * 2 * math.pi * f * np.cos(2 * math.pi * f * t + ph)))
    return c, np.array([1.0, 0, 0, 0]), v, np.zeros(3)


def small_scene(seed: int = 11, nf=(14, 9, 8), precision: str = "f32", with_soft=True,
                with_body=True, perturb=True, n_tank=(24, 14, 16), spacing=0.02) -> Scene:
    """A small coupled scene for parity tests: a tank, a fluid block of
    nf[0] x nf[1] x nf[2] sites, optionally a 4^3 soft cube with springs and a
    kinematic cube, with seeded velocity and position perturbations."""
    s = spacing
    h = 2 * s
    nx, ny, nz = n_tank
    tank = tank_sites(nx, ny, nz).astype(np.float64) * s
    occ = set()
    parts = []
    soft_ijk = None
    if with_soft:
        soft_ijk = _grid(nx - 6, nx - 3, 2, 5, 1, 4)
        occ |= set(map(tuple, soft_ijk.tolist()))
    body_ijk = None
    if with_body:
        body_ijk = block_surface_sites(nx - 9, nx - 7, ny - 5, ny - 3, 2, 4)
        occ |= set(map(tuple, _grid(nx - 9, nx - 7, ny - 5, ny - 3, 2, 4).tolist()))
    fl_ijk = _grid(1, nf[0], 1, nf[1], 1, nf[2])
    fl_ijk = np.asarray([t for t in fl_ijk.tolist() if tuple(t) not in occ], np.int64).reshape(-1, 3)
    fl = fl_ijk.astype(np.float64) * s
    m = 1000.0 * s ** 3
    rng = SplitMix64(seed, P_PERTURB)
    if perturb:
        fl = fl + (2.0 * rng.uniform(fl.size).reshape(fl.shape) - 1.0) * 0.15 * s
    parts.append((fl, FLUID, -1, m))
    springs = None
    nfl = fl.shape[0]
    if with_soft:
        soft = soft_ijk.astype(np.float64) * s
        if perturb:
            soft = soft + (2.0 * rng.uniform(soft.size).reshape(soft.shape) - 1.0) * 0.05 * s
        parts.append((soft, SOFT, -1, m))
        ij = soft_cube_springs(soft_ijk)
        L0 = np.linalg.norm((soft_ijk[ij[:, 0]] - soft_ijk[ij[:, 1]]).astype(np.float64) * s, axis=1)
        ks = 0.4 * 5e4 * s
        springs = (ij + nfl, L0, np.full(len(L0), ks),
                   np.full(len(L0), 0.1 * 2.0 * math.sqrt(ks * m)))
    parts.append((tank, BOUNDARY, 0, 0.0))
    kin = [0]
    poses = [[0, 0, 0, 1, 0, 0, 0]]
    if with_body:
        body = body_ijk.astype(np.float64) * s
        parts.append((body, BOUNDARY, 1, 0.0))
        kin.append(1)
        poses.append(list(body.mean(0)) + [1, 0, 0, 0])
    lo = (-0.5 * s, -0.5 * s, -0.5 * s)
    hi = ((nx + 0.5) * s, (ny + 0.5) * s, (nz + 6.5) * s)
    params = _params(h, 1e-3 * (s / 0.02), lo, hi, precision)
    sc = _assemble(f"small_{seed}", precision, params, s, parts, kin=kin, poses=poses,
                   springs=springs, info={"body": 1 if with_body else None})
    if perturb:
        mov = sc.type != BOUNDARY
        sc.v[mov] = (2.0 * rng.uniform(3 * int(mov.sum())).reshape(-1, 3) - 1.0) * 0.3
    return sc


# --------------------------------------------------------------------------
# pose trajectories of kinematic bodies (inputs, not method arithmetic)
# --------------------------------------------------------------------------

def quat_normalize(q):
    q = np.asarray(q, np.float64)
    return q / np.linalg.norm(q)


def quat_mul(a, b):
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.array([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def stirring_pose(scene: Scene, t: float):
    """Paddle pose at time t: c = c0 + A[sin(2 pi f t + phi) - sin(phi)] e_x."""
    A, f, ph = scene.info["amplitude"], scene.info["freq"], scene.info["phase"]
    c0 = np.asarray(scene.info["c0"], np.float64)
    c = c0 + np.array([A * (math.sin(2 * math.pi * f * t + ph) - math.sin(ph)), 0.0, 0.0])
    v = np.array([A * 2 * math.pi * f * math.cos(2 * math.pi * f * t + ph), 0.0, 0.0])
    return c, np.array([1.0, 0, 0, 0]), v, np.zeros(3)


def random_walk(seed: int, n_ticks: int, c0, tick=1e-3, box_lo=WALK_BOX[0],
                box_hi=WALK_BOX[1], sig_v=0.028, sig_w=0.141, decay=0.99, q0=None, v0=None, w0=None):
    """Ornstein-Uhlenbeck random walk of a body pose sampled every `tick`
    seconds: v <- decay v + N(0, sig_v^2) per axis, w likewise; the centre is
    reflected at the box.  Starts at c0 and (q0, v0, w0), by default at rest
    in the identity orientation.  Returns arrays c, q, v, w of shape
    (n_ticks, .)."""
    rng = SplitMix64(seed, P_WALK)
    c = np.asarray(c0, np.float64).copy()
    q = np.array([1.0, 0, 0, 0]) if q0 is None else np.asarray(q0, np.float64).copy()
    v = np.zeros(3) if v0 is None else np.asarray(v0, np.float64).copy()
    w = np.zeros(3) if w0 is None else np.asarray(w0, np.float64).copy()
    lo, hi = np.asarray(box_lo), np.asarray(box_hi)
    C, Q, V, W = (np.zeros((n_ticks, 3)), np.zeros((n_ticks, 4)),
                  np.zeros((n_ticks, 3)), np.zeros((n_ticks, 3)))
    for t in range(n_ticks):
        C[t], Q[t], V[t], W[t] = c, q, v, w
        nz = rng.normal(6)
        v = decay * v + sig_v * nz[:3]
        w = decay * w + sig_w * nz[3:]
        c = c + tick * v
        for a in range(3):
            if c[a] < lo[a]:
                c[a] = 2 * lo[a] - c[a]
                v[a] = -v[a]
            elif c[a] > hi[a]:
                c[a] = 2 * hi[a] - c[a]
                v[a] = -v[a]
        q = quat_normalize(q + 0.5 * tick * quat_mul(np.array([0.0, *w]), q))
    return C, Q, V, W


def smooth_walk(seed: int, n_ticks: int, c0, box_lo, box_hi, tick=1e-3, tau_a=0.08, tau_v=0.1,
                rms_a=0.5, f_spring=1.5, tau_target=1.0, tau_alpha=0.08, tau_w=0.3, rms_alpha=6.0,
                q0=None, v0=None, w0=None):
    """Hand-like pose stream at 1 kHz.  A target point wanders over the box
    (Ornstein-Uhlenbeck, correlation time tau_target, spread 0.18 of the box
    per axis); the centre follows it through a spring of frequency f_spring
    with velocity relaxation tau_v, plus an Ornstein-Uhlenbeck
    acceleration (tau_a, RMS rms_a m/s^2); the angular velocity relaxes with
    tau_w under an Ornstein-Uhlenbeck angular acceleration (tau_alpha,
    rms_alpha rad/s^2).  The box reflects the centre (rarely reached).
    Starts at c0 and (q0, v0, w0), by default at rest in the identity
    orientation.  Returns c, q, v, w arrays (n_ticks, .)."""
    rng = SplitMix64(seed, P_WALK + 10)
    ra, rv = math.exp(-tick / tau_a), math.exp(-tick / tau_v)
    rb, rw = math.exp(-tick / tau_alpha), math.exp(-tick / tau_w)
    rt = math.exp(-tick / tau_target)
    sa, sb, st = (rms_a * math.sqrt(1 - ra * ra), rms_alpha * math.sqrt(1 - rb * rb), math.sqrt(1 - rt * rt))
    kap = (2.0 * math.pi * f_spring) ** 2
    c = np.asarray(c0, np.float64).copy()
    q = np.array([1.0, 0, 0, 0]) if q0 is None else np.asarray(q0, np.float64).copy()
    v = np.zeros(3) if v0 is None else np.asarray(v0, np.float64).copy()
    w = np.zeros(3) if w0 is None else np.asarray(w0, np.float64).copy()
    a, al = np.zeros(3), np.zeros(3)
    lo, hi = np.asarray(box_lo, np.float64), np.asarray(box_hi, np.float64)
    mid, spread = 0.5 * (lo + hi), 0.18 * (hi - lo)
    u = (c - mid) / spread                      # target in units of the spread
    C, Q, V, W = (np.zeros((n_ticks, 3)), np.zeros((n_ticks, 4)),
                  np.zeros((n_ticks, 3)), np.zeros((n_ticks, 3)))
    for t in range(n_ticks):
        C[t], Q[t], V[t], W[t] = c, q, v, w
        nz = rng.normal(9)
        a = ra * a + sa * nz[:3]
        al = rb * al + sb * nz[3:6]
        u = rt * u + st * nz[6:]
        target = np.clip(mid + spread * u, lo, hi)
        v = rv * v + tick * (a - kap * (c - target))
        w = rw * w + tick * al
        c = c + tick * v
        for k in range(3):
            if c[k] < lo[k]:
                c[k] = 2 * lo[k] - c[k]
                v[k] = -v[k]
            elif c[k] > hi[k]:
                c[k] = 2 * hi[k] - c[k]
                v[k] = -v[k]
        q = quat_normalize(q + 0.5 * tick * quat_mul(np.array([0.0, *w]), q))
    return C, Q, V, W


def random_pose_velocity(seed: int, c0, vmax=0.3, wmax=2.0):
    """A seeded rotation and rigid velocity for parity tests."""
    rng = SplitMix64(seed, P_PERTURB + 100)
    u = rng.uniform(10)
    axis = u[0:3] - 0.5
    axis = axis / np.linalg.norm(axis)
    ang = (u[3] - 0.5) * 0.6
    q = np.array([math.cos(ang / 2), *(math.sin(ang / 2) * axis)])
    v = (2 * u[4:7] - 1) * vmax
    w = (2 * u[7:10] - 1) * wmax
    return np.asarray(c0, np.float64), q, v, w


WORKLOADS = {
    "dam_break": dam_break,
    "stirring_tank": stirring_tank,
    "coupled_1m": coupled_1m,
}
