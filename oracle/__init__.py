"""FP64 CPU oracle of the SPHaptics SPH step (arXiv 2511.15908).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library (``paper_2511_15908_amd``); the two meet only in the seeded
scene arrays of ``paper_2511_15908_amd.scenes``, which hold no arithmetic of
the method.

The arithmetic lives in ``sph_oracle.c`` (plain C, binary64, OpenMP over
independent targets); this file marshals arrays and sequences one step in the
order of the paper's simulation loop (Alg. 2; Sec. 3.2 rigid placement; Alg. 1
density pass, force pass, integration; Sec. 3.3 rolling average).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "sph_oracle.c"
_LIB = _HERE / "_build" / "liboracle.so"

FLUID, SOFT, BOUNDARY = 0, 1, 2
CLAMP_NEG_PRESSURE, BOUNDARY_SINGLE_TERM, NO_BOUNDARY_VISCOSITY, UNIFIED_BOUNDARY = 1, 2, 4, 8


def build(force: bool = True) -> Path:
    """Compile the oracle with gcc (binary64, no contraction, no fast-math)."""
    _LIB.parent.mkdir(parents=True, exist_ok=True)
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                        "-fPIC", "-shared", "-o", str(tmp), str(_SRC), "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("precision", C.c_int32), ("flags", C.c_uint32), ("h", C.c_double),
                ("rho0", C.c_double), ("k", C.c_double), ("nu", C.c_double),
                ("g", C.c_double * 3), ("dt", C.c_double), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3)]


class _Grid(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("bits", C.c_int32), ("cs", C.c_double),
                ("inv_cs64", C.c_double), ("inv_cs32", C.c_float), ("lo32", C.c_float * 3),
                ("R2_32", C.c_float), ("R2_64", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
            build(force=True)
        L = C.CDLL(str(_LIB))
        d, i64, i32, u8, u32 = (C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                C.POINTER(C.c_uint8), C.POINTER(C.c_uint32))
        P = C.POINTER(_Params)
        L.orc_alpha3.restype = C.c_double
        L.orc_alpha3.argtypes = [C.c_double]
        L.orc_W.restype = C.c_double
        L.orc_W.argtypes = [C.c_double, C.c_double]
        L.orc_dWdr.restype = C.c_double
        L.orc_dWdr.argtypes = [C.c_double, C.c_double]
        L.orc_grid_setup.argtypes = [P, C.POINTER(_Grid)]
        L.orc_morton3.restype = C.c_uint32
        L.orc_morton3.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
        L.orc_cell_keys.argtypes = [P, C.c_int64, d, u32]
        L.orc_neighbors.restype = C.c_int64
        L.orc_neighbors.argtypes = [P, C.c_int64, d, C.c_int64, i64, C.c_int, i64, i64, C.c_int64]
        L.orc_boundary_psi.argtypes = [P, C.c_int64, d, u8, i32, i64, i64, i64, d]
        L.orc_quat_to_R.argtypes = [d, d]
        L.orc_body_frame.argtypes = [C.c_int64, d, i32, C.c_int32, d, d]
        L.orc_body_place.argtypes = [C.c_int64, i32, C.c_int32, d, d, d, d, d, d, d]
        L.orc_pose_advance.argtypes = [d, d, d, d, C.c_double]
        L.orc_body_mass_props.argtypes = [C.c_int64, d, d, i32, C.c_int32, d, d, d, d]
        L.orc_body_velocity_step.argtypes = [d, d, C.c_double, d, d, d, C.c_double, d, d]
        L.orc_density.argtypes = [P, C.c_int64, d, d, u8, d, C.c_int64, i64, i64, i64, i64, d, d]
        L.orc_probe_density.argtypes = [P, C.c_int64, d, d, u8, C.c_int64, d, d]
        L.orc_springs.argtypes = [C.c_int64, d, d, C.c_int64, u32, d, d, d, d]
        L.orc_forces.argtypes = [P, C.c_int64, d, d, d, u8, d, d, d, d, C.c_int64, i64, i64, i64,
                                 i64, d]
        L.orc_wrench.argtypes = [C.c_int64, i32, C.c_int32, d, d, d, d, d]
        L.orc_integrate.argtypes = [P, C.c_int64, u8, d, d, d, d]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_params(params: dict, precision: str) -> _Params:
    P = _Params()
    P.precision = 0 if precision == "f32" else 1
    P.flags = int(params.get("flags", 0))
    P.h, P.rho0, P.k, P.nu = params["h"], params["rho0"], params["k_pressure"], params["nu"]
    P.g[:] = list(params["gravity"])
    P.dt = params["dt"]
    P.lo[:] = list(params["domain_lo"])
    P.hi[:] = list(params["domain_hi"])
    return P


# --------------------------------------------------------------------------
# thin wrappers
# --------------------------------------------------------------------------

def W(r, h):
    return lib().orc_W(float(r), float(h))


def dWdr(r, h):
    return lib().orc_dWdr(float(r), float(h))


def grid_info(params: dict, precision: str) -> dict:
    g = _Grid()
    P = make_params(params, precision)
    lib().orc_grid_setup(C.byref(P), C.byref(g))
    return {"dims": tuple(g.dims), "bits": g.bits, "cs": g.cs, "inv_cs32": g.inv_cs32,
            "R2_32": g.R2_32, "R2_64": g.R2_64}


def morton3(cx, cy, cz, bits):
    return lib().orc_morton3(int(cx), int(cy), int(cz), int(bits))


def cell_keys(params, precision, x):
    x = _f64(x)
    out = np.zeros(x.shape[0], np.uint32)
    P = make_params(params, precision)
    lib().orc_cell_keys(C.byref(P), x.shape[0], _p(x, C.c_double), _p(out, C.c_uint32))
    return out


def neighbors(params, precision, x, targets=None, use_grid=True):
    """Neighbour lists (self included, ascending id) of the targets (all
    particles when None).  Returns (counts, offsets, ids)."""
    x = _f64(x)
    n = x.shape[0]
    P = make_params(params, precision)
    if targets is None:
        tptr, nt = None, n
    else:
        targets = np.ascontiguousarray(targets, np.int64)
        tptr, nt = _p(targets, C.c_int64), targets.shape[0]
    counts = np.zeros(nt, np.int64)
    total = lib().orc_neighbors(C.byref(P), n, _p(x, C.c_double), nt, tptr, int(use_grid),
                                _p(counts, C.c_int64), None, 0)
    ids = np.zeros(max(total, 1), np.int64)
    lib().orc_neighbors(C.byref(P), n, _p(x, C.c_double), nt, tptr, int(use_grid),
                        _p(counts, C.c_int64), _p(ids, C.c_int64), total)
    offs = np.zeros(nt, np.int64)
    if nt:
        offs[1:] = np.cumsum(counts)[:-1]
    return counts, offs, ids[:total]


def probe_density(params, precision, x, mass, type_, points):
    """Density of fluid and soft particles at world points (Eq. density at a
    free point), brute force over all particles."""
    P = make_params(params, precision)
    x, mass = _f64(x), _f64(mass)
    t = np.ascontiguousarray(type_, np.uint8)
    pts = _f64(points).reshape(-1, 3)
    out = np.zeros(pts.shape[0])
    lib().orc_probe_density(C.byref(P), x.shape[0], _p(x, C.c_double), _p(mass, C.c_double),
                            _p(t, C.c_uint8), pts.shape[0], _p(pts, C.c_double), _p(out, C.c_double))
    return out


def quat_to_R(q):
    q = _f64(q)
    R = np.zeros(9)
    lib().orc_quat_to_R(_p(q, C.c_double), _p(R, C.c_double))
    return R.reshape(3, 3)


def body_mass_props(x, mass, obj, o, q0):
    """Mass, centre of mass and body-frame inertia of object o's particles."""
    x, mass = _f64(x), _f64(mass)
    obj = np.ascontiguousarray(obj, np.int32)
    com, m, I = np.zeros(3), np.zeros(1), np.zeros(9)
    lib().orc_body_mass_props(x.shape[0], _p(x, C.c_double), _p(mass, C.c_double), _p(obj, C.c_int32), int(o),
                              _p(_f64(q0), C.c_double), _p(com, C.c_double), _p(m, C.c_double), _p(I, C.c_double))
    return float(m[0]), com, I.reshape(3, 3)


def body_velocity_step(F, T, m, I_body, q, g, dt, v, w):
    """Semi-implicit Euler velocity step of a free body; returns new (v, w)."""
    v, w = _f64(v).copy(), _f64(w).copy()
    lib().orc_body_velocity_step(_p(_f64(F), C.c_double), _p(_f64(T), C.c_double), float(m),
                                 _p(_f64(np.asarray(I_body).ravel()), C.c_double), _p(_f64(q), C.c_double),
                                 _p(_f64(g), C.c_double), float(dt), _p(v, C.c_double), _p(w, C.c_double))
    return v, w


def pose_advance(c, q, v, w, dt):
    c, q, v, w = _f64(c).copy(), _f64(q).copy(), _f64(v), _f64(w)
    lib().orc_pose_advance(_p(c, C.c_double), _p(q, C.c_double), _p(v, C.c_double),
                           _p(w, C.c_double), float(dt))
    return c, q


def springs(n, x, v, ij, L0, ks, cs):
    x, v = _f64(x), _f64(v)
    ij = np.ascontiguousarray(ij, np.uint32)
    L0, ks, cs = _f64(L0), _f64(ks), _f64(cs)
    f = np.zeros((n, 3))
    lib().orc_springs(n, _p(x, C.c_double), _p(v, C.c_double), ij.shape[0], _p(ij, C.c_uint32),
                      _p(L0, C.c_double), _p(ks, C.c_double), _p(cs, C.c_double), _p(f, C.c_double))
    return f


def density(params, precision, x, mass, type_, psi, targets, nbr=None):
    """rho and p of the targets (Eqs. density, pressure)."""
    P = make_params(params, precision)
    x, mass, psi = _f64(x), _f64(mass), _f64(psi)
    type_ = np.ascontiguousarray(type_, np.uint8)
    targets = np.ascontiguousarray(targets, np.int64)
    if nbr is None:
        nbr = neighbors(params, precision, x, targets)
    counts, offs, ids = nbr
    rho = np.zeros(targets.shape[0])
    pr = np.zeros(targets.shape[0])
    lib().orc_density(C.byref(P), x.shape[0], _p(x, C.c_double), _p(mass, C.c_double),
                      _p(type_, C.c_uint8), _p(psi, C.c_double), targets.shape[0],
                      _p(targets, C.c_int64), _p(counts, C.c_int64), _p(offs, C.c_int64),
                      _p(ids, C.c_int64), _p(rho, C.c_double), _p(pr, C.c_double))
    return rho, pr


def forces(params, precision, x, v, mass, type_, psi, rho_full, p_full, fspring, targets, nbr=None):
    """Force on the targets (Alg. 1 second pass); rho_full/p_full by id."""
    P = make_params(params, precision)
    x, v, mass, psi = _f64(x), _f64(v), _f64(mass), _f64(psi)
    rho_full, p_full = _f64(rho_full), _f64(p_full)
    type_ = np.ascontiguousarray(type_, np.uint8)
    targets = np.ascontiguousarray(targets, np.int64)
    if nbr is None:
        nbr = neighbors(params, precision, x, targets)
    counts, offs, ids = nbr
    fs = _f64(fspring) if fspring is not None else np.zeros((x.shape[0], 3))
    f = np.zeros((targets.shape[0], 3))
    lib().orc_forces(C.byref(P), x.shape[0], _p(x, C.c_double), _p(v, C.c_double),
                     _p(mass, C.c_double), _p(type_, C.c_uint8), _p(psi, C.c_double),
                     _p(rho_full, C.c_double), _p(p_full, C.c_double), _p(fs, C.c_double),
                     targets.shape[0], _p(targets, C.c_int64), _p(counts, C.c_int64),
                     _p(offs, C.c_int64), _p(ids, C.c_int64), _p(f, C.c_double))
    return f


def boundary_psi(params, precision, x, type_, obj):
    """psi_b = rho0 / sum_{same object} W (boundary volumes)."""
    P = make_params(params, precision)
    x = _f64(x)
    type_ = np.ascontiguousarray(type_, np.uint8)
    obj = np.ascontiguousarray(obj, np.int32)
    n = x.shape[0]
    bids = np.nonzero(type_ == BOUNDARY)[0]
    psi = np.zeros(n)
    if bids.size == 0:
        return psi
    counts, offs, ids = neighbors(params, precision, x, bids)
    fc = np.zeros(n, np.int64)
    fo = np.zeros(n, np.int64)
    fc[bids] = counts
    fo[bids] = offs
    lib().orc_boundary_psi(C.byref(P), n, _p(x, C.c_double), _p(type_, C.c_uint8),
                           _p(obj, C.c_int32), _p(fc, C.c_int64), _p(fo, C.c_int64),
                           _p(ids, C.c_int64), _p(psi, C.c_double))
    return psi


def wrench(object_, o, q, r_loc, f):
    """F = sum f_b, T = sum (R(q) r_loc) x f_b over the particles of object o."""
    obj = np.ascontiguousarray(object_, np.int32)
    q, r_loc, f = _f64(q), _f64(r_loc), _f64(f)
    F, T = np.zeros(3), np.zeros(3)
    lib().orc_wrench(obj.shape[0], _p(obj, C.c_int32), int(o), _p(q, C.c_double),
                     _p(r_loc, C.c_double), _p(f, C.c_double), _p(F, C.c_double), _p(T, C.c_double))
    return F, T


def integrate(params, precision, type_, mass, f, x, v):
    """Semi-implicit Euler (Eq. euler) in place on copies; returns (x, v)."""
    P = make_params(params, precision)
    x, v = _f64(x).copy(), _f64(v).copy()
    type_ = np.ascontiguousarray(type_, np.uint8)
    lib().orc_integrate(C.byref(P), x.shape[0], _p(type_, C.c_uint8), _p(_f64(mass), C.c_double),
                        _p(_f64(f), C.c_double), _p(x, C.c_double), _p(v, C.c_double))
    return x, v


def round_to(a, precision):
    return np.asarray(a, np.float32).astype(np.float64) if precision == "f32" else np.asarray(a, np.float64)


# --------------------------------------------------------------------------
# one simulation, stepped in the paper's order
# --------------------------------------------------------------------------

class Oracle:
    """Holds a scene's state (binary64) and steps it.

    The state starts from the scene rounded to the run's precision (the same
    rounding the GPU library applies at initialisation).  Kinematic objects
    carry a pose (c, q, v, w); between pose updates the pose is advanced by
    c += v dt, q <- normalise(q + dt/2 (0,w) q) after every step.  Dynamic
    objects (object_kinematic 2) carry the pose of their centre of mass and,
    while not grabbed, first update v and w from the step's wrench, gravity
    and their inertia (body_velocity_step).
    """

    def __init__(self, scene, precision=None):
        self.sc = scene
        self.prec = precision or scene.precision
        self.params = dict(scene.params)
        self.P = make_params(self.params, self.prec)
        self.n = scene.n
        self.x = round_to(scene.x, self.prec).copy()
        self.v = round_to(scene.v, self.prec).copy()
        # the particle state holds masses (and, below, boundary volumes) at the
        # run's precision too; rigid-body mass properties use the scene's FP64
        # masses
        self.mass = round_to(scene.mass, self.prec).copy()
        self.type = np.ascontiguousarray(scene.type, np.uint8)
        self.obj = np.ascontiguousarray(scene.object, np.int32)
        self.kin = [o for o in range(len(scene.object_kinematic)) if scene.object_kinematic[o]]
        self.pose = {}
        self.free = {}          # dynamic objects: True while integrated, False while grabbed
        self.body = {}          # dynamic objects: (mass, body-frame inertia)
        self.r_loc = np.zeros((self.n, 3))
        for o in self.kin:
            p0 = _f64(scene.object_pose0[o]).copy()
            if scene.object_kinematic[o] == 2:
                m, com, I = body_mass_props(scene.x, scene.mass, self.obj, o, p0[3:])
                p0[:3] = com
                self.body[o] = (m, I)
                self.free[o] = True
            lib().orc_body_frame(self.n, _p(_f64(scene.x), C.c_double), _p(self.obj, C.c_int32), o,
                                 _p(p0, C.c_double), _p(self.r_loc, C.c_double))
            q = p0[3:] / np.linalg.norm(p0[3:])
            self.pose[o] = [p0[:3].copy(), q, np.zeros(3), np.zeros(3)]
        self.psi = round_to(self._psi(), self.prec).copy()
        self.K = int(self.params.get("smoothing_window", 20))
        self.unified = bool(int(self.params.get("flags", 0)) & UNIFIED_BOUNDARY)
        self.samples = {o: [] for o in self.kin}
        self.nsteps = 0

    # boundary volumes from the initial configuration
    def _psi(self):
        return boundary_psi(self.params, self.prec, self.x, self.type, self.obj)

    def grab(self, o):
        """A dynamic object follows set_pose from now on (smoothing restarts)."""
        self.free[o] = False
        self.samples[o] = []

    def release(self, o):
        """A grabbed dynamic object moves under its wrench again."""
        self.free[o] = True
        self.samples[o] = []

    def set_pose(self, o, c, q, v, w):
        q = _f64(q)
        self.pose[o] = [_f64(c).copy(), q / np.linalg.norm(q), _f64(v).copy(), _f64(w).copy()]

    def place(self):
        for o in self.kin:
            c, q, v, w = self.pose[o]
            lib().orc_body_place(self.n, _p(self.obj, C.c_int32), o, _p(c, C.c_double),
                                 _p(q, C.c_double), _p(v, C.c_double), _p(w, C.c_double),
                                 _p(self.r_loc, C.c_double), _p(self.x, C.c_double),
                                 _p(self.v, C.c_double))

    def _springs(self):
        sc = self.sc
        if sc.spring_ij.shape[0] == 0:
            return np.zeros((self.n, 3))
        return springs(self.n, self.x, self.v, sc.spring_ij, sc.spring_L0, sc.spring_k, sc.spring_c)

    def density(self, targets, nbr):
        counts, offs, ids = nbr
        targets = np.ascontiguousarray(targets, np.int64)
        rho = np.zeros(targets.shape[0])
        pr = np.zeros(targets.shape[0])
        lib().orc_density(C.byref(self.P), self.n, _p(self.x, C.c_double), _p(self.mass, C.c_double),
                          _p(self.type, C.c_uint8), _p(self.psi, C.c_double), targets.shape[0],
                          _p(targets, C.c_int64), _p(counts, C.c_int64), _p(offs, C.c_int64),
                          _p(ids, C.c_int64), _p(rho, C.c_double), _p(pr, C.c_double))
        return rho, pr

    def forces(self, targets, nbr, rho_full, p_full, fspring):
        counts, offs, ids = nbr
        targets = np.ascontiguousarray(targets, np.int64)
        f = np.zeros((targets.shape[0], 3))
        fs = _f64(fspring)
        lib().orc_forces(C.byref(self.P), self.n, _p(self.x, C.c_double), _p(self.v, C.c_double),
                         _p(self.mass, C.c_double), _p(self.type, C.c_uint8), _p(self.psi, C.c_double),
                         _p(rho_full, C.c_double), _p(p_full, C.c_double), _p(fs, C.c_double),
                         targets.shape[0], _p(targets, C.c_int64), _p(counts, C.c_int64),
                         _p(offs, C.c_int64), _p(ids, C.c_int64), _p(f, C.c_double))
        return f

    def wrench(self, o, f_full):
        F, T = np.zeros(3), np.zeros(3)
        q = self.pose[o][1]
        lib().orc_wrench(self.n, _p(self.obj, C.c_int32), o, _p(q, C.c_double),
                         _p(self.r_loc, C.c_double), _p(_f64(f_full), C.c_double),
                         _p(F, C.c_double), _p(T, C.c_double))
        return F, T

    def probe_points_world(self, points, frame):
        """World coordinates of probe points given in world (frame -1) or in
        the frame of kinematic object `frame` (c + R p), with the current
        poses."""
        pts = _f64(points).reshape(-1, 3).copy()
        for t, o in enumerate(np.asarray(frame, np.int64)):
            if o >= 0:
                c, q = self.pose[int(o)][0], self.pose[int(o)][1]
                pts[t] = c + quat_to_R(q).reshape(3, 3) @ pts[t]
        return pts

    def step(self, keep_neighbors=False, probes=None):
        """One step: placement, keys, neighbours, springs, density, forces,
        wrench, integration, pose advance.  Returns the quantities computed
        from the pre-integration state and updates x, v, poses.  `probes` =
        (points, frame) adds the probe densities of that state as "probe"."""
        self.place()
        out = {"x_pre": self.x.copy(), "v_pre": self.v.copy()}
        if probes is not None:
            w = self.probe_points_world(*probes)
            out["probe"] = probe_density(self.params, self.prec, self.x, self.mass, self.type, w)
        out["keys"] = cell_keys(self.params, self.prec, self.x)
        nbr = neighbors(self.params, self.prec, self.x)
        if keep_neighbors:
            out["nbr"] = nbr
        counts, offs, ids = nbr
        fspring = self._springs()
        mov = np.nonzero(self.type != BOUNDARY)[0]
        rho_full = np.zeros(self.n)
        p_full = np.zeros(self.n)
        sub = lambda idx: (counts[idx], offs[idx], ids)   # noqa: E731
        # unified reading: boundary particles carry their own density and
        # pressure (Eq. density with psi_b as their mass)
        dens_t = np.arange(self.n) if self.unified else mov
        r, p = self.density(dens_t, sub(dens_t))
        rho_full[dens_t], p_full[dens_t] = r, p
        kin_b = np.nonzero((self.type == BOUNDARY) & np.isin(self.obj, self.kin))[0]
        tg = np.concatenate([mov, kin_b])
        f_t = self.forces(tg, sub(tg), rho_full, p_full, fspring)
        f_full = np.zeros((self.n, 3))
        f_full[tg] = f_t
        out.update(rho=rho_full, p=p_full, f=f_full, fspring=fspring)
        out["wrench"] = {}
        for o in self.kin:
            F, T = self.wrench(o, f_full)
            out["wrench"][o] = (F, T)
            self.samples[o].append(np.concatenate([F, T]))
        lib().orc_integrate(C.byref(self.P), self.n, _p(self.type, C.c_uint8),
                            _p(self.mass, C.c_double), _p(f_full, C.c_double),
                            _p(self.x, C.c_double), _p(self.v, C.c_double))
        for o in self.kin:
            c, q, v, w = self.pose[o]
            if self.free.get(o, False):
                m, I = self.body[o]
                F, T = out["wrench"][o]
                v, w = body_velocity_step(F, T, m, I, q, self.params["gravity"], self.params["dt"], v, w)
            c2, q2 = pose_advance(c, q, v, w, self.params["dt"])
            self.pose[o] = [c2, q2, v, w]
        self.nsteps += 1
        out["x"], out["v"] = self.x.copy(), self.v.copy()
        return out

    def smoothed_wrench(self, o):
        """Rolling average (Sec. 3.3) of the last min(K, count) samples."""
        s = self.samples[o]
        if not s:
            return np.zeros(6)
        return np.mean(np.asarray(s[-self.K:]), axis=0)

    def sampled(self, targets):
        """Density and force of selected targets from the current state
        (after placement), for full-size checks where a whole-scene pass is
        too slow: density is computed for the targets and all their
        neighbours, forces for the targets only."""
        targets = np.ascontiguousarray(targets, np.int64)
        self.place()
        nb_t = neighbors(self.params, self.prec, self.x, targets)
        mark = np.zeros(self.n, bool)
        mark[targets] = True
        mark[nb_t[2]] = True
        union = np.nonzero(mark)[0]
        union_mov = union if self.unified else union[self.type[union] != BOUNDARY]
        nb_u = neighbors(self.params, self.prec, self.x, union_mov)
        rho_full = np.zeros(self.n)
        p_full = np.zeros(self.n)
        r, p = self.density(union_mov, nb_u)
        rho_full[union_mov], p_full[union_mov] = r, p
        fspring = self._springs()
        f = self.forces(targets, nb_t, rho_full, p_full, fspring)
        return {"rho": rho_full[targets], "p": p_full[targets], "f": f, "nbr": nb_t}
