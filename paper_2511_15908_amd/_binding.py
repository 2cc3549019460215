"""ctypes binding of libsph.so (include/sph.h).

Argument marshalling only: every step of the SPH path runs in the HIP kernels
of libsph.so.  PyTorch provides the device workspace (one uint8 tensor) and
the stream.  There is no CPU fallback: without the built library every entry
point raises.
"""
from __future__ import annotations

import ctypes as C
import os
from pathlib import Path

import numpy as np

_PKG = Path(__file__).resolve().parent
LIB_PATH = Path(os.environ.get("SPH_LIB", _PKG / "libsph.so"))

SPH_ABI_VERSION = 1
SPH_STATIC_WORKSPACE_BYTES = 128 << 20
SPH_FP32, SPH_FP64 = 0, 1
SPH_FLUID, SPH_SOFT, SPH_BOUNDARY = 0, 1, 2
(SPH_FLAG_CLAMP_NEG_PRESSURE, SPH_FLAG_BOUNDARY_SINGLE_TERM, SPH_FLAG_NO_BOUNDARY_VISCOSITY,
 SPH_FLAG_UNIFIED_BOUNDARY) = 1, 2, 4, 8
(SPH_FIELD_X, SPH_FIELD_V, SPH_FIELD_RHO, SPH_FIELD_PRESSURE, SPH_FIELD_FORCE, SPH_FIELD_PSI,
 SPH_FIELD_KEY, SPH_FIELD_SPRING) = range(8)
FIELD_NAMES = {"x": SPH_FIELD_X, "v": SPH_FIELD_V, "rho": SPH_FIELD_RHO, "p": SPH_FIELD_PRESSURE,
               "f": SPH_FIELD_FORCE, "psi": SPH_FIELD_PSI, "key": SPH_FIELD_KEY,
               "fspring": SPH_FIELD_SPRING}
STATUS = {0: "SPH_OK", 1: "SPH_ERR_ARG", 2: "SPH_ERR_WORKSPACE", 3: "SPH_ERR_DEVICE",
          4: "SPH_ERR_STATE", 5: "SPH_ERR_UNSTABLE", 6: "SPH_ERR_UNSUPPORTED", 7: "SPH_ERR_CAPACITY"}
N_PHASES = 10

EXPORTED = ["sph_workspace_size", "sph_init", "sph_init_static", "sph_set_body_pose", "sph_step", "sph_get_body_wrench",
            "sph_reset_smoothing", "sph_read_field", "sph_debug_neighbors", "sph_debug_neighbors_of",
            "sph_get_stats", "sph_get_info",
            "sph_synchronize", "sph_profile_begin", "sph_profile_begin_sampled", "sph_profile_read",
            "sph_profile_phase_name",
            "sph_set_probes", "sph_read_probes", "sph_grab_body", "sph_release_body", "sph_get_body_state",
            "sph_batch_workspace_size", "sph_batch_init", "sph_read_log", "sph_read_probe_log", "sph_set_graph",
            "sph_set_body_track", "sph_destroy", "sph_status_string", "sph_last_error"]


class SphError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {msg}")


class SphParams(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("precision", C.c_int32), ("flags", C.c_uint32),
                ("smoothing_window", C.c_uint32), ("h", C.c_double), ("rho0", C.c_double),
                ("k_pressure", C.c_double), ("nu", C.c_double), ("gravity", C.c_double * 3),
                ("dt", C.c_double), ("domain_lo", C.c_double * 3), ("domain_hi", C.c_double * 3),
                ("v_max", C.c_double), ("max_probes", C.c_uint32), ("log_steps", C.c_uint32),
                ("track_steps", C.c_uint32), ("reserved", C.c_uint32 * 5)]


class SphScene(C.Structure):
    _fields_ = [("n", C.c_uint32), ("x", C.POINTER(C.c_double)), ("v", C.POINTER(C.c_double)),
                ("mass", C.POINTER(C.c_double)), ("type", C.POINTER(C.c_uint8)),
                ("object", C.POINTER(C.c_int32)), ("n_objects", C.c_uint32),
                ("object_kinematic", C.POINTER(C.c_uint8)), ("object_pose0", C.POINTER(C.c_double)),
                ("n_springs", C.c_uint32), ("spring_ij", C.POINTER(C.c_uint32)),
                ("spring_L0", C.POINTER(C.c_double)), ("spring_k", C.POINTER(C.c_double)),
                ("spring_c", C.POINTER(C.c_double))]


class SphInfo(C.Structure):
    _fields_ = [("n", C.c_uint32), ("n_fluid", C.c_uint32), ("n_soft", C.c_uint32),
                ("n_boundary", C.c_uint32), ("n_body_particles", C.c_uint32),
                ("n_kinematic", C.c_uint32), ("grid_dims", C.c_uint32 * 3), ("grid_bits", C.c_uint32),
                ("cell_slots", C.c_uint32), ("max_candidates", C.c_uint32), ("steps", C.c_uint64),
                ("cell_size", C.c_double)]


_lib = None


def load_library(path=None):
    """Load libsph.so and declare its prototypes; raise if it is not built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = Path(path) if path else LIB_PATH
    if not p.exists():
        raise RuntimeError(f"libsph.so not built ({p}); run `python -m paper_2511_15908_amd.build`")
    L = C.CDLL(str(p))
    vp, sz = C.c_void_p, C.c_size_t
    d3 = C.POINTER(C.c_double)
    L.sph_workspace_size.argtypes = [C.POINTER(SphParams), C.POINTER(SphScene), C.POINTER(sz)]
    L.sph_init.argtypes = [C.POINTER(SphParams), C.POINTER(SphScene), vp, sz, vp, C.POINTER(vp)]
    L.sph_init_static.argtypes = [C.POINTER(SphParams), C.POINTER(SphScene), vp, C.POINTER(vp)]
    L.sph_set_body_pose.argtypes = [vp, C.c_uint32, d3, d3, d3, d3]
    L.sph_step.argtypes = [vp, C.c_uint32, vp]
    L.sph_get_body_wrench.argtypes = [vp, C.c_uint32, d3, d3, C.c_int]
    L.sph_reset_smoothing.argtypes = [vp, C.c_uint32]
    L.sph_read_field.argtypes = [vp, C.c_int, vp, sz]
    L.sph_debug_neighbors.argtypes = [vp, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), sz,
                                      C.POINTER(sz)]
    L.sph_debug_neighbors_of.argtypes = [vp, C.c_uint32, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                         C.POINTER(C.c_uint32), sz, C.POINTER(sz)]
    L.sph_get_info.argtypes = [vp, C.POINTER(SphInfo)]
    L.sph_get_stats.argtypes = [vp, C.POINTER(C.c_uint64)]
    L.sph_synchronize.argtypes = [vp]
    L.sph_profile_begin.argtypes = [vp, C.c_uint32]
    L.sph_profile_begin_sampled.argtypes = [vp, C.c_uint32, C.c_uint32]
    L.sph_profile_read.argtypes = [vp, d3, C.POINTER(C.c_uint32), C.c_uint32]
    L.sph_profile_phase_name.argtypes = [C.c_uint32]
    L.sph_profile_phase_name.restype = C.c_char_p
    L.sph_set_probes.argtypes = [vp, C.c_uint32, d3, C.POINTER(C.c_int32)]
    L.sph_read_probes.argtypes = [vp, d3, C.c_uint32]
    L.sph_grab_body.argtypes = [vp, C.c_uint32]
    L.sph_batch_workspace_size.argtypes = [C.POINTER(SphParams), C.POINTER(SphScene), C.c_uint32, C.POINTER(sz)]
    L.sph_batch_init.argtypes = [C.POINTER(SphParams), C.POINTER(SphScene), C.c_uint32, vp, sz, vp, C.POINTER(vp)]
    L.sph_read_log.argtypes = [vp, d3, sz, C.POINTER(C.c_uint32)]
    L.sph_read_probe_log.argtypes = [vp, d3, sz, C.POINTER(C.c_uint32)]
    L.sph_set_graph.argtypes = [vp, C.c_int]
    L.sph_set_body_track.argtypes = [vp, C.c_uint32, C.c_uint32, d3]
    L.sph_release_body.argtypes = [vp, C.c_uint32]
    L.sph_get_body_state.argtypes = [vp, C.c_uint32, d3, d3, d3, d3]
    L.sph_destroy.argtypes = [vp]
    L.sph_status_string.argtypes = [C.c_int]
    L.sph_status_string.restype = C.c_char_p
    L.sph_last_error.argtypes = [vp]
    L.sph_last_error.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("sph_profile_phase_name", "sph_status_string", "sph_last_error"):
            getattr(L, name).restype = C.c_int
    if path is None:
        _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None and a.size else None


def make_params(params: dict, precision: str, v_max: float = 0.0, max_probes: int = 0,
                log_steps: int = 0, track_steps: int = 0) -> SphParams:
    P = SphParams()
    P.abi_version = SPH_ABI_VERSION
    P.precision = SPH_FP64 if precision == "f64" else SPH_FP32
    P.flags = int(params.get("flags", 0))
    P.smoothing_window = int(params.get("smoothing_window", 20))
    P.h, P.rho0, P.k_pressure, P.nu = params["h"], params["rho0"], params["k_pressure"], params["nu"]
    P.gravity[:] = list(params["gravity"])
    P.dt = params["dt"]
    P.domain_lo[:] = list(params["domain_lo"])
    P.domain_hi[:] = list(params["domain_hi"])
    P.v_max = float(v_max)
    P.max_probes = int(max_probes)
    P.log_steps = int(log_steps)
    P.track_steps = int(track_steps)
    return P


class _SceneArrays:
    """Keeps the numpy arrays alive while the C struct points at them."""

    def __init__(self, scene):
        n = scene.n
        self.x = np.ascontiguousarray(scene.x, np.float64).reshape(n, 3)
        self.v = np.ascontiguousarray(scene.v, np.float64).reshape(n, 3)
        self.mass = np.ascontiguousarray(scene.mass, np.float64)
        self.type = np.ascontiguousarray(scene.type, np.uint8)
        self.object = np.ascontiguousarray(scene.object, np.int32)
        self.kin = np.ascontiguousarray(scene.object_kinematic, np.uint8)
        self.pose0 = np.ascontiguousarray(scene.object_pose0, np.float64).reshape(-1, 7)
        self.ij = np.ascontiguousarray(scene.spring_ij, np.uint32).reshape(-1, 2)
        self.L0 = np.ascontiguousarray(scene.spring_L0, np.float64)
        self.k = np.ascontiguousarray(scene.spring_k, np.float64)
        self.c = np.ascontiguousarray(scene.spring_c, np.float64)
        S = SphScene()
        S.n = n
        S.x, S.v, S.mass = _dp(self.x), _dp(self.v), _dp(self.mass)
        S.type = self.type.ctypes.data_as(C.POINTER(C.c_uint8)) if n else None
        S.object = self.object.ctypes.data_as(C.POINTER(C.c_int32)) if n else None
        S.n_objects = self.kin.shape[0]
        S.object_kinematic = self.kin.ctypes.data_as(C.POINTER(C.c_uint8)) if self.kin.size else None
        S.object_pose0 = _dp(self.pose0)
        S.n_springs = self.ij.shape[0]
        S.spring_ij = self.ij.ctypes.data_as(C.POINTER(C.c_uint32)) if self.ij.size else None
        S.spring_L0, S.spring_k, S.spring_c = _dp(self.L0), _dp(self.k), _dp(self.c)
        self.struct = S


def workspace_size(scene, precision=None, v_max=0.0) -> int:
    L = load_library()
    P = make_params(scene.params, precision or scene.precision, v_max)
    A = _SceneArrays(scene)
    out = C.c_size_t(0)
    st = L.sph_workspace_size(C.byref(P), C.byref(A.struct), C.byref(out))
    if st:
        raise SphError(st, "sph_workspace_size")
    return int(out.value)


class Sim:
    """One simulation context on a GPU.

    scene: a paper_2511_15908_amd.scenes.Scene, or a list of them (a batch
    stepped together; particle and object ids of scene k follow those of the
    earlier scenes).  The workspace is a torch uint8 tensor on `device`;
    kernels run on torch's current stream of that device (or `stream`, a
    torch.cuda.Stream).  static_workspace=True (one scene) uses the library's
    own per-device workspace instead (sph_init_static: nothing is allocated;
    one such context per device at a time).
    """

    def __init__(self, scene, precision=None, device="cuda", stream=None, v_max=0.0, params=None, max_probes=0,
                 log_steps=0, track_steps=0, static_workspace=False):
        import torch
        self.torch = torch
        self.L = load_library()
        scenes = list(scene) if isinstance(scene, (list, tuple)) else [scene]
        self.precision = precision or scenes[0].precision
        self.device = torch.device(device)
        self._stream = stream
        ns = len(scenes)
        self.P = (SphParams * ns)()
        self._arrays = [_SceneArrays(sc) for sc in scenes]
        S = (SphScene * ns)()
        for k, sc in enumerate(scenes):
            pr = dict(sc.params)
            if params:
                pr.update(params)
            self.P[k] = make_params(pr, self.precision, v_max, max_probes, log_steps, track_steps)
            S[k] = self._arrays[k].struct
        self.ctx = C.c_void_p()
        if static_workspace:
            if ns != 1:
                raise ValueError("static_workspace takes one scene")
            self.ws, self.ws_bytes = None, 0
            with torch.cuda.device(self.device):
                st = self.L.sph_init_static(self.P, S, self.stream_handle(), C.byref(self.ctx))
            if st:
                raise SphError(st, "sph_init_static")
        else:
            out = C.c_size_t(0)
            st = self.L.sph_batch_workspace_size(self.P, S, ns, C.byref(out))
            if st:
                raise SphError(st, "sph_batch_workspace_size")
            self.ws_bytes = int(out.value)
            self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            base = self.ws.data_ptr()
            aligned = (base + 255) & ~255
            st = self.L.sph_batch_init(self.P, S, ns, C.c_void_p(aligned), self.ws_bytes, self.stream_handle(),
                                       C.byref(self.ctx))
            if st:
                raise SphError(st, "sph_batch_init")
        self.n = sum(sc.n for sc in scenes)
        self.part0 = np.cumsum([0] + [sc.n for sc in scenes])
        self.obj0 = np.cumsum([0] + [len(sc.object_kinematic) for sc in scenes])
        self.kinematic = [int(self.obj0[k]) + o for k, sc in enumerate(scenes)
                          for o in range(len(sc.object_kinematic)) if sc.object_kinematic[o]]
        self.log_steps = int(log_steps)

    # -- plumbing
    def stream_handle(self):
        s = self._stream if self._stream is not None else self.torch.cuda.current_stream(self.device)
        return C.c_void_p(s.cuda_stream)

    def _check(self, st, what):
        if st:
            msg = self.L.sph_last_error(self.ctx)
            raise SphError(st, f"{what}: {msg.decode() if msg else ''}")

    # -- the C ABI
    def step(self, n=1):
        self._check(self.L.sph_step(self.ctx, int(n), self.stream_handle()), "sph_step")

    def set_body_pose(self, obj, c, q, v=(0, 0, 0), w=(0, 0, 0)):
        arr = [np.ascontiguousarray(a, np.float64) for a in (c, q, v, w)]
        self._check(self.L.sph_set_body_pose(self.ctx, int(obj), *[_dp(a) for a in arr]),
                    "sph_set_body_pose")

    def wrench(self, obj, smoothed=False, check=True):
        F = np.zeros(3)
        T = np.zeros(3)
        st = self.L.sph_get_body_wrench(self.ctx, int(obj), _dp(F), _dp(T), int(bool(smoothed)))
        if check:
            self._check(st, "sph_get_body_wrench")
        return F, T

    def set_body_track(self, obj, poses):
        """poses: [n][13] (c, q, v, w) for the next n steps, taken on the device."""
        p = np.ascontiguousarray(poses, np.float64).reshape(-1, 13)
        self._check(self.L.sph_set_body_track(self.ctx, int(obj), p.shape[0], _dp(p)), "sph_set_body_track")

    def set_graph(self, enable=True):
        """Replay steps as a captured two-step HIP graph (non-default stream)."""
        self._check(self.L.sph_set_graph(self.ctx, int(bool(enable))), "sph_set_graph")

    def read_log(self):
        """Per-step body records [steps][bodies][20] (c, q, v, w, F, T, step),
        oldest first; empties the log."""
        nb = len(self.kinematic)
        out = np.zeros(max(self.log_steps, 1) * max(nb, 1) * 20)
        m = C.c_uint32(0)
        self._check(self.L.sph_read_log(self.ctx, _dp(out), out.size, C.byref(m)), "sph_read_log")
        return out[:m.value * nb * 20].reshape(m.value, nb, 20)

    def read_probe_log(self):
        """Per-step probe densities [steps][n_probes] of the steps read_log
        would return (oldest first); does not empty the log."""
        npr = getattr(self, "n_probes", 0)
        out = np.zeros(max(self.log_steps, 1) * max(npr, 1))
        m = C.c_uint32(0)
        self._check(self.L.sph_read_probe_log(self.ctx, _dp(out), out.size, C.byref(m)), "sph_read_probe_log")
        return out[:m.value * npr].reshape(m.value, npr)

    def grab(self, obj):
        """A free rigid body follows set_body_pose until release()."""
        self._check(self.L.sph_grab_body(self.ctx, int(obj)), "sph_grab_body")

    def release(self, obj):
        self._check(self.L.sph_release_body(self.ctx, int(obj)), "sph_release_body")

    def body_state(self, obj):
        """(c, q, v, w) of a kinematic or free body (synchronises)."""
        c, q, v, w = np.zeros(3), np.zeros(4), np.zeros(3), np.zeros(3)
        self._check(self.L.sph_get_body_state(self.ctx, int(obj), _dp(c), _dp(q), _dp(v), _dp(w)),
                    "sph_get_body_state")
        return c, q, v, w

    def reset_smoothing(self, obj):
        self._check(self.L.sph_reset_smoothing(self.ctx, int(obj)), "sph_reset_smoothing")

    def read(self, field, check=True):
        fid = FIELD_NAMES[field] if isinstance(field, str) else int(field)
        if fid == SPH_FIELD_KEY:
            out = np.zeros(self.n, np.uint32)
        elif fid in (SPH_FIELD_X, SPH_FIELD_V, SPH_FIELD_FORCE, SPH_FIELD_SPRING):
            out = np.zeros((self.n, 3), np.float64)
        else:
            out = np.zeros(self.n, np.float64)
        st = self.L.sph_read_field(self.ctx, fid, out.ctypes.data_as(C.c_void_p) if out.size else None,
                                   out.nbytes)
        if check:
            self._check(st, "sph_read_field")
        return out

    def neighbors(self):
        """(counts, offsets, ids) of the last density pass, in particle-id order."""
        counts = np.zeros(max(self.n, 1), np.uint32)
        tot = C.c_size_t(0)
        self._check(self.L.sph_debug_neighbors(self.ctx, counts.ctypes.data_as(C.POINTER(C.c_uint32)),
                                               None, 0, C.byref(tot)), "sph_debug_neighbors")
        ids = np.zeros(max(tot.value, 1), np.uint32)
        self._check(self.L.sph_debug_neighbors(self.ctx, counts.ctypes.data_as(C.POINTER(C.c_uint32)),
                                               ids.ctypes.data_as(C.POINTER(C.c_uint32)), ids.size,
                                               C.byref(tot)), "sph_debug_neighbors")
        counts = counts[:self.n].astype(np.int64)
        offs = np.zeros(self.n, np.int64)
        if self.n:
            offs[1:] = np.cumsum(counts)[:-1]
        return counts, offs, ids[:tot.value].astype(np.int64)

    def neighbors_of(self, targets):
        """(counts, offsets, ids) of the given particle ids, in their order."""
        t = np.ascontiguousarray(targets, np.uint32)
        counts = np.zeros(max(t.size, 1), np.uint32)
        tot = C.c_size_t(0)
        P = C.POINTER(C.c_uint32)
        self._check(self.L.sph_debug_neighbors_of(self.ctx, t.size, t.ctypes.data_as(P), counts.ctypes.data_as(P),
                                                  None, 0, C.byref(tot)), "sph_debug_neighbors_of")
        ids = np.zeros(max(tot.value, 1), np.uint32)
        self._check(self.L.sph_debug_neighbors_of(self.ctx, t.size, t.ctypes.data_as(P), counts.ctypes.data_as(P),
                                                  ids.ctypes.data_as(P), ids.size, C.byref(tot)),
                    "sph_debug_neighbors_of")
        counts = counts[:t.size].astype(np.int64)
        offs = np.zeros(t.size, np.int64)
        if t.size:
            offs[1:] = np.cumsum(counts)[:-1]
        return counts, offs, ids[:tot.value].astype(np.int64)

    def set_probes(self, points, frame=None):
        """Density probe points ([n,3]); frame[i] = kinematic object id of the
        body whose frame point i is given in, or -1 for world coordinates."""
        pts = np.ascontiguousarray(points, np.float64).reshape(-1, 3)
        fr = np.full(pts.shape[0], -1, np.int32) if frame is None else np.ascontiguousarray(frame, np.int32)
        self._check(self.L.sph_set_probes(self.ctx, pts.shape[0], _dp(pts),
                                          fr.ctypes.data_as(C.POINTER(C.c_int32)) if fr.size else None),
                    "sph_set_probes")
        self.n_probes = pts.shape[0]

    def read_probes(self):
        out = np.zeros(getattr(self, "n_probes", 0))
        self._check(self.L.sph_read_probes(self.ctx, _dp(out), out.size), "sph_read_probes")
        return out

    def info(self) -> dict:
        I = SphInfo()
        self._check(self.L.sph_get_info(self.ctx, C.byref(I)), "sph_get_info")
        return {k: (list(getattr(I, k)) if k == "grid_dims" else getattr(I, k)) for k, _ in I._fields_}

    def stats(self) -> dict:
        """Cumulative device work counters of the density pass."""
        v = (C.c_uint64 * 6)()
        self._check(self.L.sph_get_stats(self.ctx, v), "sph_get_stats")
        return {"pairs_density": v[0], "pairs_force": v[1], "candidates": v[2], "waves": v[3],
                "iter_density": v[4], "iter_force": v[5]}

    def synchronize(self):
        self._check(self.L.sph_synchronize(self.ctx), "sph_synchronize")

    def profile_begin(self, max_steps, every=1):
        """Per-phase event timing on the next max_steps steps, recorded on
        every `every`-th of them."""
        self._check(self.L.sph_profile_begin_sampled(self.ctx, int(max_steps), int(every)),
                    "sph_profile_begin_sampled")

    def profile_read(self) -> dict:
        ms = np.zeros(N_PHASES)
        cnt = np.zeros(N_PHASES, np.uint32)
        self._check(self.L.sph_profile_read(self.ctx, _dp(ms), cnt.ctypes.data_as(C.POINTER(C.c_uint32)),
                                            N_PHASES), "sph_profile_read")
        return {self.L.sph_profile_phase_name(k).decode(): (float(ms[k]), int(cnt[k]))
                for k in range(N_PHASES)}

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.L.sph_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
