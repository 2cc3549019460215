"""ctypes binding of the wrench-surrogate MLP (include/sph_mlp.h, in libsph.so).

Argument marshalling only: the products, activations, loss, gradients,
Adam and the haptic-tick chain run in the HIP kernels of libsph.so.  Device
arrays are torch tensors (float32, contiguous); the workspace is one torch
uint8 tensor.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from ._binding import load_library

MLP_ABI_VERSION = 1
STATUS = {0: "MLP_OK", 1: "MLP_ERR_ARG", 2: "MLP_ERR_WORKSPACE", 3: "MLP_ERR_DEVICE", 4: "MLP_ERR_STATE",
          5: "MLP_ERR_NONFINITE"}
EXPORTED = ["mlp_workspace_size", "mlp_init", "mlp_param_count", "mlp_set_params", "mlp_get_params",
            "mlp_fit_normalizer", "mlp_set_normalizer", "mlp_get_normalizer", "mlp_forward", "mlp_gradients",
            "mlp_adam_step", "mlp_train_step", "mlp_last_loss", "mlp_predict_one", "mlp_predict_one_device",
            "mlp_gemm_bf16", "mlp_destroy", "mlp_last_error", "mlp_set_input_range", "mlp_get_input_range",
            "mlp_set_guard", "mlp_guard_count"]


class MlpError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {msg}")


class MlpConfig(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("n_in", C.c_uint32), ("n_out", C.c_uint32),
                ("hidden", C.c_uint32), ("layers", C.c_uint32), ("max_batch", C.c_uint32),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float), ("residual_from", C.c_uint32),
                ("reserved", C.c_uint32 * 6)]


_declared = False


def lib():
    global _declared
    L = load_library()
    if not _declared:
        vp, f32p, d = C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_double)
        L.mlp_workspace_size.argtypes = [C.POINTER(MlpConfig), C.POINTER(C.c_size_t)]
        L.mlp_init.argtypes = [C.POINTER(MlpConfig), vp, C.c_size_t, vp, C.POINTER(vp)]
        L.mlp_param_count.argtypes = [vp]
        L.mlp_param_count.restype = C.c_size_t
        L.mlp_set_params.argtypes = [vp, f32p, C.c_size_t]
        L.mlp_get_params.argtypes = [vp, f32p, C.c_size_t]
        L.mlp_fit_normalizer.argtypes = [vp, vp, vp, C.c_uint32]
        L.mlp_set_normalizer.argtypes = [vp, f32p, f32p, f32p, f32p]
        L.mlp_get_normalizer.argtypes = [vp, f32p, f32p, f32p, f32p]
        L.mlp_forward.argtypes = [vp, vp, C.c_uint32, vp]
        L.mlp_gradients.argtypes = [vp, vp, vp, C.c_uint32, f32p, d]
        L.mlp_adam_step.argtypes = [vp, f32p, C.c_size_t, C.c_float]
        L.mlp_train_step.argtypes = [vp, vp, vp, C.c_uint32, C.c_float]
        L.mlp_last_loss.argtypes = [vp, d]
        L.mlp_predict_one.argtypes = [vp, f32p, f32p]
        L.mlp_predict_one_device.argtypes = [vp, vp, vp]
        L.mlp_gemm_bf16.argtypes = [vp, C.c_int, C.c_int, vp, C.c_uint32, vp, C.c_uint32, C.c_uint32, C.c_uint32,
                                    C.c_uint32, vp, C.c_uint32]
        L.mlp_set_input_range.argtypes = [vp, f32p, f32p]
        L.mlp_get_input_range.argtypes = [vp, f32p, f32p]
        L.mlp_set_guard.argtypes = [vp, C.c_float]
        L.mlp_guard_count.argtypes = [vp, C.POINTER(C.c_uint64)]
        L.mlp_destroy.argtypes = [vp]
        L.mlp_last_error.argtypes = [vp]
        L.mlp_last_error.restype = C.c_char_p
        for name in EXPORTED:
            if name not in ("mlp_param_count", "mlp_last_error"):
                getattr(L, name).restype = C.c_int
        _declared = True
    return L


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _dev(t):
    return C.c_void_p(t.data_ptr())


class Mlp:
    """A network of `layers` hidden layers of `hidden` units on one GPU."""

    def __init__(self, n_in, n_out, hidden=256, layers=3, max_batch=4096, device="cuda", stream=None,
                 beta1=0.9, beta2=0.999, eps=1e-8, residual_col=None):
        import torch
        self.torch = torch
        self.L = lib()
        self.device = torch.device(device)
        self._stream = stream
        cfg = MlpConfig()
        cfg.abi_version = MLP_ABI_VERSION
        cfg.n_in, cfg.n_out, cfg.hidden, cfg.layers, cfg.max_batch = n_in, n_out, hidden, layers, max_batch
        cfg.beta1, cfg.beta2, cfg.eps = beta1, beta2, eps
        cfg.residual_from = 0 if residual_col is None else int(residual_col) + 1
        self.cfg = cfg
        nb = C.c_size_t(0)
        st = self.L.mlp_workspace_size(C.byref(cfg), C.byref(nb))
        if st:
            raise MlpError(st, "mlp_workspace_size")
        self.ws = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        base = (self.ws.data_ptr() + 255) & ~255
        self.ctx = C.c_void_p()
        st = self.L.mlp_init(C.byref(cfg), C.c_void_p(base), int(nb.value), self.stream_handle(), C.byref(self.ctx))
        if st:
            raise MlpError(st, "mlp_init")
        self.n_params = int(self.L.mlp_param_count(self.ctx))
        self.n_in, self.n_out = n_in, n_out
        self._px = np.zeros(n_in, np.float32)
        self._py = np.zeros(n_out, np.float32)

    def stream_handle(self):
        s = self._stream if self._stream is not None else self.torch.cuda.current_stream(self.device)
        return C.c_void_p(s.cuda_stream)

    def _check(self, st, what):
        if st:
            msg = self.L.mlp_last_error(self.ctx)
            raise MlpError(st, f"{what}: {msg.decode() if msg else ''}")

    def _f32(self, t, cols):
        t = t.to(device=self.device, dtype=self.torch.float32).contiguous()
        assert t.dim() == 2 and t.shape[1] == cols, t.shape
        return t

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        self._check(self.L.mlp_set_params(self.ctx, _fp(p), p.size), "mlp_set_params")

    def get_params(self):
        p = np.zeros(self.n_params, np.float32)
        self._check(self.L.mlp_get_params(self.ctx, _fp(p), p.size), "mlp_get_params")
        return p

    def fit_normalizer(self, X, Y):
        X, Y = self._f32(X, self.n_in), self._f32(Y, self.n_out)
        self._check(self.L.mlp_fit_normalizer(self.ctx, _dev(X), _dev(Y), X.shape[0]), "mlp_fit_normalizer")

    def set_normalizer(self, mu_x, sd_x, mu_y, sd_y):
        a = [np.ascontiguousarray(v, np.float32) for v in (mu_x, sd_x, mu_y, sd_y)]
        self._check(self.L.mlp_set_normalizer(self.ctx, *[_fp(v) for v in a]), "mlp_set_normalizer")

    def get_normalizer(self):
        a = [np.zeros(self.n_in, np.float32), np.zeros(self.n_in, np.float32),
             np.zeros(self.n_out, np.float32), np.zeros(self.n_out, np.float32)]
        self._check(self.L.mlp_get_normalizer(self.ctx, *[_fp(v) for v in a]), "mlp_get_normalizer")
        return a

    def set_input_range(self, lo, hi):
        a = [np.ascontiguousarray(v, np.float32) for v in (lo, hi)]
        self._check(self.L.mlp_set_input_range(self.ctx, *[_fp(v) for v in a]), "mlp_set_input_range")

    def get_input_range(self):
        a = [np.zeros(self.n_in, np.float32), np.zeros(self.n_in, np.float32)]
        self._check(self.L.mlp_get_input_range(self.ctx, *[_fp(v) for v in a]), "mlp_get_input_range")
        return a

    def set_guard(self, margin):
        """Plain-SPH fallback: rows outside the training range (widened by
        margin x range per side) return the residual base; margin < 0: off."""
        self._check(self.L.mlp_set_guard(self.ctx, float(margin)), "mlp_set_guard")
        self.guard_margin = float(margin) if margin >= 0 else -1.0

    def guard_count(self):
        """(rows checked by guarded calls, rows that fell back) since init."""
        v = (C.c_uint64 * 2)()
        self._check(self.L.mlp_guard_count(self.ctx, v), "mlp_guard_count")
        return int(v[0]), int(v[1])

    def forward(self, X):
        X = self._f32(X, self.n_in)
        out = self.torch.empty((X.shape[0], self.n_out), dtype=self.torch.float32, device=self.device)
        self._check(self.L.mlp_forward(self.ctx, _dev(X), X.shape[0], _dev(out)), "mlp_forward")
        return out

    def gradients(self, X, Y):
        X, Y = self._f32(X, self.n_in), self._f32(Y, self.n_out)
        g = np.zeros(self.n_params, np.float32)
        loss = C.c_double(0.0)
        self._check(self.L.mlp_gradients(self.ctx, _dev(X), _dev(Y), X.shape[0], _fp(g), C.byref(loss)),
                    "mlp_gradients")
        return g, loss.value

    def adam_step(self, grad, lr):
        g = np.ascontiguousarray(grad, np.float32)
        self._check(self.L.mlp_adam_step(self.ctx, _fp(g), g.size, float(lr)), "mlp_adam_step")

    def train_step(self, X, Y, lr):
        """X, Y: float32 contiguous device tensors (not copied)."""
        self._check(self.L.mlp_train_step(self.ctx, _dev(X), _dev(Y), X.shape[0], float(lr)), "mlp_train_step")

    def last_loss(self):
        v = C.c_double(0.0)
        self._check(self.L.mlp_last_loss(self.ctx, C.byref(v)), "mlp_last_loss")
        return v.value

    def predict_one(self, x):
        self._px[:] = x
        self._check(self.L.mlp_predict_one(self.ctx, _fp(self._px), _fp(self._py)), "mlp_predict_one")
        return self._py.copy()

    def predict_one_device(self, x, y):
        self._check(self.L.mlp_predict_one_device(self.ctx, _dev(x), _dev(y)), "mlp_predict_one_device")

    def close(self):
        if getattr(self, "ctx", None):
            self.L.mlp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gemm_bf16(A_bits, B_bits, M, N, K, a_layout=0, b_layout=0, lda=None, ldb=None):
    """C = A B with BF16 operands given as int16 bit-pattern device tensors
    (layouts as in mlp_gemm_bf16); returns an FP32 M x N tensor."""
    import torch
    L = lib()
    lda = lda if lda is not None else (K if a_layout == 0 else M)
    ldb = ldb if ldb is not None else (K if b_layout == 0 else N)
    Cm = torch.empty((M, N), dtype=torch.float32, device=A_bits.device)
    s = torch.cuda.current_stream(A_bits.device)
    st = L.mlp_gemm_bf16(C.c_void_p(s.cuda_stream), a_layout, b_layout, _dev(A_bits), lda, _dev(B_bits), ldb,
                         M, N, K, _dev(Cm), N)
    if st:
        raise MlpError(st, "mlp_gemm_bf16")
    return Cm
