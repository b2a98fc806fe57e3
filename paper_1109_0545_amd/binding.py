"""ctypes binding of libqdpath.so (argument marshalling only).

Every computation runs in the HIP kernels behind the C-ABI declared in
``include/qdpath.h``; this module converts numpy arrays and torch tensors to
pointers, checks status codes and raises ``QdpError`` with the library's
message.  If the shared library is missing the import fails loudly: there is
no fallback implementation.
"""

from __future__ import annotations

import ctypes as ct
import os
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqdpath.so")

QDP_F64, QDP_DD, QDP_QD = 1, 2, 4
SOLVE_FULL, SOLVE_MIXED_IR = 0, 1
PRED_SECANT, PRED_LEARNED, PRED_QUADRATIC = 0, 1, 2
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENONFINITE", 5: "EUNSUPPORTED"}

ARITH_OPS = {"add": 0, "sub": 1, "mul": 2, "div": 3, "cadd": 10, "csub": 11, "cmul": 12, "cdiv": 13, "cfms": 14,
             "cinv": 15, "pivot": 16}


class QdpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qdpath {STATUS.get(status, status)}: {msg}")
        self.status = status


class NewtonInfo(ct.Structure):
    _fields_ = [
        ("iterations", ct.c_int32),
        ("success", ct.c_int32),
        ("singular", ct.c_int32),
        ("nonfinite", ct.c_int32),
        ("residual_first", ct.c_double),
        ("residual_last", ct.c_double),
        ("cond_est", ct.c_double),
        ("dz_norm", ct.c_double),
        ("refine_err", ct.c_double),
        ("refine_steps", ct.c_int32),
        ("pad", ct.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class TrackParams(ct.Structure):
    _fields_ = [
        ("lambda0", ct.c_double),
        ("lambda_min", ct.c_double),
        ("lambda_max", ct.c_double),
        ("shrink", ct.c_double),
        ("expand", ct.c_double),
        ("expand_after", ct.c_int32),
        ("max_it_path", ct.c_int32),
        ("eps_path", ct.c_double),
        ("eps_end", ct.c_double),
        ("max_it_end", ct.c_int32),
        ("predictor", ct.c_int32),
        ("max_steps", ct.c_int64),
        ("mode", ct.c_int32),
        ("probe", ct.c_int32),
        ("policy", ct.c_void_p),
        ("lambda_max_learned", ct.c_double),
        ("accept_threshold", ct.c_double),
        ("policy_rule", ct.c_int32),
        ("pad2", ct.c_int32),
    ]


class TrackStats(ct.Structure):
    _fields_ = [
        ("fail", ct.c_int32),
        ("end_success", ct.c_int32),
        ("t_final", ct.c_double),
        ("succ_corrections", ct.c_int64),
        ("corrections", ct.c_int64),
        ("newton_iterations", ct.c_int64),
        ("avg_step", ct.c_double),
        ("min_step", ct.c_double),
        ("seconds", ct.c_double),
        ("end_residual", ct.c_double),
        ("policy_used", ct.c_int64),
        ("policy_rejected", ct.c_int64),
        ("log_count", ct.c_int64),
        ("probe_corrections", ct.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


N_FEATURES = 16
N_MULT = 5


class StepRecord(ct.Structure):
    _fields_ = [
        ("t", ct.c_double),
        ("lam", ct.c_double),
        ("rho_first", ct.c_double),
        ("rho_last", ct.c_double),
        ("dz_first", ct.c_double),
        ("cond_est", ct.c_double),
        ("znorm", ct.c_double),
        ("pred_dist", ct.c_double),
        ("blend_label", ct.c_double),
        ("features", ct.c_float * N_FEATURES),
        ("iterations", ct.c_int32),
        ("accepted", ct.c_int32),
        ("kind", ct.c_int32),
        ("probe_ok", ct.c_int32),
    ]


_P = ct.c_void_p
_D = ct.POINTER(ct.c_double)

# name -> (restype, argtypes)
SIGNATURES = {
    "qdp_system_create": (ct.c_int, [ct.c_int32, _P, _P, _P, ct.c_int, ct.POINTER(_P)]),
    "qdp_system_destroy": (None, [_P]),
    "qdp_homotopy_create": (ct.c_int, [_P, _P, ct.POINTER(_P)]),
    "qdp_homotopy_destroy": (None, [_P]),
    "qdp_eval_jacobian": (ct.c_int, [_P, _P, ct.c_int, _P, _P, _P]),
    "qdp_eval_jacobian_dev": (ct.c_int, [_P, _P, ct.c_int, _P, _P, _P]),
    "qdp_eval_homotopy": (ct.c_int, [_P, ct.c_double, _P, ct.c_int, _P, _P, _P, _P]),
    "qdp_eval_homotopy_dev": (ct.c_int, [_P, ct.c_double, _P, ct.c_int, _P, _P, _P, _P]),
    "qdp_newton_step": (ct.c_int, [_P, ct.c_double, _P, ct.c_int, ct.c_int, ct.c_double, ct.c_int32,
                                   ct.POINTER(NewtonInfo), _P]),
    "qdp_newton_step_dev": (ct.c_int, [_P, ct.c_double, _P, ct.c_int, ct.c_int, ct.c_double, ct.c_int32, _P]),
    "qdp_newton_step_noalloc_dev": (ct.c_int, [_P, ct.c_double, _P, ct.c_int, ct.c_int, ct.c_double, ct.c_int32,
                                               _P, _P]),
    "qdp_homotopy_last_info": (ct.c_int, [_P, ct.c_int, ct.POINTER(NewtonInfo), _P]),
    "qdp_eval_homotopy_batch_dev": (ct.c_int, [_P, ct.c_double, _P, ct.c_int32, ct.c_int, _P, _P, _P, _P]),
    "qdp_newton_batch_dev": (ct.c_int, [_P, ct.c_double, _P, ct.c_int32, ct.c_int, ct.c_int, ct.c_double,
                                        ct.c_int32, _P]),
    "qdp_homotopy_last_info_batch": (ct.c_int, [_P, ct.c_int, ct.c_int32, ct.POINTER(NewtonInfo), _P]),
    "qdp_track_params_default": (ct.c_int, [ct.POINTER(TrackParams)]),
    "qdp_track_path": (ct.c_int, [_P, _P, ct.c_int, ct.POINTER(TrackParams), ct.POINTER(TrackStats),
                                  ct.POINTER(StepRecord), ct.c_int64, _P]),
    "qdp_track_paths": (ct.c_int, [_P, _P, ct.c_int32, ct.c_int, ct.POINTER(TrackParams), ct.POINTER(TrackStats),
                                   _P]),
    "qdp_arith_batch": (ct.c_int, [ct.c_int32, ct.c_int, ct.c_int64, _P, _P, _P, _P, _P]),
    "qdp_set_timing": (ct.c_int, [ct.c_int32]),
    "qdp_set_elimination": (ct.c_int, [ct.c_int32]),
    "qdp_homotopy_last_timing": (ct.c_int, [_P, ct.c_int, _D, _D, ct.POINTER(ct.c_int32), _P]),
    "qdp_policy_create": (ct.c_int, [ct.c_int32, _P, _P, _P, _P, ct.POINTER(_P)]),
    "qdp_policy_destroy": (None, [_P]),
    "qdp_policy_get_params": (ct.c_int, [_P, _P]),
    "qdp_policy_save": (ct.c_int, [_P, ct.c_char_p]),
    "qdp_policy_load": (ct.c_int, [ct.c_char_p, ct.POINTER(_P)]),
    "qdp_policy_gradient": (ct.c_int, [_P, _P, _P, _P, ct.c_int32, _P, _P, _P]),
    "qdp_policy_adam_step": (ct.c_int, [_P, _P, ct.c_float, ct.c_float, ct.c_float, ct.c_float, _P]),
    "qdp_policy_train_step": (ct.c_int, [_P, _P, _P, _P, ct.c_int32, ct.c_float, ct.c_float, ct.c_float,
                                         ct.c_float, _P, _P]),
    "qdp_policy_forward": (ct.c_int, [_P, _P, ct.c_int32, ct.c_int32, _P, _P]),
    "qdp_policy_infer_host": (ct.c_int, [_P, _P, _P, _P]),
    "qdp_last_error": (ct.c_char_p, []),
    "qdp_version": (ct.c_char_p, []),
}

_lib = None


def lib():
    """Load libqdpath.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built: run python -m paper_1109_0545_amd.build")
        L = ct.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise QdpError(status, lib().qdp_last_error().decode())


def _ptr(a) -> int:
    """Address of a contiguous host numpy array (None passes through)."""
    if a is None:
        return None
    if not isinstance(a, np.ndarray):
        raise QdpError(1, f"expected a numpy array, got {type(a).__name__}")
    if not a.flags["C_CONTIGUOUS"]:
        raise QdpError(1, "array must be C-contiguous")
    return a.ctypes.data


def _dev(a, name: str, numel: int, dtype: str = "float64", nullable: bool = False):
    """Device address of a torch tensor that a kernel will touch for ``numel``
    elements of ``dtype``: raises QdpError before any launch unless the tensor
    is on the GPU, has that dtype, is contiguous and holds at least ``numel``
    elements (a wrong buffer would otherwise become an out-of-bounds access)."""
    if a is None:
        if nullable:
            return None
        raise QdpError(1, f"{name}: a device tensor is required")
    import torch

    if not isinstance(a, torch.Tensor):
        raise QdpError(1, f"{name}: expected a torch tensor on the GPU, got {type(a).__name__}")
    if not a.is_cuda:
        raise QdpError(1, f"{name}: tensor is on {a.device}, not on the GPU")
    if a.dtype != getattr(torch, dtype):
        raise QdpError(1, f"{name}: dtype {a.dtype}, expected torch.{dtype}")
    if not a.is_contiguous():
        raise QdpError(1, f"{name}: tensor must be contiguous")
    if a.numel() < numel:
        raise QdpError(1, f"{name}: {a.numel()} elements, the call touches {numel}")
    return a.data_ptr()


def _host_point(x, shape, name: str = "x") -> np.ndarray:
    """A C-contiguous float64 copy of a host array of exactly ``shape``."""
    x = np.array(x, dtype=np.float64, copy=True, order="C")
    if x.shape != tuple(shape):
        raise QdpError(1, f"{name}: shape {x.shape}, expected {tuple(shape)}")
    return x


def _count(B) -> int:
    B = int(B)
    if B < 1:
        raise QdpError(1, f"batch size {B} < 1")
    return B


def _stream(s) -> Optional[int]:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


# ------------------------------------------------------------------ handles


class System:
    """Device copy of a sparse system (``qdp_system``)."""

    def __init__(self, n: int, poly_offsets, exps, coefs, prec: int):
        self.n = int(n)
        self.prec = int(prec)
        self._off = np.ascontiguousarray(poly_offsets, dtype=np.int32)
        self._exps = np.ascontiguousarray(exps, dtype=np.uint8)
        self._coefs = np.ascontiguousarray(coefs, dtype=np.float64)
        if self.n < 1 or self._off.shape != (self.n + 1,):
            raise QdpError(1, f"poly_offsets must hold n + 1 = {self.n + 1} entries")
        terms = int(self._off[-1])
        if self._exps.shape != (terms, self.n):
            raise QdpError(1, f"exps: shape {self._exps.shape}, expected [{terms}][{self.n}]")
        if self._coefs.shape != (terms, 2, self.prec):
            raise QdpError(1, f"coefs: shape {self._coefs.shape}, expected [{terms}][2][{self.prec}]")
        h = _P()
        _check(lib().qdp_system_create(self.n, _ptr(self._off), _ptr(self._exps), _ptr(self._coefs), self.prec,
                                       ct.byref(h)))
        self.handle = h

    @classmethod
    def from_synth(cls, s, prec: Optional[int] = None):
        prec = prec or s.L
        coefs = np.ascontiguousarray(s.coefs[:, :, :prec])
        return cls(s.n, s.poly_offsets, s.exps, coefs, prec)

    def close(self):
        if getattr(self, "handle", None):
            lib().qdp_system_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Homotopy:
    """Total-degree homotopy t f + (1-t) gamma (x^d - 1) (``qdp_homotopy``)."""

    def __init__(self, system: System, gamma):
        self.system = system
        g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64)[:, : system.prec])
        h = _P()
        _check(lib().qdp_homotopy_create(system.handle, _ptr(g), ct.byref(h)))
        self.handle = h
        self.n = system.n

    def close(self):
        if getattr(self, "handle", None):
            lib().qdp_homotopy_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Policy:
    """Step-size network (``qdp_policy``): FP32 master parameters on the device."""

    def __init__(self, widths, params, feat_mean, feat_std):
        self.widths = np.ascontiguousarray(widths, dtype=np.int32)
        p = np.ascontiguousarray(params, dtype=np.float32)
        mu = np.ascontiguousarray(feat_mean, dtype=np.float32)
        sd = np.ascontiguousarray(feat_std, dtype=np.float32)
        h = _P()
        _check(lib().qdp_policy_create(len(self.widths), _ptr(self.widths), _ptr(p), _ptr(mu), _ptr(sd),
                                       ct.byref(h)))
        self.handle = h
        self.n_params = p.size
        self.feat_mean, self.feat_std = mu, sd

    @classmethod
    def load(cls, path: str) -> "Policy":
        """qdp_policy_load: a network from a file written by save()."""
        h = _P()
        _check(lib().qdp_policy_load(os.fsencode(path), ct.byref(h)))
        self = cls.__new__(cls)
        self.handle = h
        # widths and normalisation back from the file's header (read by the library above)
        with open(path, "rb") as fh:
            fh.read(8)
            nw = int(np.frombuffer(fh.read(4), dtype="<i4")[0])
            self.widths = np.frombuffer(fh.read(4 * nw), dtype="<i4").astype(np.int32)
        self.n_params = int(sum(o * i + o for i, o in zip(self.widths[:-1], self.widths[1:])))
        with open(path, "rb") as fh:
            fh.seek(12 + 4 * nw + 4 * self.n_params)
            w0 = int(self.widths[0])
            self.feat_mean = np.frombuffer(fh.read(4 * w0), dtype="<f4").copy()
            self.feat_std = np.frombuffer(fh.read(4 * w0), dtype="<f4").copy()
        return self

    def save(self, path: str) -> None:
        """qdp_policy_save: widths, parameters and feature normalisation to a file."""
        _check(lib().qdp_policy_save(self.handle, os.fsencode(path)))

    def params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().qdp_policy_get_params(self.handle, _ptr(out)))
        return out

    def _batch(self, X, Y=None, M=None):
        B = _count(X.shape[0]) if hasattr(X, "shape") and len(X.shape) else _count(0)
        ni, no = int(self.widths[0]), int(self.widths[-1])
        ptrs = [_dev(X, "X", B * ni, "float32")]
        if Y is not None or M is not None:
            ptrs += [_dev(Y, "Y", B * no, "float32"), _dev(M, "M", B * no, "float32")]
        return B, ptrs

    def gradient(self, X, Y, M, grad_out=None, stream=None):
        """Device tensors in; returns the loss (float); gradient into grad_out (device) if given."""
        B, (px, py, pm) = self._batch(X, Y, M)
        pg = _dev(grad_out, "grad_out", self.n_params, "float32", nullable=True)
        loss = ct.c_float()
        _check(lib().qdp_policy_gradient(self.handle, px, py, pm, B, pg, ct.byref(loss), _stream(stream)))
        return loss.value

    def adam_step(self, grad=None, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        pg = _dev(grad, "grad", self.n_params, "float32", nullable=True)
        _check(lib().qdp_policy_adam_step(self.handle, pg, lr, b1, b2, eps, _stream(stream)))

    def train_step(self, X, Y, M, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, want_loss=False, stream=None):
        B, (px, py, pm) = self._batch(X, Y, M)
        loss = ct.c_float()
        _check(lib().qdp_policy_train_step(self.handle, px, py, pm, B, lr, b1, b2, eps,
                                           ct.byref(loss) if want_loss else None, _stream(stream)))
        return loss.value if want_loss else None

    def forward(self, X, bf16=True, stream=None):
        import torch

        B, (px,) = self._batch(X)
        Y = torch.empty((B, int(self.widths[-1])), dtype=torch.float32, device=X.device)
        _check(lib().qdp_policy_forward(self.handle, px, B, 1 if bf16 else 0, Y.data_ptr(), _stream(stream)))
        return Y

    def close(self):
        if getattr(self, "handle", None):
            lib().qdp_policy_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ calls


def eval_jacobian(system: System, x: np.ndarray, prec: int, stream=None) -> Tuple[np.ndarray, np.ndarray]:
    n = system.n
    x = _host_point(x, (n, 2, prec))
    y = np.zeros((n, 2, prec))
    J = np.zeros((n, n, 2, prec))
    _check(lib().qdp_eval_jacobian(system.handle, _ptr(x), prec, _ptr(y), _ptr(J), _stream(stream)))
    return y, J


def eval_jacobian_dev(system: System, x, prec: int, y, jac, stream=None) -> None:
    v = system.n * 2 * prec
    px, py, pj = _dev(x, "x", v), _dev(y, "y", v), _dev(jac, "jac", system.n * v)
    _check(lib().qdp_eval_jacobian_dev(system.handle, px, prec, py, pj, _stream(stream)))


def eval_homotopy(h: Homotopy, t: float, x: np.ndarray, prec: int, stream=None):
    n = h.n
    x = _host_point(x, (n, 2, prec))
    y = np.zeros((n, 2, prec))
    J = np.zeros((n, n, 2, prec))
    S = np.zeros(n)
    _check(lib().qdp_eval_homotopy(h.handle, float(t), _ptr(x), prec, _ptr(y), _ptr(J), _ptr(S), _stream(stream)))
    return y, J, S


def eval_homotopy_dev(h: Homotopy, t: float, x, prec: int, y, jac, scale=None, stream=None) -> None:
    v = h.n * 2 * prec
    px, py, pj = _dev(x, "x", v), _dev(y, "y", v), _dev(jac, "jac", h.n * v)
    ps = _dev(scale, "scale", h.n, nullable=True)
    _check(lib().qdp_eval_homotopy_dev(h.handle, float(t), px, prec, py, pj, ps, _stream(stream)))


def eval_homotopy_batch_dev(h: Homotopy, t: float, x, B: int, prec: int, y, jac, scale=None, stream=None) -> None:
    """B points x [B][n][2][prec] (device) -> y [B][n][2][prec], jac [B][n][n][2][prec], scale [B][n]."""
    B = _count(B)
    v = B * h.n * 2 * prec
    px, py, pj = _dev(x, "x", v), _dev(y, "y", v), _dev(jac, "jac", h.n * v)
    ps = _dev(scale, "scale", B * h.n, nullable=True)
    _check(lib().qdp_eval_homotopy_batch_dev(h.handle, float(t), px, B, prec, py, pj, ps, _stream(stream)))


def newton_batch_dev(h: Homotopy, t: float, x, B: int, prec: int, mode: int = SOLVE_FULL, eps: float = 1e-10,
                     max_it: int = 4, stream=None) -> None:
    B = _count(B)
    px = _dev(x, "x", B * h.n * 2 * prec)
    _check(lib().qdp_newton_batch_dev(h.handle, float(t), px, B, prec, mode, float(eps), int(max_it),
                                      _stream(stream)))


def last_info_batch(h: Homotopy, prec: int, B: int, stream=None) -> list:
    infos = (NewtonInfo * B)()
    _check(lib().qdp_homotopy_last_info_batch(h.handle, prec, int(B), infos, _stream(stream)))
    return [infos[b].as_dict() for b in range(B)]


def newton_step(h: Homotopy, t: float, x: np.ndarray, prec: int, mode: int = SOLVE_FULL, eps: float = 1e-10,
                max_it: int = 4, stream=None):
    """Returns (new x, info dict)."""
    x = _host_point(x, (h.n, 2, prec))
    info = NewtonInfo()
    _check(lib().qdp_newton_step(h.handle, float(t), _ptr(x), prec, mode, float(eps), int(max_it), ct.byref(info),
                                 _stream(stream)))
    return x, info.as_dict()


def newton_step_dev(h: Homotopy, t: float, x, prec: int, mode: int = SOLVE_FULL, eps: float = 1e-10,
                    max_it: int = 4, stream=None) -> None:
    px = _dev(x, "x", h.n * 2 * prec)
    _check(lib().qdp_newton_step_dev(h.handle, float(t), px, prec, mode, float(eps), int(max_it),
                                     _stream(stream)))


def newton_step_noalloc_dev(h: Homotopy, t: float, x, prec: int, mode: int = SOLVE_FULL, eps: float = 1e-10,
                            max_it: int = 4, info=None, stream=None) -> None:
    """qdp_newton_step_noalloc_dev: x a device tensor (in/out); info an optional
    device uint8 tensor of at least sizeof(qdp_newton_info) bytes (decode with
    info_from_bytes after synchronising).  Allocates nothing."""
    px = _dev(x, "x", h.n * 2 * prec)
    pi = _dev(info, "info", ct.sizeof(NewtonInfo), "uint8", nullable=True)
    _check(lib().qdp_newton_step_noalloc_dev(h.handle, float(t), px, prec, mode, float(eps), int(max_it), pi,
                                             _stream(stream)))


def info_from_bytes(raw) -> dict:
    """A qdp_newton_info from its bytes (host numpy uint8 array)."""
    return NewtonInfo.from_buffer_copy(bytes(np.asarray(raw, dtype=np.uint8)[: ct.sizeof(NewtonInfo)])).as_dict()


def last_info(h: Homotopy, prec: int, stream=None) -> dict:
    info = NewtonInfo()
    _check(lib().qdp_homotopy_last_info(h.handle, prec, ct.byref(info), _stream(stream)))
    return info.as_dict()


def default_track_params(**overrides) -> TrackParams:
    p = TrackParams()
    _check(lib().qdp_track_params_default(ct.byref(p)))
    for k, v in overrides.items():
        if k == "policy" and v is not None and not isinstance(v, int):
            v = v.handle.value if hasattr(v.handle, "value") else v.handle
        setattr(p, k, v)
    return p


def track_path(h: Homotopy, x0: np.ndarray, prec: int, params: Optional[TrackParams] = None, log_cap: int = 0,
               stream=None):
    """Returns (endpoint, stats dict, step log list or None)."""
    x = _host_point(x0, (h.n, 2, prec), "x0")
    st = TrackStats()
    p = params if params is not None else default_track_params()
    log = (StepRecord * log_cap)() if log_cap > 0 else None
    _check(lib().qdp_track_path(h.handle, _ptr(x), prec, ct.byref(p), ct.byref(st), log, int(log_cap),
                                _stream(stream)))
    recs = None
    if log is not None:
        recs = []
        for i in range(st.log_count):
            r = log[i]
            d = {f: getattr(r, f) for f, _ in StepRecord._fields_ if f != "features"}
            d["features"] = np.ctypeslib.as_array(r.features).copy()
            recs.append(d)
    return x, st.as_dict(), recs


def track_paths(h: Homotopy, x0: np.ndarray, prec: int, params: Optional[TrackParams] = None, stream=None):
    """B paths at once: x0 [B][n][2][prec] start solutions.  Returns (end points, list of stats dicts)."""
    x = np.array(x0, dtype=np.float64, copy=True, order="C")
    if x.ndim != 4 or x.shape[1:] != (h.n, 2, prec):
        raise QdpError(1, f"x0: shape {x.shape}, expected [B][{h.n}][2][{prec}]")
    nb = _count(x.shape[0])
    st = (TrackStats * nb)()
    p = params if params is not None else default_track_params()
    _check(lib().qdp_track_paths(h.handle, _ptr(x), nb, prec, ct.byref(p), st, _stream(stream)))
    return x, [st[b].as_dict() for b in range(nb)]


def arith_batch(op: str, prec: int, a, b=None, c=None, stream=None):
    """Elementwise multiword op on device tensors (float64, [count][L] or [count][2][L])."""
    import torch

    if op not in ARITH_OPS:
        raise QdpError(1, f"unknown op {op}")
    count = int(a.shape[0])
    pa = _dev(a, "a", max(a.numel(), count))
    pb = _dev(b, "b", a.numel(), nullable=True)
    pc = _dev(c, "c", a.numel(), nullable=True)
    out = torch.empty((count, prec), dtype=a.dtype, device=a.device) if op == "pivot" else torch.empty_like(a)
    _check(lib().qdp_arith_batch(ARITH_OPS[op], prec, count, pa, pb, pc, out.data_ptr(), _stream(stream)))
    return out


ELIM_AUTO, ELIM_POINT, ELIM_COLUMNS, ELIM_BLOCKS = 0, 1, 2, 3


def set_elimination(policy: int) -> None:
    """qdp_set_elimination: ELIM_AUTO, ELIM_POINT (one workgroup per point),
    ELIM_COLUMNS (one workgroup per column) or ELIM_BLOCKS (blocks of columns
    per workgroup), process-wide."""
    _check(lib().qdp_set_elimination(int(policy)))


def set_timing(on: bool) -> None:
    _check(lib().qdp_set_timing(1 if on else 0))


def last_timing(h: Homotopy, prec: int, stream=None):
    """(eval ms summed, solve ms summed, iterations timed) of the last Newton call."""
    a, b, k = ct.c_double(), ct.c_double(), ct.c_int32()
    _check(lib().qdp_homotopy_last_timing(h.handle, prec, ct.byref(a), ct.byref(b), ct.byref(k), _stream(stream)))
    return a.value, b.value, k.value


def version() -> str:
    return lib().qdp_version().decode()
