"""Python binding of the MI355X LSKUM library (argument marshalling only).

Every computation runs in ``liblskum.so`` (hand-written HIP for gfx950);
this module converts arguments, owns nothing but handles, and raises
``LskumError`` with the library's message on a non-zero status.  Device
memory and streams may come from PyTorch (tensors' ``data_ptr()``, streams'
``cuda_stream``); host arrays are numpy.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import cloudgen

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblskum.so")

OK, ERR_ARG, ERR_CONNECTIVITY, ERR_DEGENERATE, ERR_COLOURING = 0, -1, -2, -3, -4
ERR_NONPHYSICAL, ERR_NOT_CONVERGED, ERR_HIP, ERR_OOM = -5, -6, -7, -8
JVP_EXACT, JVP_FLUXDIFF = 0, 1
FP64, MIXED = 0, 1
ANANDH, MANISH = 0, 1
IMPLICIT, EXPLICIT = 0, 1
ORDER_COLOUR, ORDER_WALL_FIRST = 0, 1
FARFIELD_DIRICHLET, FARFIELD_KINETIC = 0, 1


class LskumError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lskum error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("cfl", C.c_double), ("inner_iters", C.c_int32),
                ("jvp_mode", C.c_int32), ("precision", C.c_int32), ("check_every", C.c_int32),
                ("tol_rel", C.c_double), ("max_iters", C.c_int32), ("sweep_lanes", C.c_int32),
                ("residual_lanes", C.c_int32), ("limiter", C.c_int32), ("limiter_k", C.c_double),
                ("variant", C.c_int32), ("scheme", C.c_int32), ("order", C.c_int32),
                ("farfield", C.c_int32), ("qgrad_lanes", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("res_fs", C.c_double),
                ("res_first", C.c_double), ("res_final", C.c_double), ("seconds", C.c_double),
                ("cl", C.c_double), ("cd", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

# name -> (restype, argtypes); mirrors include/lskum.h
_SIGS = {
    "lskum_default_params": (None, [C.c_void_p]),
    "lskum_cloud_create": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lskum_cloud_info": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lskum_cloud_colours": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lskum_cloud_destroy": (None, [C.c_void_p]),
    "lskum_state_create": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "lskum_state_destroy": (None, [C.c_void_p]),
    "lskum_state_set_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lskum_state_set_U": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "lskum_state_get_U": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "lskum_state_get_dU": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "lskum_residual": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "lskum_q_derivatives": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "lskum_lusgs_step": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lskum_step_timed": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lskum_solve": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lskum_forces": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lskum_batch_create": (C.c_int, [C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lskum_batch_info": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lskum_batch_set_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lskum_batch_set_cfl": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lskum_batch_get_cfl": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lskum_batch_set_cfl_control": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_double]),
    "lskum_batch_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lskum_batch_step_timed": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lskum_batch_get_U": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int]),
    "lskum_batch_set_U": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int]),
    "lskum_batch_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                       C.c_void_p]),
    "lskum_batch_destroy": (None, [C.c_void_p]),
    "lskum_mlp_create": (C.c_int, [C.c_uint64, C.c_int64, C.c_void_p, C.c_void_p]),
    "lskum_mlp_destroy": (None, [C.c_void_p]),
    "lskum_mlp_get_params": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "lskum_mlp_set_params": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "lskum_mlp_forward": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "lskum_mlp_gradient": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "lskum_mlp_train_step": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_float,
                                       C.c_void_p]),
    "lskum_mlp_train": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int32,
                                  C.c_int32, C.c_float, C.c_float, C.c_uint64, C.c_void_p,
                                  C.c_void_p]),
    "lskum_state_features": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lskum_batch_features": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lskum_mlp_warm_start": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lskum_mlp_warm_start_batch": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lskum_residual_noalloc": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lskum_residual_noalloc_max_points": (C.c_int64, []),
    "lskum_last_error": (C.c_char_p, []),
    "lskum_build_hash": (C.c_char_p, []),
}


def lib():
    """Loads the in-tree HIP library; raises if it has not been built or was
    built from other sources than the ones in the tree."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2406_07441_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        from . import build
        built, now = L.lskum_build_hash().decode(), build.source_hash()
        if built != now:
            raise RuntimeError(f"{LIB_PATH} was built from other sources (hash {built}, tree "
                               f"{now}): rebuild it with `python -m paper_2406_07441_amd.build`")
        _lib = L
    return _lib


def _check(code: int):
    if code != OK:
        raise LskumError(code, lib().lskum_last_error().decode())


def default_params(**kw) -> Params:
    p = Params()
    lib().lskum_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _ptr(a: np.ndarray):
    return a.ctypes.data


class Cloud:
    """Device copy of a point cloud (geometry, CSR, colours)."""

    def __init__(self, cloud: cloudgen.Cloud, colours: np.ndarray | None = None):
        self.src = cloud
        arrs = [np.ascontiguousarray(cloud.x, np.float64), np.ascontiguousarray(cloud.y, np.float64),
                np.ascontiguousarray(cloud.type, np.int8), np.ascontiguousarray(cloud.tx, np.float64),
                np.ascontiguousarray(cloud.ty, np.float64),
                np.ascontiguousarray(cloud.nbr_off, np.int32),
                np.ascontiguousarray(cloud.nbr_idx, np.int32)]
        col = None if colours is None else np.ascontiguousarray(colours, np.int32)
        h = C.c_void_p()
        _check(lib().lskum_cloud_create(cloud.n, *[_ptr(a) for a in arrs],
                                        None if col is None else _ptr(col), C.byref(h)))
        self.h = h
        n, nnz, nc, nd = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int64()
        _check(lib().lskum_cloud_info(h, C.byref(n), C.byref(nnz), C.byref(nc), C.byref(nd)))
        self.n, self.nnz, self.n_colours, self.n_degenerate = n.value, nnz.value, nc.value, nd.value

    def colours(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int32)
        _check(lib().lskum_cloud_colours(self.h, _ptr(out)))
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().lskum_cloud_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def residual_noalloc(cloud: Cloud, mach: float, aoa_deg: float, params: Params, U, R, res,
                     stream=None):
    """lskum_residual_noalloc: U ([4][n] float64 device tensor) -> R (same
    shape, or None) and res (2 float64 on the device: the norm, and 1.0 if a
    non-physical state was met).  Enqueued on `stream` (torch stream or raw
    handle; None = the default stream); nothing is synchronised."""
    handle = None
    if stream is not None:
        handle = stream if isinstance(stream, int) else stream.cuda_stream
    _check(lib().lskum_residual_noalloc(cloud.h, float(mach), float(aoa_deg), C.byref(params),
                                        U.data_ptr(), None if R is None else R.data_ptr(),
                                        res.data_ptr(), handle))


def residual_noalloc_max_points() -> int:
    return int(lib().lskum_residual_noalloc_max_points())


class State:
    """One flow condition on a cloud: U and the iteration's work arrays.

    ``stream`` is a torch.cuda.Stream (or a raw hipStream_t int); by default
    the library uses a private stream of default priority.
    """

    def __init__(self, cloud: Cloud, mach: float, aoa_deg: float, params: Params | None = None,
                 stream=None):
        self.cloud = cloud
        self.params = params if params is not None else default_params()
        handle = None
        if stream is not None:
            handle = stream if isinstance(stream, int) else stream.cuda_stream
        h = C.c_void_p()
        _check(lib().lskum_state_create(cloud.h, float(mach), float(aoa_deg),
                                        C.byref(self.params), handle, C.byref(h)))
        self.h = h
        self.n = cloud.n

    def close(self):
        if getattr(self, "h", None):
            lib().lskum_state_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: Params):
        _check(lib().lskum_state_set_params(self.h, C.byref(params)))
        self.params = params

    # -- fields ----------------------------------------------------------------
    def set_U(self, U):
        if isinstance(U, np.ndarray):
            U = np.ascontiguousarray(U, np.float64)
            assert U.shape == (4, self.n)
            _check(lib().lskum_state_set_U(self.h, _ptr(U), 0))
        else:  # torch tensor on the device
            import torch
            assert U.is_cuda and U.dtype == torch.float64 and U.shape == (4, self.n)
            U = U.contiguous()
            torch.cuda.current_stream().synchronize()
            _check(lib().lskum_state_set_U(self.h, U.data_ptr(), 1))

    def _get(self, fn, device: bool):
        if device:
            import torch
            out = torch.empty((4, self.n), dtype=torch.float64, device="cuda")
            torch.cuda.current_stream().synchronize()
            _check(fn(self.h, out.data_ptr(), 1))
            return out
        out = np.empty((4, self.n))
        _check(fn(self.h, _ptr(out), 0))
        return out

    def get_U(self, device: bool = False):
        return self._get(lib().lskum_state_get_U, device)

    def get_dU(self, device: bool = False):
        return self._get(lib().lskum_state_get_dU, device)

    # -- hot path ----------------------------------------------------------------
    def residual(self, want_R: bool = True):
        res = C.c_double()
        R = np.empty((4, self.n)) if want_R else None
        _check(lib().lskum_residual(self.h, None if R is None else _ptr(R), 0, C.byref(res)))
        return R, res.value

    def q_derivatives(self):
        qx, qy = np.empty((4, self.n)), np.empty((4, self.n))
        _check(lib().lskum_q_derivatives(self.h, _ptr(qx), _ptr(qy), 0))
        return qx, qy

    def step(self, want_res: bool = True):
        if not want_res:
            _check(lib().lskum_lusgs_step(self.h, None))
            return None
        res = C.c_double()
        _check(lib().lskum_lusgs_step(self.h, C.byref(res)))
        return res.value

    PHASES = ("q_derivatives", "residual", "norm", "forward_sweep", "backward_sweep", "update")

    def step_timed(self) -> dict:
        """One step with per-phase GPU times (ms) from HIP events."""
        ms = np.zeros(6)
        _check(lib().lskum_step_timed(self.h, _ptr(ms)))
        return dict(zip(self.PHASES, ms.tolist()))

    def solve(self, raise_on_error: bool = False) -> Report:
        rep = Report()
        code = lib().lskum_solve(self.h, C.byref(rep))
        if code != OK and (raise_on_error or code not in (ERR_NOT_CONVERGED, ERR_NONPHYSICAL)):
            _check(code)
        return rep

    def forces(self):
        cl, cd = C.c_double(), C.c_double()
        _check(lib().lskum_forces(self.h, C.byref(cl), C.byref(cd)))
        return cl.value, cd.value

    def features(self, targets: bool = False):
        """Warm-start features [n][5] (and targets [n][4]) as device tensors."""
        return _features(lib().lskum_state_features, self.h, self.n, targets)


class Batch:
    """Many flow conditions iterated together (one launch per kernel/phase).

    ``clouds``: list of ``Cloud``; condition k uses ``clouds[cond_cloud[k]]``
    at (``mach[k]``, ``aoa[k]``).
    """

    def __init__(self, clouds, cond_cloud, mach, aoa, params: Params | None = None, stream=None):
        self.clouds = list(clouds)
        self.params = params if params is not None else default_params()
        cc = np.ascontiguousarray(cond_cloud, np.int32)
        m = np.ascontiguousarray(mach, np.float64)
        a = np.ascontiguousarray(aoa, np.float64)
        assert cc.shape == m.shape == a.shape
        arr = (C.c_void_p * len(self.clouds))(*[c.h.value for c in self.clouds])
        handle = None
        if stream is not None:
            handle = stream if isinstance(stream, int) else stream.cuda_stream
        h = C.c_void_p()
        _check(lib().lskum_batch_create(len(self.clouds), arr, len(cc), _ptr(cc), _ptr(m), _ptr(a),
                                        C.byref(self.params), handle, C.byref(h)))
        self.h = h
        self.n_cond = len(cc)
        self.sizes = [self.clouds[k].n for k in cc]
        npt, nnz, nc = C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib().lskum_batch_info(h, C.byref(npt), C.byref(nnz), C.byref(nc)))
        self.n_points, self.nnz, self.n_colours = npt.value, nnz.value, nc.value

    def close(self):
        if getattr(self, "h", None):
            lib().lskum_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: Params):
        _check(lib().lskum_batch_set_params(self.h, C.byref(params)))
        self.params = params

    def set_cfl(self, cfl):
        """CFL number per condition (n_cond values > 0)."""
        cfl = np.ascontiguousarray(cfl, dtype=np.float64)
        assert cfl.shape == (self.n_cond,)
        _check(lib().lskum_batch_set_cfl(self.h, cfl.ctypes.data))

    def get_cfl(self) -> np.ndarray:
        out = np.empty(self.n_cond)
        _check(lib().lskum_batch_get_cfl(self.h, _ptr(out)))
        return out

    def set_cfl_control(self, window: int, factor: float = 0.3, cfl_min: float = 1.0):
        """Residual-driven per-condition CFL control (window 0 switches it off)."""
        _check(lib().lskum_batch_set_cfl_control(self.h, int(window), float(factor),
                                                 float(cfl_min)))

    def solve(self):
        """Returns (list of Report dicts, total seconds)."""
        reps = (Report * self.n_cond)()
        tot = C.c_double()
        code = lib().lskum_batch_solve(self.h, reps, C.byref(tot))
        if code not in (OK, ERR_NOT_CONVERGED, ERR_NONPHYSICAL):
            _check(code)
        return [r.as_dict() for r in reps], tot.value

    def step_timed(self) -> dict:
        ms = np.zeros(6)
        _check(lib().lskum_batch_step_timed(self.h, _ptr(ms)))
        return dict(zip(State.PHASES, ms.tolist()))

    def get_U(self, k: int) -> np.ndarray:
        out = np.empty((4, self.sizes[k]))
        _check(lib().lskum_batch_get_U(self.h, int(k), _ptr(out), 0))
        return out

    def set_U(self, k: int, U: np.ndarray):
        U = np.ascontiguousarray(U, np.float64)
        assert U.shape == (4, self.sizes[k])
        _check(lib().lskum_batch_set_U(self.h, int(k), _ptr(U), 0))

    def autotune(self, iters: int = 3):
        """Times the lane counts and the q-derivative kernel form and keeps the
        fastest; returns (sweep_lanes, residual_lanes, qgrad_lanes)."""
        sl, rl, ql = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().lskum_batch_autotune(self.h, int(iters), C.byref(sl), C.byref(rl),
                                          C.byref(ql)))
        self.params.sweep_lanes, self.params.residual_lanes = sl.value, rl.value
        self.params.qgrad_lanes = ql.value
        return sl.value, rl.value, ql.value

    def features(self, targets: bool = False):
        """Features [n_points][5] (and targets [n_points][4]) of all conditions."""
        return _features(lib().lskum_batch_features, self.h, self.n_points, targets)


def _features(fn, h, n, targets):
    import torch
    X = torch.empty((n, MLP_FEATURES), dtype=torch.float32, device="cuda")
    T = torch.empty((n, MLP_OUTPUTS), dtype=torch.float32, device="cuda") if targets else None
    torch.cuda.current_stream().synchronize()
    _check(fn(h, X.data_ptr(), None if T is None else T.data_ptr()))
    return (X, T) if targets else X


MLP_PARAMS, MLP_FEATURES, MLP_OUTPUTS = 34308, 5, 4


def _f32_dev(t, cols):
    import torch
    assert t.is_cuda and t.dtype == torch.float32 and t.dim() == 2 and t.shape[1] == cols
    return t.contiguous()


class MLP:
    """Per-point warm-start network (BF16 weights/activations, FP32 accumulate).

    Feature, target and prediction arrays are float32 torch tensors on the
    device, [m][5] and [m][4]; parameters are exchanged as numpy float32.
    """

    def __init__(self, seed: int = 0, max_rows: int = 65536, stream=None):
        handle = None
        if stream is not None:
            handle = stream if isinstance(stream, int) else stream.cuda_stream
        h = C.c_void_p()
        _check(lib().lskum_mlp_create(int(seed) & (2**64 - 1), int(max_rows), handle, C.byref(h)))
        self.h = h
        self.max_rows = int(max_rows)

    def close(self):
        if getattr(self, "h", None):
            lib().lskum_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.empty(MLP_PARAMS, np.float32)
        _check(lib().lskum_mlp_get_params(self.h, _ptr(out), 0))
        return out

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, np.float32)
        assert th.shape == (MLP_PARAMS,)
        _check(lib().lskum_mlp_set_params(self.h, _ptr(th), 0))

    def forward(self, X):
        import torch
        X = _f32_dev(X, MLP_FEATURES)
        Y = torch.empty((X.shape[0], MLP_OUTPUTS), dtype=torch.float32, device=X.device)
        torch.cuda.current_stream().synchronize()
        _check(lib().lskum_mlp_forward(self.h, X.shape[0], X.data_ptr(), Y.data_ptr()))
        return Y

    def gradient(self, X, T):
        """(loss, gradient as numpy float32) without changing the parameters."""
        import torch
        X, T = _f32_dev(X, MLP_FEATURES), _f32_dev(T, MLP_OUTPUTS)
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
        loss = C.c_double()
        torch.cuda.current_stream().synchronize()
        _check(lib().lskum_mlp_gradient(self.h, X.shape[0], X.data_ptr(), T.data_ptr(),
                                        g.data_ptr(), C.byref(loss)))
        return loss.value, g.cpu().numpy()

    def train_step(self, X, T, lr: float) -> float:
        import torch
        X, T = _f32_dev(X, MLP_FEATURES), _f32_dev(T, MLP_OUTPUTS)
        loss = C.c_double()
        torch.cuda.current_stream().synchronize()
        _check(lib().lskum_mlp_train_step(self.h, X.shape[0], X.data_ptr(), T.data_ptr(),
                                          float(lr), C.byref(loss)))
        return loss.value

    def train(self, X, T, steps: int, batch: int, lr: float, lr_final: float = 0.0,
              seed: int = 0):
        """Minibatch Adam; returns (loss history, seconds)."""
        import torch
        X, T = _f32_dev(X, MLP_FEATURES), _f32_dev(T, MLP_OUTPUTS)
        assert X.shape[0] == T.shape[0]
        hist = np.zeros(max(int(steps), 1))
        secs = C.c_double()
        torch.cuda.current_stream().synchronize()
        _check(lib().lskum_mlp_train(self.h, X.shape[0], X.data_ptr(), T.data_ptr(), int(steps),
                                     int(batch), float(lr), float(lr_final),
                                     int(seed) & (2**64 - 1), _ptr(hist), C.byref(secs)))
        return hist[:int(steps)], secs.value

    def warm_start(self, target):
        """Warm-starts a State or Batch; returns (fallback flags, residual norms)."""
        if isinstance(target, Batch):
            k = target.n_cond
            fn = lib().lskum_mlp_warm_start_batch
        else:
            k = 1
            fn = lib().lskum_mlp_warm_start
        fb = np.zeros(k, np.int32)
        res = np.zeros(k)
        _check(fn(self.h, target.h, _ptr(fb), _ptr(res)))
        return fb, res
