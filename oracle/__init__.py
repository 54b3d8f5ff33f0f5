"""CPU oracle of the implicit LSKUM iteration (test infrastructure).

A ctypes binding of ``lskum_oracle.cpp``: the serial FP64 reference that the
HIP library is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the library never does.
It shares no code with the HIP path (inputs come from the seeded generator in
``paper_2406_07441_amd.cloudgen``, which holds no arithmetic of the method).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lskum_oracle.cpp")
_LIB = os.path.join(_HERE, "liblskum_oracle.so")

GAMMA = 1.4
OK, ERR_ARG, ERR_CONN, ERR_DEGEN, ERR_COLOUR, ERR_NONPHYS = 0, -1, -2, -3, -4, -5


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no fused multiply-add, no fast math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c++17",
               "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Cloud(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("tx", C.c_void_p),
                ("ty", C.c_void_p), ("type", C.c_void_p), ("off", C.c_void_p),
                ("idx", C.c_void_p), ("colour", C.c_void_p), ("ncolour", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("cfl", C.c_double), ("mach", C.c_double),
                ("aoa_deg", C.c_double), ("inner_iters", C.c_int32), ("jvp_mode", C.c_int32),
                ("limiter", C.c_int32), ("variant", C.c_int32), ("limiter_k", C.c_double),
                ("order", C.c_int32), ("farfield", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P, D, I32, I64 = C.c_void_p, C.c_double, C.c_int32, C.c_int64
        sig = {
            "ora_colour": (I32, [I64, P, P, P]),
            "ora_split_flux": (None, [P, D, D, I32, D, P]),
            "ora_flux_jvp": (None, [P, P, D, D, I32, P, P]),
            "ora_q_from_U": (None, [I64, P, D, P]),
            "ora_U_from_q": (None, [I64, P, D, P]),
            "ora_split_weights": (I32, [P, I64, I32, I32, P, P, P, I32]),
            "ora_split_dirs": (I32, [P, I64, P, I32]),
            "ora_free_stream": (None, [P, P, P]),
            "ora_q_grad_pass": (I32, [P, P, P, P, P, P]),
            "ora_q_derivatives": (I32, [P, P, P, P, P]),
            "ora_residual": (I32, [P, P, P, P, P, P]),
            "ora_flux_residual": (I32, [P, P, P, P, P, P]),
            "ora_limit_gradients": (None, [P, P, P, P, P]),
            "ora_timestep_diag": (None, [P, P, P, P, P]),
            "ora_lusgs": (None, [P, P, P, P, P, P]),
            "ora_residual_norm": (D, [P, P]),
            "ora_iteration": (I32, [P, P, P, P, P, P]),
            "ora_unsplit_jvp": (None, [P, P, D, D, P, P]),
            "ora_explicit_iteration": (I32, [P, P, P, P, P]),
            "ora_manish_source": (None, [P, P, P, P, P]),
            "ora_solve": (I32, [P, P, P, I32, D, P]),
            "ora_forces": (I32, [P, P, P, P, P]),
            "ora_set_threads": (None, [I32]),
            "ora_threads": (I32, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    """Threads of the oracle's per-point loops (results do not depend on it)."""
    lib().ora_set_threads(int(n))


def threads() -> int:
    return int(lib().ora_threads())


def colour(cloud) -> tuple[np.ndarray, int]:
    """Algorithm 4 colouring: (0-based colours, number of colours)."""
    col = np.empty(cloud.n, dtype=np.int32)
    nc = lib().ora_colour(cloud.n, _p(cloud.nbr_off), _p(cloud.nbr_idx), _p(col))
    return col, int(nc)


def split_flux(U, d, s, gamma=GAMMA):
    U = _f64(U)
    G = np.empty(4)
    lib().ora_split_flux(_p(U), float(d[0]), float(d[1]), int(s), gamma, _p(G))
    return G


ANANDH, MANISH = 0, 1
COLOUR_ORDER, WALL_FIRST = 0, 1


DIRICHLET, KINETIC = 0, 1


def params(mach=0.63, aoa_deg=2.0, cfl=100.0, inner_iters=1, jvp_mode=0, gamma=GAMMA, limiter=0,
           limiter_k=5.0, variant=ANANDH, order=COLOUR_ORDER, farfield=DIRICHLET):
    return _Params(gamma, cfl, mach, aoa_deg, inner_iters, jvp_mode, limiter, variant, limiter_k,
                   order, farfield)


def unsplit_jvp(U, dU, d, jvp_mode=0, gamma=GAMMA):
    """Unsplit Euler flux Jacobian product A_d(U) dU (exact or flux difference)."""
    J = np.empty(4)
    prm = params(jvp_mode=jvp_mode, gamma=gamma)
    lib().ora_unsplit_jvp(_p(_f64(U)), _p(_f64(dU)), float(d[0]), float(d[1]), C.byref(prm),
                          _p(J))
    return J


def flux_jvp(U, dU, d, s, jvp_mode=0, gamma=GAMMA):
    U, dU = _f64(U), _f64(dU)
    J = np.empty(4)
    prm = params(jvp_mode=jvp_mode, gamma=gamma)
    lib().ora_flux_jvp(_p(U), _p(dU), float(d[0]), float(d[1]), int(s), C.byref(prm), _p(J))
    return J


def q_from_U(U, gamma=GAMMA):
    U = _f64(U)
    n = U.shape[-1]
    q = np.empty((4, n))
    lib().ora_q_from_U(n, _p(U), gamma, _p(q))
    return q


def U_from_q(q, gamma=GAMMA):
    q = _f64(q)
    n = q.shape[-1]
    U = np.empty((4, n))
    lib().ora_U_from_q(n, _p(q), gamma, _p(U))
    return U


class Oracle:
    """Oracle bound to one cloud and one flow condition."""

    def __init__(self, cloud, mach=0.63, aoa_deg=2.0, cfl=100.0, inner_iters=1, jvp_mode=0,
                 gamma=GAMMA, colours=None, limiter=0, limiter_k=5.0, variant=ANANDH,
                 order=COLOUR_ORDER, farfield=DIRICHLET):
        self.cloud = cloud
        self._keep = [_f64(cloud.x), _f64(cloud.y), _f64(cloud.tx), _f64(cloud.ty),
                      np.ascontiguousarray(cloud.type, dtype=np.int8),
                      np.ascontiguousarray(cloud.nbr_off, dtype=np.int32),
                      np.ascontiguousarray(cloud.nbr_idx, dtype=np.int32)]
        if colours is None:
            col, nc = colour(cloud)
        else:
            col = np.ascontiguousarray(colours, dtype=np.int32)
            nc = int(col.max()) + 1
        self.colours, self.ncolour = col, nc
        k = self._keep
        self.c = _Cloud(cloud.n, _p(k[0]), _p(k[1]), _p(k[2]), _p(k[3]), _p(k[4]), _p(k[5]),
                        _p(k[6]), _p(col), nc)
        self.prm = params(mach, aoa_deg, cfl, inner_iters, jvp_mode, gamma, limiter, limiter_k,
                          variant, order, farfield)
        self.n = cloud.n

    # -- state -------------------------------------------------------------
    def free_stream(self):
        U = np.empty((4, self.n))
        lib().ora_free_stream(C.byref(self.c), C.byref(self.prm), _p(U))
        return U

    # -- steps ---------------------------------------------------------------
    def q_grad_pass(self, q, qx_in=None, qy_in=None):
        q = _f64(q)
        qx, qy = np.empty((4, self.n)), np.empty((4, self.n))
        st = lib().ora_q_grad_pass(C.byref(self.c), _p(q), _p(None if qx_in is None else _f64(qx_in)),
                                   _p(None if qy_in is None else _f64(qy_in)), _p(qx), _p(qy))
        if st:
            raise RuntimeError(f"q_grad_pass status {st}")
        return qx, qy

    def q_derivatives(self, q):
        q = _f64(q)
        qx, qy = np.empty((4, self.n)), np.empty((4, self.n))
        st = lib().ora_q_derivatives(C.byref(self.c), C.byref(self.prm), _p(q), _p(qx), _p(qy))
        if st:
            raise RuntimeError(f"q_derivatives status {st}")
        return qx, qy

    def residual(self, U, check=True):
        U = _f64(U)
        R = np.empty((4, self.n))
        res = C.c_double(0.0)
        ndeg = C.c_int64(0)
        st = lib().ora_residual(C.byref(self.c), C.byref(self.prm), _p(U), _p(R), C.byref(res),
                                C.byref(ndeg))
        if check and st:
            raise RuntimeError(f"residual status {st}")
        self.degenerate = int(ndeg.value)
        return R, float(res.value)

    def limit_gradients(self, q, qx, qy):
        qx, qy = _f64(qx).copy(), _f64(qy).copy()
        lib().ora_limit_gradients(C.byref(self.c), C.byref(self.prm), _p(_f64(q)), _p(qx), _p(qy))
        return qx, qy

    def flux_residual(self, q, qx, qy):
        R = np.empty((4, self.n))
        st = lib().ora_flux_residual(C.byref(self.c), C.byref(self.prm), _p(_f64(q)), _p(_f64(qx)),
                                     _p(_f64(qy)), _p(R))
        if st:
            raise RuntimeError(f"flux_residual status {st}")
        return R

    def timestep_diag(self, U):
        dt, D = np.empty(self.n), np.empty(self.n)
        lib().ora_timestep_diag(C.byref(self.c), C.byref(self.prm), _p(_f64(U)), _p(dt), _p(D))
        return dt, D

    def lusgs(self, U, R, D):
        dU = np.empty((4, self.n))
        lib().ora_lusgs(C.byref(self.c), C.byref(self.prm), _p(_f64(U)), _p(_f64(R)), _p(_f64(D)),
                        _p(dU))
        return dU

    def residual_norm(self, R):
        return float(lib().ora_residual_norm(C.byref(self.c), _p(_f64(R))))

    def manish_source(self, U, dU_prev):
        S = np.empty((4, self.n))
        lib().ora_manish_source(C.byref(self.c), C.byref(self.prm), _p(_f64(U)),
                                _p(None if dU_prev is None else _f64(dU_prev)), _p(S))
        return S

    def iteration(self, U, dU_prev=None):
        """One iteration; returns (U_new, R, dU, res).  dU_prev: the previous
        iteration's increment (Manish variant; None = zero)."""
        U = _f64(U).copy()
        R = np.empty((4, self.n))
        dU = np.zeros((4, self.n)) if dU_prev is None else _f64(dU_prev).copy()
        res = C.c_double(0.0)
        st = lib().ora_iteration(C.byref(self.c), C.byref(self.prm), _p(U), _p(R), _p(dU),
                                 C.byref(res))
        if st:
            raise RuntimeError(f"iteration status {st}")
        return U, R, dU, float(res.value)

    def explicit_iteration(self, U):
        """One explicit iteration U - dt R; returns (U_new, R, res)."""
        U = _f64(U).copy()
        R = np.empty((4, self.n))
        res = C.c_double(0.0)
        st = lib().ora_explicit_iteration(C.byref(self.c), C.byref(self.prm), _p(U), _p(R),
                                          C.byref(res))
        if st:
            raise RuntimeError(f"explicit iteration status {st}")
        return U, R, float(res.value)

    def solve(self, U, max_iters, tol_abs=0.0):
        """Iterate in place; returns (U, iterations, residual history)."""
        U = _f64(U).copy()
        hist = np.zeros(max_iters)
        it = lib().ora_solve(C.byref(self.c), C.byref(self.prm), _p(U), int(max_iters),
                             float(tol_abs), _p(hist))
        if it < 0:
            raise RuntimeError(f"solve status {it}")
        return U, int(it), hist[:it]

    def forces(self, U):
        cl, cd = C.c_double(0.0), C.c_double(0.0)
        st = lib().ora_forces(C.byref(self.c), C.byref(self.prm), _p(_f64(U)), C.byref(cl),
                              C.byref(cd))
        if st:
            raise RuntimeError(f"forces status {st}")
        return float(cl.value), float(cd.value)

    def split_stencil(self, p, k, cap=64):
        nb = np.empty(cap, dtype=np.int32)
        w = np.empty(cap)
        ls1 = C.c_double(0.0)
        m = lib().ora_split_weights(C.byref(self.c), int(p), int(k), cap, _p(nb), _p(w),
                                    C.byref(ls1), int(self.prm.farfield))
        if m < 0:
            raise IndexError("no such split")
        if m > cap:
            raise ValueError(f"split stencil of point {p} has {m} members, more than cap={cap}")
        return nb[:m].copy(), w[:m].copy(), float(ls1.value)

    def split_dirs(self, p):
        out = np.empty(12)
        ns = lib().ora_split_dirs(C.byref(self.c), int(p), _p(out), int(self.prm.farfield))
        return [((out[3 * k], out[3 * k + 1]), int(out[3 * k + 2])) for k in range(ns)]
