"""ctypes wrapper of the FP64 CPU oracle (oracle/bssn_oracle.c).

Test infrastructure only.  Arrays are numpy float64 buffers in the layout of
the shared input module (flat, front pad included); grids are any object
with n, ghost, sy, sz, sf, off0, total, origin, h, bc attributes.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
NSLOT = 25


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("ghost", ctypes.c_int32),
                ("sy", ctypes.c_int64), ("sz", ctypes.c_int64),
                ("sf", ctypes.c_int64), ("origin", ctypes.c_double * 3),
                ("h", ctypes.c_double * 3), ("bc", ctypes.c_int32)]


class _Params(ctypes.Structure):
    _fields_ = [("fd_order", ctypes.c_int32), ("ko_eps", ctypes.c_double),
                ("lapse_f", ctypes.c_double), ("shift_G", ctypes.c_double),
                ("eta", ctypes.c_double), ("eta_R", ctypes.c_double),
                ("lapse_static", ctypes.c_int32),
                ("shift_static", ctypes.c_int32)]


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        _lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        d = P(ctypes.c_double)
        g, p = P(_Grid), P(_Params)
        _lib.oracle_rhs.argtypes = [g, p, d, d]
        _lib.oracle_rhs_points.argtypes = [g, p, d, ctypes.c_int,
                                           P(ctypes.c_int32), d]
        _lib.oracle_rk4_step.argtypes = [g, p, ctypes.c_double, d, d]
        _lib.oracle_constraints.argtypes = [g, p, d, d, d, d, d, ctypes.c_int,
                                            ctypes.c_double, d]
        _lib.oracle_num_threads.restype = ctypes.c_int
        _lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _lib.oracle_set_num_threads.restype = None
        _lib.oracle_point_ops.argtypes = [g, p, d, ctypes.c_int,
                                          P(ctypes.c_int32), d, d]
    return _lib


def params(fd_order=4, ko_eps=0.1, lapse_f=2.0, shift_G=0.75, eta=0.5,
           eta_R=0.0, lapse_static=0, shift_static=0):
    """Gauge and dissipation parameters (paper defaults: 1+log f = 2/alpha,
    Gamma-driver G = 3/(4 alpha^2), eta = 1/2, q = 1)."""
    return dict(fd_order=fd_order, ko_eps=ko_eps, lapse_f=lapse_f,
                shift_G=shift_G, eta=eta, eta_R=eta_R,
                lapse_static=lapse_static, shift_static=shift_static)


def _g(grid):
    s = _Grid()
    s.n[:] = list(grid.n)
    s.ghost = grid.ghost
    s.sy, s.sz, s.sf = grid.sy, grid.sz, grid.sf
    s.origin[:] = list(grid.origin)
    s.h[:] = list(grid.h)
    s.bc = grid.bc
    return s


def _p(prm):
    s = _Params()
    for k, v in prm.items():
        setattr(s, k, v)
    return s


def _ptr(a, off):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return ctypes.cast(a.ctypes.data + 8 * off, ctypes.POINTER(ctypes.c_double))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


def rhs(grid, prm, u):
    """Right-hand side at every interior point (flat buffer, ghosts 0)."""
    out = np.zeros(grid.total)
    _check(lib().oracle_rhs(_g(grid), _p(prm), _ptr(u, grid.off0),
                            _ptr(out, grid.off0)), "rhs")
    return out


def rhs_points(grid, prm, u, pts):
    """Right-hand side at interior points pts (N x 3 ints) -> (N, 25)."""
    pts = np.ascontiguousarray(pts, dtype=np.int32)
    out = np.zeros((len(pts), NSLOT))
    _check(lib().oracle_rhs_points(
        _g(grid), _p(prm), _ptr(u, grid.off0), len(pts),
        pts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "rhs_points")
    return out


def rk4_step(grid, prm, dt, u):
    """One classical RK4 step; returns the new flat buffer."""
    out = np.zeros(grid.total)
    _check(lib().oracle_rk4_step(_g(grid), _p(prm), dt, _ptr(u, grid.off0),
                                 _ptr(out, grid.off0)), "rk4_step")
    return out


def rk4_steps(grid, prm, dt, u, nsteps):
    for _ in range(nsteps):
        u = rk4_step(grid, prm, dt, u)
    return u


def constraints(grid, prm, u, centres=(), r_exc=0.0):
    """H (1 slot), M (3 slots), G (3 slots) flat buffers and the 8 norms
    (H_rms, H_max, M_rms, M_max, G_rms, G_max, N_used, N_nonfinite)."""
    H = np.zeros(grid.total)
    M = np.zeros(grid.total)
    G = np.zeros(grid.total)
    c = np.ascontiguousarray(np.asarray(centres, dtype=np.float64).reshape(-1))
    if c.size == 0:
        c = np.zeros(3)
        ncent = 0
    else:
        ncent = c.size // 3
    norms = np.zeros(8)
    _check(lib().oracle_constraints(
        _g(grid), _p(prm), _ptr(u, grid.off0), _ptr(H, grid.off0),
        _ptr(M, grid.off0), _ptr(G, grid.off0), _ptr(c, 0), ncent, r_exc,
        _ptr(norms, 0)), "constraints")
    return H, M, G, norms


def point_ops(grid, prm, u, slot, p, beta=(1.0, 1.0, 1.0)):
    """The discrete operators of one slot at one interior point: first
    derivatives (3), second derivatives (3x3), lopsided derivatives for
    the signs of beta (3), Kreiss-Oliger terms (3)."""
    out = np.zeros(18)
    pp = np.ascontiguousarray(p, dtype=np.int32)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    _check(lib().oracle_point_ops(
        _g(grid), _p(prm), _ptr(u, grid.off0), slot,
        pp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(b, 0),
        _ptr(out, 0)), "point_ops")
    return dict(d1=out[0:3], d2=out[3:12].reshape(3, 3), up=out[12:15],
                ko=out[15:18])


def num_threads():
    return lib().oracle_num_threads()


def set_num_threads(n):
    """Threads of the oracle's parallel loops from now on."""
    lib().oracle_set_num_threads(int(n))
