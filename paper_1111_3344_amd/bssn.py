"""Python binding of the C ABI in include/bssn.h (argument marshalling only).

Every function here has the name of the C entry point it calls; all GPU work
runs in the HIP library (libbssn_hip.so, built in-tree by build.py).  There
is no fallback: if the library is missing, loading raises.

State buffers are flat torch float64 tensors on the GPU laid out as described
in ``paper_1111_3344_amd.inputs`` (front pad ``grid.off0`` elements, then 25
slots); the pointer handed to the library is the ghost corner of slot 0.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbssn_hip.so")

BSSN_OK, BSSN_EINVAL, BSSN_ENOMEM, BSSN_EHIP, BSSN_ESTALE, \
    BSSN_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
BSSN_FP64, BSSN_MIXED = 0, 1
BSSN_BC_STATIC, BSSN_BC_PERIODIC = 0, 1
BSSN_PATH_AUTO, BSSN_PATH_DIRECT = 0, 1


BSSN_BATCH_PER_PATCH = 0x200


def BSSN_BATCH_TILE(v):
    """batch_patches_plan autotune value forcing tile v for every class."""
    return 0x100 | int(v)


class BssnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class bssn_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("ghost", ctypes.c_int32),
                ("sy", ctypes.c_int64), ("sz", ctypes.c_int64),
                ("sf", ctypes.c_int64), ("origin", ctypes.c_double * 3),
                ("h", ctypes.c_double * 3), ("bc", ctypes.c_int32)]


class bssn_amr_patch(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("grid", bssn_grid)]


class bssn_params(ctypes.Structure):
    _fields_ = [("fd_order", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("ko_eps", ctypes.c_double), ("lapse_f", ctypes.c_double),
                ("shift_G", ctypes.c_double), ("eta", ctypes.c_double),
                ("eta_R", ctypes.c_double), ("lapse_static", ctypes.c_int32),
                ("shift_static", ctypes.c_int32),
                ("fp64_alpha_threshold", ctypes.c_double)]


@dataclasses.dataclass
class Params:
    """bssn_params with the paper's gauge defaults."""
    fd_order: int = 4
    precision: int = BSSN_FP64
    ko_eps: float = 0.1
    lapse_f: float = 2.0
    shift_G: float = 0.75
    eta: float = 0.5
    eta_R: float = 0.0
    lapse_static: int = 0
    shift_static: int = 0
    fp64_alpha_threshold: float = 0.3

    def c(self):
        p = bssn_params()
        for f in dataclasses.fields(self):
            setattr(p, f.name, getattr(self, f.name))
        return p


_lib = None


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "paper_1111_3344_amd.build.build() (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        g, p = P(bssn_grid), P(bssn_params)
        L.bssn_abi_version.restype = ctypes.c_int
        L.bssn_last_error.restype = ctypes.c_char_p
        L.bssn_set_path.argtypes = [ctypes.c_int]
        L.bssn_rhs.argtypes = [g, p, vp, vp, vp]
        L.rk4_stage.argtypes = [g, p, ctypes.c_int, ctypes.c_double, vp, vp,
                                vp, vp, vp]
        L.bssn_constraints.argtypes = [g, p, vp, vp, vp, vp,
                                       P(ctypes.c_double), ctypes.c_int,
                                       ctypes.c_double, vp, vp]
        L.bssn_constraints_noalloc.argtypes = [g, p, vp, vp, vp, vp,
                                       P(ctypes.c_double), ctypes.c_int,
                                       ctypes.c_double, vp, vp]
        L.bssn_mixed_tile_count.argtypes = [g, p, vp, P(ctypes.c_int64),
                                            P(ctypes.c_int64), vp]
        L.bssn_from_adm.argtypes = [g, p, vp, vp, vp]
        L.bssn_track_punctures.argtypes = [g, vp, ctypes.c_int, vp,
                                           ctypes.c_double, vp]
        L.bssn_amr_plan_create.argtypes = [P(bssn_amr_patch), ctypes.c_int,
                                           P(vp)]
        L.bssn_amr_plan_counts.argtypes = [vp, ctypes.c_int,
                                           P(ctypes.c_int64)]
        L.bssn_amr_fill_ghosts.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int,
                                           P(vp), P(ctypes.c_double),
                                           ctypes.c_double, vp]
        L.bssn_amr_restrict.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        L.bssn_amr_plan_destroy.argtypes = [vp]
        L.bssn_multipole.argtypes = [g, vp, vp, P(ctypes.c_double),
                                     ctypes.c_double, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     vp, vp, vp]
        L.rk4_stage_radiative.argtypes = [
            g, p, ctypes.c_int, ctypes.c_double, P(ctypes.c_double),
            P(ctypes.c_double), ctypes.c_int, vp, vp, vp, vp, vp, vp]
        L.bssn_psi4.argtypes = [g, ctypes.c_int, vp, P(ctypes.c_double),
                                vp, vp]
        L.bssn_radiative_rhs.argtypes = [g, P(ctypes.c_double),
                                         P(ctypes.c_double), ctypes.c_int,
                                         vp, vp, vp]
        if hasattr(L, "batch_patches_plan"):
            L.batch_patches_plan.argtypes = [
                ctypes.c_int, P(bssn_grid), p, P(vp), P(vp), P(vp), P(vp),
                P(ctypes.c_double), ctypes.c_int, P(vp), vp]
            L.batch_patches_plan_out.argtypes = [
                ctypes.c_int, P(bssn_grid), p, P(vp), P(vp), P(vp), P(vp),
                P(vp), P(ctypes.c_double), ctypes.c_int, P(vp), vp]
            L.batch_patches_stage.argtypes = [vp, ctypes.c_int, vp]
            L.batch_patches.argtypes = [vp, ctypes.c_int, vp]
            L.batch_patches_unbatched.argtypes = [vp, ctypes.c_int, vp]
            L.batch_patches_describe.argtypes = [vp, ctypes.c_int,
                                                 P(ctypes.c_int32)]
            L.batch_patches_destroy.argtypes = [vp]
            L.batch_patches_launch_mode.argtypes = [vp]
        _lib = L
    return _lib


def c_grid(grid):
    """bssn_grid from a GridSpec-like object."""
    s = bssn_grid()
    s.n[:] = list(grid.n)
    s.ghost = grid.ghost
    s.sy, s.sz, s.sf = grid.sy, grid.sz, grid.sf
    s.origin[:] = list(grid.origin)
    s.h[:] = list(grid.h)
    s.bc = grid.bc
    return s


def _params(prm):
    if prm is None:
        prm = Params()
    if isinstance(prm, dict):
        prm = Params(**prm)
    return prm.c()


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def ptr(grid, t, nslot=25):
    """Device address of the ghost corner of slot 0 of flat tensor t (or of
    a raw device address t that holds such a flat buffer).  A tensor must be
    a contiguous float64 device tensor holding at least off0 + nslot * sf
    elements (nslot: the slots the call reads or writes), since the kernels
    address every slot from this one pointer."""
    if t is None:
        return None
    if isinstance(t, int):
        return ctypes.c_void_p(t + 8 * grid.off0)
    if t.dtype.itemsize != 8 or not t.dtype.is_floating_point:
        raise TypeError("state buffers are float64")
    if not t.is_cuda:
        raise TypeError("state buffers are device tensors")
    if not t.is_contiguous():
        raise TypeError("state buffers are contiguous")
    need = grid.off0 + nslot * grid.sf
    if t.numel() < need:
        raise ValueError(f"buffer of {t.numel()} elements is shorter than "
                         f"the {need} that {nslot} slots of this grid need")
    return ctypes.c_void_p(t.data_ptr() + 8 * grid.off0)


def _check(rc):
    if rc != BSSN_OK:
        raise BssnError(rc, bssn_last_error())


def bssn_abi_version():
    return lib().bssn_abi_version()


def bssn_set_path(path):
    _check(lib().bssn_set_path(int(path)))


def bssn_last_error():
    return lib().bssn_last_error().decode()


def bssn_rhs(grid, params, u, rhs, stream=None):
    _check(lib().bssn_rhs(ctypes.byref(c_grid(grid)),
                          ctypes.byref(_params(params)), ptr(grid, u),
                          ptr(grid, rhs), _stream(stream)))


def rk4_stage(grid, params, stage, dt, u_n, u_s, acc, u_out, stream=None):
    _check(lib().rk4_stage(ctypes.byref(c_grid(grid)),
                           ctypes.byref(_params(params)), int(stage),
                           float(dt), ptr(grid, u_n), ptr(grid, u_s),
                           ptr(grid, acc), ptr(grid, u_out), _stream(stream)))


def rk4_step(grid, params, dt, u, a, b, acc, stream=None):
    """One classical RK4 step in place on u (four rk4_stage calls)."""
    rk4_stage(grid, params, 0, dt, u, u, acc, a, stream)
    rk4_stage(grid, params, 1, dt, u, a, acc, b, stream)
    rk4_stage(grid, params, 2, dt, u, b, acc, a, stream)
    rk4_stage(grid, params, 3, dt, u, a, acc, u, stream)


def bssn_constraints(grid, params, u, norms, H=None, M=None, G=None,
                     centres=(), r_exc=0.0, stream=None):
    """norms: device float64 tensor of >= 8 elements; H/M/G: flat state-shaped
    tensors (their slots 0, 0..2, 0..2 receive the fields) or None."""
    flat = [float(v) for c in centres for v in c]
    arr = (ctypes.c_double * max(1, len(flat)))(*flat)
    _check(lib().bssn_constraints(
        ctypes.byref(c_grid(grid)), ctypes.byref(_params(params)),
        ptr(grid, u), ptr(grid, H, 1), ptr(grid, M, 3), ptr(grid, G, 3),
        arr,
        len(flat) // 3, float(r_exc), ctypes.c_void_p(norms.data_ptr()),
        _stream(stream)))


def bssn_constraints_noalloc(grid, params, u, norms, H=None, M=None, G=None,
                             centres=(), r_exc=0.0, stream=None):
    """bssn_constraints without device allocation (the library's fixed
    partials array; grids of at most 262,144 constraint blocks)."""
    flat = [float(v) for c in centres for v in c]
    arr = (ctypes.c_double * max(1, len(flat)))(*flat)
    _check(lib().bssn_constraints_noalloc(
        ctypes.byref(c_grid(grid)), ctypes.byref(_params(params)),
        ptr(grid, u), ptr(grid, H, 1), ptr(grid, M, 3), ptr(grid, G, 3),
        arr, len(flat) // 3, float(r_exc), ctypes.c_void_p(norms.data_ptr()),
        _stream(stream)))


def bssn_mixed_tile_count(grid, params, u, stream=None):
    a, b = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().bssn_mixed_tile_count(
        ctypes.byref(c_grid(grid)), ctypes.byref(_params(params)),
        ptr(grid, u), ctypes.byref(a), ctypes.byref(b), _stream(stream)))
    return a.value, b.value


def bssn_from_adm(grid, params, adm, u, stream=None):
    """BSSN state u (flat state-shaped tensor) from the ADM variables adm
    (flat tensor of off0 + 16 sf elements: g_ij, K_ij, alpha, beta^i)."""
    _check(lib().bssn_from_adm(ctypes.byref(c_grid(grid)),
                               ctypes.byref(_params(params)), ptr(grid, adm, 16),
                               ptr(grid, u), _stream(stream)))


def bssn_track_punctures(grid, u, pos, dt, stream=None):
    """One Euler step of dx/dt = -beta(x) for the punctures in pos (device
    float64 tensor of shape (n, 3), updated in place)."""
    if pos.dtype.itemsize != 8 or pos.numel() % 3 or not pos.is_contiguous():
        raise TypeError("pos must be a contiguous float64 (n, 3) tensor")
    _check(lib().bssn_track_punctures(
        ctypes.byref(c_grid(grid)), ptr(grid, u), pos.numel() // 3,
        ctypes.c_void_p(pos.data_ptr()), float(dt), _stream(stream)))


def bssn_multipole(grid, re, im, centre, radius, spin, lmax, ntheta, nphi,
                   re_slot=0, im_slot=0, stream=None):
    """C^{lm} (complex numpy array indexed l*l + l + m) of the field whose
    real part is slot re_slot of flat tensor re (im likewise; im may be
    None) on the sphere of the given radius around centre."""
    import numpy as np
    import torch
    for t in (re, im):
        if t is not None and (t.dtype.itemsize != 8 or not t.is_cuda):
            raise TypeError("fields are float64 device tensors")
    chunks = min(64, (ntheta * nphi + 255) // 256)
    work = torch.empty(2 * ntheta * (nphi + 1) + 2 * (lmax + 1) ** 2 * chunks,
                       dtype=torch.float64, device=re.device)
    coeffs = torch.empty(2 * (lmax + 1) ** 2, dtype=torch.float64,
                         device=re.device)
    c = (ctypes.c_double * 3)(*[float(x) for x in centre])
    rp = ctypes.c_void_p(ptr(grid, re, re_slot + 1).value +
                         8 * re_slot * grid.sf)
    ip = (None if im is None else
          ctypes.c_void_p(ptr(grid, im, im_slot + 1).value +
                          8 * im_slot * grid.sf))
    _check(lib().bssn_multipole(ctypes.byref(c_grid(grid)), rp, ip, c,
                                float(radius), int(spin), int(lmax),
                                int(ntheta), int(nphi),
                                ctypes.c_void_p(work.data_ptr()),
                                ctypes.c_void_p(coeffs.data_ptr()),
                                _stream(stream)))
    out = coeffs.cpu().numpy()
    return out[0::2] + 1j * out[1::2]


# Values at infinity and wave speeds of the radiative boundary, per slot:
# the flat-space values (1 for the diagonal conformal metric and the lapse,
# 0 otherwise); speed 1, and sqrt(2) for the lapse and K, which the 1+log
# condition propagates at sqrt(f alpha) = sqrt(2) near alpha = 1.
RADIATIVE_X0 = tuple(1.0 if s in (1, 4, 6, 17) else 0.0 for s in range(25))
RADIATIVE_V0 = tuple(2.0 ** 0.5 if s in (7, 17) else 1.0 for s in range(25))


def rk4_stage_radiative(grid, params, stage, dt, u_n, u_s, acc, u_out, k,
                        x0=None, v0=None, power=2, stream=None):
    """One RK4 stage with the radiative outer boundary evolved (k: a state-
    sized work buffer)."""
    x0 = RADIATIVE_X0 if x0 is None else x0
    v0 = RADIATIVE_V0 if v0 is None else v0
    cx = (ctypes.c_double * 25)(*[float(v) for v in x0])
    cv = (ctypes.c_double * 25)(*[float(v) for v in v0])
    _check(lib().rk4_stage_radiative(
        ctypes.byref(c_grid(grid)), ctypes.byref(_params(params)), int(stage),
        float(dt), cx, cv, int(power), ptr(grid, u_n), ptr(grid, u_s),
        ptr(grid, acc), ptr(grid, u_out), ptr(grid, k), _stream(stream)))


def rk4_step_radiative(grid, params, dt, u, a, b, acc, k, x0=None, v0=None,
                       power=2, stream=None):
    """One RK4 step of state u (in place) with the radiative boundary; a, b,
    acc, k are state-sized work buffers."""
    for s, (us, uo) in enumerate(((u, a), (a, b), (b, a), (a, u))):
        rk4_stage_radiative(grid, params, s, dt, u, us, acc, uo, k, x0, v0,
                            power, stream)


def bssn_psi4(grid, fd_order, u, out, centre=(0.0, 0.0, 0.0), stream=None):
    """Psi_4 of state u at the interior points: Re in slot 0 and Im in slot 1
    of out (a flat float64 device tensor of at least off0 + 2 sf elements,
    grid layout)."""
    c = (ctypes.c_double * 3)(*[float(v) for v in centre])
    _check(lib().bssn_psi4(ctypes.byref(c_grid(grid)), int(fd_order),
                           ptr(grid, u), c, ptr(grid, out, nslot=2),
                           _stream(stream)))


def bssn_radiative_rhs(grid, u, rhs, x0=RADIATIVE_X0, v0=RADIATIVE_V0,
                       power=2, stream=None):
    """Radiative outer boundary: fills the ghost layers of rhs (flat
    state-shaped tensor whose interior holds the interior right-hand side)
    from the state u."""
    a = (ctypes.c_double * 25)(*[float(v) for v in x0])
    b = (ctypes.c_double * 25)(*[float(v) for v in v0])
    _check(lib().bssn_radiative_rhs(ctypes.byref(c_grid(grid)), a, b,
                                    int(power), ptr(grid, u), ptr(grid, rhs),
                                    _stream(stream)))


class BatchPlan:
    """Owner of a bssn_batch_plan*; the buffers must outlive it."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep

    def __del__(self):
        self.destroy()

    def destroy(self):
        if getattr(self, "handle", None):
            lib().batch_patches_destroy(self.handle)
            self.handle = None


def batch_patches_plan(grids, params, u, a, b, acc, dt, autotune=True,
                       stream=None, u_new=None):
    """A batch plan; with u_new (one buffer per patch) its steps write
    u_{n+1} there (batch_patches_plan_out) instead of into u."""
    n = len(grids)
    G = (bssn_grid * n)(*[c_grid(g) for g in grids])
    arrs = []
    for bufs in (u, a, b, acc) + ((u_new,) if u_new is not None else ()):
        arrs.append((ctypes.c_void_p * n)(*[ptr(g, t) for g, t in
                                             zip(grids, bufs)]))
    # dt: one value for every patch, or one per patch
    dts = ([float(dt)] * n if isinstance(dt, (int, float)) else
           [float(x) for x in dt])
    if len(dts) != n:
        raise ValueError(f"{len(dts)} time steps for {n} patches")
    dta = (ctypes.c_double * n)(*dts)
    h = ctypes.c_void_p()
    if u_new is None:
        _check(lib().batch_patches_plan(n, G, ctypes.byref(_params(params)),
                                        arrs[0], arrs[1], arrs[2], arrs[3],
                                        dta, int(autotune),
                                        ctypes.byref(h), _stream(stream)))
        return BatchPlan(h, (u, a, b, acc))
    _check(lib().batch_patches_plan_out(n, G, ctypes.byref(_params(params)),
                                        arrs[0], arrs[4], arrs[1], arrs[2],
                                        arrs[3], dta, int(autotune),
                                        ctypes.byref(h), _stream(stream)))
    return BatchPlan(h, (u, a, b, acc, u_new))


def batch_patches_stage(plan, stage, stream=None):
    _check(lib().batch_patches_stage(plan.handle, int(stage),
                                     _stream(stream)))


def batch_patches(plan, nsteps, stream=None):
    _check(lib().batch_patches(plan.handle, int(nsteps), _stream(stream)))


def batch_patches_unbatched(plan, nsteps, stream=None):
    _check(lib().batch_patches_unbatched(plan.handle, int(nsteps),
                                         _stream(stream)))


def batch_patches_describe(plan, max_classes=64):
    """[(class extent, tile_x, tile_y, z-block depth), ...]"""
    out = (ctypes.c_int32 * (4 * max_classes))()
    n = lib().batch_patches_describe(plan.handle, max_classes, out)
    if n < 0:
        raise BssnError(n, bssn_last_error())
    return [tuple(out[4 * i:4 * i + 4]) for i in range(min(n, max_classes))]


def batch_patches_launch_mode(plan):
    m = lib().batch_patches_launch_mode(plan.handle)
    if m < 0:
        raise BssnError(m, bssn_last_error())
    return m


def batch_patches_destroy(plan):
    plan.destroy()


# ---- device buffers -------------------------------------------------------
class AmrPlan:
    """Glue plan of a refinement hierarchy: hier is a list of (level, grid)
    pairs; state lists below are indexed like hier (None where a call does
    not read the entry)."""

    def __init__(self, hier):
        import torch
        self.hier = list(hier)
        arr = (bssn_amr_patch * len(self.hier))()
        for i, (lv, g) in enumerate(self.hier):
            arr[i].level = lv
            arr[i].grid = c_grid(g)
        h = ctypes.c_void_p()
        _check(lib().bssn_amr_plan_create(arr, len(self.hier),
                                          ctypes.byref(h)))
        self.h = h
        self._torch = torch
        # device pointer tables, one per distinct tuple of pointers: a
        # stepping driver rotates a few buffers, so the tables are built
        # once (a table is never freed while the plan lives, so a launch
        # still queued keeps a valid one)
        self._tables = {}

    def _table(self, states):
        vals = tuple(0 if t is None else ptr(g, t).value
                     for (lv, g), t in zip(self.hier, states))
        tab = self._tables.get(vals)
        if tab is None:
            if len(self._tables) >= 4096:
                raise RuntimeError("more than 4096 distinct state sets")
            tab = self._torch.tensor(list(vals), dtype=self._torch.int64,
                                     device="cuda")
            self._tables[vals] = tab
        return ctypes.c_void_p(tab.data_ptr())

    def counts(self, level):
        c = (ctypes.c_int64 * 3)()
        _check(lib().bssn_amr_plan_counts(self.h, int(level), c))
        return tuple(c)

    def fill_ghosts(self, level, states, coarse_levels, t_src, t,
                    stream=None):
        ut = self._table(states)
        tabs = (ctypes.c_void_p * len(coarse_levels))(
            *[self._table(c).value for c in coarse_levels])
        ts = (ctypes.c_double * len(t_src))(*[float(x) for x in t_src])
        _check(lib().bssn_amr_fill_ghosts(self.h, int(level), ut,
                                          len(coarse_levels), tabs, ts,
                                          float(t), _stream(stream)))

    def restrict(self, level, fine_states, coarse_states, stream=None):
        _check(lib().bssn_amr_restrict(self.h, int(level),
                                       self._table(fine_states),
                                       self._table(coarse_states),
                                       _stream(stream)))

    def destroy(self):
        if self.h:
            lib().bssn_amr_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def to_device(flat, device="cuda"):
    import torch
    return torch.from_numpy(flat).to(device)


def empty_state(grid, device="cuda"):
    import torch
    return torch.zeros(grid.total, dtype=torch.float64, device=device)
