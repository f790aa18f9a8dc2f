"""C ABI checks that need no GPU: the library loads, exports every entry
point include/bssn.h declares, and rejects invalid arguments before any HIP
call is made."""
import ctypes
import os
import re

import pytest

from paper_1111_3344_amd import bssn as B
from paper_1111_3344_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bssn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("bssn_rhs", "rk4_stage", "bssn_constraints", "batch_patches",
              "batch_patches_plan", "batch_patches_destroy",
              "bssn_abi_version", "bssn_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = B.lib()
    for n in _declared():
        assert hasattr(L, n), f"{n} declared in bssn.h but not exported"
    assert B.bssn_abi_version() == 2


def _grid(**kw):
    g = I.cell_centred(8, -1, 1, 3)
    return B.c_grid(g), g


P = ctypes.c_void_p


def _stage(grid, prm, stage=0, dt=0.1, un=1, us=1, acc=2, out=3):
    return B.lib().rk4_stage(ctypes.byref(grid), ctypes.byref(prm), stage,
                             dt, P(un), P(us), P(acc), P(out), None)


def test_validation_rejects_before_launch():
    cg, g = _grid()
    prm = B.Params().c()
    # fake non-NULL device addresses: validation must fail before any use
    assert _stage(cg, prm, stage=4) == B.BSSN_EINVAL
    assert "stage" in B.bssn_last_error()
    assert _stage(cg, prm, dt=float("nan")) == B.BSSN_EINVAL
    assert _stage(cg, prm, un=0) == B.BSSN_EINVAL
    assert _stage(cg, prm, out=1, us=1, un=5) == B.BSSN_EINVAL  # u_out == u_s
    assert _stage(cg, prm, acc=1) == B.BSSN_EINVAL             # acc == u_n
    assert _stage(cg, prm, stage=1, out=1, us=7) == B.BSSN_EINVAL
    bad = B.c_grid(g)
    bad.ghost = 2
    assert _stage(bad, prm) == B.BSSN_EINVAL
    assert "ghost" in B.bssn_last_error()
    bad = B.c_grid(g)
    bad.sy = 4
    assert _stage(bad, prm) == B.BSSN_EINVAL
    bad = B.c_grid(g)
    bad.h[1] = 0.0
    assert _stage(bad, prm) == B.BSSN_EINVAL
    bad = B.c_grid(g)
    bad.bc = 7
    assert _stage(bad, prm) == B.BSSN_EINVAL
    p8 = B.Params(fd_order=8).c()
    assert _stage(cg, p8) == B.BSSN_EINVAL          # ghost 3 < 5
    p6 = B.Params(fd_order=6).c()
    assert _stage(cg, p6) == B.BSSN_EINVAL
    pp = B.Params(precision=3).c()
    assert _stage(cg, pp) == B.BSSN_EINVAL
    pk = B.Params(ko_eps=-1.0).c()
    assert _stage(cg, pk) == B.BSSN_EINVAL
    assert B.lib().bssn_rhs(ctypes.byref(cg), ctypes.byref(prm), P(1), P(1),
                            None) == B.BSSN_EINVAL
    assert B.lib().rk4_stage(None, ctypes.byref(prm), 0, 0.1, P(1), P(1),
                             P(2), P(3), None) == B.BSSN_EINVAL


def test_constraints_validation():
    cg, g = _grid()
    prm = B.Params().c()
    c = (ctypes.c_double * 3)(0, 0, 0)
    L = B.lib()
    assert L.bssn_constraints(ctypes.byref(cg), ctypes.byref(prm), P(1), None,
                              None, None, c, 17, 0.0, P(2),
                              None) == B.BSSN_EINVAL
    assert L.bssn_constraints(ctypes.byref(cg), ctypes.byref(prm), P(1), None,
                              None, None, c, 0, 0.0, None,
                              None) == B.BSSN_EINVAL
    assert L.bssn_constraints(ctypes.byref(cg), ctypes.byref(prm), P(1), P(1),
                              None, None, c, 0, 0.0, P(2),
                              None) == B.BSSN_EINVAL


def test_radiative_validation():
    L = B.lib()
    x0 = (ctypes.c_double * 25)(*([0.0] * 25))
    v0 = (ctypes.c_double * 25)(*([1.0] * 25))

    def call(g, power=2, u=1, rhs=2, a=x0, b=v0):
        return L.bssn_radiative_rhs(ctypes.byref(B.c_grid(g)), a, b, power,
                                    P(u), P(rhs), None)

    g = I.cell_centred(8, -1, 1, 3)
    assert call(g, u=1, rhs=1) == B.BSSN_EINVAL          # rhs == u
    assert call(g, u=0) == B.BSSN_EINVAL
    assert call(g, power=-1) == B.BSSN_EINVAL
    assert call(g, power=17) == B.BSSN_EINVAL
    assert call(g, a=None) == B.BSSN_EINVAL
    bad = (ctypes.c_double * 25)(*([1.0] * 24 + [-1.0]))
    assert call(g, b=bad) == B.BSSN_EINVAL
    assert "slot 24" in B.bssn_last_error()
    nan = (ctypes.c_double * 25)(*([float("nan")] + [0.0] * 24))
    assert call(g, a=nan) == B.BSSN_EINVAL
    gp = I.cell_centred(8, -1, 1, 3, I.BC_PERIODIC)
    assert call(gp) == B.BSSN_EINVAL
    assert "static" in B.bssn_last_error()
    # interior point 0 at (2h, 2h, 2h): the coordinate origin is the ghost
    # point two steps below it on every axis (every case above and this one
    # is rejected before anything is launched)
    h = 0.1
    go = I.GridSpec((6, 6, 6), 3, (h, h, h), (2 * h, 2 * h, 2 * h),
                    I.BC_STATIC)
    assert call(go) == B.BSSN_EINVAL
    assert "origin" in B.bssn_last_error()


def test_from_adm_validation():
    L = B.lib()
    prm = B.Params().c()

    def call(g, prm=prm, adm=1, u=2):
        return L.bssn_from_adm(ctypes.byref(B.c_grid(g)), ctypes.byref(prm),
                               P(adm), P(u), None)

    g = I.cell_centred(8, -1, 1, 3)
    assert call(g, adm=1, u=1) == B.BSSN_EINVAL
    assert call(g, adm=0) == B.BSSN_EINVAL
    assert call(g, prm=B.Params(fd_order=8).c()) == B.BSSN_EINVAL  # ghost 3
    thin = I.GridSpec((8, 3, 8), 3, (0.1,) * 3, (0.0,) * 3, I.BC_STATIC)
    assert call(thin) == B.BSSN_EINVAL
    assert "n[1]" in B.bssn_last_error()


def test_track_punctures_validation():
    L = B.lib()
    g = I.cell_centred(8, -1, 1, 3)

    def call(n=2, u=1, pos=2, dt=0.1):
        return L.bssn_track_punctures(ctypes.byref(B.c_grid(g)), P(u), n,
                                      P(pos), dt, None)

    assert call(n=0) == B.BSSN_EINVAL
    assert call(n=65537) == B.BSSN_EINVAL
    assert call(u=0) == B.BSSN_EINVAL
    assert call(pos=0) == B.BSSN_EINVAL
    assert call(dt=float("nan")) == B.BSSN_EINVAL


def _amr_create(hier):
    arr = (B.bssn_amr_patch * len(hier))()
    for i, (lv, g) in enumerate(hier):
        arr[i].level = lv
        arr[i].grid = B.c_grid(g)
    h = ctypes.c_void_p()
    rc = B.lib().bssn_amr_plan_create(arr, len(hier), ctypes.byref(h))
    return rc, h


def test_amr_plan_validation():
    """Hierarchies the plan must refuse, before it allocates anything."""
    from tests import amr_hier as H
    L = B.lib()
    c = I.GridSpec((12, 12, 12), 3, (0.2,) * 3, (0.0, 0.0, 0.0),
                   I.BC_STATIC)
    f = H.child(c, (3, 3, 3), (8, 8, 8))
    h = ctypes.c_void_p()
    assert L.bssn_amr_plan_create(None, 1, ctypes.byref(h)) == B.BSSN_EINVAL
    assert _amr_create([])[0] == B.BSSN_EINVAL
    # a level without patches
    assert _amr_create([(0, c), (2, f)])[0] == B.BSSN_EINVAL
    # spacing not half of the coarser level's
    bad_h = I.GridSpec(f.n, 3, (0.09,) * 3, f.origin, I.BC_STATIC)
    assert _amr_create([(0, c), (1, bad_h)])[0] == B.BSSN_EINVAL
    # fine points on the coarse points (vertex-style), not a quarter off
    bad_o = I.GridSpec(f.n, 3, f.h, (0.6, 0.6, 0.6), I.BC_STATIC)
    assert _amr_create([(0, c), (1, bad_o)])[0] == B.BSSN_EINVAL
    # a sibling off its level's lattice
    off = H.sibling(f, (0, 0, 0))
    off = I.GridSpec(off.n, 3, off.h, (off.origin[0] + 0.03,) +
                     off.origin[1:], I.BC_STATIC)
    assert _amr_create([(0, c), (1, f), (1, off)])[0] == B.BSSN_EINVAL
    # a fine patch whose ghosts leave the coarse storage
    out = H.child(c, (-3, 0, 0), (8, 8, 8))
    rc, _ = _amr_create([(0, c), (1, out)])
    assert rc == B.BSSN_EINVAL
    assert "ghost point" in B.bssn_last_error()
    # periodic patches are refused
    per = I.GridSpec(c.n, 3, c.h, c.origin, I.BC_PERIODIC)
    assert _amr_create([(0, per)])[0] == B.BSSN_EINVAL
    # calls on a NULL plan
    assert L.bssn_amr_fill_ghosts(None, 1, P(1), 1, None, None, 0.0,
                                  None) == B.BSSN_EINVAL
    assert L.bssn_amr_restrict(None, 1, P(1), P(2), None) == B.BSSN_EINVAL
    assert L.bssn_amr_plan_counts(None, 1, None) == B.BSSN_EINVAL
    assert L.bssn_amr_plan_destroy(None) == B.BSSN_OK


def test_multipole_validation():
    L = B.lib()
    g = I.cell_centred(8, -1, 1, 3)
    c = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    bad_c = (ctypes.c_double * 3)(0.0, float("nan"), 0.0)

    def call(re=1, im=None, cen=c, r=0.5, s=-2, lmax=4, nt=8, nph=16,
             work=2, coeffs=3):
        return L.bssn_multipole(ctypes.byref(B.c_grid(g)), P(re), P(im),
                                cen, r, s, lmax, nt, nph, P(work), P(coeffs),
                                None)

    assert call(re=0) == B.BSSN_EINVAL
    assert call(work=0) == B.BSSN_EINVAL
    assert call(coeffs=0) == B.BSSN_EINVAL
    assert call(cen=bad_c) == B.BSSN_EINVAL
    assert call(r=0.0) == B.BSSN_EINVAL
    assert call(r=float("inf")) == B.BSSN_EINVAL
    assert call(s=9) == B.BSSN_EINVAL
    assert call(lmax=17) == B.BSSN_EINVAL
    assert call(nt=0) == B.BSSN_EINVAL
    assert call(nph=4097) == B.BSSN_EINVAL


def test_rk4_stage_radiative_validation():
    L = B.lib()
    g = I.cell_centred(8, -1, 1, 3)
    prm = B.Params().c()
    x0 = (ctypes.c_double * 25)(*B.RADIATIVE_X0)
    v0 = (ctypes.c_double * 25)(*B.RADIATIVE_V0)
    bad_v = (ctypes.c_double * 25)(*([-1.0] + [1.0] * 24))

    def call(stage=0, dt=0.1, cx=x0, cv=v0, power=2, un=1, us=1, acc=2,
             out=3, k=4, grid=g):
        return L.rk4_stage_radiative(
            ctypes.byref(B.c_grid(grid)), ctypes.byref(prm), stage, dt, cx,
            cv, power, P(un), P(us), P(acc), P(out), P(k), None)

    assert call(stage=4) == B.BSSN_EINVAL
    assert call(dt=float("inf")) == B.BSSN_EINVAL
    assert call(k=0) == B.BSSN_EINVAL
    assert call(k=2) == B.BSSN_EINVAL                 # k aliases acc
    assert call(k=1) == B.BSSN_EINVAL                 # k aliases u_s
    assert call(out=1) == B.BSSN_EINVAL               # u_out aliases u_s
    assert call(acc=1) == B.BSSN_EINVAL
    assert call(cv=bad_v) == B.BSSN_EINVAL
    assert call(cx=None) == B.BSSN_EINVAL
    assert call(power=17) == B.BSSN_EINVAL
    gp = I.cell_centred(8, -1, 1, 3, I.BC_PERIODIC)
    assert call(grid=gp) == B.BSSN_EINVAL
    # the coordinate origin on the outermost interior layer: r = 0 at a root
    go = I.GridSpec((6, 6, 6), 3, (0.5,) * 3, (0.0, -1.0, -1.0), I.BC_STATIC)
    assert call(grid=go) == B.BSSN_EINVAL
    assert "outermost interior layer" in B.bssn_last_error()


def test_batch_stage_and_plan_out_validation():
    L = B.lib()
    g = I.cell_centred(8, -1, 1, 3)
    G = (B.bssn_grid * 1)(B.c_grid(g))
    prm = B.Params().c()
    arr = lambda v: (ctypes.c_void_p * 1)(v)
    dt = (ctypes.c_double * 1)(0.1)
    h = ctypes.c_void_p()
    # u_new aliasing a / acc, or NULL, is rejected before any allocation
    for un in (1 << 20, 3 << 20, None):
        rc = L.batch_patches_plan_out(1, G, ctypes.byref(prm), arr(1 << 20),
                                      None if un is None else arr(un),
                                      arr(2 << 20), arr(4 << 20),
                                      arr(3 << 20), dt, 0, ctypes.byref(h),
                                      None)
        if un == 1 << 20:
            # u_new == u is allowed: fails later, on the fake pointers
            assert rc != B.BSSN_OK
        else:
            assert rc == B.BSSN_EINVAL
    assert L.batch_patches_stage(None, 0, None) == B.BSSN_EINVAL


def test_psi4_validation():
    L = B.lib()
    g = I.cell_centred(8, -1, 1, 3)
    c = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    bad_c = (ctypes.c_double * 3)(0.0, 0.0, float("inf"))
    base = 1 << 30

    def call(order=4, u=base, out=base + 64 * g.sf, cen=c, grid=g):
        return L.bssn_psi4(ctypes.byref(B.c_grid(grid)), order, P(u), cen,
                           P(out), None)

    assert call(order=6) == B.BSSN_EINVAL
    assert call(order=8) == B.BSSN_EINVAL          # ghost 3 < 5
    assert call(u=0) == B.BSSN_EINVAL
    assert call(out=0) == B.BSSN_EINVAL
    assert call(cen=None) == B.BSSN_EINVAL
    assert call(cen=bad_c) == B.BSSN_EINVAL
    # the two output slots may not overlap the 25 state slots
    assert call(out=base + 8 * 24 * g.sf) == B.BSSN_EINVAL
    assert "overlaps" in B.bssn_last_error()
    assert call(out=base - 8 * g.sf) == B.BSSN_EINVAL
    g8 = I.cell_centred(8, -1, 1, 5)
    assert call(order=8, grid=g8, out=0) == B.BSSN_EINVAL  # reaches out=0


def test_periodic_grid_must_cover_stencil():
    g = I.GridSpec((2, 8, 8), 3, (0.1,) * 3, (0,) * 3, I.BC_PERIODIC)
    assert _stage(B.c_grid(g), B.Params().c()) == B.BSSN_EINVAL


def _plan(grids, prm, bufs=None, dt=0.1, autotune=0, out=True):
    n = len(grids)
    G = (B.bssn_grid * max(1, n))(*[B.c_grid(g) for g in grids])
    if bufs is None:
        bufs = [[8 * (4 * p + i + 1) for p in range(n)] for i in range(4)]
    arrs = [(ctypes.c_void_p * max(1, n))(*b) for b in bufs]
    dts = dt if isinstance(dt, (list, tuple)) else [dt] * max(1, n)
    dta = None if dt is None else (ctypes.c_double * len(dts))(*dts)
    h = ctypes.c_void_p()
    return B.lib().batch_patches_plan(n, G, ctypes.byref(prm), *arrs, dta,
                                      autotune,
                                      ctypes.byref(h) if out else None, None)


def L_mode_null():
    return B.lib().batch_patches_launch_mode(None)


def test_batch_plan_validation():
    g = I.cell_centred(8, -1, 1, 3)
    prm = B.Params().c()
    assert _plan([], prm) == B.BSSN_EINVAL
    assert _plan([g], prm, out=False) == B.BSSN_EINVAL
    assert _plan([g], prm, dt=float("inf")) == B.BSSN_EINVAL
    # per-patch time steps: every entry finite and >= 0, the array present
    assert _plan([g], prm, dt=None) == B.BSSN_EINVAL
    assert _plan([g, g], prm, dt=[0.1, float("nan")]) == B.BSSN_EINVAL
    assert "patch 1" in B.bssn_last_error()
    assert _plan([g, g], prm, dt=[-0.05, 0.1]) == B.BSSN_EINVAL
    assert "patch 0" in B.bssn_last_error()
    assert _plan([g], prm, autotune=2) == B.BSSN_EINVAL
    assert _plan([g], prm, autotune=B.BSSN_BATCH_TILE(5)) == B.BSSN_EINVAL
    assert _plan([g], prm, autotune=0x400) == B.BSSN_EINVAL
    assert _plan([g], prm, autotune=0x201) == B.BSSN_EINVAL  # tile w/o 0x100
    assert L_mode_null() == B.BSSN_EINVAL
    gp = I.cell_centred(8, -1, 1, 3, I.BC_PERIODIC)
    assert _plan([g, gp], prm) == B.BSSN_EINVAL
    assert "patch 1" in B.bssn_last_error()
    assert _plan([g], prm, bufs=[[8], [8], [16], [24]]) == B.BSSN_EINVAL
    assert "alias" in B.bssn_last_error()
    assert _plan([g], prm, bufs=[[8], [0], [16], [24]]) == B.BSSN_EINVAL
    assert _plan([g], B.Params(fd_order=8).c()) == B.BSSN_EINVAL
    L = B.lib()
    assert L.batch_patches(None, 1, None) == B.BSSN_EINVAL
    assert L.batch_patches_unbatched(None, 1, None) == B.BSSN_EINVAL
    assert L.batch_patches_describe(None, 0, None) == B.BSSN_EINVAL


def test_constraints_noalloc_rejects_oversize_grid():
    """The allocation-free constraints hold partial norms for at most
    262,144 blocks: a 512^3 grid (8 x 128 x 512 blocks) is rejected on the
    host before anything touches a device (fake device pointers)."""
    g = I.cell_centred(512, -1, 1, 3)
    norms = (ctypes.c_double * 8)()
    rc = B.lib().bssn_constraints_noalloc(
        ctypes.byref(B.c_grid(g)), ctypes.byref(B.Params().c()),
        ctypes.c_void_p(64), None, None, None, None, 0, 0.0,
        ctypes.c_void_p(128), None)
    assert rc == B.BSSN_EINVAL
    assert "262144" in B.bssn_last_error()
    # the shared argument checks still apply
    rc = B.lib().bssn_constraints_noalloc(
        ctypes.byref(B.c_grid(g)), ctypes.byref(B.Params().c()), None, None,
        None, None, None, 0, 0.0, ctypes.c_void_p(128), None)
    assert rc == B.BSSN_EINVAL
