"""HIP path vs the FP64 CPU oracle, through the C ABI (needs an MI355X).

Tolerances (FP64 path):
  * right-hand side: per slot f, max|gpu - oracle| <= 1e-12 * D_f, with D_f
    the largest |oracle| value of slot f (or of all slots when slot f is
    identically zero).  Both sides difference from the centre value, so the
    only disagreement is rounding order (~1e-15 of D_f).
  * RK4 states: the update is u_n + dt * (weighted k), rounded at |u|.  An
    error of 1e-12 D in k moves the state by at most 1e-12 * |u - u_n|, and
    the final roundings add a few ulp of |u|:
        max|gpu - oracle| <= 1e-12 * max|u - u_n| + 8 ulp(max|u|)  per slot
    (per step, summed over steps).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1111_3344_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_3344_amd import bssn
    bssn.lib()
    return bssn


def oparams(p):
    return O.params(fd_order=p.fd_order, ko_eps=p.ko_eps, lapse_f=p.lapse_f,
                    shift_G=p.shift_G, eta=p.eta, eta_R=p.eta_R,
                    lapse_static=p.lapse_static,
                    shift_static=p.shift_static)


def rhs_err(grid, a, b):
    """Per-slot normwise error of flat buffers a (gpu) vs b (oracle)."""
    ai, bi = grid.interior(a), grid.interior(b)
    D = np.abs(bi).reshape(25, -1).max(axis=1)
    Dall = D.max()
    D = np.where(D > 0, D, Dall if Dall > 0 else 1.0)
    return np.abs(ai - bi).reshape(25, -1).max(axis=1) / D


def gpu_rhs(B, grid, prm, u):
    du = B.to_device(u)
    out = torch.zeros_like(du)
    B.bssn_rhs(grid, prm, du, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def gpu_steps(B, grid, prm, dt, u, nsteps):
    du = B.to_device(u)
    a, b, acc = du.clone(), du.clone(), torch.zeros_like(du)
    for _ in range(nsteps):
        B.rk4_step(grid, prm, dt, du, a, b, acc)
    torch.cuda.synchronize()
    return du.cpu().numpy()


def state_tol(grid, u0, u1, nsteps):
    d = np.abs(grid.interior(u1) - grid.interior(u0)).reshape(25, -1).max(1)
    m = np.abs(grid.interior(u1)).reshape(25, -1).max(1)
    return nsteps * (1e-12 * d + 8 * EPS * np.maximum(m, 1e-300))


CASES = {
    # name: (grid, data, params kwargs)
    "noise-periodic-32": (
        lambda: I.cell_centred(32, -1.6, 1.6, 3, I.BC_PERIODIC),
        lambda g: I.minkowski_noise(g), {}),
    "smooth-static-ragged": (
        lambda: I.GridSpec((70, 38, 29), 3, (0.11, 0.13, 0.12),
                           (-3.8, -2.4, -1.7), I.BC_STATIC),
        lambda g: I.smooth_random(g, seed=7), {}),
    "smooth-periodic": (
        lambda: I.GridSpec((20, 24, 18), 3, (0.1, 0.09, 0.12),
                           (0.0, 0.0, 0.0), I.BC_PERIODIC),
        lambda g: I.smooth_random(g, seed=8), {}),
    "smooth-static-qR-gauges": (
        lambda: I.GridSpec((36, 21, 17), 3, (0.1, 0.1, 0.1),
                           (-1.7, -1.0, -0.8), I.BC_STATIC),
        lambda g: I.smooth_random(g, seed=9),
        dict(eta_R=1.2, eta=0.7)),
    "smooth-static-frozen-gauge": (
        lambda: I.GridSpec((33, 19, 13), 3, (0.1, 0.1, 0.1),
                           (-1.7, -1.0, -0.8), I.BC_STATIC),
        lambda g: I.smooth_random(g, seed=10),
        dict(lapse_static=1, shift_static=1)),
    "bl-two-punctures-48": (
        lambda: I.cell_centred(48, -16, 16, 3),
        lambda g: I.brill_lindquist(g, (0.5, 0.5), ((3, 0, 0), (-3, 0, 0))),
        {}),
    "order8-smooth-static": (
        lambda: I.GridSpec((67, 22, 15), 5, (0.1, 0.11, 0.12),
                           (-3.3, -1.2, -0.9), I.BC_STATIC),
        lambda g: I.smooth_random(g, seed=11), dict(fd_order=8)),
    "order8-noise-periodic": (
        lambda: I.GridSpec((24, 20, 16), 5, (0.1,) * 3, (0.0,) * 3,
                           I.BC_PERIODIC),
        lambda g: I.minkowski_noise(g, seed=3), dict(fd_order=8)),
    "order8-bl-40": (
        lambda: I.cell_centred(40, -24, 24, 5),
        lambda g: I.brill_lindquist(g, (0.6, 0.4), ((4, 0, 0), (-4, 0, 0))),
        dict(fd_order=8)),
    # tile grid 8 x 16 x 10: the LDS kernel takes its blocked walk (4x4x2
    # blocks, one per XCD), with a ragged x edge (124 = 7.75 tiles)
    "smooth-static-blocked": (
        lambda: I.GridSpec((124, 64, 40), 3, (0.1, 0.11, 0.12),
                           (-6.1, -3.5, -2.4), I.BC_STATIC),
        lambda g: I.smooth_random(g, seed=12), {}),
    "order8-smooth-blocked": (
        lambda: I.GridSpec((124, 64, 40), 5, (0.1, 0.11, 0.12),
                           (-6.1, -3.5, -2.4), I.BC_STATIC),
        lambda g: I.smooth_random(g, seed=13), dict(fd_order=8)),
    # tile grid 8 x 8 x 12: blocks of 4 x 2 x 4 tiles, 4 deep in z
    "smooth-static-blocked-z4": (
        lambda: I.GridSpec((124, 32, 48), 3, (0.1, 0.11, 0.12),
                           (-6.1, -1.7, -2.8), I.BC_STATIC),
        lambda g: I.smooth_random(g, seed=14), {}),
}


@pytest.fixture(params=["auto", "direct"])
def path(request, B):
    """Both kernels: the LDS-pipelined one (auto on static grids) and the
    direct-load one."""
    B.bssn_set_path(B.BSSN_PATH_AUTO if request.param == "auto"
                    else B.BSSN_PATH_DIRECT)
    yield request.param
    B.bssn_set_path(B.BSSN_PATH_AUTO)


@pytest.mark.parametrize("case", list(CASES))
def test_rhs_matches_oracle(B, case, path):
    gfn, dfn, kw = CASES[case]
    g = gfn()
    u = dfn(g)
    prm = B.Params(**kw)
    print(f"[rhs] {case} n={g.n} path={path}", flush=True)
    ref = O.rhs(g, oparams(prm), u)
    got = gpu_rhs(B, g, prm, u)
    e = rhs_err(g, got, ref)
    assert e.max() <= 1e-12, (e.max(), int(e.argmax()))
    # ghosts of the output are untouched (zero-initialised here)
    v = g.view(got)
    gh = g.ghost
    v2 = v.copy()
    v2[:, gh:-gh, gh:-gh, gh:-gh] = 0
    assert np.all(v2 == 0)


@pytest.mark.parametrize("case,nsteps,dt", [
    ("noise-periodic-32", 1, 0.025),
    ("smooth-static-ragged", 2, 0.02),
    ("smooth-periodic", 2, 0.02),
    ("bl-two-punctures-48", 2, 0.1),
    ("order8-smooth-static", 1, 0.02),
    ("smooth-static-blocked", 2, 0.02),
    ("smooth-static-blocked-z4", 1, 0.02)])
def test_rk4_steps_match_oracle(B, case, nsteps, dt, path):
    gfn, dfn, kw = CASES[case]
    g = gfn()
    u0 = dfn(g)
    prm = B.Params(**kw)
    print(f"[rk4] {case} n={g.n} steps={nsteps} path={path}", flush=True)
    ref = O.rk4_steps(g, oparams(prm), dt, u0, nsteps)
    got = gpu_steps(B, g, prm, dt, u0, nsteps)
    tol = state_tol(g, u0, ref, nsteps)
    err = np.abs(g.interior(got) - g.interior(ref)).reshape(25, -1).max(1)
    assert np.all(err <= tol), (err / tol).max()
    if g.bc == I.BC_STATIC:  # static ghosts are never written
        gh = g.ghost
        mask = np.ones(g.view(u0).shape[1:], bool)
        mask[gh:-gh, gh:-gh, gh:-gh] = False
        assert np.array_equal(g.view(got)[:, mask], g.view(u0)[:, mask])


def test_minkowski_rhs_is_exactly_zero(B, path):
    for prec in (B.BSSN_FP64, B.BSSN_MIXED):
        for order, gh in ((4, 3), (8, 5)):
            g = I.GridSpec((40, 9, 7), gh, (0.1,) * 3, (0.0,) * 3,
                           I.BC_STATIC)
            got = gpu_rhs(B, g, B.Params(fd_order=order, precision=prec),
                          I.minkowski(g))
            assert np.all(got == 0.0)


def test_periodic_translation_invariance_bitwise(B):
    g = I.GridSpec((24, 20, 18), 3, (0.1,) * 3, (0.0,) * 3, I.BC_PERIODIC)
    u = I.smooth_random(g, seed=21)
    r1 = gpu_rhs(B, g, B.Params(), u)
    u2 = g.empty()
    g.interior(u2)[...] = np.roll(g.interior(u), (1, 2), axis=(1, 3))
    r2 = gpu_rhs(B, g, B.Params(), u2)
    np.testing.assert_array_equal(g.interior(r2),
                                  np.roll(g.interior(r1), (1, 2), axis=(1, 3)))


def test_runs_are_bitwise_reproducible(B, path):
    g = I.GridSpec((70, 38, 29), 3, (0.11, 0.13, 0.12), (-3.8, -2.4, -1.7),
                   I.BC_STATIC)
    u = I.smooth_random(g, seed=7)
    a = gpu_steps(B, g, B.Params(), 0.02, u, 2)
    b = gpu_steps(B, g, B.Params(), 0.02, u, 2)
    assert np.array_equal(a, b)


# ---- full-size configurations: sampled points ------------------------------
FULL = {
    "bl1-128": (lambda: I.cell_centred(128, -8, 8, 3),
               lambda g: I.brill_lindquist(g, (1.0,), ((0, 0, 0),)), 4),
    "bl2-256": (lambda: I.cell_centred(256, -16, 16, 3),
               lambda g: I.brill_lindquist(g, (0.5, 0.5),
                                           ((3, 0, 0), (-3, 0, 0))), 4),
    "bl2-384-order8": (lambda: I.cell_centred(384, -24, 24, 5),
                      lambda g: I.brill_lindquist(g, (0.6, 0.4),
                                                  ((4, 0, 0), (-4, 0, 0))),
                      8),
}


def _sample_points(g, n=400, seed=0):
    rng = np.random.default_rng(seed)
    pts = np.stack([rng.integers(0, g.n[a], size=n) for a in range(3)], 1)
    # always include corners and faces (stencils reaching into ghosts) and
    # points next to the punctures
    extra = [(0, 0, 0), tuple(v - 1 for v in g.n), (0, g.n[1] // 2, 3),
             (g.n[0] // 2, g.n[1] // 2, g.n[2] // 2),
             (g.n[0] // 2 - 1, g.n[1] // 2 - 1, g.n[2] // 2 - 1)]
    return np.concatenate([pts, np.array(extra)], 0).astype(np.int32)


@pytest.mark.parametrize("case", list(FULL))
def test_full_size_stage0_sampled(B, case, path):
    """At the benchmark sizes, stage 0 of RK4 (same launch as the
    benchmark) against the oracle evaluated point by point."""
    gfn, dfn, order = FULL[case]
    g = gfn()
    print(f"[full] {case} n={g.n}", flush=True)
    u = dfn(g)
    prm = B.Params(fd_order=order)
    dt = 0.03125
    du = B.to_device(u)
    acc = torch.zeros_like(du)
    out = du.clone()
    B.rk4_stage(g, prm, 0, dt, du, du, acc, out)
    torch.cuda.synchronize()
    pts = _sample_points(g)
    k = O.rhs_points(g, oparams(prm), u, pts)             # (N, 25)
    idx = (g.off0 + np.arange(25)[None, :] * g.sf
           + (pts[:, 2:3] + g.ghost) * g.sz + (pts[:, 1:2] + g.ghost) * g.sy
           + (pts[:, 0:1] + g.ghost))
    un = u[idx]
    it = torch.from_numpy(idx.reshape(-1)).to(out.device)
    gout = out[it].cpu().numpy().reshape(idx.shape)
    gacc = acc[it].cpu().numpy().reshape(idx.shape)
    del du, acc, out
    ref_out = un + (dt / 2) * k
    ref_acc = un + (dt / 6) * k
    D = np.abs(k).max(0)
    D = np.where(D > 0, D, D.max())
    for got, ref, c in ((gout, ref_out, dt / 2), (gacc, ref_acc, dt / 6)):
        tol = 1e-12 * c * D + 4 * EPS * np.abs(ref).max(0)
        assert np.all(np.abs(got - ref).max(0) <= tol)


# ---- constraints -------------------------------------------------------------
@pytest.mark.parametrize("case", ["smooth-static-ragged",
                                  "bl-two-punctures-48", "smooth-periodic",
                                  "order8-smooth-static"])
def test_constraints_match_oracle(B, case):
    gfn, dfn, kw = CASES[case]
    g = gfn()
    u = dfn(g)
    prm = B.Params(**kw)
    cent = [(3.0, 0.0, 0.0), (-3.0, 0.0, 0.0)]
    H0, M0, G0, n0 = O.constraints(g, oparams(prm), u, cent, 1.5)
    du = B.to_device(u)
    H, M, G = (torch.zeros_like(du) for _ in range(3))
    norms = torch.zeros(8, dtype=torch.float64, device="cuda")
    B.bssn_constraints(g, prm, du, norms, H, M, G, cent, 1.5)
    torch.cuda.synchronize()
    for a, b, ns in ((H, H0, 1), (M, M0, 3), (G, G0, 3)):
        ai = g.interior(a.cpu().numpy(), nslot=25)[:ns]
        bi = g.interior(b, nslot=25)[:ns]
        D = max(np.abs(bi).max(), 1e-300)
        assert np.abs(ai - bi).max() <= 1e-12 * D
    got = norms.cpu().numpy()
    np.testing.assert_array_equal(got[6:], n0[6:])
    np.testing.assert_allclose(got[:6], n0[:6], rtol=1e-12, atol=0)


def test_constraints_nonfinite_counted(B):
    g = I.GridSpec((20, 12, 10), 3, (0.1,) * 3, (0.0,) * 3, I.BC_STATIC)
    u = I.smooth_random(g, seed=4)
    g.interior(u)[I.TRK, 5, 6, 7] = np.nan
    du = B.to_device(u)
    norms = torch.zeros(8, dtype=torch.float64, device="cuda")
    B.bssn_constraints(g, B.Params(), du, norms)
    n = norms.cpu().numpy()
    _, _, _, n0 = O.constraints(g, O.params(), u)
    assert n[7] == n0[7] >= 1 and n[6] == n0[6]
    assert np.isfinite(n[:6]).all()


@pytest.mark.parametrize("nan", [False, True])
def test_constraint_norms_closed_form(B, nan):
    """The GPU's norms on the closed-form state of the oracle's norm pins
    (flat metric, K linear in x, constant Gt^x; two centres whose excised
    sets are counted by hand, one NaN reaching 10 points): N_used and
    N_nonfinite exactly, the RMS and maxima to 1e-13."""
    import test_oracle_norms as T
    g = T._grid()
    u = T._state(g)
    used = np.ones((T.N,) * 3, bool)
    for cx in (3, 4):
        for d in [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
                  (0, 0, 1), (0, 0, -1)]:
            used[3 + d[2], 3 + d[1], cx + d[0]] = False
    bad = 0
    if nan:
        g.interior(u)[I.TRK, 1, 1, 5] = np.nan
        for x, y, z in [(5, 1, 1), (4, 1, 1), (6, 1, 1), (3, 1, 1), (5, 0, 1),
                        (5, 2, 1), (5, 3, 1), (5, 1, 0), (5, 1, 2), (5, 1, 3)]:
            used[z, y, x] = False
        bad = 10
    du = B.to_device(u)
    norms = torch.zeros(8, dtype=torch.float64, device="cuda")
    B.bssn_constraints(g, B.Params(), du, norms,
                       centres=[(0.0, 0.0, 0.0), (0.5, 0.0, 0.0)], r_exc=0.5)
    torch.cuda.synchronize()
    T._check(norms.cpu().numpy(), T._closed_form_norms(used), nonfinite=bad)
