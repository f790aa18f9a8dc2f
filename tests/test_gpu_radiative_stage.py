"""RK4 stages with the radiative outer boundary evolved (rk4_stage_radiative)
against the oracle, through the C ABI (needs an MI355X).

  * Whole steps on small grids: every storage point (interior and ghost
    layers) after one and three steps equals classical RK4 on the oracle's
    right-hand side with the oracle's radiative boundary
    (f(u) = radiative_rhs(rhs(u))), increments within 1e-11 of their largest
    value per slot.
  * Each stage at the 128^3 benchmark grid: the FP64 right-hand side the
    call leaves in k at the outermost interior layer (all 96,776 points)
    against the oracle point by point; acc and u_out at all 308,952 ghost
    points against the stage update of the oracle's radiative right-hand
    side (built from those oracle values), per point within 1e-12 of the
    slot's largest increment plus the rounding of the stored sum
    (4 eps |value|: the increments, O(dt k), sit on O(1) values whose
    last bit is larger than 1e-12 of a small slot's increment); the
    interior bitwise equal to
    rk4_stage's on the same inputs (the same fused launch).
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import radiative as R
from paper_1111_3344_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_3344_amd import bssn
    bssn.lib()
    bssn.bssn_set_path(bssn.BSSN_PATH_AUTO)
    return bssn


def _oracle_steps(g, u0, order, dt, nsteps, x0, v0):
    prm = O.params(fd_order=order)

    def f(u):
        return R.radiative_rhs(g, u, O.rhs(g, prm, u), x0, v0, 2)

    u = u0
    for _ in range(nsteps):
        k1 = f(u)
        k2 = f(u + 0.5 * dt * k1)
        k3 = f(u + 0.5 * dt * k2)
        k4 = f(u + dt * k3)
        u = u + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return u


STEP_CASES = {
    "bl-20": (lambda: I.cell_centred(20, -3, 3, 3),
              lambda g: I.brill_lindquist(g, (0.8,), ((0.2, 0.1, -0.1),)), 4),
    "smooth-ragged": (
        lambda: I.GridSpec((23, 14, 11), 3, (0.11, 0.13, 0.12),
                           (-1.3, -0.9, -0.7), I.BC_STATIC),
        lambda g: I.smooth_random(g, seed=31), 4),
    "smooth-o8-ghost5": (
        lambda: I.GridSpec((17, 15, 19), 5, (0.1, 0.12, 0.09),
                           (0.6, -0.8, -0.9), I.BC_STATIC),
        lambda g: I.smooth_random(g, seed=32), 8),
}


@pytest.mark.parametrize("path", ["lds", "direct"])
@pytest.mark.parametrize("nsteps", [1, 3])
@pytest.mark.parametrize("case", list(STEP_CASES))
def test_steps_match_oracle(B, case, nsteps, path):
    """Both kernel paths: the LDS stage kernels leave the roots' right-hand
    side in k themselves; the direct-load stage has the shell kernel compute
    it first."""
    gfn, dfn, order = STEP_CASES[case]
    g = gfn()
    u0 = dfn(g)
    x0, v0 = np.array(B.RADIATIVE_X0), np.array(B.RADIATIVE_V0)
    dt = 0.25 * min(g.h)
    ref = _oracle_steps(g, u0, order, dt, nsteps, x0, v0)
    print(f"[radstage] {case} steps={nsteps} path={path}", flush=True)
    du = B.to_device(u0)
    a, b, acc, k = (torch.zeros_like(du) for _ in range(4))
    prm = B.Params(fd_order=order)
    B.bssn_set_path(B.BSSN_PATH_DIRECT if path == "direct"
                    else B.BSSN_PATH_AUTO)
    try:
        for _ in range(nsteps):
            B.rk4_step_radiative(g, prm, dt, du, a, b, acc, k)
        torch.cuda.synchronize()
    finally:
        B.bssn_set_path(B.BSSN_PATH_AUTO)
    got = du.cpu().numpy()
    inc_ref = g.view(ref - u0).reshape(25, -1)
    inc_got = g.view(got - u0).reshape(25, -1)
    D = np.abs(inc_ref).max(1)
    D = np.where(D > 0, D, D.max())
    e = np.abs(inc_got - inc_ref).max(1) / D
    print(f"[radstage] {case} steps={nsteps} path={path}: max normwise "
          f"increment error {e.max():.2e}", flush=True)
    assert np.all(e <= 1e-11), (e.max(), int(e.argmax()))
    layer, _ = R.layers(g)
    assert np.abs(g.view(ref - u0)[:, layer > 0]).max() > 0


def _shell_points(g):
    n = g.n
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]),
                          indexing="ij")
    m = ((x == 0) | (x == n[0] - 1) | (y == 0) | (y == n[1] - 1) |
         (z == 0) | (z == n[2] - 1))
    return np.stack([x[m], y[m], z[m]], 1)


@pytest.mark.parametrize("stage", [0, 1, 2, 3])
def test_stage_full_size(B, stage):
    g = I.cell_centred(128, -8.0, 8.0, 3)
    x0, v0 = np.array(B.RADIATIVE_X0), np.array(B.RADIATIVE_V0)
    dt = 0.03125
    u_n = I.brill_lindquist(g, (1.0,), ((0.0, 0.0, 0.0),))
    # smooth_random minus its backgrounds (nmodes=0): a pure perturbation
    u_s = u_n + 1e-3 * (I.smooth_random(g, seed=41) -
                        I.smooth_random(g, seed=41, nmodes=0))
    acc0 = u_n + 1e-2 * (I.smooth_random(g, seed=42) -
                         I.smooth_random(g, seed=42, nmodes=0))
    prm = B.Params()
    print(f"[radstage] full size stage {stage}", flush=True)
    dn, ds = B.to_device(u_n), B.to_device(u_s)
    acc = B.to_device(acc0)
    out = torch.zeros_like(dn)
    k = torch.zeros_like(dn)
    outn = dn if stage == 3 else out
    B.rk4_stage_radiative(g, prm, stage, dt, dn, ds, acc, outn, k)
    # the plain fused stage on the same inputs
    acc2 = B.to_device(acc0)
    dn2 = B.to_device(u_n)
    out2 = dn2 if stage == 3 else torch.zeros_like(dn2)
    B.rk4_stage(g, prm, stage, dt, dn2, ds, acc2, out2)
    torch.cuda.synchronize()
    got_out = outn.cpu().numpy()
    got_acc = acc.cpu().numpy()
    got_k = k.cpu().numpy()
    # interior: the same fused launch
    assert np.array_equal(g.interior(got_out), g.interior(out2.cpu().numpy()))
    if stage != 3:
        assert np.array_equal(g.interior(got_acc),
                              g.interior(acc2.cpu().numpy()))
    # the roots' right-hand side
    pts = _shell_points(g)
    kref = O.rhs_points(g, O.params(), u_s, pts)              # (N, 25)
    kv = g.view(got_k)[:, pts[:, 2] + g.ghost, pts[:, 1] + g.ghost,
                       pts[:, 0] + g.ghost].T
    D = np.abs(kref).max(0)
    D = np.where(D > 0, D, D.max())
    ek = (np.abs(kv - kref).max(0) / D).max()
    assert ek <= 1e-12, ek
    # the ghost layers: stage update of the oracle's radiative right-hand side
    rin = g.empty()
    g.view(rin)[:, pts[:, 2] + g.ghost, pts[:, 1] + g.ghost,
                pts[:, 0] + g.ghost] = kref.T
    kr = g.view(R.radiative_rhs(g, u_s, rin, x0, v0, 2))
    layer, _ = R.layers(g)
    m = layer > 0
    un, ac = g.view(u_n)[:, m], g.view(acc0)[:, m]
    kb = kr[:, m]
    if stage == 0:
        want_acc, want_out = un + dt / 6 * kb, un + dt / 2 * kb
    elif stage == 3:
        want_acc, want_out = None, ac + dt / 6 * kb
    else:
        c = dt / 2 if stage == 1 else dt
        want_acc, want_out = ac + dt / 3 * kb, un + c * kb
    base = ac if stage == 3 else un

    def err(got, want, base):
        # per point: within 1e-12 of the slot's largest increment, plus the
        # rounding of the stored sum base + increment (4 eps |want|)
        inc_w = want - base
        D = np.abs(inc_w).max(1, keepdims=True)
        D = np.where(D > 0, D, D.max())
        tol = 1e-12 * D + 4 * np.finfo(float).eps * np.abs(want)
        return (np.abs(got - want) / tol).max()
    e_out = err(g.view(got_out)[:, m], want_out, base)
    e_acc = 0.0 if want_acc is None else err(g.view(got_acc)[:, m], want_acc,
                                             ac if stage else un)
    print(f"[radstage] full size stage {stage}: roots {ek:.2e} (normwise); "
          f"ghost u_out {e_out:.3f}, acc {e_acc:.3f} of the tolerance",
          flush=True)
    assert e_out <= 1.0 and e_acc <= 1.0


def test_mixed_precision_tracks_fp64(B):
    """Three radiative steps in mixed precision (FP32 tiles, the roots' right-
    hand side from the tiles as computed) stay within 1e-5 of FP64, per slot
    relative to the slot's largest increment, interior and boundary."""
    g = I.cell_centred(40, -4, 4, 3)
    u0 = I.brill_lindquist(g, (0.8,), ((0.2, 0.1, -0.1),))
    dt = 0.25 * g.h[0]
    res = []
    for prec in (B.BSSN_FP64, B.BSSN_MIXED):
        du = B.to_device(u0)
        a, b, acc, k = (torch.zeros_like(du) for _ in range(4))
        for _ in range(3):
            B.rk4_step_radiative(g, B.Params(precision=prec), dt, du, a, b,
                                 acc, k)
        torch.cuda.synchronize()
        res.append(du.cpu().numpy())
    inc64 = g.view(res[0] - u0).reshape(25, -1)
    incm = g.view(res[1] - u0).reshape(25, -1)
    D = np.abs(inc64).max(1)
    D = np.where(D > 0, D, D.max())
    e = np.abs(incm - inc64).max(1) / D
    print(f"[radstage] mixed vs FP64, 3 steps: max normwise {e.max():.2e}",
          flush=True)
    assert np.isfinite(res[1]).all()
    assert e.max() <= 1e-5, (e.max(), int(e.argmax()))
