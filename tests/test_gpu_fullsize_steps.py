"""Full-size parity of whole RK4 steps, in the launch configurations the
benchmark times (needs an MI355X).

  * every stage (0..3) of one RK4 step on the 128^3, 256^3 and 384^3
    (8th-order) workloads, FP64 and mixed precision: acc and the stage
    output at sampled points against the oracle's right-hand side of the
    same stage input, evaluated on the stencil cube gathered around each
    sample (the cube is a one-point grid whose ghosts are the sample's
    neighbours, so the oracle sees exactly the values the kernel read);
  * ten whole RK4 steps on the full 128^3 grid against the oracle's ten
    steps, every interior point;
  * one batched step (the benchmark's autotuned plan) of all 256 uneven
    patches against the oracle: at sampled points of every patch, the
    oracle's RK4 step of a sub-box around the point.  One RK4 step moves
    information by 3R points after the first stage (each of stages 1..3
    reads its input R points away, and stage 0 reads the initial data,
    which the sub-box's ghosts hold), so a sub-box reaching 3R points
    beyond the sample in every direction (or to the patch's own ghosts)
    gives the exact step at the sample.

Tolerances are those of the single-patch parity tests: FP64 k within
1e-12 of the oracle per slot (normwise), states within 1e-12 of their
change plus a few ulps; mixed-precision k within 1e-5.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1111_3344_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
MIXED_RHS_TOL = 1e-5
DT = 0.03125


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_3344_amd import bssn
    bssn.lib()
    bssn.bssn_set_path(bssn.BSSN_PATH_AUTO)
    return bssn


GRIDS = {
    "bl1-128": (lambda: I.cell_centred(128, -8, 8, 3), (1.0,),
                ((0.0, 0.0, 0.0),), 4),
    "bl2-256": (lambda: I.cell_centred(256, -16, 16, 3), (0.5, 0.5),
                ((3.0, 0.0, 0.0), (-3.0, 0.0, 0.0)), 4),
    "bl2-384-o8": (lambda: I.cell_centred(384, -24, 24, 5), (0.6, 0.4),
                   ((4.0, 0.0, 0.0), (-4.0, 0.0, 0.0)), 8),
}


def sample_points(g, centres, n=240, seed=9):
    """Random interior points, the 8 corners, and points around each
    puncture (whose tiles mixed precision routes to FP64)."""
    rng = np.random.default_rng(seed)
    pts = [np.stack([rng.integers(0, g.n[a], size=n) for a in range(3)], 1)]
    pts.append(np.array([[x, y, z] for x in (0, g.n[0] - 1)
                         for y in (0, g.n[1] - 1) for z in (0, g.n[2] - 1)]))
    for c in centres:
        ic = [int((c[a] - g.origin[a]) / g.h[a]) for a in range(3)]
        for d in ((-2, 0, 0), (0, 0, 0), (1, 1, 1), (0, -1, 2)):
            pts.append(np.array([[ic[a] + d[a] for a in range(3)]]))
    return np.concatenate(pts, 0).astype(np.int64)


def point_index(g, pts):
    """Flat indices (N, 25) of every slot at interior points pts."""
    gh = g.ghost
    return (g.off0 + np.arange(25)[None, :] * g.sf
            + (pts[:, 2:3] + gh) * g.sz + (pts[:, 1:2] + gh) * g.sy
            + (pts[:, 0:1] + gh))


def cube_index(g, p):
    """Flat indices (25, 2g+1, 2g+1, 2g+1) of the storage cube around
    interior point p ([slot][z][y][x])."""
    w = 2 * g.ghost + 1
    d = np.arange(w)
    return (g.off0 + np.arange(25)[:, None, None, None] * g.sf
            + (p[2] + d)[None, :, None, None] * g.sz
            + (p[1] + d)[None, None, :, None] * g.sy
            + (p[0] + d)[None, None, None, :])


def oracle_k_at(g, prm, cubes, pts):
    """The oracle's right-hand side at each sample from its stencil cube:
    a grid of one interior point with the grid's ghost width, placed at
    the sample's coordinates."""
    out = np.empty((len(pts), 25))
    for i, p in enumerate(pts):
        gc = I.GridSpec((1, 1, 1), g.ghost, g.h,
                        tuple(g.origin[a] + p[a] * g.h[a] for a in range(3)),
                        I.BC_STATIC)
        u = gc.empty()
        gc.view(u)[...] = cubes[i]
        out[i] = gc.interior(O.rhs(gc, prm, u))[:, 0, 0, 0]
    return out


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", list(GRIDS))
def test_full_size_every_stage_sampled(B, name, precision):
    gfn, masses, centres, order = GRIDS[name]
    g = gfn()
    print(f"[stages] {name} n={g.n} precision={precision}", flush=True)
    du = B.to_device(I.brill_lindquist(g, masses, centres))
    a, b, acc = du.clone(), du.clone(), torch.zeros_like(du)
    prm = B.Params(fd_order=order, precision=precision)
    oprm = O.params(fd_order=order)
    pts = sample_points(g, centres)
    pidx = torch.from_numpy(point_index(g, pts).reshape(-1)).to("cuda")
    cidx = torch.from_numpy(np.stack([cube_index(g, p) for p in pts])
                            .reshape(-1)).to("cuda")
    cshape = (len(pts), 25) + (2 * g.ghost + 1,) * 3
    bufs = [(du, du, a), (du, a, b), (du, b, a), (du, a, du)]
    tile_f64 = None
    if precision:
        al = g.interior(du.cpu().numpy())[I.ALP]  # routing of stage 0
        nz, ny, nx = al.shape
        p = np.pad(al, ((0, -nz % 4), (0, -ny % 4), (0, -nx % 16)),
                   constant_values=np.inf)
        tmin = p.reshape(p.shape[0] // 4, 4, p.shape[1] // 4, 4,
                         p.shape[2] // 16, 16).min(axis=(1, 3, 5))
        tile_f64 = tmin[pts[:, 2] // 4, pts[:, 1] // 4, pts[:, 0] // 16] < 0.3
        assert tile_f64.sum() >= 4
    for s, (un, us, uo) in enumerate(bufs):
        cubes = us[cidx].cpu().numpy().reshape(cshape)
        u_n = un[pidx].cpu().numpy().reshape(-1, 25)
        acc_in = acc[pidx].cpu().numpy().reshape(-1, 25)
        B.rk4_stage(g, prm, s, DT, un, us, acc, uo)
        torch.cuda.synchronize()
        out = uo[pidx].cpu().numpy().reshape(-1, 25)
        acc_out = acc[pidx].cpu().numpy().reshape(-1, 25)
        k = oracle_k_at(g, oprm, cubes, pts)
        base, c = ((u_n, DT / 2) if s < 2 else (u_n, DT) if s == 2
                   else (acc_in, DT / 6))
        ref_out = base + c * k
        checks = [(out, ref_out, c)]
        if s < 3:
            ca = DT / 6 if s == 0 else DT / 3
            ref_acc = (u_n if s == 0 else acc_in) + ca * k
            checks.append((acc_out, ref_acc, ca))
        D = np.abs(k).max(0)
        D = np.where(D > 0, D, D.max())
        for got, ref, cc in checks:
            err = np.abs(got - ref)  # (N, 25)
            tol64 = 1e-12 * cc * D + 4 * EPS * np.abs(ref).max(0)
            if precision:
                tol = MIXED_RHS_TOL * cc * D + 4 * EPS * np.abs(ref).max(0)
                assert np.all(err <= tol), (s, (err / tol).max())
                if s == 0:  # the FP64-routed tiles take the FP64 method
                    assert np.all(err[tile_f64] <= tol64), s
            else:
                assert np.all(err <= tol64), (s, (err / tol64).max())
        print(f"[stages] {name} stage {s}: max |k| error / D = "
              f"{(np.abs((out - base) / c - k) / D).max():.2e}", flush=True)
    del du, a, b, acc
    torch.cuda.empty_cache()


def test_ten_steps_full_128_grid(B):
    """Ten FP64 RK4 steps of the 128^3 single-puncture workload, every
    interior point against the oracle's ten steps."""
    gfn, masses, centres, order = GRIDS["bl1-128"]
    g = gfn()
    u0 = I.brill_lindquist(g, masses, centres)
    du = B.to_device(u0)
    a, b, acc = du.clone(), du.clone(), torch.zeros_like(du)
    prm = B.Params()
    for _ in range(10):
        B.rk4_step(g, prm, DT, du, a, b, acc)
    torch.cuda.synchronize()
    got = du.cpu().numpy()
    del du, a, b, acc
    print("[ten steps] oracle on 128^3 ...", flush=True)
    ref = O.rk4_steps(g, O.params(), DT, u0, 10)
    gi, ri, i0 = g.interior(got), g.interior(ref), g.interior(u0)
    d = np.abs(ri - i0).reshape(25, -1).max(1)
    m = np.abs(ri).reshape(25, -1).max(1)
    tol = 10 * (1e-12 * d + 8 * EPS * np.maximum(m, 1e-300))
    err = np.abs(gi - ri).reshape(25, -1).max(1)
    print(f"[ten steps] max error / tolerance {(err / tol).max():.3f}",
          flush=True)
    assert np.all(err <= tol), (err / tol).max()


def subbox_step_value(g, u, p, margin, prm, dt):
    """The oracle's RK4 step of the sub-box of grid g whose interior is the
    points within `margin` of p (clipped to the grid); returns the 25 slots
    at p."""
    lo = [max(0, p[a] - margin) for a in range(3)]
    hi = [min(g.n[a] - 1, p[a] + margin) for a in range(3)]
    n = tuple(hi[a] - lo[a] + 1 for a in range(3))
    gs = I.GridSpec(n, g.ghost, g.h,
                    tuple(g.origin[a] + lo[a] * g.h[a] for a in range(3)),
                    I.BC_STATIC)
    us = gs.empty()
    gs.view(us)[...] = g.view(u)[:, lo[2]:hi[2] + 2 * g.ghost + 1,
                                 lo[1]:hi[1] + 2 * g.ghost + 1,
                                 lo[0]:hi[0] + 2 * g.ghost + 1]
    out = O.rk4_step(gs, prm, dt, us)
    return gs.interior(out)[:, p[2] - lo[2], p[1] - lo[1], p[0] - lo[0]]


def test_batched_step_every_patch(B):
    """One step of the benchmark's batch plan (FP64, autotuned) over the
    256 uneven patches: four points of every patch (two corners, two
    random) against the oracle's step of a sub-box with margin 3R."""
    specs = I.patches(256)
    grids = [g for g, _, _ in specs]
    hosts = [I.brill_lindquist(g, (m,), (c,)) for g, m, c in specs]
    u = [torch.from_numpy(x).to("cuda") for x in hosts]
    a = [t.clone() for t in u]
    b = [t.clone() for t in u]
    acc = [torch.zeros_like(t) for t in u]
    plan = B.batch_patches_plan(grids, B.Params(), u, a, b, acc, DT,
                                autotune=True)
    for i, x in enumerate(hosts):  # autotuning ran stage 0 into a and acc
        u[i].copy_(torch.from_numpy(x))
    B.batch_patches(plan, 1)
    torch.cuda.synchronize()
    rng = np.random.default_rng(17)
    prm = O.params()
    margin = 3 * 3
    print("[batched] oracle sub-boxes on 256 patches ...", flush=True)
    got, ref, old, where = [], [], [], []
    for p, (g, x) in enumerate(zip(grids, hosts)):
        pts = [(0, 0, 0), (g.n[0] - 1, g.n[1] - 1, g.n[2] - 1)]
        pts += [tuple(int(rng.integers(0, g.n[a])) for a in range(3))
                for _ in range(2)]
        view = g.view(u[p].cpu().numpy())
        gh = g.ghost
        for q in pts:
            ref.append(subbox_step_value(g, x, q, margin, prm, DT))
            got.append(view[:, q[2] + gh, q[1] + gh, q[0] + gh])
            old.append(g.view(x)[:, q[2] + gh, q[1] + gh, q[0] + gh])
            where.append((p, q))
    plan.destroy()
    got, ref, old = np.array(got), np.array(ref), np.array(old)
    # per slot: 1e-12 of the slot's largest change over the samples plus
    # a few ulps of its largest value (the single-patch state tolerance)
    tol = (1e-12 * np.abs(ref - old).max(0) +
           8 * EPS * np.abs(ref).max(0))
    err = np.abs(got - ref)
    bad = np.argwhere(err > tol)
    assert len(bad) == 0, [(where[i], s) for i, s in bad[:5]]
    live = tol > 0  # slot A is identically zero: no error and no tolerance
    print(f"[batched] {len(got)} points, max error / tolerance "
          f"{(err[:, live] / tol[live]).max():.3f}", flush=True)


def test_evolved_constraints_converge_fourth_order(B):
    """Brill-Lindquist M = 1 on [-8, 8]^3 at n = 64, 128, 256 (h = 1/4, 1/8,
    1/16), evolved in FP64 to t = 1 with dt = h/4: the Hamiltonian and
    momentum constraint RMS over 2 < r < 6, |x|_inf < 6 (away from the
    puncture, whose non-smooth data converge at lower order, and from the
    static outer boundary, whose mismatch with the evolution enters from
    |x| = 8 at the gauge speed sqrt(2)) fall by 2^4 per halving of h."""
    rms = []
    for n in (64, 128, 256):
        g = I.cell_centred(n, -8, 8, 3)
        h = 16.0 / n
        du = B.to_device(I.brill_lindquist(g, (1.0,), ((0.0, 0.0, 0.0),)))
        a, b, acc = du.clone(), du.clone(), torch.zeros_like(du)
        prm = B.Params()
        nst = int(round(4 / h))
        for _ in range(nst):
            B.rk4_step(g, prm, h / 4, du, a, b, acc)
        H, M = torch.zeros_like(du), torch.zeros_like(du)
        norms = torch.zeros(8, dtype=torch.float64, device="cuda")
        B.bssn_constraints(g, prm, du, norms, H, M)
        torch.cuda.synchronize()
        Hi = g.interior(H.cpu().numpy(), 1)[0]
        Mi = np.sqrt((g.interior(M.cpu().numpy(), 3) ** 2).sum(0))
        gh = g.ghost
        X, Y, Z = [np.asarray(v)[gh:-gh, gh:-gh, gh:-gh] for v in g.mesh()]
        r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
        box = np.maximum(np.maximum(np.abs(X), np.abs(Y)), np.abs(Z))
        m = (r > 2) & (r < 6) & (box < 6)
        rms.append((np.sqrt((Hi[m] ** 2).mean()), np.sqrt((Mi[m] ** 2).mean())))
        del du, a, b, acc, H, M
        torch.cuda.empty_cache()
    rh = [rms[i][0] / rms[i + 1][0] for i in range(2)]
    rm = [rms[i][1] / rms[i + 1][1] for i in range(2)]
    print(f"[convergence t=1] H rms {[f'{x[0]:.3e}' for x in rms]} ratios "
          f"{rh[0]:.2f} {rh[1]:.2f}; M rms {[f'{x[1]:.3e}' for x in rms]} "
          f"ratios {rm[0]:.2f} {rm[1]:.2f}", flush=True)
    for q in rh + rm:
        assert 13.0 < q < 19.5, (rh, rm)
