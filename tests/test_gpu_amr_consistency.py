"""Refinement does not disturb the coarse solution (needs an MI355X).

A Brill-Lindquist puncture is evolved for several level-0 steps twice:
on one coarse grid, and with a refined level over its central half
(Berger-Oliger stepping, paper_1111_3344_amd.amr).  Away from the
refined region the two coarse solutions differ only by what the better
resolved centre sends out in that time, so the difference must be far
below the solution's own change there, and the refined run must stay
finite everywhere.  Doubling the resolution of both runs must shrink the
difference (the glue is consistent: no O(1) error at the seams).
"""
import numpy as np
import pytest

from paper_1111_3344_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _run(n, steps):
    from paper_1111_3344_amd import amr
    from paper_1111_3344_amd import bssn as B
    g = I.cell_centred(n, -4.0, 4.0, 3)
    h = g.h[0]
    f = I.GridSpec(g.n, 3, (h / 2,) * 3,
                   tuple(g.origin[a] + (n // 4 - 0.25) * h for a in range(3)),
                   I.BC_STATIC)
    m, c = (0.5,), ((0.05, -0.03, 0.02),)
    u0 = I.brill_lindquist(g, m, c)
    dt = 0.25 * h
    # uniform coarse run
    single = amr.BergerOliger([(0, g)], B.Params(), dt, [B.to_device(u0)])
    two = amr.BergerOliger([(0, g), (1, f)], B.Params(), dt,
                           [B.to_device(u0),
                            B.to_device(I.brill_lindquist(f, m, c))])
    for _ in range(steps):
        single.step()
        two.step()
    torch.cuda.synchronize()
    a = g.view(single.u[0].cpu().numpy())
    b = g.view(two.u[0].cpu().numpy())
    assert np.isfinite(b).all() and np.isfinite(f.view(
        two.u[1].cpu().numpy())).all()
    # outer shell of the level-0 interior: outside the refined region
    X, Y, Z = g.mesh()
    r = np.maximum(np.maximum(np.abs(X), np.abs(Y)), np.abs(Z))
    outer = r > 3.0
    diff = np.abs(a - b)[:, outer].max()
    change = np.abs(a - g.view(u0))[:, outer].max()
    return diff, change


def test_refinement_keeps_the_coarse_solution():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d1, c1 = _run(32, 4)
    d2, c2 = _run(64, 8)    # same physical time
    print(f"[amr-consistency] n=32: diff {d1:.3e} change {c1:.3e}; "
          f"n=64: diff {d2:.3e} change {c2:.3e}", flush=True)
    assert d1 < 0.1 * c1
    assert d2 < 0.1 * c2
    assert d2 < d1


def test_refined_run_in_mixed_precision_tracks_fp64():
    """The same two-level run with the mixed-precision stages: every
    patch's change within 1e-5 relative per slot (normwise) of the FP64
    run, the bar of the single-grid mixed path."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_3344_amd import amr
    from paper_1111_3344_amd import bssn as B
    n = 48
    g = I.cell_centred(n, -4.0, 4.0, 3)
    h = g.h[0]
    f = I.GridSpec(g.n, 3, (h / 2,) * 3,
                   tuple(g.origin[a] + (n // 4 - 0.25) * h for a in range(3)),
                   I.BC_STATIC)
    hier = [(0, g), (1, f)]
    m, c = (0.5,), ((0.05, -0.03, 0.02),)
    u0 = [I.brill_lindquist(gr, m, c) for _, gr in hier]
    runs = {}
    for name, prec in (("f64", B.BSSN_FP64), ("mixed", B.BSSN_MIXED)):
        d = amr.BergerOliger(hier, B.Params(precision=prec), 0.25 * h,
                             [B.to_device(x) for x in u0])
        for _ in range(3):
            d.step()
        torch.cuda.synchronize()
        runs[name] = [x.cpu().numpy() for x in d.u]
    worst = 0.0
    for p, (_, gr) in enumerate(hier):
        a = gr.view(runs["f64"][p] - u0[p]).reshape(25, -1)
        b = gr.view(runs["mixed"][p] - u0[p]).reshape(25, -1)
        D = np.abs(a).max(1)
        D = np.where(D > 0, D, 1.0)
        worst = max(worst, (np.abs(a - b).max(1) / D).max())
    print(f"[amr-mixed] max normwise change difference {worst:.2e}",
          flush=True)
    assert worst <= 1e-5
