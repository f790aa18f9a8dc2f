"""Berger-Oliger time stepping with subcycling (paper_1111_3344_amd.amr) on
the GPU against the same schedule built from the oracle's pieces (needs an
MI355X).

The oracle side: the oracle's right-hand side on each patch, classical RK4
with separate k buffers, the oracle's ghost fill at each stage time and
after each step, its restriction after the two fine steps.  Two level-0
steps on a hierarchy with two coarse patches sharing a face and two fine
siblings across the coarse seam (sibling exchange on both levels,
prolongation from either coarse patch, two and then three coarse time
levels, restriction) from Brill-Lindquist data.  Every patch's change of
state must match to 1e-10 relative per slot (normwise): the two sides
differ by the rounding of about a hundred right-hand-side evaluations and
fills, not by any term.
"""
import numpy as np
import pytest

from oracle import amr as M
from oracle import oracle as O
from paper_1111_3344_amd import inputs as I
from tests import amr_hier as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

C = (0.0, 0.5, 0.5, 1.0)


def _oracle_bo(hr, prm, dt0, u0, nsteps):
    nl = 1 + max(lv for lv, _ in hr)
    u = [x.copy() for x in u0]
    prev = [x.copy() for x in u0]
    prev2 = [x.copy() for x in u0]
    time = [0.0] * nl
    ns = [0] * nl

    def level(L, lst):
        return [x if lv == L else None for (lv, _), x in zip(hr, lst)]

    def fill(L, states, t):
        if L == 0:
            M.fill_ghosts(hr, 0, states, None, None, t)
            return
        c = L - 1
        dt = dt0 / 2 ** c
        if ns[c] >= 2:
            tabs = [level(c, prev2), level(c, prev), level(c, u)]
            ts = [time[c] - 2 * dt, time[c] - dt, time[c]]
        else:
            tabs = [level(c, prev), level(c, u)]
            ts = [time[c] - dt, time[c]]
        M.fill_ghosts(hr, L, states, tabs, ts, t)

    def advance(L):
        dt = dt0 / 2 ** L
        T = time[L]
        idx = [p for p, (lv, _) in enumerate(hr) if lv == L]
        for p in idx:
            prev2[p], prev[p] = prev[p], u[p]
        y = list(prev)
        ks = {p: [] for p in idx}
        for s in range(4):
            fill(L, level(L, y), T + C[s] * dt)
            for p in idx:
                ks[p].append(O.rhs(hr[p][1], prm, y[p]))
            if s < 3:
                f = (0.5, 0.5, 1.0)[s] * dt
                y = list(y)
                for p in idx:
                    y[p] = prev[p] + f * ks[p][s]
        for p in idx:
            k1, k2, k3, k4 = ks[p]
            u[p] = prev[p] + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
        fill(L, level(L, u), T + dt)
        time[L] = T + dt
        ns[L] += 1
        if L + 1 < nl:
            advance(L + 1)
            advance(L + 1)
            M.restrict(hr, L + 1, level(L + 1, u), level(L, u))

    for _ in range(nsteps):
        advance(0)
    return u


def test_berger_oliger_two_steps_match_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_3344_amd import amr
    from paper_1111_3344_amd import bssn as B
    B.lib()
    hr = H.bo_level()
    m, c = (0.3,), ((0.02, -0.07, -0.05),)
    u0 = [I.brill_lindquist(g, m, c) for _, g in hr]
    dt0 = 0.25 * hr[0][1].h[0]
    want = _oracle_bo(hr, O.params(), dt0, u0, 2)
    drv = amr.BergerOliger(hr, B.Params(), dt0, [B.to_device(x) for x in u0])
    drv.step()
    drv.step()
    torch.cuda.synchronize()
    worst = 0.0
    for p, (lv, g) in enumerate(hr):
        got = drv.u[p].cpu().numpy()
        inc_w = g.view(want[p] - u0[p]).reshape(25, -1)
        inc_g = g.view(got - u0[p]).reshape(25, -1)
        D = np.abs(inc_w).max(1)
        D = np.where(D > 0, D, 1.0)
        e = (np.abs(inc_g - inc_w).max(1) / D).max()
        print(f"[bo] patch {p} (level {lv}): max normwise increment error "
              f"{e:.2e}, max |increment| {np.abs(inc_w).max():.2e}",
              flush=True)
        worst = max(worst, e)
        assert np.abs(inc_w).max() > 0
    assert worst <= 1e-10, worst
    assert drv.time == [2 * dt0, 2 * dt0]


@pytest.mark.parametrize("hname,precision", [("two_level", 0),
                                             ("three_level", 0),
                                             ("two_level", 1)])
def test_batched_level_stages_bitwise(hname, precision):
    """The stepper with every level's stages batched over its patches
    (batch_patches_stage of per-level plans; a level of one patch calls its
    rk4_stage) equals the one launching rk4_stage per patch, bitwise, over
    three level-0 steps: the same kernel arithmetic, the same fills and
    restrictions."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_3344_amd import amr
    from paper_1111_3344_amd import bssn as B
    B.lib()
    hr = getattr(H, hname)()
    m, c = (0.3,), ((0.02, -0.07, -0.05),)
    u0 = [I.brill_lindquist(g, m, c) for _, g in hr]
    dt0 = 0.25 * hr[0][1].h[0]
    prm = B.Params(precision=precision)
    print(f"[bo] batched vs per patch: {hname}, precision {precision}",
          flush=True)
    res = []
    for batched in (True, False):
        drv = amr.BergerOliger(hr, prm, dt0, [B.to_device(x) for x in u0],
                               batched=batched)
        for _ in range(3):
            drv.step()
        torch.cuda.synchronize()
        res.append([x.cpu().numpy() for x in drv.u])
        if batched:
            # plans exactly for the levels of several patches (a level of
            # one patch calls its rk4_stage)
            multi = {lv for lv, _ in hr
                     if sum(1 for l2, _ in hr if l2 == lv) > 1}
            assert {L for L, _ in drv._plans} == multi
    for p in range(len(hr)):
        assert np.array_equal(res[0][p], res[1][p]), p
        assert not np.array_equal(res[0][p], u0[p])
