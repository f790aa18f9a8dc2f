"""Mesh-refinement glue on the GPU (bssn_amr_*) against the oracle
(oracle/amr.py), through the C ABI (needs an MI355X).

Every patch holds its own seeded smooth state (so a sibling copy, a
prolongation from either coarse patch and a restriction give different
values).  Level 0 only exchanges the faces its patches share.  Ghost points filled by a copy must match the oracle bitwise;
prolonged ghost points and restricted coarse points to 1e-13 relative per
slot (normwise over the points compared: both sides sum the same 64 or 192
products, in a different contraction); nothing else may change.
"""
import functools

import numpy as np
import pytest

from oracle import amr as M
from paper_1111_3344_amd import inputs as I
from tests import amr_hier as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_3344_amd import bssn
    bssn.lib()
    return bssn


def _states(hr, seed):
    return [I.smooth_random(g, seed=seed + 7 * p) for p, (_, g) in
            enumerate(hr)]


def _ghost_mask(g):
    m = np.ones(tuple(g.ext[::-1]), bool)
    c = g.ghost
    m[c:-c, c:-c, c:-c] = False
    return m


def _rel(a, b):
    D = np.abs(b).reshape(25, -1).max(1)
    D = np.where(D > 0, D, 1.0)
    return (np.abs(a - b).reshape(25, -1).max(1) / D).max()


CASES = {
    "two-level-one-time": (H.two_level, [0.0], 0.0),
    "two-level-three-times": (H.two_level, [0.0, 0.5, 1.0], 0.75),
    "three-level-two-times": (H.three_level, [0.0, 1.0], 0.5),
    # the ghost width of 8th-order grids: wider shells, more tiles
    "two-level-ghost5-two-times": (functools.partial(H.two_level, ghost=5),
                                   [0.0, 1.0], 0.3),
    "three-level-ghost5-three-times": (
        functools.partial(H.three_level, ghost=5), [0.0, 0.5, 1.0], 0.8),
}


@pytest.mark.parametrize("case", list(CASES))
def test_fill_ghosts_matches_oracle(B, case):
    hfn, ts, t = CASES[case]
    hr = hfn()
    plan = B.AmrPlan(hr)
    top = max(lv for lv, _ in hr)
    for level in range(0, top + 1):
        states = _states(hr, 100 + level)
        levels = [_states(hr, 200 + 13 * l) for l in range(len(ts))]
        ref = [u.copy() for u in states]
        M.fill_ghosts(hr, level, ref, levels, ts, t)
        d_states = [B.to_device(u) for u in states]
        d_levels = [[B.to_device(u) for u in lv] for lv in levels]
        print(f"[amr] fill {case} level {level} counts "
              f"{plan.counts(level)}", flush=True)
        plan.fill_ghosts(level, d_states, d_levels, ts, t)
        torch.cuda.synchronize()
        nf, ncopy, _ = plan.counts(level)
        seen_f = seen_c = 0
        for p, (lv, g) in enumerate(hr):
            got = d_states[p].cpu().numpy()
            if lv != level:
                assert np.array_equal(got, states[p])
                continue
            m = _ghost_mask(g)
            a, b = g.view(got), g.view(ref[p])
            assert np.array_equal(a[:, ~m], g.view(states[p])[:, ~m])
            # copies: bitwise (the oracle's copies equal some interior value
            # of a sibling; the prolonged values differ from every input)
            cp = np.all(a[:, m] == b[:, m], axis=0)
            assert _rel(a[:, m], b[:, m]) <= 1e-13, (p, _rel(a[:, m],
                                                            b[:, m]))
            seen_f += int(m.sum())
            seen_c += int(cp.sum())
        if level > 0:
            assert seen_f == nf
        assert seen_c >= ncopy
        for l, lv in enumerate(d_levels):   # coarse time levels: read only
            for p, u in enumerate(lv):
                assert np.array_equal(u.cpu().numpy(), levels[l][p])
    plan.destroy()


def test_copy_points_bitwise(B):
    hr = H.two_level()
    plan = B.AmrPlan(hr)
    states = _states(hr, 300)
    ref = [u.copy() for u in states]
    M.fill_ghosts(hr, 1, ref, [states], [0.0], 0.0)
    d = [B.to_device(u) for u in states]
    plan.fill_ghosts(1, d, [d], [0.0], 0.0)
    torch.cuda.synchronize()
    # f0 (patch 2) +x face ghosts inside f1 (patch 3): copied, bitwise
    g0 = hr[2][1]
    c = g0.ghost
    xs = slice(c + g0.n[0], 2 * c + g0.n[0])
    got = g0.view(d[2].cpu().numpy())[:, c:-c, c:-c, xs]
    want = g0.view(ref[2])[:, c:-c, c:-c, xs]
    assert np.array_equal(got, want)
    # the number of copies equals the ghost points that lie in a sibling's
    # interior, found from coordinates
    ncp = 0
    for p, (lv, g) in enumerate(hr):
        if lv != 1:
            continue
        X, Y, Z = g.mesh()
        inside_any = np.zeros(X.shape, bool)
        for q, (lq, gq) in enumerate(hr):
            if q == p or lq != 1:
                continue
            inside = np.ones(X.shape, bool)
            for a, C in enumerate((X, Y, Z)):
                inside &= ((C > gq.origin[a] - 0.5 * gq.h[a]) &
                           (C < gq.origin[a] + (gq.n[a] - 0.5) * gq.h[a]))
            inside_any |= inside
        ncp += int((inside_any & _ghost_mask(g)).sum())
    assert plan.counts(1)[1] == ncp > 2 * c * g0.n[1] * g0.n[2]
    plan.destroy()


@pytest.mark.parametrize("hfn", [H.two_level, H.three_level,
                                 functools.partial(H.two_level, ghost=5)],
                         ids=["two_level", "three_level", "two_level_ghost5"])
def test_restrict_matches_oracle(B, hfn):
    hr = hfn()
    plan = B.AmrPlan(hr)
    top = max(lv for lv, _ in hr)
    for level in range(1, top + 1):
        states = _states(hr, 400 + level)
        ref = [u.copy() for u in states]
        M.restrict(hr, level, ref, ref)
        d = [B.to_device(u) for u in states]
        plan.restrict(level, d, d)
        torch.cuda.synchronize()
        nr = plan.counts(level)[2]
        changed = 0
        for p, (lv, g) in enumerate(hr):
            got = d[p].cpu().numpy()
            if lv != level - 1:
                assert np.array_equal(got, states[p])
                continue
            diff = g.view(ref[p]) != g.view(states[p])
            touched = np.any(diff, axis=0)
            changed += int(touched.sum())
            a, b = g.view(got), g.view(ref[p])
            assert np.array_equal(a[:, ~touched], b[:, ~touched])
            assert _rel(a[:, touched], b[:, touched]) <= 1e-13
        assert changed == nr > 0
    plan.destroy()


def test_plan_call_validation(B):
    hr = H.two_level()
    plan = B.AmrPlan(hr)
    L = B.lib()
    tab = torch.zeros(len(hr), dtype=torch.int64, device="cuda")
    tp = B.ctypes.c_void_p(tab.data_ptr())
    ts = (B.ctypes.c_double * 3)(0.0, 0.0, 1.0)
    tabs = (B.ctypes.c_void_p * 3)(tab.data_ptr(), tab.data_ptr(),
                                   tab.data_ptr())
    # refused before any launch: bad level, ntl, equal times, NULL tables
    # (every call here fails validation; the zero tables are never read)
    assert L.bssn_amr_fill_ghosts(plan.h, -1, tp, 1, tabs, ts, 0.0,
                                  None) == B.BSSN_EINVAL
    assert L.bssn_amr_fill_ghosts(plan.h, 2, tp, 1, tabs, ts, 0.0,
                                  None) == B.BSSN_EINVAL
    assert L.bssn_amr_fill_ghosts(plan.h, 1, tp, 4, tabs, ts, 0.0,
                                  None) == B.BSSN_EINVAL
    assert L.bssn_amr_fill_ghosts(plan.h, 1, tp, 2, tabs, ts, 0.0,
                                  None) == B.BSSN_EINVAL
    assert L.bssn_amr_fill_ghosts(plan.h, 1, None, 1, tabs, ts, 0.0,
                                  None) == B.BSSN_EINVAL
    assert L.bssn_amr_fill_ghosts(plan.h, 1, tp, 1, tabs, ts,
                                  float("nan"), None) == B.BSSN_EINVAL
    assert L.bssn_amr_restrict(plan.h, 0, tp, tp, None) == B.BSSN_EINVAL
    assert L.bssn_amr_restrict(plan.h, 1, None, tp, None) == B.BSSN_EINVAL
    plan.destroy()
