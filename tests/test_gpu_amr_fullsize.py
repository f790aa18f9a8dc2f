"""Refinement glue at the benchmark's size and launch configuration (needs
an MI355X): three nested levels of the 128^3 + 3 ghost grid on [-8, 8]^3
(spacings h, h/2, h/4), three coarse time levels, one bssn_amr_fill_ghosts
call per refined level and one bssn_amr_restrict call per level pair.

Inputs are seeded normal values (the work does not depend on them).  The
oracle computes sampled outputs one by one (oracle.amr.ghost_value,
restricted_value): 300 ghost points per refined level and 300 restricted
points per pair, plus the faces, edges and corners of each shell, to
1e-13 relative per slot; the number of points each call changed must equal
the plan's counts.
"""
import numpy as np
import pytest

from oracle import amr as M
from paper_1111_3344_amd import inputs as I
from tests import amr_hier as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TS, T = [0.0, 1.0, 2.0], 1.25


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_full_size_fill_and_restrict_sampled():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_3344_amd import bssn as B
    B.lib()
    g = I.cell_centred(128, -8.0, 8.0, 3)
    hier = H.nested(g)
    rng = np.random.default_rng(20240)
    cur = [rng.standard_normal(gr.total) for _, gr in hier]
    tl = [[rng.standard_normal(gr.total) for _, gr in hier] for _ in TS]
    dcur = [B.to_device(x) for x in cur]
    dtl = [[B.to_device(x) for x in lv] for lv in tl]
    plan = B.AmrPlan(hier)
    tw = M.lagrange(T, TS)
    for level in (1, 2):
        print(f"[amr-full] fill level {level}", flush=True)
        plan.fill_ghosts(level, dcur, dtl, TS, T)
        torch.cuda.synchronize()
        gr = hier[level][1]
        got = gr.view(dcur[level].cpu().numpy())
        before = gr.view(cur[level])
        changed = int(np.any(got != before, axis=0).sum())
        assert changed == plan.counts(level)[0]
        N = [gr.n[a] + 2 * gr.ghost for a in range(3)]
        gh = gr.ghost
        pts = set()
        while len(pts) < 300:
            i, j, k = (int(rng.integers(0, N[a])) for a in range(3))
            if all(gh <= v < gh + gr.n[a] for a, v in enumerate((i, j, k))):
                continue
            pts.add((i, j, k))
        for i in (0, gh - 1, N[0] - 1):          # faces, edges, corners
            for j in (0, N[1] // 2, N[1] - 1):
                for k in (0, N[2] // 2, N[2] - 1):
                    if not (i == N[0] // 2 and j == N[1] // 2):
                        pts.add((i, j, k))
        err = 0.0
        for (i, j, k) in sorted(pts):
            want = M.ghost_value(hier, level, cur, tl, tw, level, i, j, k)
            err = max(err, _rel(got[:, k, j, i], want))
        print(f"[amr-full] fill level {level}: {len(pts)} sampled points, "
              f"max rel error {err:.2e}", flush=True)
        assert err <= 1e-13
    # restriction, level 1 into 0 first (it reads level 1 before the
    # second call writes it).  Sampled coarse points whose 4 x 4 x 4 fine
    # stencil lies in the fine interior, which the fills did not change, so
    # the oracle reads the test's own fine inputs; stencils that reach the
    # fine ghosts are covered by the whole-patch tests at small size.
    for level in (1, 2):
        print(f"[amr-full] restrict level {level}", flush=True)
        plan.restrict(level, dcur, dcur)
        torch.cuda.synchronize()
        cg = hier[level - 1][1]
        got = cg.view(dcur[level - 1].cpu().numpy())
        gh = cg.ghost
        lo, hi = gh + cg.n[0] // 4 + 1, gh + 3 * cg.n[0] // 4 - 1
        fine = [None] * len(hier)
        fine[level] = cur[level]
        err = 0.0
        for _ in range(300):
            i, j, k = (int(rng.integers(lo, hi)) for _ in range(3))
            want = M.restricted_value(hier, level, fine, level - 1, i, j, k)
            assert want is not None
            err = max(err, _rel(got[:, k, j, i], want))
        changed = int(np.any(got != cg.view(cur[level - 1]), axis=0).sum())
        print(f"[amr-full] restrict level {level}: max rel error {err:.2e}, "
              f"{changed} points changed", flush=True)
        assert err <= 1e-13
        # level 0 has no ghosts filled; level 1 also had its shell filled
        fills = plan.counts(level - 1)[0] if level - 1 > 0 else 0
        assert changed == plan.counts(level)[2] + fills
    plan.destroy()
