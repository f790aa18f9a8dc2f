"""bssn_constraints_noalloc (the allocation-free constraints) against
bssn_constraints through the C ABI (needs an MI355X): the same fields and
norms, bitwise (same kernels, same partial records, fixed-order fold), on
two calls in a row, the second on a smaller grid, so that the shared device
array holds the first call's records when the second runs."""
import ctypes

import numpy as np
import pytest

from paper_1111_3344_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_3344_amd import bssn
    bssn.lib()
    return bssn


def _both(B, g, u, order, centres, r_exc):
    du = B.to_device(u)
    prm = B.Params(fd_order=order)
    res = []
    for fn in (B.bssn_constraints, B.bssn_constraints_noalloc):
        H, M, G = (torch.zeros_like(du) for _ in range(3))
        norms = torch.full((8,), -1.0, dtype=torch.float64, device="cuda")
        fn(g, prm, du, norms, H, M, G, centres, r_exc)
        torch.cuda.synchronize()
        res.append([x.cpu().numpy() for x in (norms, H, M, G)])
    return res


def test_noalloc_equals_allocating_entry_point_twice(B):
    cases = [
        (I.GridSpec((150, 97, 61), 3, (0.1, 0.11, 0.12), (-7.0, -5.0, -3.5),
                    I.BC_STATIC), 4, [(1.0, 0.5, 0.0), (-2.0, 0.0, 0.3)], 0.8),
        (I.GridSpec((40, 21, 13), 5, (0.1, 0.1, 0.1), (-2.0, -1.0, -0.6),
                    I.BC_STATIC), 8, [(0.1, 0.0, 0.0)], 0.3),
    ]
    for g, order, centres, r_exc in cases:
        print(f"[noalloc] n={g.n} order={order}", flush=True)
        u = I.smooth_random(g, seed=3 + order)  # H, M and G all non-zero
        (n0, H0, M0, G0), (n1, H1, M1, G1) = _both(B, g, u, order, centres,
                                                   r_exc)
        assert n0[6] > 0 and np.isfinite(n0).all()
        assert n0[0] > 0 and n0[2] > 0 and n0[4] > 0
        assert np.array_equal(n0, n1), (n0, n1)
        for a, b in ((H0, H1), (M0, M1), (G0, G1)):
            assert np.array_equal(a, b)
