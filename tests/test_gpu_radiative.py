"""Radiative outer boundary on the GPU (bssn_radiative_rhs) against the
oracle (oracle/radiative.py), through the C ABI (needs an MI355X).

Both sides get the same input: the state and an interior right-hand side
made by the oracle.  The ghost layers must match to 1e-12 relative per slot
(normwise over the boundary points), and the interior must come back
unchanged.  One classical RK4 step with evolved boundary points (interior
from bssn_rhs, boundary from bssn_radiative_rhs, the update in torch)
matches the same step built from the oracle's pieces.
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


CASES = {
    "bl-puncture-32": (
        lambda: I.cell_centred(32, -4, 4, 3),
        lambda g: I.brill_lindquist(g, (1.0,), ((0.1, -0.2, 0.05),)), 4),
    "smooth-ragged": (
        lambda: I.GridSpec((37, 22, 17), 3, (0.11, 0.13, 0.12),
                           (-2.1, -1.4, -0.9), I.BC_STATIC),
        lambda g: I.smooth_random(g, seed=21), 4),
    "smooth-off-origin-ghost5": (
        lambda: I.GridSpec((23, 18, 29), 5, (0.1, 0.12, 0.09),
                           (1.3, 0.4, -1.1), I.BC_STATIC),
        lambda g: I.smooth_random(g, seed=22), 8),
}


def _boundary(g):
    layer, _ = R.layers(g)
    return layer > 0


@pytest.mark.parametrize("case", list(CASES))
def test_radiative_matches_oracle(B, case):
    gfn, dfn, order = CASES[case]
    g = gfn()
    u = dfn(g)
    x0, v0 = np.array(B.RADIATIVE_X0), np.array(B.RADIATIVE_V0)
    rhs_in = O.rhs(g, O.params(fd_order=order), u)   # interior from the oracle
    ref = R.radiative_rhs(g, u, rhs_in, x0, v0, 2)
    du = B.to_device(u)
    dr = B.to_device(rhs_in)
    print(f"[radiative] {case} n={g.n} ghost={g.ghost}", flush=True)
    B.bssn_radiative_rhs(g, du, dr)
    torch.cuda.synchronize()
    got = dr.cpu().numpy()
    assert np.array_equal(g.interior(got), g.interior(rhs_in))
    m = _boundary(g)
    a, b = g.view(got)[:, m], g.view(ref)[:, m]
    D = np.abs(b).max(1)
    D = np.where(D > 0, D, D.max())
    e = np.abs(a - b).max(1) / D
    assert np.all(e <= 1e-12), (e.max(), int(e.argmax()))
    # the state is only read
    assert np.array_equal(du.cpu().numpy(), u)


def test_rk4_step_with_radiative_boundary(B):
    g = I.cell_centred(20, -3, 3, 3)
    u0 = I.brill_lindquist(g, (0.8,), ((0.2, 0.1, -0.1),))
    x0, v0 = np.array(B.RADIATIVE_X0), np.array(B.RADIATIVE_V0)
    prm = O.params()
    dt = 0.25 * g.h[0]

    def f_oracle(u):
        return R.radiative_rhs(g, u, O.rhs(g, prm, u), x0, v0, 2)

    # reference: classical RK4 on every storage point from the oracle
    k1 = f_oracle(u0)
    k2 = f_oracle(u0 + 0.5 * dt * k1)
    k3 = f_oracle(u0 + 0.5 * dt * k2)
    k4 = f_oracle(u0 + dt * k3)
    ref = u0 + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)

    bp = B.Params()
    du = B.to_device(u0)

    def f_gpu(u):
        k = torch.zeros_like(u)
        B.bssn_rhs(g, bp, u, k)
        B.bssn_radiative_rhs(g, u, k)
        return k

    g1 = f_gpu(du)
    g2 = f_gpu(du + 0.5 * dt * g1)
    g3 = f_gpu(du + 0.5 * dt * g2)
    g4 = f_gpu(du + dt * g3)
    got = (du + dt / 6.0 * (g1 + 2 * g2 + 2 * g3 + g4)).cpu().numpy()
    torch.cuda.synchronize()
    # the increment is compared (the state is O(1), its change O(dt))
    inc_ref = g.view(ref - u0)
    inc_got = g.view(got - u0)
    D = np.abs(inc_ref).reshape(25, -1).max(1)
    D = np.where(D > 0, D, D.max())
    e = np.abs(inc_got - inc_ref).reshape(25, -1).max(1) / D
    print(f"[radiative] RK4 step, max normwise increment error {e.max():.2e}",
          flush=True)
    assert np.all(e <= 1e-11), (e.max(), int(e.argmax()))
    m = _boundary(g)
    assert np.abs(inc_ref[:, m]).max() > 0   # the boundary does evolve
