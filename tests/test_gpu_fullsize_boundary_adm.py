"""The radiative boundary and the ADM -> BSSN conversion at the benchmark's
size (the 128^3 + 3 ghost grid on [-8, 8]^3, the bench's launch
configuration), against the oracle at every point (needs an MI355X).

Radiative: the Brill-Lindquist state and a seeded random interior
right-hand side; every boundary point to 1e-12 relative per slot
(normwise), the interior unchanged.  Conversion: smooth seeded ADM data
(non-zero K_ij and off-diagonal metric); every slot at interior points and
every slot but Gt on the ghosts to 1e-12, Gt on ghost layer k to
1e-12 * 15^(k-1) (the growth bound of the layered extrapolation).
"""
import numpy as np
import pytest

from oracle import adm as A
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
    return bssn


def _grid():
    return I.cell_centred(128, -8.0, 8.0, 3)


def test_radiative_full_size(B):
    g = _grid()
    u = I.brill_lindquist(g, (1.0,), ((0.0, 0.0, 0.0),))
    rng = np.random.default_rng(7)
    rhs = g.empty()
    g.interior(rhs)[:] = rng.standard_normal(g.interior(rhs).shape)
    x0, v0 = np.array(B.RADIATIVE_X0), np.array(B.RADIATIVE_V0)
    ref = R.radiative_rhs(g, u, rhs, x0, v0, 2)
    dr = B.to_device(rhs)
    print("[full] radiative 128^3", flush=True)
    B.bssn_radiative_rhs(g, B.to_device(u), dr)
    torch.cuda.synchronize()
    got = dr.cpu().numpy()
    assert np.array_equal(g.interior(got), g.interior(rhs))
    layer, _ = R.layers(g)
    m = layer > 0
    a, b = g.view(got)[:, m], g.view(ref)[:, m]
    D = np.abs(b).max(1)
    D = np.where(D > 0, D, D.max())
    e = (np.abs(a - b).max(1) / D).max()
    print(f"[full] radiative: {int(m.sum())} boundary points, max normwise "
          f"error {e:.2e}", flush=True)
    assert e <= 1e-12


def test_from_adm_full_size(B):
    g = _grid()
    rng = np.random.default_rng(8)
    X, Y, Z = g.mesh()
    adm = np.zeros(g.off0 + 16 * g.sf)
    v = g.view(adm, 16)
    for s in range(16):
        k = rng.uniform(0.1, 0.4, 3)
        ph = rng.uniform(0, 2 * np.pi)
        w = np.sin(k[0] * X + k[1] * Y + k[2] * Z + ph)
        v[s] = (1.0 + 0.2 * w if s in (0, 3, 5) else
                0.05 * w if s < 6 else 1.0 + 0.1 * w if s == 12 else 0.1 * w)
    del X, Y, Z
    ref = A.from_adm(g, adm, 4)
    du = torch.zeros(g.total, dtype=torch.float64, device="cuda")
    print("[full] ADM conversion 128^3", flush=True)
    B.bssn_from_adm(g, B.Params(), torch.from_numpy(adm).to("cuda"), du)
    torch.cuda.synchronize()
    a, b = g.view(du.cpu().numpy()), g.view(ref)
    D = np.abs(b).reshape(25, -1).max(1)
    D = np.where(D > 0, D, 1.0).reshape(25, 1, 1, 1)
    e = np.abs(a - b) / D
    layer, _ = R.layers(g)
    rest = [s for s in range(25) if not A.GAMX <= s < A.GAMX + 3]
    e_in, e_rest = e[:, layer == 0].max(), e[rest].max()
    print(f"[full] ADM: interior {e_in:.2e}, non-Gt slots {e_rest:.2e}",
          flush=True)
    assert e_in <= 1e-12 and e_rest <= 1e-12
    gam = slice(A.GAMX, A.GAMX + 3)
    for k in range(1, g.ghost + 1):
        ek = e[gam][:, layer == k].max()
        print(f"[full] ADM: Gt ghost layer {k}: {ek:.2e}", flush=True)
        assert ek <= 1e-12 * 15.0 ** (k - 1)
