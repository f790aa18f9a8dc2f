"""ADM -> BSSN initial conversion on the GPU (bssn_from_adm) against the
oracle (oracle/adm.py), through the C ABI (needs an MI355X).

Every slot at every interior point, and every slot but Gt on the ghost
layers, must match the oracle to 1e-12 relative per slot (normwise); Gt on
ghost layer k to 1e-12 * 15^(k-1), the growth bound of the layered cubic
extrapolation;
Brill-Lindquist ADM data must give the closed-form BSSN state that the
input module builds directly (phi = ln psi, conformally flat, Gt = 0).
Puncture tracking (bssn_track_punctures) must move positions inside, near
and beyond the edge of the storage grid as the oracle does, to 1e-13 of the
coordinates' size.
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


def _adm_smooth(g, seed):
    rng = np.random.default_rng(seed)
    X, Y, Z = g.mesh()
    adm = np.zeros(g.off0 + 16 * g.sf)
    v = g.view(adm, 16)
    for s in range(16):
        k = rng.uniform(0.5, 1.5, 3)
        ph = rng.uniform(0, 2 * np.pi)
        w = np.sin(k[0] * X + k[1] * Y + k[2] * Z + ph)
        v[s] = (1.0 + 0.2 * w if s in (0, 3, 5) else
                0.05 * w if s < 6 else 1.0 + 0.1 * w if s == 12 else 0.1 * w)
    return adm


CASES = {
    "smooth-ragged-order4": (
        lambda: I.GridSpec((29, 18, 13), 3, (0.11, 0.13, 0.12),
                           (-1.6, -1.2, -0.7), I.BC_STATIC), 4, 31),
    "smooth-order8": (
        lambda: I.GridSpec((21, 16, 19), 5, (0.1, 0.12, 0.09),
                           (-1.0, -0.9, -0.8), I.BC_STATIC), 8, 32),
}


@pytest.mark.parametrize("case", list(CASES))
def test_from_adm_matches_oracle(B, case):
    gfn, order, seed = CASES[case]
    g = gfn()
    adm = _adm_smooth(g, seed)
    ref = A.from_adm(g, adm, order)
    dadm = torch.from_numpy(adm).to("cuda")
    du = torch.zeros(g.total, dtype=torch.float64, device="cuda")
    print(f"[adm] {case} n={g.n} ghost={g.ghost}", flush=True)
    B.bssn_from_adm(g, B.Params(fd_order=order), dadm, du)
    torch.cuda.synchronize()
    got = du.cpu().numpy()
    a, b = g.view(got), g.view(ref)
    D = np.abs(b).reshape(25, -1).max(1)
    D = np.where(D > 0, D, 1.0)
    e = np.abs(a - b) / D.reshape(25, 1, 1, 1)
    # interior points (every slot) and every slot but Gt: 1e-12
    layer, _ = R.layers(g)
    gam = slice(A.GAMX, A.GAMX + 3)
    assert e[:, layer == 0].max() <= 1e-12, e[:, layer == 0].max()
    rest = [s for s in range(25) if not A.GAMX <= s < A.GAMX + 3]
    assert e[rest].max() <= 1e-12, e[rest].max()
    # Gt on ghost layer k: each cubic extrapolation step multiplies a
    # difference of its inputs by at most |4| + |6| + |4| + |1| = 15, so the
    # rounding differences of the interior grow by up to 15 per layer
    for k in range(1, g.ghost + 1):
        ek = e[gam][:, layer == k].max()
        print(f"[adm] {case} ghost layer {k}: Gt error {ek:.2e}", flush=True)
        assert ek <= 1e-12 * 15.0 ** (k - 1), (k, ek)
    assert np.array_equal(dadm.cpu().numpy(), adm)   # input only read


def test_brill_lindquist_adm_gives_the_bssn_data(B):
    g = I.cell_centred(40, -4, 4, 3)
    m, c = (0.7, 0.3), ((0.6, 0.2, -0.1), (-0.9, -0.3, 0.4))
    X, Y, Z = g.mesh()
    psi = 1.0 + sum(mi / (2 * np.maximum(np.sqrt((X - ci[0]) ** 2 +
                                                 (Y - ci[1]) ** 2 +
                                                 (Z - ci[2]) ** 2),
                                         0.5 * g.h[0]))
                    for mi, ci in zip(m, c))
    adm = np.zeros(g.off0 + 16 * g.sf)
    v = g.view(adm, 16)
    for s in (0, 3, 5):
        v[s] = psi ** 4
    v[12] = psi ** -2
    du = torch.zeros(g.total, dtype=torch.float64, device="cuda")
    B.bssn_from_adm(g, B.Params(), torch.from_numpy(adm).to("cuda"), du)
    torch.cuda.synchronize()
    got = g.view(du.cpu().numpy())
    want = g.view(I.brill_lindquist(g, m, c))
    err = np.abs(got - want).reshape(25, -1).max(1)
    print(f"[adm] Brill-Lindquist: max |converted - closed form| per slot "
          f"{err.max():.2e}", flush=True)
    # Gt is 0 in exact arithmetic; the differences of gt = 1 + rounding give
    # ~1e-14, and each extrapolated layer multiplies that by up to 15
    gam = [I.GAMX, I.GAMY, I.GAMZ]
    other = [s for s in range(25) if s not in gam]
    assert np.all(err[other] <= 1e-12), (err[other].max(),)
    assert np.all(err[gam] <= 1e-9), (err[gam].max(),)


def test_track_punctures_matches_oracle(B):
    g = I.GridSpec((21, 18, 25), 3, (0.2, 0.15, 0.25), (-2.1, -1.3, -3.0),
                   I.BC_STATIC)
    u = I.smooth_random(g, seed=41)
    rng = np.random.default_rng(8)
    lo = np.array([g.origin[a] - g.ghost * g.h[a] for a in range(3)])
    hi = np.array([g.origin[a] + (g.n[a] + g.ghost - 1) * g.h[a]
                   for a in range(3)])
    pos = rng.uniform(lo - 0.3, hi + 0.3, size=(50, 3))   # some outside
    pos[0] = [g.origin[a] + 4 * g.h[a] for a in range(3)]  # on a node
    dt = 0.07
    want = A.track_punctures(g, u, pos, dt)
    dpos = torch.from_numpy(pos.copy()).to("cuda")
    B.bssn_track_punctures(g, B.to_device(u), dpos, dt)
    torch.cuda.synchronize()
    got = dpos.cpu().numpy()
    step = np.abs(want - pos).max()
    assert np.abs(got - want).max() <= 1e-13 * max(1.0, np.abs(pos).max())
    assert step > 0
