"""Multipole coefficients on the GPU (bssn_multipole) against the oracle
(oracle/multipole.py), through the C ABI (needs an MI355X).

Both sides get the same grid functions (two slots of a seeded smooth
state).  Coefficients must match to 1e-12 of the largest coefficient: the
sums run over at most a few thousand products in a different order, and
the two sides take their Gauss-Legendre nodes from different routines
(Newton iteration in the kernel, numpy in the oracle), both converged to
rounding.  A polynomial field must give its textbook coefficient.
"""
import math

import numpy as np
import pytest

from oracle import multipole as MP
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


CASES = {
    # name: (centre, radius, spin, lmax, ntheta, nphi, imaginary part)
    "psi4-like-s-2": ((0.1, -0.05, 0.02), 1.3, -2, 6, 16, 32, True),
    "real-s0": ((0.0, 0.2, -0.1), 1.1, 0, 4, 9, 18, False),
    "beyond-the-grid-s2": ((0.0, 0.0, 0.0), 2.7, 2, 5, 12, 20, True),
    "one-point": ((0.05, 0.0, 0.0), 0.9, 0, 2, 1, 1, True),
}


@pytest.mark.parametrize("case", list(CASES))
def test_multipole_matches_oracle(B, case):
    c, r, s, lmax, nt, nph, use_im = CASES[case]
    g = I.GridSpec((16, 15, 17), 3, (0.25,) * 3, (-2.0, -1.9, -2.1),
                   I.BC_STATIC)
    u = I.smooth_random(g, seed=61)
    v = g.view(u)
    re, im = v[17], (v[7] if use_im else None)    # alpha and K
    want = MP.multipole(g, re, im, c, r, s, lmax, nt, nph)
    du = B.to_device(u)
    print(f"[multipole] {case}", flush=True)
    got = B.bssn_multipole(g, du, du if use_im else None, c, r, s, lmax, nt,
                           nph, re_slot=17, im_slot=7)
    scale = max(np.abs(want).max(), 1e-300)
    err = np.abs(got - want).max() / scale
    print(f"[multipole] {case}: max error / max |C| = {err:.2e}", flush=True)
    assert err <= 1e-12
    for l in range(abs(s)):
        assert np.all(got[l * l:(l + 1) ** 2] == 0)


def test_polynomial_field_textbook_coefficient(B):
    g = I.GridSpec((16, 15, 17), 3, (0.25,) * 3, (-2.0, -1.9, -2.1),
                   I.BC_STATIC)
    c, r = (0.1, -0.05, 0.02), 1.3
    u = g.empty()
    X, Y, Z = g.mesh()
    g.view(u)[0] = Z - c[2]
    got = B.bssn_multipole(g, B.to_device(u), None, c, r, 0, 3, 6, 12)
    want = np.zeros(16, complex)
    want[2] = r ** 3 * math.sqrt(4 * math.pi / 3)
    assert np.allclose(got, want, rtol=0, atol=1e-12), got


def test_maximum_sizes_closed_form(B):
    """ntheta = 1024, nphi = 4096, l <= 16: the field z - c_z still projects
    onto C^{10} = r^3 sqrt(4 pi / 3) alone.  Goldberg's alternating sum
    loses digits at high l (about 1e-12 absolute at l = 16 against scipy's
    harmonics), hence 1e-9 of C^{10} for the other coefficients."""
    g = I.GridSpec((16, 15, 17), 3, (0.25,) * 3, (-2.0, -1.9, -2.1),
                   I.BC_STATIC)
    c, r = (0.1, -0.05, 0.02), 1.3
    u = g.empty()
    X, Y, Z = g.mesh()
    g.view(u)[0] = Z - c[2]
    print("[multipole] maximum sizes", flush=True)
    got = B.bssn_multipole(g, B.to_device(u), None, c, r, 0, 16, 1024, 4096)
    c10 = r ** 3 * math.sqrt(4 * math.pi / 3)
    assert abs(got[2] - c10) <= 1e-12 * c10
    rest = np.delete(got, 2)
    print(f"[multipole] maximum sizes: max |other C| / C10 = "
          f"{np.abs(rest).max() / c10:.2e}", flush=True)
    assert np.abs(rest).max() <= 1e-9 * c10
