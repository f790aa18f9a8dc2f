"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module only lays out memory and draws or evaluates initial data; it holds
none of the evolution method's arithmetic (no derivative, no right-hand side,
no time step).  Both the HIP binding and the oracle's tests take the arrays
built here and nothing else.

Layout of one state buffer (structure of arrays, float64):
    element (slot, z, y, x) of the storage grid, ghosts included, sits at
    flat index  off0 + slot*sf + z*sz + y*sy + x
with sy a multiple of 16 elements and off0 chosen so that the first interior
point of every row (x = ghost) starts on a 128-byte boundary whenever the
flat buffer itself does.  ``view`` returns the 4-D (slot, z, y, x) window.

Initial data recipes (the paper's workloads, synthetic and seeded):
  * Minkowski (ADMBase defaults: unit metric, zero curvature, unit lapse,
    zero shift) plus uniform noise on every slot;
  * Brill-Lindquist punctures: the TwoPunctures split with zero extrinsic
    curvature, where the regular part is identically one, so
    psi = 1 + sum_a m_a / (2 r_a), taken here with a pre-collapsed lapse
    alpha = psi^-2 and zero shift;
  * Kasner (the Gowdy T^3 example with P = Q = lambda = 0), in BSSN variables
    at time t;
  * smooth seeded perturbations of every slot, used to make every term of the
    right-hand side non-zero in parity tests;
  * uneven AMR-style patches for the batched path.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

NSLOT = 25

# slot numbers (phi, gt_ij, K, At_ij, Gt^i, alpha, beta^i, B^i, A)
PHI, GXX, GXY, GXZ, GYY, GYZ, GZZ, TRK = 0, 1, 2, 3, 4, 5, 6, 7
AXX, AXY, AXZ, AYY, AYZ, AZZ = 8, 9, 10, 11, 12, 13
GAMX, GAMY, GAMZ, ALP, BETX, BETY, BETZ, BX, BY, BZ, ADOT = range(14, 25)
SLOT_NAMES = ["phi", "gxx", "gxy", "gxz", "gyy", "gyz", "gzz", "K",
              "Axx", "Axy", "Axz", "Ayy", "Ayz", "Azz", "Gamx", "Gamy",
              "Gamz", "alpha", "betax", "betay", "betaz", "Bx", "By", "Bz",
              "A"]

BC_STATIC, BC_PERIODIC = 0, 1


@dataclasses.dataclass(frozen=True)
class GridSpec:
    """A uniform Cartesian patch: interior points, ghost width, spacing."""

    n: tuple            # interior points (nx, ny, nz)
    ghost: int
    h: tuple            # spacing (hx, hy, hz)
    origin: tuple       # coordinate of interior point (0, 0, 0)
    bc: int = BC_STATIC

    @property
    def ext(self):
        g = self.ghost
        return (self.n[0] + 2 * g, self.n[1] + 2 * g, self.n[2] + 2 * g)

    @property
    def sy(self):
        return -(-self.ext[0] // 16) * 16

    @property
    def sz(self):
        return self.sy * self.ext[1]

    @property
    def sf(self):
        return self.sz * self.ext[2]

    @property
    def off0(self):
        return (16 - self.ghost % 16) % 16

    @property
    def total(self):
        """Elements of one flat buffer (front pad + 25 slots)."""
        return self.off0 + NSLOT * self.sf

    @property
    def npoints(self):
        return self.n[0] * self.n[1] * self.n[2]

    def empty(self):
        return np.zeros(self.total, dtype=np.float64)

    def view(self, flat, nslot=NSLOT):
        """(slot, z, y, x) window of a flat buffer, ghosts included."""
        ex = self.ext
        a = flat[self.off0:self.off0 + nslot * self.sf]
        return a.reshape(nslot, ex[2], ex[1], self.sy)[..., :ex[0]]

    def interior(self, flat, nslot=NSLOT):
        g = self.ghost
        v = self.view(flat, nslot)
        return v[:, g:g + self.n[2], g:g + self.n[1], g:g + self.n[0]]

    def body(self, flat):
        """Flat buffer without the front pad: element (0,0,0,0) first."""
        return flat[self.off0:]

    def coords(self):
        """1-D coordinates of every storage point along x, y, z."""
        g = self.ghost
        return tuple(self.origin[a] + (np.arange(self.ext[a]) - g) * self.h[a]
                     for a in range(3))

    def mesh(self):
        x, y, z = self.coords()
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        return X, Y, Z


def cell_centred(n, lo, hi, ghost, bc=BC_STATIC):
    """Grid of n^3 (or n=(nx,ny,nz)) cell-centred points on [lo, hi]^3."""
    if np.isscalar(n):
        n = (int(n),) * 3
    h = tuple((hi - lo) / n[a] for a in range(3))
    origin = tuple(lo + 0.5 * h[a] for a in range(3))
    return GridSpec(tuple(int(v) for v in n), int(ghost), h, origin, bc)


def fill_periodic_ghosts(grid, flat):
    """Copy interior values into the ghost layers periodically (in place)."""
    v = grid.view(flat)
    g = grid.ghost
    for ax in range(3):
        n = grid.n[ax]
        axis = 3 - ax
        ext = grid.ext[ax]
        idx = (np.arange(ext) - g) % n + g
        v[...] = np.take(v, idx, axis=axis)
    return flat


def minkowski(grid):
    flat = grid.empty()
    v = grid.view(flat)
    for s in (GXX, GYY, GZZ, ALP):
        v[s] = 1.0
    return flat


def minkowski_noise(grid, amp=1e-8, seed=11113344):
    """Minkowski plus U(-amp, amp) on all 25 slots at interior points, drawn
    in C order [slot][z][y][x]; periodic grids get periodic ghosts."""
    flat = minkowski(grid)
    rng = np.random.default_rng(seed)
    noise = rng.uniform(-amp, amp, size=(NSLOT, grid.n[2], grid.n[1],
                                          grid.n[0]))
    grid.interior(flat)[...] += noise
    if grid.bc == BC_PERIODIC:
        fill_periodic_ghosts(grid, flat)
    return flat


def brill_lindquist(grid, masses, centres, lapse="precollapsed"):
    """Brill-Lindquist punctures on every storage point (ghosts included):
    psi = 1 + sum m/(2 max(r, h/2)), phi = ln psi, gt = delta, K = At = 0,
    Gt = 0, alpha = psi^-2 (or 1), beta = B = A = 0."""
    flat = grid.empty()
    v = grid.view(flat)
    X, Y, Z = grid.mesh()
    rmin = 0.5 * min(grid.h)
    psi = np.ones_like(X)
    for m, c in zip(masses, centres):
        r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
        psi += m / (2.0 * np.maximum(r, rmin))
    v[PHI] = np.log(psi)
    for s in (GXX, GYY, GZZ):
        v[s] = 1.0
    v[ALP] = psi ** -2 if lapse == "precollapsed" else 1.0
    return flat


def kasner(grid, t=1.0):
    """Kasner metric dt^2 = -dt^2 + t^(4/3)(dx^2+dy^2) + t^(-2/3) dz^2 at time
    t, in BSSN variables (unit lapse, zero shift); spatially uniform."""
    flat = grid.empty()
    v = grid.view(flat)
    v[PHI] = math.log(t) / 6.0
    v[GXX] = v[GYY] = t ** (2.0 / 3.0)
    v[GZZ] = t ** (-4.0 / 3.0)
    v[TRK] = -1.0 / t
    v[AXX] = v[AYY] = -t ** (-1.0 / 3.0) / 3.0
    v[AZZ] = 2.0 * t ** (-7.0 / 3.0) / 3.0
    v[ALP] = 1.0
    return flat


# background and amplitude of the smooth perturbation of each slot
_SMOOTH = {
    PHI: (0.0, 0.1), GXX: (1.0, 0.08), GXY: (0.0, 0.05), GXZ: (0.0, 0.05),
    GYY: (1.0, 0.08), GYZ: (0.0, 0.05), GZZ: (1.0, 0.08), TRK: (0.0, 0.1),
    AXX: (0.0, 0.1), AXY: (0.0, 0.1), AXZ: (0.0, 0.1), AYY: (0.0, 0.1),
    AYZ: (0.0, 0.1), AZZ: (0.0, 0.1), GAMX: (0.0, 0.1), GAMY: (0.0, 0.1),
    GAMZ: (0.0, 0.1), ALP: (1.0, 0.3), BETX: (0.0, 0.3), BETY: (0.0, 0.3),
    BETZ: (0.0, 0.3), BX: (0.0, 0.1), BY: (0.0, 0.1), BZ: (0.0, 0.1),
    ADOT: (0.0, 0.1)}


def smooth_random(grid, seed=1, nmodes=3, kmax=2):
    """Every slot = background + amp * sum of nmodes seeded plane waves.
    Wave numbers are integer multiples of 2 pi / L (L = n h), so the data is
    periodic on a periodic grid; shifts change sign across the grid, metric
    stays positive definite and the lapse positive."""
    rng = np.random.default_rng(seed)
    flat = grid.empty()
    v = grid.view(flat)
    X, Y, Z = grid.mesh()
    L = [grid.n[a] * grid.h[a] for a in range(3)]
    for s in range(NSLOT):
        bg, amp = _SMOOTH[s]
        acc = np.zeros_like(X)
        for _ in range(nmodes):
            m = rng.integers(-kmax, kmax + 1, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            a = rng.uniform(0.5, 1.0) / nmodes
            acc += a * np.sin(2 * np.pi * (m[0] * X / L[0] + m[1] * Y / L[1]
                                           + m[2] * Z / L[2]) + ph)
        v[s] = bg + amp * acc
    return flat


def patches(npatch=256, seed=11113348, nlo=24, nhi=96, h=0.125, ghost=3):
    """Uneven AMR-style patches: interiors U{nlo..nhi} per axis, spacing h,
    centred on the origin; per patch a puncture of mass U[0.3, 1.0] at a
    centre drawn from U[-n h/4, n h/4] per axis.  Returns a list of
    (GridSpec, mass, centre)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(npatch):
        n = tuple(int(v) for v in rng.integers(nlo, nhi + 1, size=3))
        m = float(rng.uniform(0.3, 1.0))
        c = tuple(float(rng.uniform(-n[a] * h / 4, n[a] * h / 4))
                  for a in range(3))
        origin = tuple(-0.5 * n[a] * h + 0.5 * h for a in range(3))
        out.append((GridSpec(n, ghost, (h, h, h), origin, BC_STATIC), m, c))
    return out
