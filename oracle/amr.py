"""Mesh-refinement glue between patches of a refinement hierarchy, plain
numpy/Python in FP64.  Test infrastructure only.

It follows the mesh-refinement part of the paper's section on the Cactus
framework and Carpet (Berger-Oliger time stepping with subcycling, and the
figure that shows its time stepping and fine-grid boundaries):
  * a refined level has half the spacing of the next coarser one, in space
    and in time, and takes two steps for each coarse step;
  * the boundary points of a refined patch are filled by interpolation from
    the coarser level, in space and in time;
  * after the fine steps the fine solution is put back into the coarse grid
    where the two overlap.

Readings (the paper names neither the orders nor the grid staggering):
  * patches are cell-centred grids (state layout of the main kernels); a
    fine cell is one eighth of a coarse cell, so a fine point lies a
    quarter of a coarse spacing from a coarse point along each axis;
  * a ghost point of a level-0 patch that lies in another level-0 patch's
    interior takes that patch's value (the first in list order); the
    other level-0 ghosts are the physical boundary and are left alone;
  * a ghost point of a patch on level L >= 1 takes, in this order:
      1. the value of the first other patch of level L (in list order)
         whose interior holds the same point (a copy);
      2. else the prolongation from the first patch of level L - 1 whose
         storage grid (ghosts included) holds the 4 x 4 x 4 block of
         points used: tricubic Lagrange interpolation on the coarse points
         floor(s) - 1 .. floor(s) + 2 per axis (s the point's coordinate in
         coarse index units), in time by Lagrange interpolation through the
         given coarse time levels (one, two or three);
    every ghost point must be covered by one of the two;
  * restriction: an interior point of a level L - 1 patch whose eight
    children (the fine points at +-h_f/2 per axis) lie in the interior of a
    level-L patch (the first in list order) takes the tricubic Lagrange
    interpolation of that patch's storage at its position: weights
    (-1, 9, 9, -1)/16 on the fine points two below to two above per axis.

A patch is a GridSpec-like object (n, ghost, h, origin, and the layout
strides); a hierarchy is a list of (level, grid) pairs, and states are flat
arrays in the same order.
"""
import math

import numpy as np

NSLOT = 25


def lagrange(t, nodes):
    """Weights of the polynomial through the given nodes, at t."""
    w = []
    for m, xm in enumerate(nodes):
        p = 1.0
        for l, xl in enumerate(nodes):
            if l != m:
                p *= (t - xl) / (xm - xl)
        w.append(p)
    return w


def _view(grid, flat):
    ex = [grid.n[a] + 2 * grid.ghost for a in range(3)]
    a = flat[grid.off0:grid.off0 + NSLOT * grid.sf]
    return a.reshape(NSLOT, ex[2], grid.sz // grid.sy, grid.sy)[
        :, :, :ex[1], :ex[0]]


def _coord(grid, idx, a):
    """Coordinate of storage index idx along axis a."""
    return grid.origin[a] + (idx - grid.ghost) * grid.h[a]


def _index_of(grid, x, interior):
    """Storage index of the point at coordinate x (3 values) if grid has a
    point there (within a thousandth of a spacing), and it lies in the
    interior (interior=True) or anywhere in the storage grid; else None."""
    out = []
    for a in range(3):
        s = (x[a] - grid.origin[a]) / grid.h[a]
        k = round(s)
        if abs(s - k) > 1e-3:
            return None
        lo, hi = (0, grid.n[a] - 1) if interior else (
            -grid.ghost, grid.n[a] + grid.ghost - 1)
        if not lo <= k <= hi:
            return None
        out.append(k + grid.ghost)
    return tuple(out)


def _ghost_points(grid):
    """Storage indices (i, j, k) of every ghost point of grid."""
    g = grid.ghost
    for k in range(grid.n[2] + 2 * g):
        for j in range(grid.n[1] + 2 * g):
            for i in range(grid.n[0] + 2 * g):
                if (g <= i < g + grid.n[0] and g <= j < g + grid.n[1]
                        and g <= k < g + grid.n[2]):
                    continue
                yield i, j, k


def _prolong_block(cgrid, x):
    """(base storage index per axis, weights per axis) of the tricubic
    interpolation at x from cgrid, or None if the block leaves cgrid."""
    base, wts = [], []
    for a in range(3):
        s = (x[a] - _coord(cgrid, 0, a)) / cgrid.h[a]
        b = math.floor(s) - 1
        if b < 0 or b + 3 > cgrid.n[a] + 2 * cgrid.ghost - 1:
            return None
        base.append(b)
        wts.append(lagrange(s - b, [0, 1, 2, 3]))
    return base, wts


def ghost_value(hier, level, states, coarse_states, tw, p, i, j, k):
    """The value (all slots) of ghost point (i, j, k) of patch p on level
    `level`: a sibling's copy, or the prolongation with time weights tw;
    None for a level-0 ghost that no sibling covers."""
    grid = hier[p][1]
    x = [_coord(grid, (i, j, k)[a], a) for a in range(3)]
    for q, (lq, gq) in enumerate(hier):
        if q == p or lq != level:
            continue
        idx = _index_of(gq, x, interior=True)
        if idx is not None:
            src = _view(gq, states[q])
            return src[:, idx[2], idx[1], idx[0]].copy()
    if level == 0:
        return None
    for q, (lq, gq) in enumerate(hier):
        if lq != level - 1:
            continue
        blk = _prolong_block(gq, x)
        if blk is None:
            continue
        (bx, by, bz), (wx, wy, wz) = blk
        val = np.zeros(NSLOT)
        for tl, w_t in enumerate(tw):
            c = _view(gq, coarse_states[tl][q])
            acc = np.zeros(NSLOT)
            for kk in range(4):
                for jj in range(4):
                    for ii in range(4):
                        acc += (wz[kk] * wy[jj] * wx[ii] *
                                c[:, bz + kk, by + jj, bx + ii])
            val += w_t * acc
        return val
    raise ValueError(f"ghost point {x} of patch {p} not covered")


def fill_ghosts(hier, level, states, coarse_states, t_src, t):
    """Fill the ghost points of every level-`level` patch in place.

    hier           list of (level, grid)
    states         flat states, one per patch (those of level `level` are
                   filled; the others are not touched)
    coarse_states  list over coarse time levels of lists of flat states, one
                   per patch (those of level - 1 are read)
    t_src, t       the coarse time levels' times and the target time
    """
    tw = lagrange(t, list(t_src)) if level > 0 else []
    for p, (lev, grid) in enumerate(hier):
        if lev != level:
            continue
        dst = _view(grid, states[p])
        for (i, j, k) in _ghost_points(grid):
            val = ghost_value(hier, level, states, coarse_states, tw, p, i,
                              j, k)
            if val is not None:
                dst[:, k, j, i] = val
    return states


def restricted_value(hier, level, fine_states, c, i, j, k):
    """The restricted value (all slots) of interior point (i, j, k) of the
    level - 1 patch c, or None if no level-`level` interior holds its
    eight children."""
    w = lagrange(1.5, [0, 1, 2, 3])   # (-1, 9, 9, -1) / 16
    cg = hier[c][1]
    x = [_coord(cg, (i, j, k)[a], a) for a in range(3)]
    for f, (lf, fg) in enumerate(hier):
        if lf != level:
            continue
        lo = [x[a] - fg.h[a] / 2 for a in range(3)]
        hi = [x[a] + fg.h[a] / 2 for a in range(3)]
        ilo = _index_of(fg, lo, interior=True)
        if ilo is None or _index_of(fg, hi, True) is None:
            continue
        src = _view(fg, fine_states[f])
        b = [ilo[a] - 1 for a in range(3)]
        acc = np.zeros(NSLOT)
        for kk in range(4):
            for jj in range(4):
                for ii in range(4):
                    acc += (w[kk] * w[jj] * w[ii] *
                            src[:, b[2] + kk, b[1] + jj, b[0] + ii])
        return acc
    return None


def restrict(hier, level, fine_states, coarse_states):
    """Put the level-`level` solution back into the level - 1 patches (in
    place on coarse_states) where a coarse point's children lie in a fine
    interior."""
    for c, (lc, cg) in enumerate(hier):
        if lc != level - 1:
            continue
        dst = _view(cg, coarse_states[c])
        g = cg.ghost
        for k in range(g, g + cg.n[2]):
            for j in range(g, g + cg.n[1]):
                for i in range(g, g + cg.n[0]):
                    val = restricted_value(hier, level, fine_states, c, i, j,
                                           k)
                    if val is not None:
                        dst[:, k, j, i] = val
    return coarse_states
