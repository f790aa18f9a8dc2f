"""Small two- and three-level cell-centred hierarchies for the refinement
tests (geometry only: no arithmetic of the method).

A fine patch of level L + 1 is placed by the coarse cell index m of its
first interior cell: origin_f = origin_c + (m - 1/4) h_c, h_f = h_c / 2, so
its points are the children of coarse cells m, m + 1, ...
"""
from paper_1111_3344_amd import inputs as I


def child(parent, m, nf, ghost=3):
    """Fine patch over the coarse cells m .. m + nf/2 - 1 of `parent`
    (coarse index units of the parent's interior)."""
    h = tuple(parent.h[a] / 2 for a in range(3))
    o = tuple(parent.origin[a] + (m[a] - 0.25) * parent.h[a]
              for a in range(3))
    return I.GridSpec(tuple(nf), ghost, h, o, I.BC_STATIC)


def sibling(grid, shift, n=None):
    """Patch on the same lattice as `grid`, its origin moved by `shift`
    points (integers per axis)."""
    o = tuple(grid.origin[a] + shift[a] * grid.h[a] for a in range(3))
    return I.GridSpec(tuple(n or grid.n), grid.ghost, grid.h, o,
                      I.BC_STATIC)


def two_level(h=0.2, ghost=3):
    """Two coarse patches side by side in x, three fine patches: two
    adjacent in x (each fills the other's face ghosts), one straddling the
    coarse seam."""
    c0 = I.GridSpec((12, 14, 13), ghost, (h, h, h), (-1.3, -1.1, -1.2),
                    I.BC_STATIC)
    c1 = sibling(c0, (12, 0, 0), (10, 14, 13))
    f0 = child(c0, (3, 3, 3), (8, 10, 8), ghost)
    f1 = sibling(f0, (8, 0, 0), (8, 10, 8))          # touches f0 at +x
    f2 = child(c0, (9, 8, 4), (10, 8, 10), ghost)    # straddles c0 | c1
    return [(0, c0), (0, c1), (1, f0), (1, f1), (1, f2)]


def three_level(h=0.2, ghost=3):
    c0 = I.GridSpec((14, 14, 14), ghost, (h, h, h), (-1.4, -1.3, -1.5),
                    I.BC_STATIC)
    f0 = child(c0, (3, 3, 4), (14, 12, 12), ghost)
    ff = child(f0, (3, 2, 3), (10, 12, 10), ghost)
    return [(0, c0), (1, f0), (2, ff)]


def bo_level(h=0.2, ghost=3):
    """Two coarse patches sharing a face (x), two fine siblings sharing a
    face, the fine region straddling the coarse seam: every kind of ghost
    source in a small hierarchy for time stepping."""
    c0 = I.GridSpec((8, 14, 14), ghost, (h, h, h), (-1.3, -1.3, -1.3),
                    I.BC_STATIC)
    c1 = sibling(c0, (8, 0, 0), (6, 14, 14))
    f0 = child(c0, (5, 5, 5), (6, 6, 6), ghost)
    f1 = sibling(f0, (6, 0, 0))
    return [(0, c0), (0, c1), (1, f0), (1, f1)]


def nested(g, nlevel=3):
    """Level 0 the grid g; level L + 1 a patch of the same size at half the
    spacing whose cells split the cells n/4 .. 3n/4 - 1 of level L."""
    hier = [(0, g)]
    for L in range(1, nlevel):
        par = hier[-1][1]
        hier.append((L, child(par, tuple(x // 4 for x in par.n), par.n,
                              par.ghost)))
    return hier
