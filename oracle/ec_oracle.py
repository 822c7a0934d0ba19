"""Per-level oracle (O1) for Euler-characteristic, perimeter, area and volume curves.

TEST INFRASTRUCTURE ONLY.  Nothing in the product imports this module; only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may call it.  It shares no code, table or constant with the HIP
library.

What it computes (Laky & Zavala, "A Fast and Scalable Computational Topology
Framework for the Euler Characteristic", Methodology section):

* Sublevel filtration, Eq. (2): at level c the active top cells (pixels in 2D,
  voxels in 3D) are those with value <= c.  A cell outside the field is never
  active (the "collar" discussed right after Table 1).  The superlevel
  filtration is the mirror of Eq. (2): value >= c, over falling c (the
  paper writes its sublevel sets with a minus mark, g^-_c, the superlevel sets
  being their counterpart); with integer levels the level index l stands for
  c = L - 1 - l.
* Including a face includes its edges and vertices (text after Eq. (2)), so the
  complex at a level is the union of the *closed* active cells
  (T-construction).  Its Euler characteristic is the alternating count of
  Eq. (1): chi = V - E + F (- C).  This is the 8-connected (2D) / 26-connected
  (3D) EC that the paper uses throughout (Methodology, connectivity paragraph).
* 4-connected (2D) EC is the alternating count of the complex whose vertices
  are the active pixels, whose edges join 4-neighbours and whose squares are
  fully active 2x2 blocks (V-construction).  Table 1's 4-C column is exactly
  this complex's per-vertex share.  3D 6-connectivity is not in the paper; it
  is the same construction one dimension up (vertices, face-adjacent edges,
  fully active axis-plane 2x2 squares, fully active 2x2x2 cubes).
* Perimeter (2D) is the number of unit lattice edges with exactly one active
  neighbouring pixel (Table 1 perimeter column, "computed from exterior
  edges").  Area is the number of active pixels.
* In 3D, "area" is the surface: unit faces with exactly one active voxel
  (Table 2 Area column); "volume" is the number of active voxels; "perimeter"
  is the crease measure, the sum over unit lattice edges of kappa(4 voxels
  around the edge), kappa = 1 for one or three active voxels, 2 for two
  diagonally opposite ones, 0 otherwise.  Table 2 does not define its
  Perimeter column; this reading reproduces every row of it.

The algorithm is the naive one the paper describes before introducing vertex
contributions (Methodology, paragraph before Eq. (3)): binarise the field at
every level and count cells, O(N * n_levels).  It is deliberately slow and
plain; numpy is used only for elementwise logic and sums.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "binarise",
    "ec_2d",
    "ec_3d",
    "perimeter_2d",
    "surface_3d",
    "crease_3d",
    "curves_per_level",
]


# --------------------------------------------------------------------------
# filtration
# --------------------------------------------------------------------------
def binarise(field: np.ndarray, level: int, thresholds=None, superlevel: bool = False,
             n_levels=None) -> np.ndarray:
    """Active cells at filtration level ``level`` (Eq. (2): value <= c).

    With ``thresholds`` None the levels are the integers themselves (the paper
    uses pixel values 0..M directly as levels).  Otherwise level index l means
    the float32 threshold ``thresholds[l]`` and a cell is active when
    ``float32(value) <= thresholds[l]``; NaN is never active.

    ``superlevel``: a cell is active when ``float32(value) >= thresholds[l]``
    (thresholds non-increasing); with integer levels (``thresholds`` None,
    ``n_levels`` given) when ``value >= n_levels - 1 - level``.
    """
    if superlevel:
        if thresholds is None:
            if n_levels is None:
                raise ValueError("integer superlevel levels need n_levels")
            return field.astype(np.int64) >= (int(n_levels) - 1 - int(level))
        t = np.float32(np.asarray(thresholds, dtype=np.float32)[level])
        return field.astype(np.float32) >= t
    if thresholds is None:
        return field <= level
    t = np.float32(np.asarray(thresholds, dtype=np.float32)[level])
    return field.astype(np.float32) <= t


def _pad(b: np.ndarray) -> np.ndarray:
    """Surround the active mask with one layer of never-active cells."""
    return np.pad(b, 1, mode="constant", constant_values=False)


# --------------------------------------------------------------------------
# 2D counts (Eq. (1) with C = 0)
# --------------------------------------------------------------------------
def ec_2d(b: np.ndarray, connectivity: int = 8) -> int:
    """Euler characteristic V - E + F of a binary image.

    connectivity 8: closure of the active closed unit squares.
    connectivity 4: active pixels as vertices, 4-neighbour pairs as edges,
    fully active 2x2 blocks as squares.
    """
    b = np.asarray(b, dtype=bool)
    if connectivity == 8:
        p = _pad(b)
        # lattice vertex (i, j), 0 <= i <= h, 0 <= j <= w, touches the pixels
        # (i-1..i, j-1..j); in padded coordinates p[i..i+1, j..j+1]
        v = p[:-1, :-1] | p[:-1, 1:] | p[1:, :-1] | p[1:, 1:]
        # horizontal lattice edge at row i between columns j and j+1: pixels
        # (i-1, j) and (i, j)  -> padded p[i, j+1] and p[i+1, j+1]
        eh = p[:-1, 1:-1] | p[1:, 1:-1]
        # vertical lattice edge at column j between rows i and i+1: pixels
        # (i, j-1) and (i, j)  -> padded p[i+1, j] and p[i+1, j+1]
        ev = p[1:-1, :-1] | p[1:-1, 1:]
        V = int(v.sum())
        E = int(eh.sum()) + int(ev.sum())
        F = int(b.sum())
        return V - E + F
    if connectivity == 4:
        V = int(b.sum())
        E = int((b[:, :-1] & b[:, 1:]).sum()) + int((b[:-1, :] & b[1:, :]).sum())
        F = int((b[:-1, :-1] & b[:-1, 1:] & b[1:, :-1] & b[1:, 1:]).sum())
        return V - E + F
    raise ValueError("2D connectivity must be 8 or 4")


def perimeter_2d(b: np.ndarray) -> int:
    """Unit lattice edges with exactly one active neighbouring pixel."""
    p = _pad(np.asarray(b, dtype=bool))
    return int((p[:, :-1] ^ p[:, 1:]).sum()) + int((p[:-1, :] ^ p[1:, :]).sum())


# --------------------------------------------------------------------------
# 3D counts (Eq. (1))
# --------------------------------------------------------------------------
def ec_3d(b: np.ndarray, connectivity: int = 26) -> int:
    """Euler characteristic V - E + F - C of a binary volume.

    connectivity 26: closure of the active closed unit cubes.
    connectivity 6: active voxels as vertices, face-adjacent pairs as edges,
    fully active axis-plane 2x2 blocks as squares, fully active 2x2x2 blocks
    as cubes.
    """
    b = np.asarray(b, dtype=bool)
    if connectivity == 26:
        p = _pad(b)  # shape (d+2, h+2, w+2), axes (z, y, x)
        # A lattice k-cell is present iff one of the voxels whose closure
        # contains it is active.  In padded coordinates the voxels around a
        # lattice element whose lower corner is (k, i, j) span index k..k+1
        # along every axis the element does NOT extend in, and index k+1
        # along every axis it does extend in.
        def any_over(sz, sy, sx):
            # sz/sy/sx: True  -> element extends along this axis (single voxel
            # layer, offset 1); False -> two voxel layers (offsets 0 and 1).
            out = None
            for dz in ((1,) if sz else (0, 1)):
                for dy in ((1,) if sy else (0, 1)):
                    for dx in ((1,) if sx else (0, 1)):
                        zs = slice(dz, p.shape[0] - (1 - dz) - (1 if sz else 0))
                        ys = slice(dy, p.shape[1] - (1 - dy) - (1 if sy else 0))
                        xs = slice(dx, p.shape[2] - (1 - dx) - (1 if sx else 0))
                        a = p[zs, ys, xs]
                        out = a if out is None else (out | a)
            return int(out.sum())

        V = any_over(False, False, False)
        E = any_over(False, False, True) + any_over(False, True, False) + any_over(True, False, False)
        F = any_over(False, True, True) + any_over(True, False, True) + any_over(True, True, False)
        C = int(b.sum())
        return V - E + F - C
    if connectivity == 6:
        V = int(b.sum())
        E = (int((b[:, :, :-1] & b[:, :, 1:]).sum())
             + int((b[:, :-1, :] & b[:, 1:, :]).sum())
             + int((b[:-1, :, :] & b[1:, :, :]).sum()))
        sq_xy = b[:, :-1, :-1] & b[:, :-1, 1:] & b[:, 1:, :-1] & b[:, 1:, 1:]
        sq_xz = b[:-1, :, :-1] & b[:-1, :, 1:] & b[1:, :, :-1] & b[1:, :, 1:]
        sq_yz = b[:-1, :-1, :] & b[:-1, 1:, :] & b[1:, :-1, :] & b[1:, 1:, :]
        F = int(sq_xy.sum()) + int(sq_xz.sum()) + int(sq_yz.sum())
        cube = (b[:-1, :-1, :-1] & b[:-1, :-1, 1:] & b[:-1, 1:, :-1] & b[:-1, 1:, 1:]
                & b[1:, :-1, :-1] & b[1:, :-1, 1:] & b[1:, 1:, :-1] & b[1:, 1:, 1:])
        C = int(cube.sum())
        return V - E + F - C
    raise ValueError("3D connectivity must be 26 or 6")


def surface_3d(b: np.ndarray) -> int:
    """Unit faces with exactly one active neighbouring voxel."""
    p = _pad(np.asarray(b, dtype=bool))
    return (int((p[:, :, :-1] ^ p[:, :, 1:]).sum())
            + int((p[:, :-1, :] ^ p[:, 1:, :]).sum())
            + int((p[:-1, :, :] ^ p[1:, :, :]).sum()))


def _kappa(q0, q1, q2, q3):
    """Crease weight of the 4 voxels around a lattice edge, listed cyclically.

    1 for one or three active, 2 for two diagonally opposite (q0,q2 or q1,q3),
    0 for none, four, or two side by side.
    """
    n = q0.astype(np.int64) + q1 + q2 + q3
    odd = (n == 1) | (n == 3)
    diag = (n == 2) & (q0 == q2)
    return odd.astype(np.int64) + 2 * diag.astype(np.int64)


def crease_3d(b: np.ndarray) -> int:
    """Sum over unit lattice edges of kappa(4 voxels around the edge)."""
    p = _pad(np.asarray(b, dtype=bool))
    total = 0
    # edges along x: the 4 voxels around them vary in (z, y)
    a = p[:, :, 1:-1]
    total += int(_kappa(a[:-1, :-1], a[:-1, 1:], a[1:, 1:], a[1:, :-1]).sum())
    # edges along y: vary in (z, x)
    a = p[:, 1:-1, :]
    total += int(_kappa(a[:-1, :, :-1], a[:-1, :, 1:], a[1:, :, 1:], a[1:, :, :-1]).sum())
    # edges along z: vary in (y, x)
    a = p[1:-1, :, :]
    total += int(_kappa(a[:, :-1, :-1], a[:, :-1, 1:], a[:, 1:, 1:], a[:, 1:, :-1]).sum())
    return total


# --------------------------------------------------------------------------
# curves
# --------------------------------------------------------------------------
def curves_per_level(field, n_levels: int, thresholds=None, connectivity=None,
                     levels=None, channels=("ec", "perimeter", "area", "volume"), superlevel: bool = False):
    """Binarise at every requested level and count (O(N) work per level).

    Returns a dict channel -> int64 array over ``levels`` (all n_levels by
    default).  2D channels: ec, perimeter, area.  3D channels: ec, perimeter
    (crease), area (surface), volume.
    """
    field = np.asarray(field)
    nd = field.ndim
    if nd not in (2, 3):
        raise ValueError("field must be 2D or 3D")
    if connectivity is None:
        connectivity = 8 if nd == 2 else 26
    if levels is None:
        levels = range(n_levels)
    levels = list(levels)
    want = [c for c in channels if not (nd == 2 and c == "volume")]
    out = {c: np.zeros(len(levels), dtype=np.int64) for c in want}
    for k, lvl in enumerate(levels):
        b = binarise(field, lvl, thresholds, superlevel, n_levels)
        if nd == 2:
            if "ec" in out:
                out["ec"][k] = ec_2d(b, connectivity)
            if "perimeter" in out:
                out["perimeter"][k] = perimeter_2d(b)
            if "area" in out:
                out["area"][k] = int(b.sum())
        else:
            if "ec" in out:
                out["ec"][k] = ec_3d(b, connectivity)
            if "perimeter" in out:
                out["perimeter"][k] = crease_3d(b)
            if "area" in out:
                out["area"][k] = surface_3d(b)
            if "volume" in out:
                out["volume"][k] = int(b.sum())
    return out
