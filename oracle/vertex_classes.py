"""Oracle for the vertex class counts per level (TEST INFRASTRUCTURE ONLY).

Nothing in the product imports this module; only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s checks may call it.  It shares
no code, table or constant with the HIP library.

What it computes (Laky & Zavala, Methodology: vertex contributions, Table 1
and Eq. (4)): every lattice vertex (i, j), 0 <= i <= h, 0 <= j <= w, is the
common corner of the up to four pixels (i-1..i, j-1..j); pixels outside the
field are never active (the collar after Table 1).  At a level the active
pixels among those four form the vertex's quadrant configuration, which Table 1
sorts by shape:

    class 0  one pixel
    class 1  two pixels sharing an edge
    class 2  two pixels on a diagonal
    class 3  three pixels
    class 4  four pixels

(an empty quadrant is in no class).  The counts of vertices in each class, for
every level, are the "contribution map": each column of Table 1 is a fixed
weighting of them.

Two implementations of the same definition:

* ``vertex_classes_per_level``: binarise at every level (Eq. (2)) and classify
  every vertex's quadrant; O(N * levels).
* ``vertex_classes_2d``: each vertex's quadrant only changes at the levels of
  its four pixels, so each vertex adds +1 to its new class and -1 to its old
  class at each of those levels; the counts are the running sums.  O(N + L).

3D (Table 2): the vertex (k, i, j) is the corner of the up to eight voxels
(k-1..k, i-1..i, j-1..j), its octant mask has bit dx + 2 dy + 4 dz for the
voxel at offset (dz, dy, dx) from (k-1, i-1, j-1), and its class is the orbit
of that mask under the 48 symmetries of the cube (Table 2 lists one row per
orbit).  The 21 non-empty orbits are numbered by (number of voxels, smallest
mask in the orbit).  ``vertex_classes_3d`` and ``vertex_classes_3d_per_level``
are the two forms above, one dimension up.
"""
from __future__ import annotations

import numpy as np

from .ec_oracle import binarise

CLASSES = ("one", "adjacent", "diagonal", "three", "four")


def quadrant_class(mask: int) -> int:
    """Class of a quadrant given as a 4-bit mask: bit 0 = pixel (i-1, j-1),
    bit 1 = (i-1, j), bit 2 = (i, j-1), bit 3 = (i, j); -1 when empty."""
    n = bin(mask).count("1")
    if n == 0:
        return -1
    if n == 2:
        # the two pixels share an edge unless they are (i-1,j-1)+(i,j) or (i-1,j)+(i,j-1)
        return 2 if mask in (0b1001, 0b0110) else 1
    return {1: 0, 3: 3, 4: 4}[n]


_CLASS_OF_MASK = np.array([quadrant_class(m) for m in range(16)], dtype=np.int64)


def _quadrant_masks(b: np.ndarray) -> np.ndarray:
    """4-bit quadrant mask of every lattice vertex of an active-pixel mask."""
    p = np.pad(b.astype(np.int64), 1, mode="constant", constant_values=0)
    return p[:-1, :-1] | (p[:-1, 1:] << 1) | (p[1:, :-1] << 2) | (p[1:, 1:] << 3)


def vertex_classes_per_level(field, n_levels: int, thresholds=None, superlevel: bool = False) -> np.ndarray:
    """[5, n_levels] int64: vertices per class at each level, by binarising at
    every level and classifying every quadrant."""
    field = np.asarray(field)
    if field.ndim != 2:
        raise ValueError("vertex classes are defined here for 2D fields")
    out = np.zeros((5, n_levels), dtype=np.int64)
    for lvl in range(n_levels):
        cls = _CLASS_OF_MASK[_quadrant_masks(binarise(field, lvl, thresholds, superlevel, n_levels))]
        for c in range(5):
            out[c, lvl] = int(np.count_nonzero(cls == c))
    return out


def level_index(field, n_levels: int, thresholds=None, superlevel: bool = False) -> np.ndarray:
    """Level at which each pixel becomes active (Eq. (2)); n_levels for never.

    Integer levels: the value itself when below n_levels.  Thresholds: the
    first l with float32(value) <= thresholds[l] (NaN never).  Superlevel: the
    first l with value >= t_l (non-increasing thresholds; integer levels
    t_l = n_levels - 1 - l)."""
    field = np.asarray(field)
    if superlevel:
        L = int(n_levels)
        if thresholds is None:
            v = field.astype(np.int64)
            return np.maximum(L - 1 - v, 0)
        t = np.asarray(thresholds, dtype=np.float32)
        x = field.astype(np.float32)
        lam = np.full(x.shape, L, dtype=np.int64)
        for lvl in range(L - 1, -1, -1):  # the first (smallest) l that holds wins
            lam[x >= t[lvl]] = lvl
        return lam
    if thresholds is None:
        v = field.astype(np.int64)
        return np.where(v < n_levels, v, n_levels)
    t = np.asarray(thresholds, dtype=np.float32)
    x = field.astype(np.float32)
    lam = np.searchsorted(t, x, side="left").astype(np.int64)
    lam[np.isnan(x)] = n_levels
    return lam


def vertex_classes_2d(field, n_levels: int, thresholds=None, superlevel: bool = False) -> np.ndarray:
    """[5, n_levels] int64 class counts from the per-vertex class changes."""
    field = np.asarray(field)
    if field.ndim != 2:
        raise ValueError("vertex classes are defined here for 2D fields")
    L = int(n_levels)
    lam = np.pad(level_index(field, L, thresholds, superlevel), 1, mode="constant", constant_values=L)
    # the four pixel levels around every vertex, in mask-bit order
    q = [lam[:-1, :-1].ravel(), lam[:-1, 1:].ravel(), lam[1:, :-1].ravel(), lam[1:, 1:].ravel()]
    hist = np.zeros((5, L + 1), dtype=np.int64)
    for k in range(4):  # the quadrant as it is once pixel k is active
        at = q[k]
        mask = sum(((q[b] <= at).astype(np.int64) << b) for b in range(4))
        before = sum(((q[b] < at).astype(np.int64) << b) for b in range(4))
        # pixels tied with pixel k enter together: count the change once, at
        # the lowest-numbered pixel of the tie
        first = np.ones_like(at, dtype=bool)
        for b in range(k):
            first &= q[b] != at
        sel = first & (at < L)
        new_c, old_c, lv = _CLASS_OF_MASK[mask[sel]], _CLASS_OF_MASK[before[sel]], at[sel]
        np.add.at(hist, (new_c, lv), 1)
        has_old = old_c >= 0
        np.add.at(hist, (old_c[has_old], lv[has_old]), -1)
    return np.cumsum(hist[:, :L], axis=1)


# --------------------------------------------------------------------------
# 3D
# --------------------------------------------------------------------------
def _cube_symmetries():
    """The 48 maps of octant bit positions: axis permutations with reflections."""
    import itertools
    maps = []
    for perm in itertools.permutations(range(3)):
        for flips in itertools.product((0, 1), repeat=3):
            m = []
            for b in range(8):
                c = (b & 1, b >> 1 & 1, b >> 2 & 1)
                c2 = [c[perm[a]] ^ flips[a] for a in range(3)]
                m.append(c2[0] + 2 * c2[1] + 4 * c2[2])
            maps.append(m)
    return maps


def _octant_classes():
    syms = _cube_symmetries()
    smallest = {}
    for mask in range(256):
        smallest[mask] = min(sum(1 << m[b] for b in range(8) if mask >> b & 1) for m in syms)
    reps = sorted({v for k, v in smallest.items() if k}, key=lambda r: (bin(r).count("1"), r))
    table = np.full(256, -1, dtype=np.int64)
    for mask in range(1, 256):
        table[mask] = reps.index(smallest[mask])
    return table


_CLASS_OF_OCTANT = _octant_classes()
N_CLASSES_3D = 21


def octant_class(mask: int) -> int:
    """Class (0..20) of a 3D octant mask, -1 when empty."""
    return int(_CLASS_OF_OCTANT[mask])


def _octant_masks(b: np.ndarray) -> np.ndarray:
    p = np.pad(b.astype(np.int64), 1, mode="constant", constant_values=0)
    m = np.zeros(tuple(s - 1 for s in p.shape), dtype=np.int64)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                sl = p[dz:p.shape[0] - 1 + dz, dy:p.shape[1] - 1 + dy, dx:p.shape[2] - 1 + dx]
                m |= sl << (dx + 2 * dy + 4 * dz)
    return m


def vertex_classes_3d_per_level(field, n_levels: int, thresholds=None, superlevel: bool = False) -> np.ndarray:
    """[21, n_levels] int64: vertices per octant class at each level, by
    binarising at every level and classifying every octant."""
    field = np.asarray(field)
    if field.ndim != 3:
        raise ValueError("3D field expected")
    out = np.zeros((N_CLASSES_3D, n_levels), dtype=np.int64)
    for lvl in range(n_levels):
        cls = _CLASS_OF_OCTANT[_octant_masks(binarise(field, lvl, thresholds, superlevel, n_levels))]
        cnt = np.bincount(cls[cls >= 0].ravel(), minlength=N_CLASSES_3D)
        out[:, lvl] = cnt
    return out


def vertex_classes_3d(field, n_levels: int, thresholds=None, superlevel: bool = False) -> np.ndarray:
    """[21, n_levels] int64 class counts from the per-vertex class changes."""
    field = np.asarray(field)
    if field.ndim != 3:
        raise ValueError("3D field expected")
    L = int(n_levels)
    lam = np.pad(level_index(field, L, thresholds, superlevel), 1, mode="constant", constant_values=L)
    D, H, W = lam.shape
    q = []
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):  # appended in bit order dx + 2dy + 4dz
                q.append(lam[dz:D - 1 + dz, dy:H - 1 + dy, dx:W - 1 + dx].ravel())
    hist = np.zeros((N_CLASSES_3D, L + 1), dtype=np.int64)
    for k in range(8):
        at = q[k]
        mask = sum(((q[b] <= at).astype(np.int64) << b) for b in range(8))
        before = sum(((q[b] < at).astype(np.int64) << b) for b in range(8))
        first = np.ones_like(at, dtype=bool)
        for b in range(k):
            first &= q[b] != at
        sel = first & (at < L)
        new_c, old_c, lv = _CLASS_OF_OCTANT[mask[sel]], _CLASS_OF_OCTANT[before[sel]], at[sel]
        np.add.at(hist, (new_c, lv), 1)
        has_old = old_c >= 0
        np.add.at(hist, (old_c[has_old], lv[has_old]), -1)
    return np.cumsum(hist[:, :L], axis=1)


def class_counts(field, n_levels: int, thresholds=None, superlevel: bool = False) -> np.ndarray:
    """Class counts of a 2D ([5, L]) or 3D ([21, L]) field."""
    field = np.asarray(field)
    return (vertex_classes_2d if field.ndim == 2 else vertex_classes_3d)(field, n_levels, thresholds, superlevel)

