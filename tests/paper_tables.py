"""Readers for the paper's printed vertex-contribution tables (tests/golden/).

Used by the tests to pin both the oracle (the global counts must equal the sum
of the printed per-vertex contributions over all lattice vertices) and the
library's tables (they must reproduce the printed rows).

2D masks: bit 0 = pixel (i-1, j-1), bit 1 = (i-1, j), bit 2 = (i, j-1),
bit 3 = (i, j) around lattice vertex (i, j) (row index grows downwards).
3D masks: bit (dx + 2 dy + 4 dz) = voxel at offset (dz, dy, dx) in {0,1}^3 of
the 2x2x2 block around the lattice vertex.
"""
from __future__ import annotations

import itertools
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split()


# ----------------------------------------------------------------------------
# 2D (Table 1)
# ----------------------------------------------------------------------------
def _pattern_to_mask2(p: str) -> int:
    top, bot = p.split("/")
    bits = [top[0], top[1], bot[0], bot[1]]  # (i-1,j-1), (i-1,j), (i,j-1), (i,j)
    return sum(1 << k for k, c in enumerate(bits) if c == "1")


def _sym2(mask: int):
    """All images of a 2x2 mask under the 8 symmetries of the square."""
    cells = [(0, 0), (0, 1), (1, 0), (1, 1)]
    out = set()
    for swap in (False, True):
        for fr in (False, True):
            for fc in (False, True):
                m = 0
                for k, (r, c) in enumerate(cells):
                    if mask >> k & 1:
                        r2, c2 = (c, r) if swap else (r, c)
                        r2 = 1 - r2 if fr else r2
                        c2 = 1 - c2 if fc else c2
                        m |= 1 << cells.index((r2, c2))
                out.add(m)
    return out


def table1():
    """dict mask(0..15) -> dict of Fractions: ec8, ec4, perimeter, area, V8, E8, F8, V4."""
    rows = list(_rows("table1_2d_vertex_contributions.txt"))
    out = {}
    for r in rows:
        (typ, pat, V8, E8c, E8w, F8c, F8w, EC8, V4, E4c, E4w, F4c, F4w, EC4, per, area) = r
        entry = dict(type=typ, V8=Fraction(V8), E8=Fraction(E8c) * Fraction(E8w),
                     F8=Fraction(F8c) * Fraction(F8w), ec8=Fraction(EC8), V4=Fraction(V4),
                     E4=Fraction(E4c) * Fraction(E4w), F4=Fraction(F4c) * Fraction(F4w),
                     ec4=Fraction(EC4), perimeter=Fraction(per), area=Fraction(area),
                     example=_pattern_to_mask2(pat))
        for m in _sym2(entry["example"]):
            assert m not in out, "Table 1 rows overlap under symmetry"
            out[m] = entry
    assert len(out) == 16, "Table 1 rows do not cover all 16 masks"
    return out


# ----------------------------------------------------------------------------
# 3D (Table 2)
# ----------------------------------------------------------------------------
# corner of the cube at which the paper's picture macro draws argument k (x, y, z)
MACRO_CORNER = [(0, 1, 1), (1, 1, 1), (0, 1, 0), (1, 1, 0), (0, 0, 1), (1, 0, 1), (0, 0, 0), (1, 0, 0)]


def _xyz_to_bit(x, y, z):
    return x + 2 * y + 4 * z


def _sym3_maps():
    maps = []
    for perm in itertools.permutations(range(3)):
        for flips in itertools.product((0, 1), repeat=3):
            m = []
            for b in range(8):
                c = (b & 1, b >> 1 & 1, b >> 2 & 1)
                c2 = [c[perm[a]] ^ flips[a] for a in range(3)]
                m.append(_xyz_to_bit(*c2))
            maps.append(m)
    return maps


SYM3 = _sym3_maps()


def orbit3(mask: int):
    out = set()
    for m in SYM3:
        out.add(sum(1 << m[b] for b in range(8) if mask >> b & 1))
    return out


def table2():
    """dict mask(0..255) -> dict of Fractions (ec26, perimeter, area, volume, ...)."""
    out = {}
    for r in _rows("table2_3d_vertex_contributions.txt"):
        row = int(r[0])
        args = [int(v) for v in r[1:9]]
        fadj, V, Ec, Fc, Vc, EC, per, area, area_pr, vol = r[9:19]
        mask = 0
        for k, a in enumerate(args):
            if a:
                mask |= 1 << _xyz_to_bit(*MACRO_CORNER[k])
        entry = dict(row=row, example=mask, f_adj=fadj, V=Fraction(V),
                     E=Fraction(Ec) * Fraction(1, 2), F=Fraction(Fc) * Fraction(1, 4),
                     Vox=Fraction(Vc) * Fraction(1, 8), ec26=Fraction(EC),
                     perimeter=Fraction(per), area=Fraction(area),
                     area_printed=Fraction(area_pr), volume=Fraction(vol))
        for m in orbit3(mask):
            assert m not in out, f"Table 2 row {row} overlaps another row under symmetry"
            out[m] = entry
    assert len(out) == 256, "Table 2 rows do not cover all 256 masks"
    return out


# ----------------------------------------------------------------------------
# table route: sum of per-vertex contributions over all lattice vertices
# ----------------------------------------------------------------------------
def vertex_masks_2d(b: np.ndarray) -> np.ndarray:
    p = np.pad(np.asarray(b, bool), 1).astype(np.int64)
    return p[:-1, :-1] | p[:-1, 1:] << 1 | p[1:, :-1] << 2 | p[1:, 1:] << 3


def vertex_masks_3d(b: np.ndarray) -> np.ndarray:
    p = np.pad(np.asarray(b, bool), 1).astype(np.int64)
    m = np.zeros(tuple(s - 1 for s in p.shape), dtype=np.int64)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                sl = p[dz:p.shape[0] - 1 + dz, dy:p.shape[1] - 1 + dy, dx:p.shape[2] - 1 + dx]
                m |= sl << _xyz_to_bit(dx, dy, dz)
    return m


def table_sum(masks: np.ndarray, table: dict, key: str) -> Fraction:
    counts = np.bincount(masks.ravel(), minlength=len(table))
    return sum((int(counts[m]) * table[m][key] for m in range(len(counts)) if counts[m]),
               Fraction(0))
