"""Pins of the vertex-class oracle (contribution map) and the library's class tables.

* The class of every 2x2 mask is the Table 1 row it belongs to (rows read from
  the printed table's pictures, tests/golden/, closed under the square's
  symmetries).
* Closed forms: a filled k x k square, a diagonal pair, an L of three pixels.
* Weighting the class counts by Table 1's printed columns gives the per-level
  oracle's EC (8-C and 4-C), perimeter and area, which count cells directly
  (Eq. (1)), at every level of random fields.
* The event form (per-vertex class changes, running sums) equals the
  binarise-every-level form, ties, NaN and never-entering values included.
* 3D: the octant classes are exactly the rows of Table 2 (read from the
  printed pictures), a filled box gives its corners, edges, faces and interior,
  and weighting by Table 2's printed columns gives O1's EC (26-C), crease,
  surface and volume at every level.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import ec_oracle as O1
from oracle import vertex_classes as VC
from tests import paper_tables as PT

TYPE_TO_CLASS = {"q0": -1, "q1": 0, "q2": 1, "qd": 2, "q3": 3, "q4": 4}


def test_class_assignment_matches_table1():
    t1 = PT.table1()
    for m in range(16):
        assert VC.quadrant_class(m) == TYPE_TO_CLASS[t1[m]["type"]], m


def test_library_class_table_matches_table1():
    from paper_2311_11740_amd import ecc
    t1 = PT.table1()
    assert ecc.vertex_class_table(2) == [TYPE_TO_CLASS[t1[m]["type"]] for m in range(16)]
    with pytest.raises(ecc.EccError):
        ecc.vertex_class_table(4)


def test_closed_form_square():
    n, k = 9, 4
    a = np.ones((n, n), np.uint8)
    a[2:2 + k, 3:3 + k] = 0
    for fn in (oracle.vertex_classes_per_level, oracle.vertex_classes_2d):
        c = fn(a, 2)
        assert list(c[:, 0]) == [4, 4 * (k - 1), 0, 0, (k - 1) ** 2]
        assert list(c[:, 1]) == [4, 4 * (n - 1), 0, 0, (n - 1) ** 2]


def test_closed_form_diagonal_and_three():
    a = np.array([[0, 1], [1, 0]], np.uint8)
    assert list(oracle.vertex_classes_2d(a, 1)[:, 0]) == [6, 0, 1, 0, 0]
    b = np.array([[0, 0], [0, 1]], np.uint8)
    # three pixels in an L: the inner corner is a "three" vertex, the two
    # vertices between two pixels are "adjacent", five outer corners "one",
    # the corner of the empty pixel is empty
    assert list(oracle.vertex_classes_2d(b, 1)[:, 0]) == [5, 2, 0, 1, 0]
    assert list(oracle.vertex_classes_per_level(b, 1)[:, 0]) == [5, 2, 0, 1, 0]


def _random_field(seed):
    rng = np.random.default_rng(seed)
    h, w = (int(x) for x in rng.integers(1, 14, size=2))
    kind = seed % 3
    if kind == 0:
        return rng.integers(0, 12, size=(h, w)).astype(np.uint8), 9, None
    if kind == 1:
        return rng.integers(0, 300, size=(h, w)).astype(np.uint16), 256, None
    x = rng.normal(size=(h, w)).astype(np.float32)
    x[rng.random((h, w)) < 0.1] = np.nan
    thr = np.sort(rng.normal(size=7)).astype(np.float32)
    thr[3] = thr[2]  # a repeated threshold
    x.ravel()[:3] = thr[:3]  # values exactly on thresholds
    return x, 7, thr


@pytest.mark.parametrize("seed", range(12))
def test_event_form_equals_per_level(seed):
    a, L, thr = _random_field(seed)
    assert np.array_equal(oracle.vertex_classes_2d(a, L, thr), oracle.vertex_classes_per_level(a, L, thr))


@pytest.mark.parametrize("seed", range(12))
def test_table1_weightings_give_cell_counts(seed):
    a, L, thr = _random_field(seed)
    counts = oracle.vertex_classes_2d(a, L, thr)
    t1 = PT.table1()
    example = {}
    for m, e in t1.items():
        example.setdefault(TYPE_TO_CLASS[e["type"]], e)
    ref8 = O1.curves_per_level(a, L, thr, connectivity=8)
    ref4 = O1.curves_per_level(a, L, thr, connectivity=4, channels=("ec",))
    for col, ref in (("ec8", ref8["ec"]), ("ec4", ref4["ec"]), ("perimeter", ref8["perimeter"]),
                     ("area", ref8["area"])):
        for lvl in range(L):
            s = sum(Fraction(int(counts[c, lvl])) * example[c][col] for c in range(5))
            assert s == ref[lvl], (col, lvl)


def test_all_active_covers_every_vertex():
    rng = np.random.default_rng(5)
    a = rng.integers(0, 50, size=(7, 11)).astype(np.uint8)
    c = oracle.vertex_classes_2d(a, 50)
    assert c[:, -1].sum() == 8 * 12
    assert np.all(np.diff(c.sum(axis=0)) >= 0)  # vertices never leave the complex


# ----------------------------------------------------------------------------
# 3D (Table 2)
# ----------------------------------------------------------------------------
def _row_to_class():
    """Table 2 row -> oracle class, checking that the two partitions agree."""
    t2 = PT.table2()
    mapping = {}
    for m in range(256):
        row, c = t2[m]["row"], VC.octant_class(m)
        assert mapping.setdefault(row, c) == c, f"mask {m}: Table 2 row {row} spans classes"
    assert len(set(mapping.values())) == len(mapping) == 22
    return mapping, t2


def test_octant_classes_are_table2_rows():
    mapping, _ = _row_to_class()
    assert sorted(mapping.values()) == list(range(-1, 21))


def test_library_octant_class_table():
    from paper_2311_11740_amd import ecc
    assert ecc.vertex_class_table(3) == [VC.octant_class(m) for m in range(256)]


def test_closed_form_cube():
    n, k = 7, 3
    a = np.ones((n, n, n), np.uint8)
    a[1:1 + k, 2:2 + k, 3:3 + k] = 0
    for fn in (oracle.vertex_classes_3d, oracle.vertex_classes_3d_per_level):
        c = fn(a, 2)[:, 0]
        want = np.zeros(21, np.int64)
        want[VC.octant_class(0b00000001)] = 8                 # corners: one voxel
        want[VC.octant_class(0b00000011)] = 12 * (k - 1)      # edges: two voxels sharing a face
        want[VC.octant_class(0b00001111)] = 6 * (k - 1) ** 2  # faces: a 2 x 2 square
        want[VC.octant_class(0b11111111)] = (k - 1) ** 3      # interior: full
        assert np.array_equal(c, want)


def _random_volume(seed):
    rng = np.random.default_rng(100 + seed)
    d, h, w = (int(x) for x in rng.integers(1, 7, size=3))
    if seed % 2 == 0:
        return rng.integers(0, 7, size=(d, h, w)).astype(np.uint8), 5, None
    x = rng.normal(size=(d, h, w)).astype(np.float32)
    x[rng.random(x.shape) < 0.1] = np.nan
    thr = np.sort(rng.normal(size=5)).astype(np.float32)
    thr[2] = thr[1]
    return x, 5, thr


@pytest.mark.parametrize("seed", range(8))
def test_3d_event_form_equals_per_level(seed):
    a, L, thr = _random_volume(seed)
    assert np.array_equal(oracle.vertex_classes_3d(a, L, thr), oracle.vertex_classes_3d_per_level(a, L, thr))


@pytest.mark.parametrize("seed", range(8))
def test_table2_weightings_give_cell_counts(seed):
    a, L, thr = _random_volume(seed)
    counts = oracle.vertex_classes_3d(a, L, thr)
    mapping, t2 = _row_to_class()
    entry = {}
    for m, e in t2.items():
        entry.setdefault(mapping[e["row"]], e)
    ref = O1.curves_per_level(a, L, thr, connectivity=26)
    for col, ch in (("ec26", "ec"), ("perimeter", "perimeter"), ("area", "area"), ("volume", "volume")):
        for lvl in range(L):
            s = sum(Fraction(int(counts[c, lvl])) * entry[c][col] for c in range(21))
            assert s == ref[ch][lvl], (col, lvl)
