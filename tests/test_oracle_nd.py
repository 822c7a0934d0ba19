"""Pins of the any-dimension oracle (oracle/ec_oracle_nd.py), used for 4D fields.

* For n = 2 and 3 it gives what the independently written 2D/3D oracles give:
  the closure EC = 8-C / 26-C, the face-adjacency EC = 4-C / 6-C, boundary =
  perimeter / surface, and whole curves equal to O2 (the C oracle).
* Products: the closure of A x B is the product of the closures and the face
  complex of A x B is the product of the face complexes, so
  chi(A x B) = chi(A) chi(B) for 4D sets made of two 2D images (and of a
  volume and a row).
* Duality in R^4 (Alexander duality, one point at infinity taken off):
  chi of the padded complement in the dual connectivity = 1 - chi.
* Dimension lift: a (1, d, h, w) field gives the 3D curves (boundary =
  2 x volume + surface).
* Closed forms: filled box (EC 1, boundary 2 sum of products of three sides),
  thick hollow 4-box (the 3-sphere: EC 0), two cells meeting at one vertex
  (closure 1, faces 2), a single cell.
* The per-level and all-levels forms agree (ties, NaN, never-entering
  values, both filtration directions); superlevel(f) = sublevel(-f).
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import ec_oracle as O1
from oracle import ec_oracle_nd as ND


def _rand_b(rng, shape, p=None):
    return rng.random(shape) < (rng.uniform(0.2, 0.8) if p is None else p)


@pytest.mark.parametrize("seed", range(10))
def test_nd_equals_2d_3d_oracles(seed):
    rng = np.random.default_rng(1100 + seed)
    b2 = _rand_b(rng, tuple(int(x) for x in rng.integers(1, 14, size=2)))
    assert ND.ec_closure(b2) == O1.ec_2d(b2, 8)
    assert ND.ec_faces(b2) == O1.ec_2d(b2, 4)
    assert ND.boundary(b2) == O1.perimeter_2d(b2)
    b3 = _rand_b(rng, tuple(int(x) for x in rng.integers(1, 7, size=3)))
    assert ND.ec_closure(b3) == O1.ec_3d(b3, 26)
    assert ND.ec_faces(b3) == O1.ec_3d(b3, 6)
    assert ND.boundary(b3) == O1.surface_3d(b3)


@pytest.mark.parametrize("seed", range(8))
def test_nd_all_levels_equals_c_oracle(seed, o2):
    rng = np.random.default_rng(1200 + seed)
    nd = 2 + seed % 2
    shape = tuple(int(x) for x in rng.integers(1, 12 if nd == 2 else 7, size=nd))
    sup = seed % 4 >= 2
    if seed % 3 == 0:
        f, L, thr = rng.integers(0, 20, size=shape).astype(np.uint8), 16, None
    else:
        f = rng.normal(size=shape).astype(np.float32)
        L = 11
        thr = np.sort(rng.normal(size=L)).astype(np.float32)
        thr[3] = thr[2]
        if sup:
            thr = thr[::-1].copy()
        if f.size > 1:
            f.ravel()[0] = np.nan
    for conn in ((8, 4) if nd == 2 else (26, 6)):
        a = ND.curves_all_levels(f, L, thr, conn, sup)
        b = o2(f, L, thresholds=thr, connectivity=conn, superlevel=sup)
        assert np.array_equal(a["ec"], b["ec"]), conn
        if nd == 2:
            assert np.array_equal(a["boundary"], b["perimeter"])
            assert np.array_equal(a["volume"], b["area"])
        else:
            assert np.array_equal(a["boundary"], b["area"])
            assert np.array_equal(a["volume"], b["volume"])


@pytest.mark.parametrize("seed", range(8))
def test_product_formula_4d(seed):
    rng = np.random.default_rng(1300 + seed)
    A = _rand_b(rng, tuple(int(x) for x in rng.integers(2, 7, size=2)))
    B = _rand_b(rng, tuple(int(x) for x in rng.integers(2, 7, size=2)))
    P = A[:, :, None, None] & B[None, None, :, :]
    assert ND.ec_closure(P) == O1.ec_2d(A, 8) * O1.ec_2d(B, 8)
    assert ND.ec_faces(P) == O1.ec_2d(A, 4) * O1.ec_2d(B, 4)
    V = _rand_b(rng, tuple(int(x) for x in rng.integers(2, 5, size=3)))
    row = _rand_b(rng, (int(rng.integers(2, 9)),))
    runs = int(row[0]) + int(np.sum(row[1:] & ~row[:-1]))  # chi of a set of unit segments
    Q = V[:, :, :, None] & row[None, None, None, :]
    assert ND.ec_closure(Q) == O1.ec_3d(V, 26) * runs
    assert ND.ec_faces(Q) == O1.ec_3d(V, 6) * runs


@pytest.mark.parametrize("seed", range(8))
def test_duality_4d(seed):
    rng = np.random.default_rng(1400 + seed)
    b = _rand_b(rng, tuple(int(x) for x in rng.integers(2, 5, size=4)))
    comp = ~np.pad(b, 1)
    assert ND.ec_faces(comp) == 1 - ND.ec_closure(b)
    assert ND.ec_closure(comp) == 1 - ND.ec_faces(b)


@pytest.mark.parametrize("seed", range(4))
def test_dimension_lift_4d(seed, o2):
    rng = np.random.default_rng(1500 + seed)
    v = rng.integers(0, 12, size=tuple(int(x) for x in rng.integers(1, 6, size=3))).astype(np.uint8)
    f4 = v[None]
    for c4, c3 in ((80, 26), (8, 6)):
        a = ND.curves_all_levels(f4, 10, connectivity=c4)
        r = o2(v, 10, connectivity=c3)
        assert np.array_equal(a["ec"], r["ec"])
        assert np.array_equal(a["volume"], r["volume"])
        assert np.array_equal(a["boundary"], 2 * r["volume"] + r["area"])


def test_closed_forms_4d():
    full = np.ones((2, 3, 4, 5), bool)
    assert ND.ec_closure(full) == ND.ec_faces(full) == 1
    assert ND.boundary(full) == 2 * (3 * 4 * 5 + 2 * 4 * 5 + 2 * 3 * 5 + 2 * 3 * 4)
    shell = np.ones((5, 5, 5, 5), bool)
    shell[1:-1, 1:-1, 1:-1, 1:-1] = False  # a thick-walled hollow 4-box: the 3-sphere
    assert ND.ec_closure(shell) == 0
    assert ND.ec_faces(shell) == 0
    diag = np.zeros((2, 2, 2, 2), bool)
    diag[0, 0, 0, 0] = diag[1, 1, 1, 1] = True  # two cells sharing one vertex
    assert ND.ec_closure(diag) == 1 and ND.ec_faces(diag) == 2
    one = np.zeros((3, 3, 3, 3), bool)
    one[1, 1, 1, 1] = True
    assert ND.ec_closure(one) == ND.ec_faces(one) == 1
    assert ND.boundary(one) == 8


@pytest.mark.parametrize("seed", range(8))
def test_per_level_equals_all_levels_4d(seed):
    rng = np.random.default_rng(1600 + seed)
    shape = tuple(int(x) for x in rng.integers(1, 6, size=4))
    sup = seed % 2 == 1
    if seed % 4 < 2:
        f, L, thr = rng.integers(0, 14, size=shape).astype(np.uint16), 12, None
    else:
        f = rng.normal(size=shape).astype(np.float32)
        L = 9
        thr = np.sort(rng.normal(size=L)).astype(np.float32)
        thr[4] = thr[3]
        if sup:
            thr = thr[::-1].copy()
        f.ravel()[::7] = np.nan
    for conn in (80, 8):
        a = ND.curves_per_level(f, L, thr, conn, sup)
        b = ND.curves_all_levels(f, L, thr, conn, sup)
        for k in a:
            assert np.array_equal(a[k], b[k]), (k, conn)


def test_superlevel_negation_4d():
    rng = np.random.default_rng(1700)
    f = rng.normal(size=(3, 4, 5, 6)).astype(np.float32)
    t = np.linspace(1.5, -1.5, 13).astype(np.float32)
    for conn in (80, 8):
        a = ND.curves_all_levels(f, 13, t, conn, superlevel=True)
        b = ND.curves_all_levels(-f, 13, -t, conn)
        for k in a:
            assert np.array_equal(a[k], b[k])
