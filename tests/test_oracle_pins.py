"""Pins for the test oracle against what the paper and the mathematics fix.

Nothing here touches the GPU library.  Each group targets a different way the
oracle could be wrong (a dropped term, a wrong sign, a shifted index, a
transposed operand):

* the paper's printed per-vertex contributions (Tables 1 and 2, fixtures in
  tests/golden/) summed over all lattice vertices must equal the oracle's
  global counts, channel by channel;
* closed forms (filled boxes, annulus, shells, tori, blobs);
* Betti numbers from connected-component labelling (scipy.ndimage.label);
* the nerve / inclusion-exclusion of Eq. (3) on unions of closed cells;
* Alexander duality between 8/4 (2D) and 26/6 (3D) connectivity;
* symmetry, relabelling, padding, additivity and dimension-lift invariants;
* O1 (per level) == O2 (all levels) on small random inputs.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np
import pytest
from scipy import ndimage

from oracle import ec_oracle as O1
from tests import paper_tables as PT


# ----------------------------------------------------------------------------
# the fixtures themselves, re-derived from the definitions the paper states
# ----------------------------------------------------------------------------
def _edges2(mask):
    """The 4 lattice edges at a 2D vertex, as the pairs of pixel bits beside them."""
    # bits: 0 (i-1,j-1) 1 (i-1,j) 2 (i,j-1) 3 (i,j)
    return [(0, 1), (2, 3), (0, 2), (1, 3)]  # up, down, left, right half-edges


def test_table1_rows_follow_from_cell_counting():
    t1 = PT.table1()
    for m, e in t1.items():
        act = [m >> k & 1 for k in range(4)]
        V8 = 1 if any(act) else 0
        E = sum(1 for a, b in _edges2(m) if act[a] or act[b])
        F = sum(act)
        # 4-C vertex count: 4-connected components of the active pixels in the window
        comps = 0
        seen = set()
        nb = {0: (1, 2), 1: (0, 3), 2: (0, 3), 3: (1, 2)}
        for k in range(4):
            if act[k] and k not in seen:
                comps += 1
                stack = [k]
                while stack:
                    u = stack.pop()
                    if u in seen:
                        continue
                    seen.add(u)
                    stack.extend(v for v in nb[u] if act[v])
        per = sum(1 for a, b in _edges2(m) if act[a] != act[b])
        assert e["V8"] == V8 and e["E8"] == Fraction(E, 2) and e["F8"] == Fraction(F, 4)
        assert e["ec8"] == V8 - Fraction(E, 2) + Fraction(F, 4)
        assert e["V4"] == comps
        assert e["ec4"] == comps - Fraction(E, 2) + Fraction(F, 4)
        assert e["perimeter"] == Fraction(per, 2)
        assert e["area"] == Fraction(F, 4)


def _faces3():
    """12 lattice faces at a 3D vertex as pairs of octant bits (differ in one axis)."""
    out = []
    for b in range(8):
        for a in range(3):
            if not b >> a & 1:
                out.append((b, b | 1 << a))
    return out


def _edges3():
    """6 lattice edges at a 3D vertex as cyclic 4-tuples of octant bits."""
    out = []
    for a in range(3):
        o1, o2 = [x for x in range(3) if x != a]
        for s in (0, 1):
            base = s << a
            out.append((base, base | 1 << o1, base | 1 << o1 | 1 << o2, base | 1 << o2))
    return out


def _kappa(act, cyc):
    q = [act[c] for c in cyc]
    n = sum(q)
    if n in (1, 3):
        return 1
    if n == 2 and q[0] == q[2]:
        return 2
    return 0


def test_table2_rows_follow_from_cell_counting():
    t2 = PT.table2()
    rows_seen = set()
    for m, e in t2.items():
        act = [m >> k & 1 for k in range(8)]
        V = 1 if any(act) else 0
        E = sum(1 for cyc in _edges3() if any(act[c] for c in cyc))
        F = sum(1 for a, b in _faces3() if act[a] or act[b])
        C = sum(act)
        assert e["V"] == V, e["row"]
        assert e["E"] == Fraction(E, 2), e["row"]
        assert e["F"] == Fraction(F, 4), e["row"]
        assert e["Vox"] == Fraction(C, 8), e["row"]
        assert e["ec26"] == V - Fraction(E, 2) + Fraction(F, 4) - Fraction(C, 8), e["row"]
        assert e["volume"] == Fraction(C, 8), e["row"]
        # surface: faces at the vertex with exactly one active octant, a quarter each
        assert e["area"] == Fraction(sum(1 for a, b in _faces3() if act[a] != act[b]), 4), e["row"]
        # crease: half of kappa over the 6 lattice edges at the vertex
        assert e["perimeter"] == Fraction(sum(_kappa(act, cyc) for cyc in _edges3()), 2), e["row"]
        rows_seen.add(e["row"])
    assert rows_seen == set(range(1, 23))


def test_table2_area_typo_reading():
    """The claw row prints Area 1.75; every other row's printed area is reproduced."""
    rows = {e["row"]: e for e in PT.table2().values()}
    for r, e in rows.items():
        if r == 10:
            assert e["area_printed"] == Fraction(7, 4) and e["area"] == Fraction(3, 2)
        else:
            assert e["area_printed"] == e["area"]


def test_table2_fadj_column():
    """Eq. (4): sum of pairwise distances of the active (or, daggered, empty) octants."""
    for e in {v["row"]: v for v in PT.table2().values()}.values():
        m = e["example"]
        dag = e["f_adj"].endswith("+")
        sel = [b for b in range(8) if bool(m >> b & 1) != dag]
        pts = [np.array((b & 1, b >> 1 & 1, b >> 2 & 1), float) for b in sel]
        s = sum(np.linalg.norm(p - q) for p, q in itertools.combinations(pts, 2))
        assert abs(s - float(e["f_adj"].rstrip("+"))) < 2e-3, e["row"]


# ----------------------------------------------------------------------------
# oracle == sum of the printed per-vertex contributions
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(12))
def test_oracle_2d_equals_table1_route(seed):
    rng = np.random.default_rng(seed)
    h, w = rng.integers(1, 14, size=2)
    b = rng.random((h, w)) < rng.uniform(0.1, 0.9)
    t1 = PT.table1()
    vm = PT.vertex_masks_2d(b)
    assert O1.ec_2d(b, 8) == PT.table_sum(vm, t1, "ec8")
    assert O1.ec_2d(b, 4) == PT.table_sum(vm, t1, "ec4")
    assert O1.perimeter_2d(b) == PT.table_sum(vm, t1, "perimeter")
    assert b.sum() == PT.table_sum(vm, t1, "area")


@pytest.mark.parametrize("seed", range(12))
def test_oracle_3d_equals_table2_route(seed):
    rng = np.random.default_rng(100 + seed)
    d, h, w = rng.integers(1, 8, size=3)
    b = rng.random((d, h, w)) < rng.uniform(0.1, 0.9)
    t2 = PT.table2()
    vm = PT.vertex_masks_3d(b)
    assert O1.ec_3d(b, 26) == PT.table_sum(vm, t2, "ec26")
    assert O1.crease_3d(b) == PT.table_sum(vm, t2, "perimeter")
    assert O1.surface_3d(b) == PT.table_sum(vm, t2, "area")
    assert b.sum() == PT.table_sum(vm, t2, "volume")


# ----------------------------------------------------------------------------
# closed forms
# ----------------------------------------------------------------------------
def test_closed_forms_2d():
    z = np.zeros((6, 7), bool)
    assert O1.ec_2d(z, 8) == 0 and O1.ec_2d(z, 4) == 0 and O1.perimeter_2d(z) == 0
    f = np.ones((6, 7), bool)
    assert O1.ec_2d(f, 8) == 1 and O1.ec_2d(f, 4) == 1
    assert O1.perimeter_2d(f) == 2 * (6 + 7)
    ann = np.ones((7, 7), bool)
    ann[2:5, 2:5] = False
    assert O1.ec_2d(ann, 8) == 0 and O1.ec_2d(ann, 4) == 0
    assert O1.perimeter_2d(ann) == 4 * 7 + 4 * 3
    # k disjoint blobs
    b = np.zeros((9, 20), bool)
    for k in range(5):
        b[1 + (k % 2) * 4:3 + (k % 2) * 4, 1 + 4 * k:3 + 4 * k] = True
    assert O1.ec_2d(b, 8) == 5 and O1.ec_2d(b, 4) == 5
    # two diagonal pixels: one component (8-C) vs two (4-C)
    dg = np.array([[1, 0], [0, 1]], bool)
    assert O1.ec_2d(dg, 8) == 1 and O1.ec_2d(dg, 4) == 2
    # an 8-connected ring of diagonal steps encloses a hole only for 8-C
    ring = np.zeros((5, 5), bool)
    for (r, c) in [(0, 2), (1, 1), (2, 0), (3, 1), (4, 2), (3, 3), (2, 4), (1, 3)]:
        ring[r, c] = True
    assert O1.ec_2d(ring, 8) == 0 and O1.ec_2d(ring, 4) == 8


def test_closed_forms_3d():
    d, h, w = 3, 4, 5
    f = np.ones((d, h, w), bool)
    assert O1.ec_3d(f, 26) == 1 and O1.ec_3d(f, 6) == 1
    assert O1.surface_3d(f) == 2 * (h * w + d * h + d * w)
    assert O1.crease_3d(f) == 4 * (d + h + w)
    z = np.zeros((3, 3, 3), bool)
    assert O1.ec_3d(z, 26) == 0 and O1.ec_3d(z, 6) == 0 and O1.crease_3d(z) == 0
    shell = np.ones((5, 5, 5), bool)
    shell[1:4, 1:4, 1:4] = False
    assert O1.ec_3d(shell, 26) == 2 and O1.ec_3d(shell, 6) == 2
    torus = np.ones((1, 5, 5), bool)
    torus[0, 1:4, 1:4] = False
    torus = np.concatenate([torus, torus], 0)
    assert O1.ec_3d(torus, 26) == 0 and O1.ec_3d(torus, 6) == 0
    blobs = np.zeros((4, 4, 12), bool)
    for k in range(3):
        blobs[1:3, 1:3, 1 + 4 * k:3 + 4 * k] = True
    assert O1.ec_3d(blobs, 26) == 3 and O1.ec_3d(blobs, 6) == 3
    # two voxels touching at a corner: one piece (26-C), two (6-C)
    c = np.zeros((2, 2, 2), bool)
    c[0, 0, 0] = c[1, 1, 1] = True
    assert O1.ec_3d(c, 26) == 1 and O1.ec_3d(c, 6) == 2
    assert O1.surface_3d(c) == 12 and O1.crease_3d(c) == 24
    # single voxel: 6 faces, 12 edges of kappa 1
    one = np.ones((1, 1, 1), bool)
    assert O1.surface_3d(one) == 6 and O1.crease_3d(one) == 12


# ----------------------------------------------------------------------------
# Betti numbers by labelling (2D), exhaustive 3x3 and random images
# ----------------------------------------------------------------------------
S8 = np.ones((3, 3), int)
S4 = ndimage.generate_binary_structure(2, 1)


def _betti_chi_2d(b, conn):
    fg, bg = (S8, S4) if conn == 8 else (S4, S8)
    b0 = ndimage.label(b, structure=fg)[1]
    holes = ndimage.label(~np.pad(b, 1), structure=bg)[1] - 1
    return b0 - holes


def test_betti_2d_exhaustive_3x3():
    for code in range(512):
        b = np.array([code >> k & 1 for k in range(9)], bool).reshape(3, 3)
        for conn in (8, 4):
            assert O1.ec_2d(b, conn) == _betti_chi_2d(b, conn), (code, conn)


@pytest.mark.parametrize("seed", range(8))
def test_betti_2d_random(seed):
    rng = np.random.default_rng(200 + seed)
    b = rng.random((int(rng.integers(4, 30)), int(rng.integers(4, 30)))) < rng.uniform(0.2, 0.8)
    for conn in (8, 4):
        assert O1.ec_2d(b, conn) == _betti_chi_2d(b, conn)


def test_betti_3d_components_and_cavities():
    """For volumes whose complement has no tunnels through the object, b1 = 0."""
    rng = np.random.default_rng(7)
    S26 = np.ones((3, 3, 3), int)
    S6 = ndimage.generate_binary_structure(3, 1)
    for _ in range(30):
        # disjoint solid boxes and hollow shells: chi = components + cavities
        b = np.zeros((12, 12, 12), bool)
        exp = 0
        for k in range(int(rng.integers(1, 4))):
            z, y, x = rng.integers(0, 3, size=3) + np.array([0, 0, 4 * k])
            s = int(rng.integers(1, 4))
            if x + s > 12:
                continue
            b[z:z + s, y:y + s, x:x + s] = True
            if s == 3 and rng.random() < 0.5:
                b[z + 1, y + 1, x + 1] = False
        b0 = ndimage.label(b, structure=S26)[1]
        b2 = ndimage.label(~np.pad(b, 1), structure=S6)[1] - 1
        exp = b0 + b2
        assert O1.ec_3d(b, 26) == exp


# ----------------------------------------------------------------------------
# nerve of the closed cells (Eq. (3) applied to all intersections)
# ----------------------------------------------------------------------------
def _nerve_chi(cells):
    """chi of a union of closed unit boxes = alternating count of the cliques of
    the 'closed boxes meet' graph (axis-parallel boxes that meet pairwise share a
    point, so every clique is a nonempty intersection)."""
    n = len(cells)
    cells = [np.asarray(c) for c in cells]
    adj = [[bool(np.all(np.abs(cells[i] - cells[j]) <= 1)) for j in range(n)] for i in range(n)]
    total = 0

    def grow(clique, cand):
        nonlocal total
        for k, j in enumerate(cand):
            c2 = clique + [j]
            total += 1 if len(c2) % 2 == 1 else -1
            grow(c2, [x for x in cand[k + 1:] if adj[j][x]])

    grow([], list(range(n)))
    return total


@pytest.mark.parametrize("seed", range(10))
def test_nerve_2d(seed):
    rng = np.random.default_rng(300 + seed)
    b = rng.random((6, 6)) < 0.45
    assert O1.ec_2d(b, 8) == _nerve_chi(list(zip(*np.nonzero(b))))


@pytest.mark.parametrize("seed", range(10))
def test_nerve_3d(seed):
    rng = np.random.default_rng(400 + seed)
    b = rng.random((3, 4, 4)) < 0.35
    assert O1.ec_3d(b, 26) == _nerve_chi(list(zip(*np.nonzero(b))))


# ----------------------------------------------------------------------------
# duality between the two connectivities
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(10))
def test_duality(seed):
    rng = np.random.default_rng(500 + seed)
    b = rng.random((7, 9)) < rng.uniform(0.2, 0.8)
    comp = ~np.pad(b, 1)
    assert O1.ec_2d(comp, 4) == 1 - O1.ec_2d(b, 8)
    assert O1.ec_2d(comp, 8) == 1 - O1.ec_2d(b, 4)
    v = rng.random((4, 5, 4)) < rng.uniform(0.2, 0.8)
    compv = ~np.pad(v, 1)
    assert O1.ec_3d(compv, 6) == 1 + O1.ec_3d(v, 26)
    assert O1.ec_3d(compv, 26) == 1 + O1.ec_3d(v, 6)


# ----------------------------------------------------------------------------
# invariants
# ----------------------------------------------------------------------------
def _all_channels(field, L, thr=None, conn=None):
    return O1.curves_per_level(field, L, thresholds=thr, connectivity=conn)


def test_symmetry_2d():
    rng = np.random.default_rng(11)
    f = rng.integers(0, 9, size=(7, 7)).astype(np.uint8)
    for conn in (8, 4):
        ref = _all_channels(f, 9, conn=conn)
        for g in (f.T, f[::-1], f[:, ::-1], f[::-1, ::-1].T, np.rot90(f)):
            got = _all_channels(np.ascontiguousarray(g), 9, conn=conn)
            for k in ref:
                assert (ref[k] == got[k]).all()


def test_symmetry_3d():
    rng = np.random.default_rng(12)
    f = rng.integers(0, 7, size=(4, 4, 4)).astype(np.uint8)
    for conn in (26, 6):
        ref = _all_channels(f, 7, conn=conn)
        for perm in itertools.permutations(range(3)):
            for flip in itertools.product((False, True), repeat=3):
                g = f.transpose(perm)
                for a, fl in enumerate(flip):
                    if fl:
                        g = np.flip(g, a)
                got = _all_channels(np.ascontiguousarray(g), 7, conn=conn)
                for k in ref:
                    assert (ref[k] == got[k]).all(), (perm, flip, k)


def test_relabel_padding_additivity():
    rng = np.random.default_rng(13)
    f = rng.integers(0, 10, size=(6, 8)).astype(np.uint8)
    ref = _all_channels(f, 10)
    # strictly monotone relabelling of values together with thresholds
    g = (f.astype(np.float32) * 3.5 - 7.0)
    thr = (np.arange(10, dtype=np.float32) * 3.5 - 7.0)
    got = _all_channels(g, 10, thr=thr)
    for k in ref:
        assert (ref[k] == got[k]).all()
    # padding with never-active cells changes nothing
    p = np.full((10, 12), 255, np.uint8)
    p[2:8, 3:11] = f
    got = _all_channels(p, 10)
    for k in ref:
        assert (ref[k] == got[k]).all()
    # two fields separated by a never-active gap add up
    f2 = rng.integers(0, 10, size=(6, 5)).astype(np.uint8)
    both = np.full((6, 8 + 1 + 5), 200, np.uint8)
    both[:, :8] = f
    both[:, 9:] = f2
    r2 = _all_channels(f2, 10)
    got = _all_channels(both, 10)
    for k in ref:
        assert (ref[k] + r2[k] == got[k]).all()


def test_dimension_lift():
    rng = np.random.default_rng(14)
    f = rng.integers(0, 8, size=(7, 9)).astype(np.uint16)
    r2 = _all_channels(f, 8, conn=8)
    r4 = _all_channels(f, 8, conn=4)
    v = f[None]
    r3 = _all_channels(v, 8, conn=26)
    r6 = _all_channels(v, 8, conn=6)
    assert (r3["ec"] == r2["ec"]).all()
    assert (r6["ec"] == r4["ec"]).all()
    assert (r3["volume"] == r2["area"]).all()
    assert (r3["area"] == 2 * r2["area"] + r2["perimeter"]).all()
    # crease of a one-voxel-thick slab: both horizontal lattice planes see the 2D
    # boundary edges, plus kappa of every 2x2 pixel block around the vertical edges
    for lvl in range(8):
        b = f <= lvl
        vm = PT.vertex_masks_2d(b)
        kap = {0: 0, 1: 1, 2: 1, 4: 1, 8: 1, 3: 0, 12: 0, 5: 0, 10: 0, 6: 2, 9: 2,
               7: 1, 11: 1, 13: 1, 14: 1, 15: 0}
        vert = sum(kap[int(m)] for m in vm.ravel())
        assert r3["perimeter"][lvl] == 2 * r2["perimeter"][lvl] + vert


def test_area_volume_are_cumulative_counts():
    rng = np.random.default_rng(15)
    f = rng.integers(0, 20, size=(5, 6, 7)).astype(np.uint16)
    r = _all_channels(f, 16)
    lam = np.minimum(f.ravel(), 16)
    assert (r["volume"] == np.cumsum(np.bincount(lam, minlength=17))[:16]).all()


# ----------------------------------------------------------------------------
# level semantics (Eq. (2), "<= c")
# ----------------------------------------------------------------------------
def test_float_levels_inclusive_and_nan():
    f = np.array([[0.5, np.nan], [1.0, 2.0]], np.float32)
    thr = np.array([0.5, 1.0, 1.5], np.float32)
    r = O1.curves_per_level(f, 3, thresholds=thr)
    assert list(r["area"]) == [1, 2, 2]  # 0.5 <= 0.5 counts; NaN and 2.0 never


# ----------------------------------------------------------------------------
# O1 == O2 on small random inputs
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(16))
def test_o1_equals_o2(seed, o2):
    rng = np.random.default_rng(600 + seed)
    nd = 2 if seed % 2 == 0 else 3
    shape = tuple(int(s) for s in rng.integers(1, 12 if nd == 2 else 6, size=nd))
    kind = seed % 4
    L = int(rng.integers(1, 14))
    thr = None
    if kind in (0, 1):
        dt = np.uint8 if kind == 0 else np.uint16
        f = rng.integers(0, L + 4, size=shape).astype(dt)  # some never-active values
    else:
        f = rng.normal(size=shape).astype(np.float32)
        thr = np.sort(rng.normal(size=L)).astype(np.float32)
        if L > 2:
            thr[1] = thr[0]  # repeated threshold
            f.ravel()[0] = thr[-1]  # equal to a threshold
        if f.size > 2:
            f.ravel()[1] = np.nan
    conns = (8, 4) if nd == 2 else (26, 6)
    for conn in conns:
        a = O1.curves_per_level(f, L, thresholds=thr, connectivity=conn)
        b = o2(f, L, thresholds=thr, connectivity=conn)
        for k in a:
            assert (a[k] == b[k]).all(), (k, conn, a[k], b[k])


# ----------------------------------------------------------------------------
# O2's threaded histogram == its single-threaded one
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(6))
def test_o2_threads_equal_single_thread(seed, o2):
    """The GPU tests and the CPU baseline run O2 with 16 threads (per-thread
    histograms over slabs of lattice rows or planes, summed): it must give
    exactly its single-thread result, with every thread owning a slab."""
    rng = np.random.default_rng(700 + seed)
    nd = 2 if seed % 2 == 0 else 3
    shape = (int(rng.integers(40, 90)), int(rng.integers(20, 60))) if nd == 2 else \
        (int(rng.integers(20, 40)), int(rng.integers(8, 20)), int(rng.integers(8, 20)))
    kind = seed % 3
    thr = None
    if kind == 0:
        L = 200
        f = rng.integers(0, 230, size=shape).astype(np.uint8)
    elif kind == 1:
        L = 1000
        f = rng.integers(0, 1100, size=shape).astype(np.uint16)
    else:
        L = 97
        f = rng.normal(size=shape).astype(np.float32)
        thr = np.sort(rng.normal(size=L)).astype(np.float32)
        f.ravel()[::17] = np.nan
    for conn in ((8, 4) if nd == 2 else (26, 6)):
        one = o2(f, L, thresholds=thr, connectivity=conn, n_threads=1)
        many = o2(f, L, thresholds=thr, connectivity=conn, n_threads=16)
        for k in one:
            assert np.array_equal(one[k], many[k]), (k, conn)
