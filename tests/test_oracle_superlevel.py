"""Pins of the oracle's superlevel filtration (the mirror of Eq. (2): a cell is
active at level l when value >= t_l, thresholds non-increasing; integer
levels t_l = L - 1 - l).

Each pin ties the superlevel route to something fixed outside it:

* Set algebra: {f >= c} = {-f <= -c}, so the superlevel curves of f equal the
  sublevel curves (already pinned to Tables 1 and 2, closed forms and Betti
  numbers) of -f at -t, in O1 and in O2, for integer and float fields (ties,
  NaN, +-inf, -0.0, values on thresholds).
* Betti numbers: at every level the superlevel set is binarised directly with
  numpy and its EC counted by labelling components and holes
  (scipy.ndimage.label), its perimeter and area by edge and cell counts.
* Complement duality between the two directions: for integer fields,
  {f >= c} and {f <= c - 1} partition the field, so by the 8/4 (26/6) duality
  of a set and its padded complement, chi4(pad({f <= c-1})) = 1 - chi8({f >= c})
  and chi6(pad(.)) = 1 + chi26(.) in 3D; the left side is a sublevel curve, the
  right side a superlevel curve.
* Closed forms: a peak (every superlevel set a digital disc or ball: EC 1),
  a ridge ring (annulus: EC 0 until the set fills the disc), a ridge shell
  (sphere: EC 2), and the last level where every cell is active (the filled
  box: EC 1, perimeter 2(h+w), area hw; in 3D surface 2(hw+hd+wd), crease
  4(d+h+w), volume dhw).
* O1 == O2 and both vertex-class forms agree in the superlevel direction, and
  Table 1 / Table 2 weightings of the superlevel class counts give the
  superlevel curves.
"""
from __future__ import annotations

import ctypes
from fractions import Fraction

import numpy as np
import pytest
from scipy import ndimage

import oracle
from oracle import ec_oracle as O1
from tests import paper_tables as PT

S8 = np.ones((3, 3), int)
S4 = ndimage.generate_binary_structure(2, 1)


def _betti_chi_2d(b, conn):
    fg, bg = (S8, S4) if conn == 8 else (S4, S8)
    b0 = ndimage.label(b, structure=fg)[1]
    holes = ndimage.label(~np.pad(b, 1), structure=bg)[1] - 1
    return b0 - holes


def _random_case(seed):
    """(field, L, thresholds or None) for the superlevel direction."""
    rng = np.random.default_rng(900 + seed)
    nd = 2 if seed % 2 == 0 else 3
    shape = tuple(int(s) for s in rng.integers(1, 13 if nd == 2 else 6, size=nd))
    kind = (seed // 2) % 3
    L = int(rng.integers(1, 15))
    if kind == 0:
        return rng.integers(0, L + 5, size=shape).astype(np.uint8), L, None
    if kind == 1:
        return rng.integers(0, L + 5, size=shape).astype(np.uint16), L, None
    f = rng.normal(size=shape).astype(np.float32)
    thr = np.sort(rng.normal(size=L)).astype(np.float32)[::-1].copy()  # non-increasing
    if L > 2:
        thr[1] = thr[0]  # repeated threshold
        f.ravel()[0] = thr[-1]  # on a threshold
    if f.size > 3:
        f.ravel()[1] = np.nan
        f.ravel()[2] = np.inf
        f.ravel()[3] = -np.inf
    if f.size > 4:
        f.ravel()[4] = -0.0
    return f, L, thr


def _negated(f, L, thr):
    """The sublevel problem with the same sets: -f at -t (integer levels:
    t_l = L - 1 - l, so -t_l = l - L + 1)."""
    neg_f = -(f.astype(np.float32))
    neg_t = (-thr) if thr is not None else np.arange(L, dtype=np.float32) - (L - 1)
    return neg_f, neg_t.astype(np.float32)


@pytest.mark.parametrize("seed", range(24))
def test_superlevel_is_sublevel_of_negation(seed, o2):
    f, L, thr = _random_case(seed)
    nf, nt = _negated(f, L, thr)
    for conn in ((8, 4) if f.ndim == 2 else (26, 6)):
        a = O1.curves_per_level(f, L, thresholds=thr, connectivity=conn, superlevel=True)
        b = O1.curves_per_level(nf, L, thresholds=nt, connectivity=conn)
        c = o2(f, L, thresholds=thr, connectivity=conn, superlevel=True)
        d = o2(nf, L, thresholds=nt, connectivity=conn)
        for k in a:
            assert np.array_equal(a[k], b[k]), (k, conn)
            assert np.array_equal(a[k], c[k]), (k, conn, a[k], c[k])
            assert np.array_equal(c[k], d[k]), (k, conn)


@pytest.mark.parametrize("seed", range(10))
def test_superlevel_betti_2d(seed, o2):
    rng = np.random.default_rng(950 + seed)
    h, w = (int(x) for x in rng.integers(3, 25, size=2))
    if seed % 2:
        f = rng.integers(0, 12, size=(h, w)).astype(np.uint8)
        L, thr = 12, None
        cs = [L - 1 - lvl for lvl in range(L)]
        sets = [f.astype(np.int64) >= c for c in cs]
    else:
        f = rng.normal(size=(h, w)).astype(np.float32)
        L = 9
        thr = np.linspace(1.5, -1.5, L).astype(np.float32)
        sets = [f >= t for t in thr]
    for conn in (8, 4):
        r = o2(f, L, thresholds=thr, connectivity=conn, superlevel=True)
        for lvl, b in enumerate(sets):
            assert r["ec"][lvl] == _betti_chi_2d(b, conn), (conn, lvl)
            p = np.pad(b, 1)
            perim = int((p[1:, :] != p[:-1, :]).sum() + (p[:, 1:] != p[:, :-1]).sum())
            assert r["perimeter"][lvl] == perim
            assert r["area"][lvl] == int(b.sum())


@pytest.mark.parametrize("seed", range(8))
def test_duality_between_directions(seed, o2):
    rng = np.random.default_rng(970 + seed)
    L = 10
    f2 = rng.integers(0, L, size=(int(rng.integers(2, 12)), int(rng.integers(2, 12)))).astype(np.uint8)
    g2 = np.pad(f2, 1, constant_values=0)  # the pad is active at every sublevel level
    f3 = rng.integers(0, L, size=tuple(int(x) for x in rng.integers(2, 6, size=3))).astype(np.uint8)
    g3 = np.pad(f3, 1, constant_values=0)
    sup8 = o2(f2, L, connectivity=8, superlevel=True)["ec"]
    sup4 = o2(f2, L, connectivity=4, superlevel=True)["ec"]
    sub4 = o2(g2, L, connectivity=4)["ec"]
    sub8 = o2(g2, L, connectivity=8)["ec"]
    sup26 = o2(f3, L, connectivity=26, superlevel=True)["ec"]
    sup6 = o2(f3, L, connectivity=6, superlevel=True)["ec"]
    sub6 = o2(g3, L, connectivity=6)["ec"]
    sub26 = o2(g3, L, connectivity=26)["ec"]
    for c in range(1, L):  # {f >= c} against the padded {f <= c - 1}
        ls, lp = c - 1, L - 1 - c
        assert sub4[ls] == 1 - sup8[lp], c
        assert sub8[ls] == 1 - sup4[lp], c
        assert sub6[ls] == 1 + sup26[lp], c
        assert sub26[ls] == 1 + sup6[lp], c


def test_closed_forms_peak_ring_shell(o2):
    # peak: every superlevel set of a cone is a digital disc
    yy, xx = np.mgrid[0:31, 0:31]
    dist = np.hypot(yy - 15, xx - 15)
    peak = np.maximum(0, 20 - np.rint(2 * dist)).astype(np.uint8)
    for conn in (8, 4):
        assert np.all(o2(peak, 21, connectivity=conn, superlevel=True)["ec"] == 1)
    # ridge ring of radius 9: {f >= c} is the annulus |round(dist) - 9| <= 20 - c
    # until it reaches the centre (c <= 11), then a disc
    ring = np.maximum(0, 20 - np.abs(np.rint(dist) - 9)).astype(np.uint8)
    ec = o2(ring, 21, connectivity=8, superlevel=True)["ec"]
    for lvl in range(21):
        c = 20 - lvl
        assert ec[lvl] == (0 if c > 11 else 1), (c, ec[lvl])
    # ridge shell of radius 6 in 3D, at least three voxels thick: a sphere
    zz, yy3, xx3 = np.mgrid[0:19, 0:19, 0:19]
    d3 = np.sqrt((zz - 9) ** 2 + (yy3 - 9) ** 2 + (xx3 - 9) ** 2)
    shell = np.maximum(0, 12 - np.abs(np.rint(d3) - 6)).astype(np.uint8)
    ec3 = o2(shell, 13, connectivity=26, superlevel=True)["ec"]
    for lvl in range(13):
        c = 12 - lvl
        k = 12 - c  # half-thickness of the shell
        if 1 <= k <= 5:
            assert ec3[lvl] == 2, (c, ec3[lvl])
        if k >= 6:
            assert ec3[lvl] == 1, (c, ec3[lvl])


def test_last_level_is_the_filled_box(o2):
    rng = np.random.default_rng(991)
    f = rng.integers(0, 200, size=(13, 21)).astype(np.uint8)
    r = o2(f, 50, superlevel=True)  # t_49 = 0: every value is >= 0
    assert (r["ec"][-1], r["perimeter"][-1], r["area"][-1]) == (1, 2 * (13 + 21), 13 * 21)
    assert r["area"][0] == int((f >= 49).sum())  # level 0: values >= L - 1
    v = rng.integers(0, 300, size=(5, 7, 9)).astype(np.uint16)
    r3 = o2(v, 40, superlevel=True)
    d, h, w = v.shape
    assert (r3["ec"][-1], r3["perimeter"][-1], r3["area"][-1], r3["volume"][-1]) == \
        (1, 4 * (d + h + w), 2 * (h * w + h * d + w * d), d * h * w)


@pytest.mark.parametrize("seed", range(12))
def test_o1_equals_o2_superlevel(seed, o2):
    f, L, thr = _random_case(100 + seed)
    for conn in ((8, 4) if f.ndim == 2 else (26, 6)):
        a = O1.curves_per_level(f, L, thresholds=thr, connectivity=conn, superlevel=True)
        b = o2(f, L, thresholds=thr, connectivity=conn, superlevel=True, n_threads=4)
        for k in a:
            assert np.array_equal(a[k], b[k]), (k, conn)


def test_oracle_rejects_increasing_superlevel_thresholds(o2):
    f = np.zeros((3, 3), np.float32)
    with pytest.raises(ValueError):
        o2(f, 3, thresholds=np.array([0, 1, 2], np.float32), superlevel=True)
    with pytest.raises(ValueError):
        o2(f, 3, thresholds=np.array([2, 1, 0], np.float32))


class _OracleField(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dtype", ctypes.c_int32), ("shape", ctypes.c_int64 * 3),
                ("data", ctypes.c_void_p), ("n_levels", ctypes.c_int32), ("connectivity", ctypes.c_int32),
                ("thresholds", ctypes.c_void_p), ("filtration", ctypes.c_int32)]


class _OracleCurves(ctypes.Structure):
    _fields_ = [("ec", ctypes.c_void_p), ("perimeter", ctypes.c_void_p), ("area", ctypes.c_void_p),
                ("volume", ctypes.c_void_p)]


@pytest.mark.parametrize("superlevel", [False, True])
def test_oracle_compute_struct_entry(superlevel, o2):
    """ecc_oracle_compute (field and curves descriptors, host pointers) gives
    what the spelled-out entry gives, and rejects bad requests with 1."""
    oracle.build_o2(force=False)
    lib = ctypes.CDLL(oracle._LIB)
    fn = lib.ecc_oracle_compute
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
    rng = np.random.default_rng(7)
    a = rng.normal(size=(6, 9, 11)).astype(np.float32)
    L = 20
    thr = np.linspace(-2, 2, L).astype(np.float32)
    if superlevel:
        thr = thr[::-1].copy()
    f = _OracleField(3, 3, (ctypes.c_int64 * 3)(*a.shape), a.ctypes.data, L, 0, thr.ctypes.data,
                     1 if superlevel else 0)
    out = {k: np.zeros(L, np.int64) for k in ("ec", "perimeter", "area", "volume")}
    cv = _OracleCurves(*(out[k].ctypes.data for k in ("ec", "perimeter", "area", "volume")))
    assert fn(ctypes.byref(f), ctypes.byref(cv), 2) == 0
    ref = o2(a, L, thresholds=thr, superlevel=superlevel)
    for k in out:
        assert np.array_equal(out[k], ref[k]), k
    f.filtration = 2
    assert fn(ctypes.byref(f), ctypes.byref(cv), 1) == 1
    f.filtration = 0 if superlevel else 1  # thresholds now run the wrong way
    assert fn(ctypes.byref(f), ctypes.byref(cv), 1) == 1


# ----------------------------------------------------------------------------
# vertex classes (contribution map) in the superlevel direction
# ----------------------------------------------------------------------------
TYPE_TO_CLASS = {"q0": -1, "q1": 0, "q2": 1, "qd": 2, "q3": 3, "q4": 4}


@pytest.mark.parametrize("seed", range(8))
def test_vertex_classes_superlevel(seed):
    f, L, thr = _random_case(200 + 2 * seed)  # 2D cases
    assert f.ndim == 2
    ev = oracle.vertex_classes_2d(f, L, thr, superlevel=True)
    assert np.array_equal(ev, oracle.vertex_classes_per_level(f, L, thr, superlevel=True))
    nf, nt = _negated(f, L, thr)
    assert np.array_equal(ev, oracle.vertex_classes_2d(nf, L, nt))
    t1 = PT.table1()
    example = {}
    for m, e in t1.items():
        example.setdefault(TYPE_TO_CLASS[e["type"]], e)
    ref8 = O1.curves_per_level(f, L, thr, connectivity=8, superlevel=True)
    ref4 = O1.curves_per_level(f, L, thr, connectivity=4, channels=("ec",), superlevel=True)
    for col, ref in (("ec8", ref8["ec"]), ("ec4", ref4["ec"]), ("perimeter", ref8["perimeter"]),
                     ("area", ref8["area"])):
        for lvl in range(L):
            s = sum(Fraction(int(ev[c, lvl])) * example[c][col] for c in range(5))
            assert s == ref[lvl], (col, lvl)


@pytest.mark.parametrize("seed", range(6))
def test_vertex_classes_3d_superlevel(seed):
    f, L, thr = _random_case(301 + 2 * seed)  # 3D cases
    assert f.ndim == 3
    ev = oracle.vertex_classes_3d(f, L, thr, superlevel=True)
    assert np.array_equal(ev, oracle.vertex_classes_3d_per_level(f, L, thr, superlevel=True))
    nf, nt = _negated(f, L, thr)
    assert np.array_equal(ev, oracle.vertex_classes_3d(nf, L, nt))
