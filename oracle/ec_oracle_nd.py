"""Oracle for fields of any dimension n (used for 4D fields), TEST INFRASTRUCTURE ONLY.

Nothing in the product imports this module; only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg may call it.
It shares no code, table or constant with the HIP library or with the 2D/3D
oracles (which pin it: for n = 2 and 3 it must give their curves).

The paper treats 2D and 3D fields and names higher dimensions (4D data such
as hyperspectral images over time) as future work (Conclusions).  The
definitions carry over unchanged (Methodology): the sublevel filtration of
Eq. (2) (or its superlevel mirror), the complex at a level is the union of
the closed active top cells (the n-cubes), and its Euler characteristic is the
alternating count of Eq. (1) over cells of every dimension.

* Closure (T-) construction, the connectivity the paper uses (8-C in 2D,
  26-C in 3D; 80-C in 4D): a lattice cell with extent e in {0,1}^n at lattice
  point p is present when any of the 2^(n-|e|) top cells around it is active.
* Face-adjacency (V-) construction (4-C, 6-C; 8-C in 4D): active top cells are
  vertices, and a block of 2^k cells spanning k axes is a k-cell when all of
  them are active.
* boundary: unit (n-1)-faces with exactly one active neighbouring top cell
  (2D perimeter, 3D surface); volume: active top cells.

``curves_per_level`` binarises at every level and counts (O1 form);
``curves_all_levels`` takes the level at which every cell enters and
histograms them (O2 form).  Both are plain numpy over shifted arrays.
"""
from __future__ import annotations

import itertools

import numpy as np

__all__ = ["level_index", "ec_closure", "ec_faces", "boundary", "curves_per_level", "curves_all_levels"]


def level_index(field, n_levels: int, thresholds=None, superlevel: bool = False) -> np.ndarray:
    """Level at which each top cell becomes active (Eq. (2) or its mirror);
    n_levels for never.  Integer levels: t_l = l (superlevel: t_l = L - 1 - l)."""
    field = np.asarray(field)
    L = int(n_levels)
    if thresholds is None:
        v = field.astype(np.int64)
        return np.maximum(L - 1 - v, 0) if superlevel else np.where(v < L, v, L)
    t = np.asarray(thresholds, dtype=np.float32)
    x = field.astype(np.float32)
    lam = np.full(x.shape, L, dtype=np.int64)
    for lvl in range(L - 1, -1, -1):  # the first l that holds wins
        lam[(x >= t[lvl]) if superlevel else (x <= t[lvl])] = lvl
    return lam


def _extents(n):
    return list(itertools.product((0, 1), repeat=n))


def _shift(a, offs):
    """a[p + offs] over the lattice points of a cell family (views of a padded array)."""
    sl = tuple(slice(o, o + s) for o, s in zip(offs, a.shape))
    return sl


def ec_closure(b: np.ndarray) -> int:
    """chi of the union of the closed active n-cubes (any n)."""
    n = b.ndim
    p = np.pad(b.astype(bool), 1)  # padded cells; lattice point q touches cells q-1 .. q (per axis)
    chi = 0
    for e in _extents(n):
        # cells with extent e: along axes with e_i = 1 the cell is one unit
        # long and lies between lattice points (index = cell index), along the
        # others it sits on a lattice point q shared by cells q-1 and q
        shape = tuple(b.shape[i] + (0 if e[i] else 1) for i in range(n))
        present = np.zeros(shape, dtype=bool)
        free = [i for i in range(n) if not e[i]]
        for d in itertools.product((0, 1), repeat=len(free)):
            offs = [1] * n  # padded index of cell i is i + 1
            for k, ax in enumerate(free):
                offs[ax] = d[k]  # cells q - 1 + d at lattice point q
            present |= p[tuple(slice(offs[i], offs[i] + shape[i]) for i in range(n))]
        chi += (-1) ** sum(e) * int(present.sum())
    return chi


def ec_faces(b: np.ndarray) -> int:
    """chi of the complex whose k-cells are fully active blocks of 2^k top
    cells spanning k axes (vertices = active cells)."""
    n = b.ndim
    b = b.astype(bool)
    chi = 0
    for e in _extents(n):
        shape = tuple(b.shape[i] - e[i] for i in range(n))
        if min(shape) <= 0:
            continue
        full = np.ones(shape, dtype=bool)
        span = [i for i in range(n) if e[i]]
        for d in itertools.product((0, 1), repeat=len(span)):
            offs = [0] * n
            for k, ax in enumerate(span):
                offs[ax] = d[k]
            full &= b[tuple(slice(offs[i], offs[i] + shape[i]) for i in range(n))]
        chi += (-1) ** sum(e) * int(full.sum())
    return chi


def boundary(b: np.ndarray) -> int:
    """Unit (n-1)-faces with exactly one active neighbouring top cell."""
    p = np.pad(b.astype(bool), 1)
    tot = 0
    for ax in range(b.ndim):
        a0 = np.take(p, range(0, p.shape[ax] - 1), axis=ax)
        a1 = np.take(p, range(1, p.shape[ax]), axis=ax)
        tot += int((a0 != a1).sum())
    return tot


def _default_conn(n):
    return 3 ** n - 1


def curves_per_level(field, n_levels: int, thresholds=None, connectivity=None, superlevel: bool = False,
                     levels=None):
    """O1 form: binarise at every requested level and count.  connectivity:
    3^n - 1 (closure, default) or 2n (face adjacency).  Returns dict with ec,
    boundary and volume over `levels` (all by default)."""
    field = np.asarray(field)
    n = field.ndim
    conn = connectivity or _default_conn(n)
    if conn not in (_default_conn(n), 2 * n):
        raise ValueError(f"connectivity must be {_default_conn(n)} or {2 * n} for {n}D fields")
    lam = level_index(field, n_levels, thresholds, superlevel)
    levels = list(range(n_levels)) if levels is None else list(levels)
    out = {k: np.zeros(len(levels), dtype=np.int64) for k in ("ec", "boundary", "volume")}
    for k, lvl in enumerate(levels):
        b = lam <= lvl
        out["ec"][k] = ec_closure(b) if conn == _default_conn(n) else ec_faces(b)
        out["boundary"][k] = boundary(b)
        out["volume"][k] = int(b.sum())
    return out


def curves_all_levels(field, n_levels: int, thresholds=None, connectivity=None, superlevel: bool = False):
    """O2 form: the level at which every lattice cell enters (closure: the
    smallest level of the top cells around it; face adjacency: the largest of
    its block), histogrammed by dimension and summed over levels."""
    field = np.asarray(field)
    n = field.ndim
    L = int(n_levels)
    conn = connectivity or _default_conn(n)
    if conn not in (_default_conn(n), 2 * n):
        raise ValueError(f"connectivity must be {_default_conn(n)} or {2 * n} for {n}D fields")
    lam = level_index(field, L, thresholds, superlevel)
    p = np.pad(lam, 1, constant_values=L)
    hist = np.zeros((3, L + 1), dtype=np.int64)  # ec, boundary, volume
    for e in _extents(n):
        sign = (-1) ** sum(e)
        if conn == _default_conn(n):
            shape = tuple(field.shape[i] + (0 if e[i] else 1) for i in range(n))
            entry = np.full(shape, L, dtype=np.int64)
            free = [i for i in range(n) if not e[i]]
            for d in itertools.product((0, 1), repeat=len(free)):
                offs = [1] * n
                for k, ax in enumerate(free):
                    offs[ax] = d[k]
                entry = np.minimum(entry, p[tuple(slice(offs[i], offs[i] + shape[i]) for i in range(n))])
        else:
            shape = tuple(field.shape[i] - e[i] for i in range(n))
            if min(shape) <= 0:
                continue
            entry = np.zeros(shape, dtype=np.int64)
            span = [i for i in range(n) if e[i]]
            for d in itertools.product((0, 1), repeat=len(span)):
                offs = [0] * n
                for k, ax in enumerate(span):
                    offs[ax] = d[k]
                entry = np.maximum(entry, lam[tuple(slice(offs[i], offs[i] + shape[i]) for i in range(n))])
        np.add.at(hist[0], entry.ravel(), sign)
    # boundary faces: +1 when the first of the two cells enters, -1 when the second does
    for ax in range(n):
        a0 = np.take(p, range(0, p.shape[ax] - 1), axis=ax).ravel()
        a1 = np.take(p, range(1, p.shape[ax]), axis=ax).ravel()
        np.add.at(hist[1], np.minimum(a0, a1), 1)
        np.add.at(hist[1], np.maximum(a0, a1), -1)
    np.add.at(hist[2], lam.ravel(), 1)
    cum = np.cumsum(hist[:, :L], axis=1)
    return {"ec": cum[0], "boundary": cum[1], "volume": cum[2]}
