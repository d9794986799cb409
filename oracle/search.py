"""Greedy angle-similarity search for low-complexity DCT rows (Sec. 3, Sec. 4.1).

TEST INFRASTRUCTURE: see the package docstring.

The method (Eq. (5), Eq. (6) and the algorithm of Sec. 3.5): for an ordering of
the DCT rows, approximate each row c_k in turn by the vector d of the search
space D = P^8 with the smallest angle to c_k among those orthogonal to every
row already chosen.  Sec. 4.1 fixes rows 1 and 5 to the trivial +-1 vectors and
runs the remaining 6! = 720 orders.

Readings taken here (the paper's algorithm listing is ambiguous on these):
  * the orthogonality filter requires every inner product with the chosen
    rows to vanish (the text of Sec. 3.4 and the constraint of Eq. (6)), not
    their sum;
  * the zero vector is not a candidate (its angle is undefined);
  * an order whose feasible set runs empty at some row is dead and yields no
    matrix (the listing would silently keep the first vector);
  * exact ties in angle are real (scalar multiples, mirror images and equal
    irrational angles).  The listing's strict '<' over an enumeration order
    that Tables 3-4 print inconsistently cannot be reproduced, so two forms
    are given: `closure` returns every matrix reachable under any resolution
    of the exact ties; `canonical` resolves them by a fixed rule (largest
    cosine, cosines within TIE_EPS grouped; then smaller squared norm; then
    smaller canonical index).
The angle is minimised through its cosine: arccos is decreasing.
"""

from __future__ import annotations

import itertools
import math

import numpy as np

from .matrices import dct_matrix

TIE_EPS = 1e-12          # cosines closer than this are an exact tie in reals
FIXED_ROWS = {0: np.array([1, 1, 1, 1, 1, 1, 1, 1]),
              4: np.array([1, -1, -1, 1, 1, -1, -1, 1])}
FREE_ROWS = (1, 2, 3, 5, 6, 7)

P1 = (0, 1, -1)
P2 = (0, 1, -1, 2, -2)
P4 = (0, 1, -1, 2, -2, 3, -3, 4, -4)


def canonical_digits(p) -> list[int]:
    """P ordered (0, 1, -1, 2, -2, ...): the digit order of the canonical index."""
    return sorted(set(int(v) for v in p), key=lambda v: (abs(v), v < 0))


def search_space(p, include_zero: bool = False) -> tuple[np.ndarray, np.ndarray]:
    """All of P^8 as an (|P|^8, 8) int64 array in canonical odometer order
    (first coordinate most significant), with their canonical indices.
    The zero vector (index 0) is dropped unless asked for."""
    digs = np.array(canonical_digits(p), dtype=np.int64)
    b = len(digs)
    idx = np.arange(b ** 8, dtype=np.int64)
    cols = [(idx // b ** (7 - k)) % b for k in range(8)]
    d = digs[np.stack(cols, axis=1)]
    if not include_zero:
        d, idx = d[1:], idx[1:]
    return d, idx


def cosines(d: np.ndarray, row: np.ndarray) -> np.ndarray:
    """cos angle(d, row) = <d, row> / (||d|| ||row||) (Sec. 3.3)."""
    d = np.asarray(d, dtype=np.float64)
    return (d @ row) / (np.sqrt(np.sum(d * d, axis=1)) * np.linalg.norm(row))


def top_group(cos: np.ndarray) -> np.ndarray:
    """Indices (into cos) of the best tie group: sort descending and extend
    while consecutive values differ by at most TIE_EPS."""
    near = np.flatnonzero(cos >= cos.max() - 1e-6)      # a superset, for speed
    order = near[np.argsort(-cos[near], kind="stable")]
    k = 1
    while k < len(order) and cos[order[k - 1]] - cos[order[k]] <= TIE_EPS:
        k += 1
    return order[:k]


class _Space:
    def __init__(self, p):
        self.d, self.idx = search_space(p)
        self.norm2 = np.sum(self.d * self.d, axis=1)
        c = dct_matrix()
        self.cos = np.stack([cosines(self.d, c[k]) for k in range(8)])

    def ortho_mask(self, t: np.ndarray) -> np.ndarray:
        return (self.d @ t) == 0


def _canonical_pick(space: _Space, cand: np.ndarray, row: int) -> int:
    grp = cand[top_group(space.cos[row, cand])]
    key = np.lexsort((space.idx[grp], space.norm2[grp]))
    return int(grp[key[0]])


def greedy_canonical(p, order, fixed: dict | None = FIXED_ROWS, space=None):
    """One greedy pass (Eq. (6)) over the rows in `order` with canonical tie
    breaking.  Returns the 8x8 matrix, or None if the order is dead."""
    space = space or _Space(p)
    fixed = fixed or {}
    rows = dict(fixed)
    mask = np.ones(len(space.d), dtype=bool)
    for t in rows.values():
        mask &= space.ortho_mask(t)
    for k in order:
        cand = np.flatnonzero(mask)
        if cand.size == 0:
            return None
        j = _canonical_pick(space, cand, k)
        rows[k] = space.d[j]
        mask &= space.ortho_mask(space.d[j])
        mask[j] = False
    return np.stack([rows[k] for k in range(8)])


def closure(p, orders=None, fixed: dict | None = FIXED_ROWS):
    """Every matrix the greedy search reaches over `orders` (default: all
    orders of the free rows) under any resolution of exact ties.

    Returns (matrices as a sorted list of 8x8 arrays, leaves, dead_leaves):
    `leaves` counts completed (order, tie-branch) paths, `dead_leaves` the
    paths that ran out of feasible candidates."""
    space = _Space(p)
    fixed = fixed or {}
    if orders is None:
        free = [k for k in range(8) if k not in fixed]
        orders = list(itertools.permutations(free))
    found: dict[bytes, np.ndarray] = {}
    stats = {"leaves": 0, "dead": 0}
    base = np.ones(len(space.d), dtype=bool)
    for t in fixed.values():
        base &= space.ortho_mask(t)
    # Walk a prefix tree of the orders so shared prefixes are expanded once.
    tree: dict = {}
    for o in orders:
        node = tree
        for k in o:
            node = node.setdefault(k, {})

    def walk(node, rows, mask):
        if not node:
            t = np.stack([rows[k] for k in range(8)])
            found[t.astype(np.int8).tobytes()] = t
            stats["leaves"] += 1
            return
        for k, child in node.items():
            cand = np.flatnonzero(mask)
            if cand.size == 0:
                stats["dead"] += _count_leaves(child)
                continue
            for j in cand[top_group(space.cos[k, cand])]:
                m2 = mask & space.ortho_mask(space.d[j])
                m2[j] = False
                walk(child, {**rows, k: space.d[j]}, m2)

    walk(tree, dict(fixed), base)
    mats = [found[k] for k in sorted(found)]
    return mats, stats["leaves"], stats["dead"]


def _count_leaves(node) -> int:
    return 1 if not node else sum(_count_leaves(c) for c in node.values())


# --------------------------------------------------------------------------
# Top-k scan over a large search space (P = {0, +-1, .., +-4}, 9^8 vectors)
# --------------------------------------------------------------------------

def _gcd_rows(d: np.ndarray) -> np.ndarray:
    g = np.abs(d[:, 0])
    for k in range(1, d.shape[1]):
        g = np.gcd(g, np.abs(d[:, k]))
    return g


def topk_scan(p, k: int, primitive: bool = True, chunk: int = 1 << 21,
              pool_factor: int = 4):
    """Per DCT row, the k candidates of P^8 with the smallest angle, in
    canonical order (cosine tie groups, then squared norm, then index).

    Reading: with `primitive`, only vectors whose entries have gcd 1 compete;
    a positive multiple of a row gives the same normalised row of S T, so the
    multiples are duplicates.  Returns a list of 8 dicts with 'vec' (k, 8),
    'idx' (k,), 'cos' (k,)."""
    digs = np.array(canonical_digits(p), dtype=np.int64)
    b = len(digs)
    total = b ** 8
    c = dct_matrix()
    pool = k * pool_factor
    keep_idx = [np.empty(0, np.int64) for _ in range(8)]
    keep_cos = [np.empty(0, np.float64) for _ in range(8)]
    for lo in range(1, total, chunk):
        idx = np.arange(lo, min(total, lo + chunk), dtype=np.int64)
        cols = [(idx // b ** (7 - q)) % b for q in range(8)]
        d = digs[np.stack(cols, axis=1)]
        if primitive:
            sel = _gcd_rows(d) == 1
            d, idx = d[sel], idx[sel]
        df = d.astype(np.float64)
        nrm = np.sqrt(np.sum(df * df, axis=1))
        cs = (df @ c.T) / nrm[:, None]
        for row in range(8):
            ci = np.concatenate([keep_cos[row], cs[:, row]])
            ii = np.concatenate([keep_idx[row], idx])
            if ci.size > pool:
                part = np.argpartition(-ci, pool - 1)[:pool]
                ci, ii = ci[part], ii[part]
            keep_cos[row], keep_idx[row] = ci, ii
    out = []
    for row in range(8):
        ci, ii = keep_cos[row], keep_idx[row]
        cols = [(ii // b ** (7 - q)) % b for q in range(8)]
        vec = digs[np.stack(cols, axis=1)]
        order = canonical_order(ci, np.sum(vec * vec, axis=1), ii)
        # the pool must extend past the tie group that straddles position k
        last = ci[order[min(k, len(order)) - 1]]
        inside = np.sum(ci >= last - TIE_EPS * 64)
        if inside >= len(ci) and len(ci) < (total - 1):
            raise RuntimeError("top-k pool too small for the tie group at the boundary")
        order = order[:k]
        out.append({"vec": vec[order], "idx": ii[order], "cos": ci[order]})
    return out


def canonical_order(cos: np.ndarray, norm2: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Canonical ranking: tie groups of cosine (single linkage within TIE_EPS on
    the sorted values, best group first), then squared norm, then index."""
    o = np.argsort(-cos, kind="stable")
    grp = np.zeros(len(o), dtype=np.int64)
    for a in range(1, len(o)):
        grp[a] = grp[a - 1] + (1 if cos[o[a - 1]] - cos[o[a]] > TIE_EPS else 0)
    key = np.lexsort((idx[o], norm2[o], grp))
    return o[key]


def orthogonal_tuples_py(lists: list[np.ndarray], limit: int | None = None) -> list[tuple]:
    """All 8-tuples (one entry per row's list, by position) whose vectors are
    pairwise orthogonal -- a plain depth-first enumeration.  Tuples come out
    in lexicographic order of positions."""
    out: list[tuple] = []
    vecs = [np.asarray(l, dtype=np.int64) for l in lists]

    def rec(row, chosen):
        if limit is not None and len(out) >= limit:
            return
        if row == len(vecs):
            out.append(tuple(chosen))
            return
        for a in range(len(vecs[row])):
            v = vecs[row][a]
            if all(int(v @ vecs[r][chosen[r]]) == 0 for r in range(row)):
                rec(row + 1, chosen + [a])

    rec(0, [])
    return out


def row_angles_deg(t: np.ndarray) -> np.ndarray:
    """Angle in degrees between each row of T and the matching DCT row."""
    c = dct_matrix()
    t = np.asarray(t, dtype=np.float64)
    cs = np.sum(t * c, axis=1) / np.linalg.norm(t, axis=1)
    return np.degrees(np.arccos(np.clip(cs, -1.0, 1.0)))
