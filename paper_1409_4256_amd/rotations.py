"""Rotation sets of the 600-cell refined d times (eq. (2.7)) and the adaptive
refinement rule of adaptive EMC (eq. (3.1)).  Host-side set-up: a rotation set is
built once per refinement level and handed to the GPU path as quaternions and
log prior weights.

The 600-cell's 120 vertices are unit quaternions; its 600 tetrahedral cells are
the 4-cliques of vertices 36 degrees apart.  Refinement d puts the points
(i v0 + j v1 + k v2 + l v3) / d, i + j + k + l = d, on every cell; a point on a
shared vertex, edge or face is the same combination of the same global vertices
in every cell holding it, so points are merged exactly by that combination.
Projected to the unit sphere and taken once per pair (q, -q) (the same rotation),
they number 10 (5 d^3 + d).

Prior weights: the points are evenly spaced on the flat cells, and the radial
projection of a cell at distance h from the origin onto the unit 3-sphere scales
volume by h / |p|^4, so w_j is proportional to |p_j|^-4 (normalised to sum 1).
"""
from __future__ import annotations

import functools
import itertools
import math

import numpy as np

PHI = (1.0 + math.sqrt(5.0)) / 2.0


def mrot(d: int) -> int:
    """Number of rotations of refinement d, eq. (2.7)."""
    return 10 * (5 * d ** 3 + d)


def _even_permutations(n):
    out = []
    for p in itertools.permutations(range(n)):
        inv = sum(1 for a in range(n) for b in range(a + 1, n) if p[a] > p[b])
        if inv % 2 == 0:
            out.append(p)
    return out


def vertices_600cell() -> np.ndarray:
    """The 120 vertices (unit quaternions (w, x, y, z)) of the 600-cell."""
    v = set()
    for i in range(4):
        for s in (1.0, -1.0):
            e = [0.0] * 4
            e[i] = s
            v.add(tuple(e))
    for signs in itertools.product((0.5, -0.5), repeat=4):
        v.add(signs)
    base = (PHI / 2.0, 0.5, 1.0 / (2.0 * PHI), 0.0)
    for p in _even_permutations(4):
        for signs in itertools.product((1.0, -1.0), repeat=3):
            vals = [base[0] * signs[0], base[1] * signs[1], base[2] * signs[2], 0.0]
            e = [0.0] * 4
            for src, dst in enumerate(p):
                e[dst] = vals[src]
            v.add(tuple(round(x, 15) + 0.0 for x in e))
    out = np.array(sorted(v))
    assert out.shape == (120, 4)
    return out


def cells_600cell(V: np.ndarray) -> np.ndarray:
    """The 600 tetrahedral cells: sorted index 4-tuples of mutually adjacent vertices
    (adjacent: 36 degrees apart, dot product phi / 2)."""
    adj = np.abs(V @ V.T - PHI / 2.0) < 1e-9
    nb = [set(np.flatnonzero(adj[a])) for a in range(len(V))]
    cells = set()
    for a in range(len(V)):
        for b in nb[a]:
            if b <= a:
                continue
            common = sorted(nb[a] & nb[b])
            for c, e in itertools.combinations(common, 2):
                if e in nb[c]:
                    cells.add(tuple(sorted((a, b, c, e))))
    out = np.array(sorted(cells))
    assert out.shape == (600, 4)
    return out


def _compositions(d: int) -> np.ndarray:
    """The (i, j, k, l) >= 0 with i + j + k + l = d, in lexicographic order."""
    return np.array([c for c in itertools.product(range(d + 1), repeat=4) if sum(c) == d], dtype=np.int64)


@functools.lru_cache(maxsize=None)
def _cells():
    V = vertices_600cell()
    C = cells_600cell(V)
    # antipode of each vertex: the 600-cell is centrally symmetric
    anti = np.array([int(np.argmin(np.abs(V + V[a]).sum(axis=1))) for a in range(len(V))])
    return V, C, anti


def rotation_set(d: int):
    """(quat [Mrot(d)][4] float64 unit quaternions, log_w [Mrot(d)] float64) of refinement d >= 1.

    Every (cell, composition) names a point by its key, the (vertex, weight) pairs
    of its non-zero weights in ascending vertex order; a pair (p, -p) is kept once,
    under the lexicographically smaller of the key and its antipode's key.  Keys
    are packed into integers (base-B digits, one per pair, missing pairs 0, so that
    integer order is the tuples' lexicographic order), so the merge is one sort."""
    if d < 1:
        raise ValueError("refinement d must be >= 1")
    V, C, anti = _cells()
    comps = _compositions(d)
    B = 121 * (d + 1) + 1               # pair code 1 + v (d + 1) + k < B
    v = np.repeat(C, len(comps), axis=0).reshape(len(C), len(comps), 4)   # [cell][comp][t]
    k = np.broadcast_to(comps[None, :, :], v.shape)

    def pack(vv, kk):
        # pairs with k > 0 in ascending vertex order, then empty digits
        code = np.where(kk > 0, 1 + vv * (d + 1) + kk, 0)
        order = np.argsort(np.where(kk > 0, vv, 1 << 20), axis=-1, kind="stable")
        code = np.take_along_axis(code, order, axis=-1)
        key = np.zeros(code.shape[:-1], dtype=np.int64)
        for t in range(4):
            key = key * B + code[..., t]
        return key, np.take_along_axis(vv, order, axis=-1), np.take_along_axis(kk, order, axis=-1)

    key, vs, ks = pack(v, k)
    akey, avs, aks = pack(anti[v], k)
    use_anti = akey < key
    key = np.where(use_anti, akey, key).reshape(-1)
    vs = np.where(use_anti[..., None], avs, vs).reshape(-1, 4)
    ks = np.where(use_anti[..., None], aks, ks).reshape(-1, 4)
    uniq, first = np.unique(key, return_index=True)      # sorted keys: the order of the set
    vs, ks = vs[first], ks[first]
    # sum of k V[v] over the key's pairs in order, then / d (empty pairs add exact zeros last)
    P = ks[:, 0, None] * V[vs[:, 0]]
    for t in range(1, 4):
        P = P + np.where(ks[:, t, None] > 0, ks[:, t, None] * V[vs[:, t]], 0.0)
    P = P / d
    r = np.linalg.norm(P, axis=1)
    quat = P / r[:, None]
    w = r ** -4.0
    log_w = np.log(w / w.sum())
    return quat, log_w


def next_refinement(L_prev: float | None, L_cur: float, d: int, d_max: int, tol: float = 0.01) -> int:
    """Adaptive EMC, eq. (3.1): raise d by one when the log-likelihood changed by at most
    tol |L^n| since the previous iteration (and d is below d_max)."""
    if L_prev is None or d >= d_max:
        return d
    return d + 1 if abs(L_cur - L_prev) <= tol * abs(L_cur) else d
