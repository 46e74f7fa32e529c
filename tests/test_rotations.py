"""600-cell rotation sets (eq. (2.7)) and the adaptive refinement rule (eq. (3.1)).

Pins: the counts the paper prints for eq. (2.7) (tests/golden/mrot_600cell.json);
the 60 rotations of d = 1 are the binary icosahedral group (closed under
quaternion products up to sign); every rotation of a refinement is distinct;
the prior weights track Haar (Voronoi) volumes estimated by Monte Carlo better
than equal weights do; spherical caps hold their Haar share ever more closely as
d grows."""
import json
import os

import numpy as np
import pytest

from paper_1409_4256_amd import rotations as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mrot_600cell.json")


def test_counts_printed_in_the_paper():
    g = json.load(open(GOLDEN))
    for d, m in zip(g["d"], g["mrot"]):
        assert R.mrot(d) == m
    for d, m in zip(g["d"][:3], g["mrot"][:3]):      # d = 5, 6, 8 built in full
        q, lw = R.rotation_set(d)
        assert q.shape == (m, 4) and lw.shape == (m,)


@pytest.mark.parametrize("d", [1, 2, 3, 4, 7])
def test_count_formula_and_unit_quaternions(d):
    q, lw = R.rotation_set(d)
    assert len(q) == 10 * (5 * d ** 3 + d)
    np.testing.assert_allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(np.exp(lw).sum(), 1.0, rtol=1e-12)
    # distinct rotations: q and -q are the same rotation, so |q . q'| < 1 for every pair
    if len(q) <= 5000:
        G = np.abs(q @ q.T)
        np.fill_diagonal(G, 0.0)
        assert G.max() < 1.0 - 1e-6
    else:   # nearest neighbour among a sample of rotations
        G = np.abs(q[::97] @ q.T)
        G[np.arange(G.shape[0]), np.arange(0, len(q), 97)] = 0.0
        assert G.max() < 1.0 - 1e-6


def _qmul(a, b):
    w1, x1, y1, z1 = a.T
    w2, x2, y2, z2 = b.T
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=-1)


def test_d1_is_the_binary_icosahedral_group():
    q, lw = R.rotation_set(1)
    assert len(q) == 60
    np.testing.assert_allclose(np.exp(lw), 1.0 / 60, rtol=1e-12)
    a = np.repeat(q, 60, axis=0)
    b = np.tile(q, (60, 1))
    prod = _qmul(a, b)
    best = np.abs(prod @ q.T).max(axis=1)           # every product is in the set (up to sign)
    np.testing.assert_allclose(best, 1.0, atol=1e-12)


def test_weights_track_haar_voronoi_volumes():
    """Monte Carlo: the Haar share of each rotation's Voronoi cell (nearest rotation,
    q ~ -q) against the prior weights, at d = 2 (420 rotations, 2e6 samples)."""
    q, lw = R.rotation_set(2)
    w = np.exp(lw)
    rng = np.random.default_rng(2024)
    cnt = np.zeros(len(q))
    for _ in range(40):
        X = rng.standard_normal((50000, 4))
        X /= np.linalg.norm(X, axis=1)[:, None]
        cnt += np.bincount(np.argmax(np.abs(X @ q.T), axis=1), minlength=len(q))
    vol = cnt / cnt.sum()
    err_w = np.sqrt(((w - vol) ** 2).mean()) / vol.mean()
    err_u = np.sqrt(((1.0 / len(q) - vol) ** 2).mean()) / vol.mean()
    assert err_w < 0.8 * err_u
    assert np.corrcoef(w, vol)[0, 1] > 0.85


def test_caps_approach_their_haar_share():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((300, 4))
    A /= np.linalg.norm(A, axis=1)[:, None]
    th = 0.35
    share = 2.0 * (2.0 * th - np.sin(2.0 * th)) / (2.0 * np.pi)   # |q . a| >= cos th on the unit 3-sphere
    errs = []
    for d in (2, 3, 5):
        q, lw = R.rotation_set(d)
        inside = np.abs(q @ A.T) >= np.cos(th)
        e = (np.exp(lw)[:, None] * inside).sum(axis=0) - share
        errs.append(np.sqrt((e ** 2).mean()) / share)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.05


def test_adaptive_rule():
    """eq. (3.1): raise d by one when |L^n - L^(n-1)| <= 0.01 |L^n|, up to d_max."""
    assert R.next_refinement(None, -100.0, 3, 8) == 3
    assert R.next_refinement(-100.0, -99.5, 3, 8) == 4        # change 0.5 <= 0.995
    assert R.next_refinement(-100.0, -98.0, 3, 8) == 3        # change 2 > 0.98
    assert R.next_refinement(-100.0, -99.5, 8, 8) == 8        # at d_max
    assert R.next_refinement(-100.0, -100.0, 5, 8, tol=0.0) == 6


def _rotation_set_by_loops(d):
    """The rotation set written as plain loops over cells and compositions (a dict
    of points keyed by their (vertex, weight) pairs): the vectorised builder must
    reproduce it bit for bit, order and signs included."""
    import itertools

    V = R.vertices_600cell()
    C = R.cells_600cell(V)
    anti = np.array([int(np.argmin(np.abs(V + V[a]).sum(axis=1))) for a in range(len(V))])
    comps = [c for c in itertools.product(range(d + 1), repeat=4) if sum(c) == d]
    points = {}
    for cell in C:
        for comp in comps:
            key = tuple(sorted((int(cell[t]), comp[t]) for t in range(4) if comp[t] > 0))
            akey = tuple(sorted((int(anti[v]), k) for v, k in key))
            if akey < key:
                key = akey
            if key not in points:
                points[key] = sum(k * V[v] for v, k in key) / d
    P = np.array([points[k] for k in sorted(points)])
    r = np.linalg.norm(P, axis=1)
    w = r ** -4.0
    return P / r[:, None], np.log(w / w.sum())


@pytest.mark.parametrize("d", [1, 2, 3, 5])
def test_vectorised_builder_equals_the_loops(d):
    q, lw = R.rotation_set(d)
    q0, lw0 = _rotation_set_by_loops(d)
    assert np.array_equal(q, q0) and np.array_equal(lw, lw0)
