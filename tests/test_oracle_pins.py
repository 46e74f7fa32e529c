"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a library routine (scipy,
mpmath), a brute-force construction from the definition of the interpolation
weights over every grid point, a closed form, an invariant of the method, or
numbers the paper prints.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import gammaln
from scipy.stats import poisson

import oracle as O
from emc_inputs import shoemake_quaternions, tiny_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(s):
    return np.random.default_rng(1000 + s)


def _scipy_R(quat):
    q = np.asarray(quat, dtype=np.float64)
    return Rotation.from_quat(np.concatenate([q[..., 1:], q[..., :1]], axis=-1)).as_matrix()


def _dense_F(q, quat, grid_n):
    """F[l, j, i] = prod_a max(0, 1 - |p_l - (R_j q_i + N/2)|_a) over EVERY grid point l.

    Positions use scipy's rotation (not the oracle's), grid points are
    enumerated with the flat index (x N + y) N + z.
    """
    R = _scipy_R(quat)
    p = np.einsum("jab,ib->jia", R, q) + grid_n / 2.0
    ax = np.arange(grid_n, dtype=np.float64)
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    pl = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)      # l = (x N + y) N + z
    d = np.abs(pl[:, None, None, :] - p[None, :, :, :])
    return np.prod(np.clip(1.0 - d, 0.0, None), axis=-1)            # [M][j][i]


# ----------------------------------------------------------------------------- rotations
def test_rotation_matches_scipy():
    quat = shoemake_quaternions(_rng(1), 50)
    np.testing.assert_allclose(O.rotation_matrix(quat), _scipy_R(quat), atol=1e-14)


def test_rotation_orthonormal_and_sign_invariant():
    quat = shoemake_quaternions(_rng(2), 40)
    R = O.rotation_matrix(quat)
    I = np.einsum("jab,jcb->jac", R, R)
    np.testing.assert_allclose(I, np.broadcast_to(np.eye(3), I.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-14)
    np.testing.assert_allclose(O.rotation_matrix(-quat), R, atol=1e-15)
    np.testing.assert_allclose(O.rotation_matrix(3.7 * quat), R, atol=1e-14)  # normalised first


def test_rotation_composes_like_hamilton_product():
    a = shoemake_quaternions(_rng(3), 20)
    b = shoemake_quaternions(_rng(4), 20)
    w1, v1 = a[:, 0], a[:, 1:]
    w2, v2 = b[:, 0], b[:, 1:]
    prod = np.concatenate([(w1 * w2 - np.sum(v1 * v2, 1))[:, None],
                           w1[:, None] * v2 + w2[:, None] * v1 + np.cross(v1, v2)], axis=1)
    np.testing.assert_allclose(O.rotation_matrix(prod),
                               O.rotation_matrix(a) @ O.rotation_matrix(b), atol=1e-14)


def test_quarter_turn_about_z():
    # (cos 45deg, 0, 0, sin 45deg) turns x into y (active, right-handed)
    R = O.rotation_matrix(np.array([math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)]))
    np.testing.assert_allclose(R @ [1.0, 0, 0], [0, 1.0, 0], atol=1e-15)


def test_positions_centre_and_norm():
    quat = shoemake_quaternions(_rng(5), 7)
    q = _rng(6).normal(size=(9, 3))
    q[0] = 0
    p = O.slice_positions(q, quat, 16)
    np.testing.assert_allclose(p[:, 0], 8.0, atol=0)
    np.testing.assert_allclose(np.linalg.norm(p - 8.0, axis=-1),
                               np.broadcast_to(np.linalg.norm(q, axis=1), p.shape[:2]), atol=1e-13)


# ----------------------------------------------------------------------------- expansion
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_expand_equals_dense_interpolation_matrix(seed):
    t = tiny_problem(seed, grid_n=6, n_pix=12, n_rot=5, n_data=3, q_radius=2.6)
    F = _dense_F(t["q"], t["quat"], 6)
    W_brute = np.einsum("lji,l->ji", F, t["model"])
    np.testing.assert_allclose(O.expand(t["model"], t["q"], t["quat"], 6), W_brute, rtol=1e-13, atol=1e-15)


def test_expand_points_partly_outside_grid_drop_missing_points():
    # pixels pushed beyond the box: grid points outside the N^3 box do not exist
    t = tiny_problem(7, grid_n=6, n_pix=10, n_rot=4, n_data=2, q_radius=3.4)
    F = _dense_F(t["q"], t["quat"], 6)
    np.testing.assert_allclose(O.expand(t["model"], t["q"], t["quat"], 6),
                               np.einsum("lji,l->ji", F, t["model"]), rtol=1e-13, atol=1e-15)


def test_expand_reproduces_multilinear_fields_exactly():
    N = 20
    ax = np.arange(N, dtype=np.float64)
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    a, b, c, d = 0.3, -1.7, 2.2, 5.0
    model = (a * X + b * Y + c * Z + d + 0.01 * X * Y * Z).ravel()
    quat = shoemake_quaternions(_rng(8), 6)
    q = _rng(9).uniform(-6, 6, size=(30, 3))
    p = O.slice_positions(q, quat, N)
    exact = a * p[..., 0] + b * p[..., 1] + c * p[..., 2] + d + 0.01 * p[..., 0] * p[..., 1] * p[..., 2]
    np.testing.assert_allclose(O.expand(model, q, quat, N), exact, rtol=1e-12)


def test_expand_uniform_model_is_constant():
    quat = shoemake_quaternions(_rng(10), 5)
    q = _rng(11).uniform(-5, 5, size=(40, 3))
    W = O.expand(np.full(16 ** 3, 2.5), q, quat, 16)
    np.testing.assert_allclose(W, 2.5, rtol=1e-14)


# ----------------------------------------------------------------------------- likelihood
def test_loglik_is_poisson_log_pmf_without_factorial():
    g = _rng(12)
    W = g.gamma(1.5, 0.7, size=(6, 25))
    K = g.poisson(0.8, size=(4, 25))
    mask = (g.random(25) > 0.2).astype(np.uint8)
    v = mask.astype(bool)
    Q = O.log_likelihood(W, K, mask)
    ref = np.array([[np.sum(poisson.logpmf(K[k, v], W[j, v]) + gammaln(K[k, v] + 1.0))
                     for k in range(4)] for j in range(6)])
    np.testing.assert_allclose(Q, ref, rtol=1e-13)


def test_loglik_floor_on_empty_slice():
    W = np.array([[0.0, 1.0, 2.0]])
    K = np.array([[3, 1, 0]])
    Q = O.log_likelihood(W, K, np.ones(3, np.uint8))
    assert Q[0, 0] == pytest.approx(3 * math.log(1e-10) + 0 - (1e-10 + 1.0 + 2.0), rel=1e-14)


def test_loglik_single_pixel_closed_form():
    Q = O.log_likelihood(np.array([[2.5]]), np.array([[4]]), np.ones(1, np.uint8))
    assert Q[0, 0] == pytest.approx(4 * math.log(2.5) - 2.5, rel=1e-15)


def test_loglik_gibbs_inequality_picks_matching_slice():
    g = _rng(13)
    W = g.gamma(2.0, 1.0, size=(8, 50))
    mask = np.ones(50, np.uint8)
    for jstar in range(8):
        Q = O.log_likelihood(W, W[jstar][None, :], mask)
        assert int(np.argmax(Q[:, 0])) == jstar


# ----------------------------------------------------------------------------- E-step
def test_estep_matches_mpmath_50_digits():
    g = _rng(14)
    Q = g.normal(scale=300.0, size=(9, 5)) - 4000.0
    Q[3, 2] = Q[5, 2] + 1e-9            # a near tie
    lw = np.log(g.dirichlet(np.ones(9)))
    P, L = O.responsibilities(Q, lw)
    mpmath.mp.dps = 50
    for k in range(5):
        terms = [mpmath.mpf(float(Q[j, k])) + mpmath.mpf(float(lw[j])) for j in range(9)]
        Lk = mpmath.log(mpmath.fsum(mpmath.exp(t) for t in terms))
        assert float(L[k]) == pytest.approx(float(Lk), rel=1e-15, abs=1e-12)
        for j in range(9):
            assert float(P[j, k]) == pytest.approx(float(mpmath.exp(terms[j] - Lk)), rel=1e-12, abs=1e-300)


def test_estep_equals_bayes_with_pmf_products():
    # posterior of the rotation from Poisson pmf products (no logs, factorials kept)
    g = _rng(15)
    W = g.gamma(2.0, 0.5, size=(5, 6))
    K = g.poisson(1.0, size=(3, 6))
    mask = np.ones(6, np.uint8)
    w = g.dirichlet(np.ones(5))
    P, _ = O.responsibilities(O.log_likelihood(W, K, mask), np.log(w))
    for k in range(3):
        like = np.array([np.prod(poisson.pmf(K[k], W[j])) for j in range(5)])
        np.testing.assert_allclose(P[:, k], w * like / np.sum(w * like), rtol=1e-12)


def test_estep_columns_sum_to_one():
    g = _rng(16)
    P, _ = O.responsibilities(g.normal(scale=50, size=(30, 12)), np.log(g.dirichlet(np.ones(30))))
    np.testing.assert_allclose(P.sum(axis=0), 1.0, atol=1e-14)


def test_uniform_model_gives_prior_responsibilities():
    t = tiny_problem(17, grid_n=12, n_pix=30, n_rot=7, n_data=5)
    W = O.expand(np.full(12 ** 3, 0.7), t["q"], t["quat"], 12)
    P, _ = O.responsibilities(O.log_likelihood(W, t["counts"], t["mask"]), t["log_w"])
    np.testing.assert_allclose(P, np.exp(t["log_w"])[:, None] * np.ones((1, 5)), rtol=1e-12)


# ----------------------------------------------------------------------------- M and c steps
@pytest.mark.parametrize("seed", [0, 1])
def test_compress_equals_dense_interpolation_matrix(seed):
    t = tiny_problem(20 + seed, grid_n=6, n_pix=11, n_rot=4, n_data=3, q_radius=2.6)
    F = _dense_F(t["q"], t["quat"], 6)
    g = _rng(21 + seed)
    Wp = g.random((4, 11))
    rho = g.random(4)
    v = t["mask"].astype(bool)
    num, den = O.compress(Wp, rho, t["q"], t["mask"], t["quat"], 6)
    np.testing.assert_allclose(num, np.einsum("lji,ji->l", F[:, :, v], Wp[:, v]), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(den, np.einsum("lji,j->l", F[:, :, v], rho), rtol=1e-13, atol=1e-15)


def test_constant_frames_give_constant_model():
    t = tiny_problem(22, grid_n=12, n_pix=40, n_rot=6, n_data=7)
    g = _rng(23)
    P = g.dirichlet(np.ones(6), size=7).T            # any normalised responsibilities
    K = np.full((7, 40), 3.0)
    Wp, rho = O.maximize(P, K, t["mask"])
    num, den = O.compress(Wp, rho, t["q"], t["mask"], t["quat"], 12)
    new = O.divide(num, den, np.zeros(12 ** 3))
    np.testing.assert_allclose(new[den > 0], 3.0, rtol=1e-13)
    assert np.all(new[den == 0] == 0)


def test_single_rotation_reproduces_mean_frame():
    # identity rotation, flat detector on integer voxels: f is a delta and the
    # touched voxels equal the mean frame exactly
    N = 10
    u = np.arange(-3, 4)
    X, Y = np.meshgrid(u, u, indexing="ij")
    q = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1).astype(np.float64)
    mask = np.ones(q.shape[0], np.uint8)
    mask[5] = 0
    K = _rng(24).poisson(4.0, size=(13, q.shape[0])).astype(np.float64)
    r = O.iterate(np.full(N ** 3, 1.0), K, q, mask, np.array([[1.0, 0, 0, 0]]), np.array([0.0]), N)
    np.testing.assert_allclose(r["P"], 1.0)
    l = ((X.ravel() + 5) * N + (Y.ravel() + 5)) * N + 5
    v = mask.astype(bool)
    np.testing.assert_allclose(r["model"][l[v]], K.mean(axis=0)[v], rtol=1e-14)
    untouched = np.ones(N ** 3, bool)
    untouched[l[v]] = False
    assert np.all(r["model"][untouched] == 1.0)


def test_frame_chunks_sum_before_division():
    t = tiny_problem(25, grid_n=10, n_pix=30, n_rot=6, n_data=11)
    a = O.iterate(t["model"], t["counts"], t["q"], t["mask"], t["quat"], t["log_w"], 10)
    b = O.iterate(t["model"], t["counts"], t["q"], t["mask"], t["quat"], t["log_w"], 10, frame_chunk=4)
    np.testing.assert_allclose(b["model"], a["model"], rtol=1e-12)
    np.testing.assert_allclose(b["P"], a["P"], rtol=1e-12, atol=1e-300)


def test_whole_iteration_against_brute_force():
    t = tiny_problem(26, grid_n=6, n_pix=9, n_rot=4, n_data=5, q_radius=2.5)
    F = _dense_F(t["q"], t["quat"], 6)                   # [M][j][i]
    v = t["mask"].astype(bool)
    K = t["counts"].astype(np.float64)
    W = np.einsum("lji,l->ji", F, t["model"])
    Wf = np.maximum(W, 1e-10)
    mpmath.mp.dps = 40
    P = np.zeros((4, 5))
    for k in range(5):
        logt = [sum(K[k, i] * math.log(Wf[j, i]) - Wf[j, i] for i in range(9) if v[i]) + t["log_w"][j]
                for j in range(4)]
        Z = mpmath.fsum(mpmath.exp(mpmath.mpf(x)) for x in logt)
        P[:, k] = [float(mpmath.exp(mpmath.mpf(x)) / Z) for x in logt]
    Wp = P @ K
    num = np.einsum("lji,ji->l", F[:, :, v], Wp[:, v])
    den = np.einsum("lji,j->l", F[:, :, v], P.sum(axis=1))
    model = np.where(den > 0, num / np.where(den > 0, den, 1.0), t["model"])
    r = O.iterate(t["model"], t["counts"], t["q"], t["mask"], t["quat"], t["log_w"], 6)
    np.testing.assert_allclose(r["P"], P, rtol=1e-11, atol=1e-300)
    np.testing.assert_allclose(r["model"], model, rtol=1e-11)


# ----------------------------------------------------------------------------- printed numbers
def test_paper_operation_count_reproduces_table_4_2():
    tab = json.load(open(os.path.join(GOLDEN, "table_4_2.json")))
    for row in tab["rows"]:
        for mpix in (4096, 16384):
            fl = O.paper_flops(tab["n_rot"], tab["n_data"], mpix)
            gf = fl / row[f"mpix{mpix}_time_s"] / row["gpus"] / 1e9
            assert abs(gf - row[f"mpix{mpix}_gflops_per_gpu"]) <= 0.1 + 1e-9


def test_600cell_rotation_counts_match_eq_2_7():
    g = json.load(open(os.path.join(GOLDEN, "eq_2_7_mrot.json")))
    assert [O.mrot_600cell(d) for d in g["d"]] == g["n_rot"]


def test_masked_pixels_have_no_influence():
    # counts in masked pixels (missing/saturated) must not reach any result
    t = tiny_problem(27, grid_n=10, n_pix=25, n_rot=5, n_data=6)
    t["mask"][[3, 11]] = 0
    t["counts"][:, [3, 11]] = 0
    K2 = t["counts"].copy()
    K2[:, t["mask"] == 0] = 50
    a = O.iterate(t["model"], t["counts"], t["q"], t["mask"], t["quat"], t["log_w"], 10)
    b = O.iterate(t["model"], K2, t["q"], t["mask"], t["quat"], t["log_w"], 10)
    for key in ("Q", "P", "L", "Wp", "rho", "num", "den", "model"):
        np.testing.assert_array_equal(a[key], b[key])
    assert np.all(b["Wp"][:, t["mask"] == 0] == 0)


def test_restricted_estep_with_all_candidates_is_the_full_estep():
    g = _rng(30)
    Q = g.normal(scale=30, size=(12, 7))
    lw = np.log(g.dirichlet(np.ones(12)))
    P, L = O.responsibilities(Q, lw)
    Pr, Lr = O.responsibilities_restricted(Q, lw, np.ones_like(Q, dtype=bool))
    np.testing.assert_allclose(Pr, P, rtol=1e-14)
    np.testing.assert_allclose(Lr, L, rtol=1e-14)


def test_restricted_estep_is_conditional_posterior():
    # restricting the sum gives the posterior conditioned on j in cand(k): P_restricted = P / recall
    g = _rng(31)
    Q = g.normal(scale=3, size=(10, 6))
    lw = np.log(g.dirichlet(np.ones(10)))
    cand = g.random((10, 6)) < 0.5
    cand[0] = True
    P, _ = O.responsibilities(Q, lw)
    Pr, _ = O.responsibilities_restricted(Q, lw, cand)
    rec = O.proposal_recall(P, cand)
    np.testing.assert_allclose(Pr, np.where(cand, P / rec[None, :], 0.0), rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(Pr.sum(0), 1.0, rtol=1e-14)


def test_iterate_proposed_with_every_rotation_a_candidate_is_the_full_iteration():
    t = tiny_problem(32, grid_n=12, n_pix=60, n_rot=15, n_data=9)
    a = O.iterate(t["model"], t["counts"], t["q"], t["mask"], t["quat"], t["log_w"], 12)
    b = O.iterate_proposed(t["model"], t["counts"], t["q"], t["mask"], t["quat"], t["log_w"], 12,
                           np.ones((15, 9), bool))
    for key in ("Q", "P", "L", "Wp", "rho", "num", "den", "model"):
        np.testing.assert_allclose(b[key], a[key], rtol=1e-13, atol=1e-300)


def test_iterate_proposed_with_one_candidate_reproduces_the_mean_frame():
    # every frame's single candidate is the identity rotation (the other rotations are
    # never proposed): its responsibility is 1, so with a flat detector on integer
    # voxels the touched voxels hold the mean frame exactly, whatever the other
    # rotations' likelihoods; the unrestricted posterior would spread the frames
    N = 10
    u = np.arange(-3, 4)
    X, Y = np.meshgrid(u, u, indexing="ij")
    q = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1).astype(np.float64)
    mask = np.ones(q.shape[0], np.uint8)
    mask[7] = 0
    K = _rng(33).poisson(4.0, size=(11, q.shape[0])).astype(np.float64)
    quat = np.concatenate([[[1.0, 0, 0, 0]], shoemake_quaternions(_rng(34), 5)])
    log_w = np.log(np.full(6, 1.0 / 6))
    cand = np.zeros((6, 11), bool)
    cand[0] = True
    model = _rng(35).random(N ** 3) + 0.5
    r = O.iterate_proposed(model, K, q, mask, quat, log_w, N, cand)
    np.testing.assert_array_equal(r["P"][1:], 0.0)
    np.testing.assert_allclose(r["P"][0], 1.0, rtol=1e-15)
    np.testing.assert_allclose(r["rho"], [11.0, 0, 0, 0, 0, 0])
    l = ((X.ravel() + 5) * N + (Y.ravel() + 5)) * N + 5
    v = mask.astype(bool)
    np.testing.assert_allclose(r["model"][l[v]], K.mean(axis=0)[v], rtol=1e-14)
    untouched = np.ones(N ** 3, bool)
    untouched[l[v]] = False
    np.testing.assert_array_equal(r["model"][untouched], model[untouched])
    # the same frames searched over every rotation do not give the mean frame
    full = O.iterate(model, K, q, mask, quat, log_w, N)
    assert np.max(np.abs(full["model"][l[v]] - K.mean(axis=0)[v])) > 1e-3


def test_iterate_proposed_log_evidence_is_over_the_candidates():
    # L_k = log sum_{j in cand(k)} w_j e^{Q_jk}: restricting can only lower it, and the
    # reported mean is the mean of those restricted values (eq. 2.1 over the searched set)
    t = tiny_problem(36, grid_n=12, n_pix=50, n_rot=12, n_data=8)
    g = _rng(37)
    cand = g.random((12, 8)) < 0.4
    cand[g.integers(0, 12, 8), np.arange(8)] = True
    a = O.iterate(t["model"], t["counts"], t["q"], t["mask"], t["quat"], t["log_w"], 12)
    b = O.iterate_proposed(t["model"], t["counts"], t["q"], t["mask"], t["quat"], t["log_w"], 12, cand)
    assert np.all(b["L"] <= a["L"] + 1e-12)
    for k in range(8):
        terms = [mpmath.mpf(float(a["Q"][j, k])) + mpmath.mpf(float(t["log_w"][j])) for j in range(12) if cand[j, k]]
        assert float(b["L"][k]) == pytest.approx(float(mpmath.log(mpmath.fsum(mpmath.exp(x) for x in terms))),
                                                 rel=1e-13)
    assert b["loglik"] == pytest.approx(float(np.mean(b["L"])), rel=1e-15)
