"""Pins of the C forms of the oracle's expansion (eq. 2.9) and c-step (eq. 2.12),
and of the chunked whole-iteration composition, against facts that do not come
from that code: the dense interpolation matrix built over every grid point with
scipy's rotation, multilinear fields (reproduced exactly by trilinear
interpolation), the partition of unity of the weights, and the pinned numpy
oracle on problems small enough for it."""
import numpy as np
import pytest

import oracle as O
from emc_inputs import shoemake_quaternions, tiny_problem
from oracle import native as ON
from test_oracle_pins import _dense_F


def _rng(s):
    return np.random.default_rng(5000 + s)


@pytest.mark.parametrize("seed,qr", [(0, 2.6), (1, 3.4)])
def test_c_expand_equals_dense_interpolation_matrix(seed, qr):
    t = tiny_problem(40 + seed, grid_n=6, n_pix=14, n_rot=5, n_data=2, q_radius=qr)
    F = _dense_F(t["q"], t["quat"], 6)
    np.testing.assert_allclose(ON.expand(t["model"], t["q"], t["quat"], 6), np.einsum("lji,l->ji", F, t["model"]),
                               rtol=1e-13, atol=1e-15)


def test_c_expand_reproduces_multilinear_fields_exactly():
    N = 18
    ax = np.arange(N, dtype=np.float64)
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    model = (0.4 * X - 1.1 * Y + 2.3 * Z + 7.0 + 0.02 * X * Y * Z).ravel()
    quat = shoemake_quaternions(_rng(1), 7)
    q = _rng(2).uniform(-5, 5, size=(40, 3))
    p = O.slice_positions(q, quat, N)
    exact = 0.4 * p[..., 0] - 1.1 * p[..., 1] + 2.3 * p[..., 2] + 7.0 + 0.02 * p[..., 0] * p[..., 1] * p[..., 2]
    np.testing.assert_allclose(ON.expand(model, q, quat, N), exact, rtol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_c_compress_equals_dense_interpolation_matrix(seed):
    t = tiny_problem(50 + seed, grid_n=6, n_pix=13, n_rot=4, n_data=2, q_radius=2.9)
    F = _dense_F(t["q"], t["quat"], 6)
    g = _rng(3 + seed)
    Wp, rho = g.random((4, 13)), g.random(4)
    v = t["mask"].astype(bool)
    num, den = ON.compress(Wp, rho, t["q"], t["mask"], t["quat"], 6)
    np.testing.assert_allclose(num, np.einsum("lji,ji->l", F[:, :, v], Wp[:, v]), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(den, np.einsum("lji,j->l", F[:, :, v], rho), rtol=1e-13, atol=1e-15)


def test_c_compress_partition_of_unity():
    # weights of a point inside the box sum to one: sum_l den_l = sum_j rho_j x valid pixels
    t = tiny_problem(52, grid_n=16, n_pix=200, n_rot=30, n_data=2)
    g = _rng(5)
    Wp, rho = g.random((30, 200)), g.random(30)
    num, den = ON.compress(Wp, rho, t["q"], t["mask"], t["quat"], 16)
    v = t["mask"].astype(bool)
    assert den.sum() == pytest.approx(rho.sum() * v.sum(), rel=1e-12)
    assert num.sum() == pytest.approx(Wp[:, v].sum(), rel=1e-12)


def test_loglik_all_rotations_is_poisson_log_pmf_of_brute_force_slices():
    from scipy.special import gammaln
    from scipy.stats import poisson

    t = tiny_problem(53, grid_n=6, n_pix=12, n_rot=9, n_data=4, q_radius=2.5)
    F = _dense_F(t["q"], t["quat"], 6)
    W = np.maximum(np.einsum("lji,l->ji", F, t["model"]), 1e-10)
    v = t["mask"].astype(bool)
    K = t["counts"]
    ref = np.array([[np.sum(poisson.logpmf(K[k, v], W[j, v]) + gammaln(K[k, v] + 1.0)) for k in range(4)]
                    for j in range(9)])
    Q = ON.loglik_all_rotations(t["model"], K, t["q"], t["mask"], t["quat"], 6, rot_chunk=4)
    np.testing.assert_allclose(Q, ref, rtol=1e-12)


def test_chunked_iteration_equals_brute_force_iteration():
    import math

    import mpmath

    t = tiny_problem(54, grid_n=6, n_pix=10, n_rot=7, n_data=5, q_radius=2.5)
    F = _dense_F(t["q"], t["quat"], 6)
    v = t["mask"].astype(bool)
    K = t["counts"].astype(np.float64)
    Wf = np.maximum(np.einsum("lji,l->ji", F, t["model"]), 1e-10)
    mpmath.mp.dps = 40
    P = np.zeros((7, 5))
    for k in range(5):
        logt = [sum(K[k, i] * math.log(Wf[j, i]) - Wf[j, i] for i in range(10) if v[i]) + t["log_w"][j]
                for j in range(7)]
        Z = mpmath.fsum(mpmath.exp(mpmath.mpf(x)) for x in logt)
        P[:, k] = [float(mpmath.exp(mpmath.mpf(x)) / Z) for x in logt]
    num = np.einsum("lji,ji->l", F[:, :, v], (P @ K)[:, v])
    den = np.einsum("lji,j->l", F[:, :, v], P.sum(axis=1))
    model = np.where(den > 0, num / np.where(den > 0, den, 1.0), t["model"])
    r = ON.iterate_chunked(t["model"], t["counts"], t["q"], t["mask"], t["quat"], t["log_w"], 6, rot_chunk=3)
    np.testing.assert_allclose(r["P"], P, rtol=1e-11, atol=1e-300)
    np.testing.assert_allclose(r["model"], model, rtol=1e-11)


def test_chunked_iteration_matches_numpy_oracle():
    t = tiny_problem(55, grid_n=14, n_pix=150, n_rot=60, n_data=40)
    a = O.iterate(t["model"], t["counts"], t["q"], t["mask"], t["quat"], t["log_w"], 14)
    b = ON.iterate_chunked(t["model"], t["counts"], t["q"], t["mask"], t["quat"], t["log_w"], 14, rot_chunk=17)
    np.testing.assert_allclose(b["Q"], a["Q"], rtol=1e-12)
    np.testing.assert_allclose(b["P"], a["P"], rtol=1e-10, atol=1e-300)
    np.testing.assert_allclose(b["model"], a["model"], rtol=1e-12)
    assert b["loglik"] == pytest.approx(a["loglik"], rel=1e-13)
