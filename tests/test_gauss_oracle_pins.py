"""Pins of the Gaussian-model oracle (eq. (2.2)-(2.3) likelihood, eq. (2.6) fluence,
eq. (2.11)-(2.12) with fluence) against facts fixed by the paper's formulas and by
the mathematics, not by the oracle's own code:

* noise-free frames K_k = a_k W_{j*(k)}: the fixed point of eq. (2.6) recovers the
  scale a_k exactly, the log-likelihood (a negative sum of squares) is 0 there and
  negative elsewhere;
* one identity rotation and a detector on integer voxels: the updated model is the
  fluence-corrected mean frame (each pixel lands on one voxel with weight 1);
* sigma -> infinity: Q -> 0 and the responsibilities become the prior weights;
* scale covariance: K / phi is all the likelihood sees, phi is homogeneous of
  degree 1 in K and -1 in W, and Q scales as 1 / sigma^2.
"""
import numpy as np

from emc_inputs import tiny_problem
from oracle import emc_oracle as E
from oracle import gauss_oracle as G


def _problem(seed, **kw):
    t = tiny_problem(seed, **kw)
    return t, E.expand(t["model"], t["q"], t["quat"], t["grid_n"])


def test_noise_free_scaled_frames_recover_scale_and_rotation():
    t, W = _problem(1, grid_n=16, n_pix=150, n_rot=40, n_data=1)
    rng = np.random.default_rng(5)
    n = 60
    jstar = rng.integers(0, 40, size=n)
    a = rng.uniform(0.5, 3.0, size=n)
    K = a[:, None] * W[jstar]                      # exact, noise-free, float frames
    mask = t["mask"]
    phi = G.fluence(W, K, mask)
    np.testing.assert_allclose(phi[jstar, np.arange(n)], a, rtol=1e-12)
    Q = G.log_likelihood(W, K, mask, phi, sigma=0.5)
    np.testing.assert_allclose(Q[jstar, np.arange(n)], 0.0, atol=1e-9)
    others = np.ones_like(Q, dtype=bool)
    others[jstar, np.arange(n)] = False
    assert Q[others].max() < -1e-6
    P, _ = E.responsibilities(Q, t["log_w"])
    np.testing.assert_array_equal(P.argmax(axis=0), jstar)


def test_single_identity_rotation_gives_fluence_corrected_mean_frame():
    N = 16
    u = np.arange(-4, 5)
    X, Y = np.meshgrid(u, u, indexing="ij")
    q = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1).astype(np.float64)
    mask = np.ones(q.shape[0], np.uint8)
    mask[[3, 40]] = 0
    rng = np.random.default_rng(7)
    K = rng.poisson(4.0, size=(25, q.shape[0])).astype(np.float64)
    phi = rng.uniform(0.5, 2.0, size=(1, 25))
    model = rng.uniform(0.5, 2.0, size=N ** 3)
    o = G.iterate(model, K, q, mask, np.array([[1.0, 0, 0, 0]]), np.array([0.0]), N, sigma=1.0, phi=phi)
    np.testing.assert_allclose(o["P"], 1.0)
    l = ((X.ravel() + 8) * N + (Y.ravel() + 8)) * N + 8
    v = mask.astype(bool)
    np.testing.assert_allclose(o["model"][l[v]], (K / phi[0][:, None]).mean(axis=0)[v], rtol=1e-12)
    # voxels no pixel reaches keep the previous model
    untouched = np.ones(N ** 3, bool)
    untouched[l[v]] = False
    np.testing.assert_array_equal(o["model"][untouched], model[untouched])


def test_large_sigma_gives_the_prior():
    t, W = _problem(2, grid_n=14, n_pix=120, n_rot=30, n_data=20, photons=100.0)
    phi = G.fluence(W, t["counts"], t["mask"])
    Q = G.log_likelihood(W, t["counts"], t["mask"], phi, sigma=1e7)
    P, _ = E.responsibilities(Q, t["log_w"])
    np.testing.assert_allclose(P, np.exp(t["log_w"])[:, None] * np.ones((1, 20)), rtol=1e-6)


def test_scale_covariance_of_likelihood_and_fluence():
    t, W = _problem(3, grid_n=14, n_pix=120, n_rot=25, n_data=15, photons=100.0)
    K = t["counts"].astype(np.float64)
    mask = t["mask"]
    phi = G.fluence(W, K, mask)
    c = 2.75
    np.testing.assert_allclose(G.fluence(W, c * K, mask), c * phi, rtol=1e-12)
    np.testing.assert_allclose(G.fluence(c * W, K, mask), phi / c, rtol=1e-12)
    Q = G.log_likelihood(W, K, mask, phi, sigma=0.7)
    np.testing.assert_allclose(G.log_likelihood(W, c * K, mask, c * phi, sigma=0.7), Q, rtol=1e-12)
    np.testing.assert_allclose(G.log_likelihood(W, K, mask, phi, sigma=1.4), Q / 4.0, rtol=1e-12)
    # masked pixels do not enter: changing their counts changes nothing
    K2 = K.copy()
    K2[:, mask == 0] += 9.0
    np.testing.assert_allclose(G.log_likelihood(W, K2, mask, phi, sigma=0.7), Q, rtol=1e-12)
    np.testing.assert_allclose(G.fluence(W, K2, mask), phi, rtol=1e-12)


def test_empty_frame_gets_unit_fluence_and_first_iteration_uses_its_own():
    t, W = _problem(4, grid_n=12, n_pix=80, n_rot=10, n_data=6, photons=60.0)
    K = t["counts"].astype(np.float64)
    K[2] = 0.0
    phi = G.fluence(W, K, t["mask"])
    np.testing.assert_array_equal(phi[:, 2], 1.0)
    o = G.iterate(t["model"], K, t["q"], t["mask"], t["quat"], t["log_w"], 12, sigma=1.0)
    np.testing.assert_array_equal(o["phi_used"], o["phi"])
    o2 = G.iterate(t["model"], K, t["q"], t["mask"], t["quat"], t["log_w"], 12, sigma=1.0, phi=o["phi"])
    np.testing.assert_allclose(o2["model"], o["model"], rtol=1e-13)


def test_likelihood_is_the_gaussian_log_density_up_to_a_frame_constant():
    """eq. (2.2): log Prob(K_ik | W_ij, phi_jk) is the normal log-density of K/phi around W with
    standard deviation sigma, up to terms that do not depend on the rotation (scipy.stats.norm)."""
    from scipy.stats import norm

    t, W = _problem(5, grid_n=12, n_pix=90, n_rot=12, n_data=8, photons=80.0)
    K = t["counts"].astype(np.float64)
    mask = t["mask"]
    v = mask.astype(bool)
    phi = np.random.default_rng(9).uniform(0.6, 1.6, size=(12, 8))
    sigma = 0.8
    Q = G.log_likelihood(W, K, mask, phi, sigma)
    ref = np.array([[norm.logpdf(K[k, v] / phi[j, k], loc=W[j, v], scale=sigma).sum() for k in range(8)]
                    for j in range(12)])
    # differences between rotations are free of the normalisation constant
    np.testing.assert_allclose(Q - Q[0:1], ref - ref[0:1], rtol=1e-10, atol=1e-9)
