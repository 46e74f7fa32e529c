"""Plain FP64 reference of one EMC iteration under the Gaussian noise model with
photon fluence (the paper's own likelihood, Section 2.2).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
the GPU library shares no code with it.

Notation as in the Poisson oracle (emc_oracle): frames K[k][i], slices W[j][i],
responsibilities and fluences P[j][k], phi[j][k].  Each function cites the
passage it follows.

Readings of points the paper leaves open:
  * sigma is a caller parameter, fixed within an iteration (the paper keeps it at
    a cautious level or decreases it gradually from one iteration to the next).
  * The E-step and the M-step numerator of iteration n use the fluence phi^(n);
    the iteration also returns phi^(n+1), the fixed-point update (eq. (2.6))
    evaluated on its own slices W^(n).  The paper gives no phi^(0): the first
    iteration takes the update evaluated on its own slices (phi = None below).
  * phi_jk = sum_i K_ik^2 / sum_i W_ij K_ik needs a positive denominator; a frame
    without photons (or a slice that is zero wherever the frame has photons) has
    no fluence information and gets phi = 1.
  * No floor on W: nothing takes its logarithm.  Masked pixels are excluded from
    every sum, as in the Poisson form.

parity pinned: see tests/test_gauss_oracle_pins.py (noise-free scaled frames,
a closed form with one rotation, the prior limit of large sigma, and the scale
covariances of eq. (2.2) and eq. (2.6)).
"""
from __future__ import annotations

import numpy as np

from . import emc_oracle as E


def fluence(W: np.ndarray, K: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """phi[j][k] = sum_{i valid} K_ik^2 / sum_{i valid} W_ij K_ik (eq. (2.6)); 1 where the
    denominator is not positive."""
    v = np.flatnonzero(mask)
    Kv = np.asarray(K, dtype=np.float64)[:, v]
    num = (Kv * Kv).sum(axis=1)                                   # [k]
    den = np.asarray(W, dtype=np.float64)[:, v] @ Kv.T            # [j][k]
    out = np.ones_like(den)
    pos = den > 0
    out[pos] = (np.broadcast_to(num[None, :], den.shape))[pos] / den[pos]
    return out


def log_likelihood(W: np.ndarray, K: np.ndarray, mask: np.ndarray, phi: np.ndarray, sigma: float,
                   rot_chunk: int = 16) -> np.ndarray:
    """Q[j][k] = -sum_{i valid} (K_ik / phi_jk - W_ij)^2 / (2 sigma^2) (eq. (2.2)-(2.3)),
    summed term by term (rotations in chunks to bound memory)."""
    v = np.flatnonzero(mask)
    Kv = np.asarray(K, dtype=np.float64)[:, v]                    # [k][i]
    Wv = np.asarray(W, dtype=np.float64)[:, v]                    # [j][i]
    phi = np.asarray(phi, dtype=np.float64)
    Q = np.empty((Wv.shape[0], Kv.shape[0]))
    for j0 in range(0, Wv.shape[0], rot_chunk):
        d = Kv[None, :, :] / phi[j0:j0 + rot_chunk, :, None] - Wv[j0:j0 + rot_chunk, None, :]
        Q[j0:j0 + rot_chunk] = -(d * d).sum(axis=2) / (2.0 * sigma * sigma)
    return Q


def maximize(P: np.ndarray, K: np.ndarray, mask: np.ndarray, phi: np.ndarray):
    """Returns (Wp[j][i] = sum_k P_jk K_ik / phi_jk on valid pixels, 0 on masked (eq. (2.11));
    rho[j] = sum_k P_jk, the c-step's weight (eq. (2.12)))."""
    P = np.asarray(P, dtype=np.float64)
    Wp = (P / np.asarray(phi, dtype=np.float64)) @ np.asarray(K, dtype=np.float64)
    Wp[:, np.asarray(mask) == 0] = 0.0
    return Wp, P.sum(axis=1)


def iterate(model, K, q, mask, quat, log_w, grid_n, sigma: float, phi=None):
    """One pass of Algorithm 1 under the Gaussian model: expansion (eq. (2.9)), E-step
    (eq. (2.4) with T = exp(Q) of eq. (2.3)) with fluence phi^(n), combined M- and
    c-step (eq. (2.11)-(2.12)) and the fluence update (eq. (2.6)).

    phi: [n_rot][n_data] fluence phi^(n), or None for the first iteration (phi^(n) is
    then the update evaluated on this iteration's slices).  Returns a dict with W, Q,
    P, L, loglik, phi_used, phi (= phi^(n+1)), Wp, rho, num, den, model."""
    W = E.expand(model, q, quat, grid_n)
    phi_next = fluence(W, K, mask)
    phi_used = phi_next if phi is None else np.asarray(phi, dtype=np.float64)
    Q = log_likelihood(W, K, mask, phi_used, sigma)
    P, L = E.responsibilities(Q, log_w)
    Wp, rho = maximize(P, K, mask, phi_used)
    num, den = E.compress(Wp, rho, q, mask, quat, grid_n)
    new = E.divide(num, den, model)
    return dict(W=W, Q=Q, P=P, L=L, loglik=float(L.mean()), phi_used=phi_used, phi=phi_next, Wp=Wp, rho=rho,
                num=num, den=den, model=new)
