"""Plain FP64 reference of one Expand-Maximize-Compress iteration (Poisson model).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
the GPU library shares no code with it.

Each function states the passage of Ekeberg, Engblom & Liu, "Machine learning
for ultrafast X-ray diffraction patterns on large-scale GPU clusters"
(arXiv:1409.4256) that it follows.  Arrays use the paper's index order: pixel
i, rotation j, frame k, grid point l.  Frames are ``K[k][i]`` (as stored),
slices ``W[j][i]``, responsibilities ``P[j][k]``.

Readings of points the paper leaves open (all shared, by written convention
only, with the GPU path):
  * likelihood: Poisson, log P(K_k | R_j) = sum_i K_ik log W_ij - W_ij - log K_ik!
    (Section 2.2 names the Poissonian model of the original EMC; eq. (2.5) and
    (2.11) with fluence phi = 1).  The log K! term is constant in j and W and is
    dropped from Q.
  * interpolation weights f (eq. (2.8)): trilinear tent
    f(d) = prod_a max(0, 1 - |d_a|), the same f in expansion and compression.
  * grid: N^3 voxels, flat index l = (x N + y) N + z, grid point p_l = (x, y, z);
    a pixel coordinate q (voxel units) sits at R q + (N/2, N/2, N/2).  Grid
    points outside the N^3 box do not exist (they contribute nothing).
  * rotation: unit quaternion (w, x, y, z), Hamilton convention, active rotation.
  * W = 0 would make log W undefined (the paper asks for care with finite
    precision in the E-step): slices are floored at 1e-10 photons before both the
    log and the sum.
  * masked pixels are excluded from every sum (Q, S, W', numerator, denominator).
  * voxels with zero denominator keep their previous value.

parity pinned: see tests/test_oracle_pins.py (library routines, brute-force dense
interpolation matrices, closed forms and invariants).
"""
from __future__ import annotations

import numpy as np

W_FLOOR = 1e-10


# ---------------------------------------------------------------------------------------
# rotations (Section 2.2: each rotation R_j given as a unit quaternion, with prior weight w_j)
# ---------------------------------------------------------------------------------------
def rotation_matrix(quat: np.ndarray) -> np.ndarray:
    """Rotation matrices [..., 3, 3] of quaternions [..., 4] = (w, x, y, z), normalised first."""
    q = np.asarray(quat, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def slice_positions(q: np.ndarray, quat: np.ndarray, grid_n: int) -> np.ndarray:
    """Grid-frame positions of R_j q_i, [n_rot][n_pix][3] (Section 2.2 notation W_ij = W(R_j q_i))."""
    R = rotation_matrix(quat)
    return np.einsum("jab,ib->jia", R, np.asarray(q, dtype=np.float64)) + grid_n / 2.0


# ---------------------------------------------------------------------------------------
# interpolation weights f (eq. (2.8)); the sum over l reduces to the 8 grid points around p
# ---------------------------------------------------------------------------------------
def tent(d: np.ndarray) -> np.ndarray:
    """f(d) = prod_a max(0, 1 - |d_a|) over the last axis."""
    return np.prod(np.maximum(0.0, 1.0 - np.abs(d)), axis=-1)


def stencil(p: np.ndarray, grid_n: int):
    """Grid points l with f(p_l - p) possibly > 0 and their weights.

    Returns (flat index [..., 8] int64, weight [..., 8] float64); grid points
    outside the N^3 box get weight 0 and index 0.
    """
    base = np.floor(p).astype(np.int64)
    idx = np.zeros(p.shape[:-1] + (8,), dtype=np.int64)
    wt = np.zeros(p.shape[:-1] + (8,))
    t = 0
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                v = base + np.array([dx, dy, dz])
                inside = np.all((v >= 0) & (v < grid_n), axis=-1)
                w = tent(v - p)
                idx[..., t] = np.where(inside, (v[..., 0] * grid_n + v[..., 1]) * grid_n + v[..., 2], 0)
                wt[..., t] = np.where(inside, w, 0.0)
                t += 1
    return idx, wt


# ---------------------------------------------------------------------------------------
# e-step: expansion, eq. (2.9)
# ---------------------------------------------------------------------------------------
def expand(model: np.ndarray, q: np.ndarray, quat: np.ndarray, grid_n: int) -> np.ndarray:
    """W_ij = sum_l f(p_l - R_j q_i) model_l, returned as W[j][i]."""
    p = slice_positions(q, quat, grid_n)
    idx, wt = stencil(p, grid_n)
    return np.sum(wt * np.asarray(model, dtype=np.float64)[idx], axis=-1)


# ---------------------------------------------------------------------------------------
# Poisson log-likelihood (Section 2.2; joint log-likelihood summed over pixels, eq. (2.3))
# ---------------------------------------------------------------------------------------
def log_likelihood(W: np.ndarray, K: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Q[j][k] = sum_{i valid} K_ik log Wf_ij - Wf_ij with Wf = max(W, 1e-10)."""
    v = np.flatnonzero(mask)
    Wf = np.maximum(np.asarray(W, dtype=np.float64)[:, v], W_FLOOR)
    Kv = np.asarray(K, dtype=np.float64)[:, v]
    return np.log(Wf) @ Kv.T - Wf.sum(axis=1)[:, None]


# ---------------------------------------------------------------------------------------
# E-step, eq. (2.4): P_jk = w_j T_jk / sum_j' w_j' T_j'k with T = exp(Q)
# ---------------------------------------------------------------------------------------
def responsibilities(Q: np.ndarray, log_w: np.ndarray):
    """Returns (P[j][k], L[k]) with L_k = log sum_j w_j exp(Q_jk) (the frame's log-evidence).

    The normalisation is evaluated as a max-shifted log-sum-exp so that no
    exponential overflows or underflows to a zero denominator.
    """
    a = np.asarray(Q, dtype=np.float64) + np.asarray(log_w, dtype=np.float64)[:, None]
    m = a.max(axis=0)
    L = m + np.log(np.exp(a - m[None, :]).sum(axis=0))
    return np.exp(a - L[None, :]), L


# ---------------------------------------------------------------------------------------
# M-step numerator, eq. (2.11) with phi = 1, and the per-rotation weight sum_k P_jk
# ---------------------------------------------------------------------------------------
def maximize(P: np.ndarray, K: np.ndarray, mask: np.ndarray):
    """Returns (Wp[j][i] = sum_k P_jk K_ik on valid pixels, 0 on masked; rho[j] = sum_k P_jk)."""
    Wp = np.asarray(P, dtype=np.float64) @ np.asarray(K, dtype=np.float64)
    Wp[:, np.asarray(mask) == 0] = 0.0
    return Wp, np.asarray(P, dtype=np.float64).sum(axis=1)


# ---------------------------------------------------------------------------------------
# c-step, eq. (2.12): numerator and denominator on the grid, then their ratio
# ---------------------------------------------------------------------------------------
def compress(Wp: np.ndarray, rho: np.ndarray, q: np.ndarray, mask: np.ndarray,
             quat: np.ndarray, grid_n: int):
    """num_l = sum_{j, i valid} f(p_l - R_j q_i) Wp_ij ; den_l = sum_{j, i valid} f(...) rho_j."""
    v = np.flatnonzero(mask)
    p = slice_positions(np.asarray(q)[v], quat, grid_n)          # [j][iv][3]
    idx, wt = stencil(p, grid_n)                                  # [j][iv][8]
    M = grid_n ** 3
    num = np.bincount(idx.ravel(), weights=(wt * np.asarray(Wp, dtype=np.float64)[:, v, None]).ravel(),
                      minlength=M)
    den = np.bincount(idx.ravel(), weights=(wt * np.asarray(rho, dtype=np.float64)[:, None, None]).ravel(),
                      minlength=M)
    return num, den


def divide(num: np.ndarray, den: np.ndarray, model_prev: np.ndarray) -> np.ndarray:
    """New model num/den where den > 0; elsewhere the previous value is kept."""
    out = np.array(model_prev, dtype=np.float64, copy=True)
    pos = den > 0
    out[pos] = num[pos] / den[pos]
    return out


# ---------------------------------------------------------------------------------------
# Algorithm 1 (one pass of the loop): expand -> E -> combined M and c
# ---------------------------------------------------------------------------------------
def iterate(model, K, q, mask, quat, log_w, grid_n, frame_chunk: int | None = None):
    """One EMC iteration.  Returns a dict with W, Q, P, L, loglik, Wp, rho, num, den, model.

    `frame_chunk` sums the M- and c-step contributions over consecutive frame
    chunks before the division (the k-direction split of Section 3.3); the
    result is the same up to rounding.
    """
    W = expand(model, q, quat, grid_n)
    n_data = np.asarray(K).shape[0]
    chunk = n_data if not frame_chunk else frame_chunk
    M = grid_n ** 3
    num, den = np.zeros(M), np.zeros(M)
    Qs, Ps, Ls = [], [], []
    Wp_tot = np.zeros_like(W)
    rho_tot = np.zeros(W.shape[0])
    for s in range(0, n_data, chunk):
        Kc = np.asarray(K[s:s + chunk], dtype=np.float64)
        Q = log_likelihood(W, Kc, mask)
        P, L = responsibilities(Q, log_w)
        Wp, rho = maximize(P, Kc, mask)
        n_c, d_c = compress(Wp, rho, q, mask, quat, grid_n)
        num += n_c
        den += d_c
        Wp_tot += Wp
        rho_tot += rho
        Qs.append(Q), Ps.append(P), Ls.append(L)
    Q = np.concatenate(Qs, axis=1)
    P = np.concatenate(Ps, axis=1)
    L = np.concatenate(Ls)
    new = divide(num, den, model)
    return dict(W=W, Q=Q, P=P, L=L, loglik=float(L.mean()), Wp=Wp_tot, rho=rho_tot,
                num=num, den=den, model=new)


def paper_flops(n_rot: int, n_data: int, n_pix: int) -> float:
    """The paper's operation count for one iteration: 27 Mrot Mdata Mpix (Section 4.2)."""
    return 27.0 * n_rot * n_data * n_pix


def mrot_600cell(d: int) -> int:
    """Number of rotations of the 600-cell refined d times, eq. (2.7)."""
    return 10 * (5 * d ** 3 + d)


# ---------------------------------------------------------------------------------------
# learned-proposal form: the same iteration with each frame's E-step restricted to its
# candidate rotations (audited frames keep the full search)
# ---------------------------------------------------------------------------------------
def responsibilities_restricted(Q: np.ndarray, log_w: np.ndarray, cand: np.ndarray):
    """eq. (2.4) with the sum over rotations limited to cand[j][k] (boolean); P = 0 elsewhere."""
    a = np.where(cand, np.asarray(Q, dtype=np.float64) + np.asarray(log_w)[:, None], -np.inf)
    m = a.max(axis=0)
    L = m + np.log(np.exp(a - m[None, :]).sum(axis=0))
    return np.exp(a - L[None, :]), L


def iterate_proposed(model, K, q, mask, quat, log_w, grid_n, cand):
    """One EMC iteration whose E-step runs over cand[j][k] only (see responsibilities_restricted)."""
    W = expand(model, q, quat, grid_n)
    Kf = np.asarray(K, dtype=np.float64)
    Q = log_likelihood(W, Kf, mask)
    P, L = responsibilities_restricted(Q, log_w, cand)
    Wp, rho = maximize(P, Kf, mask)
    num, den = compress(Wp, rho, q, mask, quat, grid_n)
    return dict(W=W, Q=Q, P=P, L=L, loglik=float(L.mean()), Wp=Wp, rho=rho, num=num, den=den,
                model=divide(num, den, model))


def proposal_recall(P_full: np.ndarray, cand: np.ndarray) -> np.ndarray:
    """recall_k = sum_{j in cand(k)} P_jk of the full-search responsibilities."""
    return (np.asarray(P_full) * cand).sum(axis=0)
