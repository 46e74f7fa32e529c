"""Plain C (FP64) forms of the oracle's expansion and c-step, and compositions of
them with the numpy oracle for problems at the full rotation count.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  The C source (emc_oracle_c.c) shares
no code with the GPU library; it is compiled with gcc into oracle/liboracle.so.

* ``expand`` / ``compress``: same arguments and results as ``emc_oracle.expand``
  (eq. 2.9) and ``emc_oracle.compress`` (eq. 2.12), in C loops over rotations
  and pixels (no [rotation][pixel][8] temporaries).
* ``loglik_all_rotations``: Q[j][k] over every rotation for a few frames
  (Section 2.2), slices expanded a chunk of rotations at a time and handed to
  ``emc_oracle.log_likelihood``.
* ``iterate_chunked``: one whole iteration (Algorithm 1) composed from the same
  oracle steps, with the sums over rotations of the M- and c-step taken a chunk
  of rotations at a time, for the full rotation count on a reduced frame share.

parity pinned: tests/test_oracle_c_pins.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import emc_oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "emc_oracle_c.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build_oracle(force: bool = False) -> str:
    """Compile liboracle.so with gcc (strict IEEE FP64: no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        build_oracle()
        lib = ctypes.CDLL(LIB)
        P, L, I = ctypes.c_void_p, ctypes.c_long, ctypes.c_int
        lib.orc_expand.argtypes = [P, I, P, L, P, L, P]
        lib.orc_expand.restype = None
        lib.orc_compress.argtypes = [P, P, P, P, L, P, L, I, P, P]
        lib.orc_compress.restype = None
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def expand(model, q, quat, grid_n: int) -> np.ndarray:
    """W[j][i] = sum_l f(p_l - R_j q_i) model_l (eq. 2.9), every pixel."""
    model, q, quat = _f64(model), _f64(q).reshape(-1, 3), _f64(quat).reshape(-1, 4)
    assert model.size == grid_n ** 3
    W = np.empty((quat.shape[0], q.shape[0]))
    _load().orc_expand(_p(model), int(grid_n), _p(q), q.shape[0], _p(quat), quat.shape[0], _p(W))
    return W


def compress(Wp, rho, q, mask, quat, grid_n: int):
    """(num, den) of eq. (2.12) over valid pixels."""
    Wp, rho, q, quat = _f64(Wp), _f64(rho), _f64(q).reshape(-1, 3), _f64(quat).reshape(-1, 4)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    assert Wp.shape == (quat.shape[0], q.shape[0]) and rho.shape == (quat.shape[0],) and m.size == q.shape[0]
    M = grid_n ** 3
    num, den = np.empty(M), np.empty(M)
    _load().orc_compress(_p(Wp), _p(rho), _p(q), _p(m), q.shape[0], _p(quat), quat.shape[0], int(grid_n),
                         _p(num), _p(den))
    return num, den


def loglik_all_rotations(model, K, q, mask, quat, grid_n: int, rot_chunk: int = 2000) -> np.ndarray:
    """Q[j][k] = sum_{i valid} K_ik log max(W_ij, 1e-10) - max(W_ij, 1e-10) for every rotation."""
    quat = _f64(quat).reshape(-1, 4)
    v = np.flatnonzero(mask)
    # the valid pixels only: the same sums, without [rotation][pixel] copies of the masked columns
    qv = _f64(q).reshape(-1, 3)[v]
    Kv = np.ascontiguousarray(np.asarray(K, dtype=np.float64)[:, v])
    ones = np.ones(v.size, np.uint8)
    Q = np.empty((quat.shape[0], Kv.shape[0]))
    for s in range(0, quat.shape[0], rot_chunk):
        Q[s:s + rot_chunk] = O.log_likelihood(expand(model, qv, quat[s:s + rot_chunk], grid_n), Kv, ones)
    return Q


def iterate_chunked(model, K, q, mask, quat, log_w, grid_n: int, rot_chunk: int = 2000) -> dict:
    """One iteration (expand -> E -> M and c -> divide), sums over rotations taken a chunk at a time."""
    quat = _f64(quat).reshape(-1, 4)
    K = np.asarray(K, dtype=np.float64)
    Q = loglik_all_rotations(model, K, q, mask, quat, grid_n, rot_chunk)
    P, L = O.responsibilities(Q, log_w)
    M = grid_n ** 3
    num, den = np.zeros(M), np.zeros(M)
    rho = np.empty(quat.shape[0])
    for s in range(0, quat.shape[0], rot_chunk):
        Wp, rho[s:s + rot_chunk] = O.maximize(P[s:s + rot_chunk], K, mask)
        n_c, d_c = compress(Wp, rho[s:s + rot_chunk], q, mask, quat[s:s + rot_chunk], grid_n)
        num += n_c
        den += d_c
    return dict(Q=Q, P=P, L=L, loglik=float(L.mean()), rho=rho, num=num, den=den,
                model=O.divide(num, den, model))
