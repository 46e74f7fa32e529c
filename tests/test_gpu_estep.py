"""The E-step (eq. 2.4) on a given G, through the C ABI, against FP64 numpy.

The log-joint a_jk = (G_jk + b_k) + (log w_j - S_j) is formed in the same FP64
order on both sides, so each frame's maximum must agree bit for bit; the sum of
exp(a - max) and L = max + log(sum) within FP64 summation-order error; P within
the precision it is stored in.  The frames mix concentrated posteriors (a few
units between rotations) with wide ones (hundreds of units: most terms beyond
the statistics pass's cutoff of 64 below the running maximum), some rotations
have zero prior weight (log w = -inf), and the padding columns of G hold NaN,
which must not reach any output.  Sizes are ragged against the kernels' frame
blocks (256 frames) and rotation strides (16 waves).
"""
import numpy as np
import pytest

from emc_inputs import tiny_problem
from paper_1409_4256_amd import emc as E

pytestmark = pytest.mark.gpu


def _problem(seed, n_rot, n_data):
    rng = np.random.default_rng([1409, 24, seed])
    t = tiny_problem(seed, grid_n=12, n_pix=64, n_rot=n_rot, n_data=n_data)
    log_w = t["log_w"].copy()
    log_w[rng.choice(n_rot, max(1, n_rot // 20), replace=False)] = -np.inf
    spread = rng.choice([0.5, 5.0, 50.0, 500.0], size=n_data)        # per-frame width of the log-joint
    G = -np.abs(rng.standard_normal((n_rot, n_data))) * spread[None, :]
    G[rng.integers(0, n_rot, n_data), np.arange(n_data)] = 0.0      # each frame's best rotation
    G += rng.normal(0.0, 30.0, n_data)[None, :]
    b = rng.normal(0.0, 1000.0, n_data)
    S = rng.uniform(0.0, 100.0, n_rot)
    return t, log_w, G.astype(np.float32), b, S


@pytest.mark.parametrize("precision", [E.EMC_PREC_FP32, E.EMC_PREC_BF16])
@pytest.mark.parametrize("seed,n_rot,n_data", [(1, 777, 1000), (2, 40, 300), (3, 3001, 257)])
def test_estep_on_given_G_matches_fp64(gpu_lib, precision, seed, n_rot, n_data):
    import torch

    from gpu_helpers import geometry

    t, log_w, G, b, S = _problem(seed, n_rot, n_data)
    geo = geometry(12, t["q"], t["mask"], t["quat"], log_w, n_data, precision)
    ds = geo.data_stride
    Gp = np.full((n_rot, ds), np.nan, dtype=np.float32)
    Gp[:, :n_data] = G
    dev = "cuda"
    Gd = torch.as_tensor(Gp.reshape(-1), device=dev)
    Sd = torch.as_tensor(S, device=dev)
    bd = torch.as_tensor(b, device=dev)
    stats = torch.empty(2 * n_data, dtype=torch.float64, device=dev)
    E.emc_responsibilities(geo, Gd, Sd, bd, E.EMC_RESP_PARTIAL, stats)
    bf16 = precision == E.EMC_PREC_BF16
    P = torch.full((n_rot * ds,), 7.0, dtype=torch.bfloat16 if bf16 else torch.float32, device=dev)
    L = torch.empty(n_data, dtype=torch.float64, device=dev)
    rho = torch.empty(n_rot, dtype=torch.float64, device=dev)
    E.emc_responsibilities(geo, Gd, Sd, bd, E.EMC_RESP_FULL, stats, P, L, rho)
    torch.cuda.synchronize()

    a = (G.astype(np.float64) + b[None, :]) + (log_w - S)[:, None]
    m_ref = a.max(axis=0)
    s_ref = np.exp(a - m_ref[None, :]).sum(axis=0)
    L_ref = m_ref + np.log(s_ref)
    st = stats.cpu().numpy().reshape(n_data, 2)
    assert np.array_equal(st[:, 0], m_ref)
    np.testing.assert_allclose(st[:, 1], s_ref, rtol=n_rot * 2.0 ** -52)
    Lg = L.cpu().numpy()
    assert np.all(np.abs(Lg - L_ref) <= n_rot * 2.0 ** -52 + 2.0 ** -52 * np.abs(L_ref))

    Pg = P.float().cpu().numpy().reshape(n_rot, ds)
    assert np.all(Pg[:, n_data:] == 0.0)          # padding frames: zeros, whatever G holds there
    Pg = Pg[:, :n_data].astype(np.float64)
    x = a - L_ref[None, :]
    P_ref = np.exp(x)
    assert np.all(Pg[~np.isfinite(log_w)] == 0.0)  # zero prior weight
    if bf16:   # FP32 exponential rounded to BF16: half a BF16 unit, plus the FP32 error
        tol = P_ref * (2.0 ** -8 + 1e-6) + 1e-38
    else:      # the FP32 exponent's rounding (|x| 2^-24 relative) and expf's own error
        tol = P_ref * (3e-7 + 6e-8 * np.abs(np.where(np.isfinite(x), x, 0.0))) + 2e-38
    err = np.abs(Pg - P_ref)
    assert np.all(err <= tol), float((err / np.maximum(tol, 1e-300)).max())
    # rho sums the stored values
    np.testing.assert_allclose(rho.cpu().numpy(), Pg.sum(axis=1), rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(Pg.sum(axis=0), 1.0, atol=4e-3 if bf16 else 1e-5)
