"""Parity at the full one-GPU share (128^3 grid, 16384 pixels, 25000 rotations,
100000 frames) with the benchmark's buffers and launch configuration.

The FP64 oracle cannot run the whole iteration at this size inside a test, so
it computes what it can one by one -- the slices of sampled rotations and the
log-likelihoods of sampled (rotation, frame) pairs -- and the rest is held to
identities that hold at any size: responsibilities sum to one per frame; the
log-evidence bounds every log-joint term; the trilinear weights sum to one, so
the denominator grid sums to Mdata x (valid pixels) and the numerator grid to
the total photon count; the M-step GEMM equals sum_k P_kj K_k in FP64.
"""
import numpy as np
import pytest

import oracle as O
from emc_inputs import WORKLOADS, make_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full(gpu_lib):
    import torch

    import bench

    emc = gpu_lib
    print("\n[fullsize] generating 128^3 / 25000 rotations / 100000 frames on the GPU", flush=True)
    inp = make_inputs(WORKLOADS[2], device="cuda", with_truth=False)
    run = bench.Run(inp)
    g, wl = run.geo, inp.wl
    n, ps, rs = wl.n_data, g.pix_stride, g.rot_stride
    rng = np.random.default_rng(7)
    ks = np.sort(rng.choice(n, 24, replace=False))
    snap = {}
    m_in = run.model[0]
    print("[fullsize] expand", flush=True)
    emc.emc_expand(g, m_in, run.c, run.slices, run.S)
    print("[fullsize] log-likelihood GEMM", flush=True)
    emc.emc_loglik(g, run.K, run.slices, run.c, run.GP, run.b)
    torch.cuda.synchronize()
    Gs = run.GP.view(n, rs)[torch.as_tensor(ks, device="cuda"), :wl.n_rot].double().cpu().numpy()
    snap["G"] = Gs
    snap["b"] = run.b.cpu().numpy()[ks]
    snap["S"] = run.S.cpu().numpy()
    snap["c"] = run.c.cpu().numpy()
    js = np.sort(rng.choice(wl.n_rot, 40, replace=False))
    jstar = np.argmax(Gs - snap["S"][None, :] + inp.log_w[None, :], axis=1)   # sample choice only
    js = np.unique(np.concatenate([js, jstar]))
    snap["js"] = js
    snap["logW_c"] = run.slices.view(wl.n_rot, ps)[torch.as_tensor(js, device="cuda")].double().cpu().numpy()
    print("[fullsize] E-step", flush=True)
    emc.emc_responsibilities(g, run.GP, run.S, run.b, emc.EMC_RESP_FULL, run.stats, run.GP, run.L, run.rho)
    torch.cuda.synchronize()
    P = run.GP.view(n, rs)
    snap["P_rowsum"] = P[:, :wl.n_rot].double().sum(1).cpu().numpy()
    snap["P_pad_max"] = float(P[:, wl.n_rot:].abs().max().item()) if rs > wl.n_rot else 0.0
    snap["P_cols"] = P[:, torch.as_tensor(js[:8], device="cuda")].double().cpu().numpy()   # [n][8]
    snap["L"] = run.L.cpu().numpy()
    snap["rho"] = run.rho.cpu().numpy()
    print("[fullsize] compress", flush=True)
    emc.emc_compress(g, run.GP, run.K, run.rho, run.slices, run.num, run.den, accumulate=False)
    torch.cuda.synchronize()
    snap["Wp"] = run.slices.view(wl.n_rot, ps)[torch.as_tensor(js[:8], device="cuda")].double().cpu().numpy()
    snap["num_sum"] = float(run.num.sum().item())
    snap["den_sum"] = float(run.den.sum().item())
    m_out = run.model[1]
    emc.emc_finalize(g, run.num, run.den, m_in, m_out, run.L, n, run.loglik)
    torch.cuda.synchronize()
    snap["model_in"] = m_in.double().cpu().numpy()
    snap["model_out"] = m_out.double().cpu().numpy()
    snap["den_pos"] = (run.den > 0).cpu().numpy()
    snap["loglik"] = run.loglik.item()
    counts = inp.counts
    snap["photons_total"] = float(counts.to(torch.int64).sum().item())
    # uint16 has no CUDA indexing kernel; int16 is the same bits for counts < 32768
    snap["K_rows"] = counts.view(torch.int16)[torch.as_tensor(ks, device="cuda")].to(torch.int32).cpu().numpy()
    snap["K_all_f64"] = None
    snap["ks"] = ks
    snap["counts_dev"] = counts
    print("[fullsize] done", flush=True)
    return inp, snap


def test_fullsize_slices_match_oracle(full):
    inp, s = full
    wl = inp.wl
    v = np.flatnonzero(inp.mask)
    q = np.asarray(inp.q, np.float32).astype(np.float64)
    quat = np.asarray(inp.quat, np.float32).astype(np.float64)[s["js"]]
    W = O.expand(s["model_in"], q[v], quat, wl.grid_n)
    logW = s["logW_c"][:, v] + s["c"][None, v]
    assert np.max(np.abs(logW - np.log(np.maximum(W, 1e-10)))) < 5e-6
    np.testing.assert_allclose(s["S"][s["js"]], np.maximum(W, 1e-10).sum(1), rtol=1e-12)
    s["W_oracle"] = W


def test_fullsize_loglik_pairs_match_oracle(full):
    inp, s = full
    wl = inp.wl
    v = np.flatnonzero(inp.mask)
    q = np.asarray(inp.q, np.float32).astype(np.float64)
    quat = np.asarray(inp.quat, np.float32).astype(np.float64)[s["js"]]
    W = s.get("W_oracle")
    if W is None:
        W = O.expand(s["model_in"], q[v], quat, wl.grid_n)
    Wfull = np.zeros((W.shape[0], wl.n_pix))
    Wfull[:, v] = W
    Q_ref = O.log_likelihood(Wfull, s["K_rows"], inp.mask)                    # [js][ks]
    Q_gpu = (s["G"][:, s["js"]] + s["b"][:, None] - s["S"][None, s["js"]]).T
    rel = np.max(np.abs(Q_gpu - Q_ref), axis=0) / np.max(np.abs(Q_ref), axis=0)
    assert rel.max() <= 1e-5, rel.max()
    # the log-evidence bounds every log-joint term of its frame
    L = s["L"][s["ks"]]
    assert np.all(L[None, :] >= Q_ref + inp.log_w[s["js"]][:, None] - 1e-6 * np.abs(L[None, :]))


def test_fullsize_responsibilities_properties(full):
    inp, s = full
    np.testing.assert_allclose(s["P_rowsum"], 1.0, atol=2e-5)
    assert s["P_pad_max"] == 0.0
    np.testing.assert_allclose(s["rho"].sum(), inp.wl.n_data, rtol=1e-5)
    assert np.isfinite(s["loglik"])


def test_fullsize_mstep_gemm_and_grid_identities(full):
    import torch

    inp, s = full
    wl = inp.wl
    v = np.flatnonzero(inp.mask)
    # M-step GEMM of sampled rotations in FP64 from the same responsibilities
    K = s["counts_dev"].to(torch.float64)
    ref = (torch.as_tensor(s["P_cols"], device="cuda").T @ K).cpu().numpy()     # [8][n_pix]
    got = s["Wp"][:, :wl.n_pix]
    assert np.linalg.norm(got[:, v] - ref[:, v]) / np.linalg.norm(ref[:, v]) <= 1e-5
    assert np.all(got[:, inp.mask == 0] == 0)
    # partition of unity of the trilinear weights
    np.testing.assert_allclose(s["den_sum"], wl.n_data * v.size, rtol=1e-5)
    np.testing.assert_allclose(s["num_sum"], s["photons_total"], rtol=1e-5)
    m = s["model_out"]
    assert np.all(np.isfinite(m))
    assert np.all(m[s["den_pos"]] >= 0)
    np.testing.assert_array_equal(m[~s["den_pos"]], s["model_in"][~s["den_pos"]])
