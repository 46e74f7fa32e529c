"""GPU (HIP, gfx950) vs FP64 oracle, element by element, through the C ABI.

Plain FP32 form: log-likelihood relative error <= 1e-5 (worst frame of
max_j |dQ| / max_j |Q|), responsibilities max-abs <= 1e-3, updated model
relative L2 <= 1e-5.
BF16 form: updated model relative L2 <= 1e-3 and top-1 orientation agreement
>= 99 %; the other errors are reported.
"""
import math

import numpy as np
import pytest

import oracle as O
from emc_inputs import WORKLOADS, make_inputs, tiny_problem
from paper_1409_4256_amd import emc as E

pytestmark = pytest.mark.gpu

Q_TOL, P_TOL, MODEL_TOL = 1e-5, 1e-3, 1e-5
MIXED_MODEL_TOL, MIXED_TOP1 = 1e-3, 0.99


def _oracle(model, counts, q, mask, quat, log_w, N):
    return O.iterate(np.asarray(model, dtype=np.float32).astype(np.float64), counts, q, mask, quat, log_w, N)


def _inputs_f32(q, quat):
    # the GPU receives FP32 coordinates and quaternions: the oracle gets the same values
    return np.asarray(q, np.float32).astype(np.float64), np.asarray(quat, np.float32).astype(np.float64)


def _check_expand(g, o, mask, tol):
    v = mask.astype(bool)
    Wf = np.log(np.maximum(o["W"], 1e-10))
    lw = g["logW_c"] + g["c"][None, :]
    assert np.max(np.abs(lw[:, v] - Wf[:, v])) < tol
    assert np.all(g["logW_c"][:, ~v] == 0) and np.all(g["logW_pad"] == 0)
    np.testing.assert_allclose(g["S"], np.maximum(o["W"], 1e-10)[:, v].sum(1), rtol=1e-12)


def _check_all(g, o, mask, tag):
    from gpu_helpers import q_rel_err, rel_l2

    _check_expand(g, o, mask, 5e-6)
    assert q_rel_err(g["Q"], o["Q"]) <= Q_TOL, (tag, q_rel_err(g["Q"], o["Q"]))
    assert np.max(np.abs(g["P"] - o["P"])) <= P_TOL, (tag, np.max(np.abs(g["P"] - o["P"])))
    assert g["P_pad_max"] == 0
    np.testing.assert_allclose(g["L"], o["L"], rtol=1e-6)
    np.testing.assert_allclose(g["P"].sum(0), 1.0, atol=1e-5)
    np.testing.assert_allclose(g["rho"], o["rho"], rtol=1e-4, atol=1e-6 * o["rho"].max())
    assert rel_l2(g["Wp"], o["Wp"]) <= 1e-5, (tag, rel_l2(g["Wp"], o["Wp"]))
    assert rel_l2(g["num"], o["num"]) <= 1e-5 and rel_l2(g["den"], o["den"]) <= 1e-5, tag
    err = rel_l2(g["model"], o["model"])
    assert err <= MODEL_TOL, (tag, err)
    assert abs(g["loglik"] - o["loglik"]) <= 1e-6 * abs(o["loglik"]), tag


@pytest.fixture(scope="module")
def cfg1():
    return make_inputs(WORKLOADS[1])


@pytest.mark.parametrize("start", ["random_smooth", "true_model"])
def test_config1_full_iteration_matches_oracle(gpu_lib, cfg1, start):
    from gpu_helpers import geometry, pack, run_steps, upload_counts

    inp = cfg1
    model = inp.model_start if start == "random_smooth" else inp.model_true
    q, quat = _inputs_f32(inp.q, inp.quat)
    geo = geometry(32, q, inp.mask, quat, inp.log_w, inp.wl.n_data)
    K = pack(geo, upload_counts(inp.counts))
    g = run_steps(geo, model, K)
    o = _oracle(model, inp.counts, q, inp.mask, quat, inp.log_w, 32)
    _check_all(g, o, inp.mask, start)


@pytest.mark.parametrize("seed,N,npx,nrot,ndata,qr", [(0, 24, 529, 300, 333, None), (1, 20, 257, 129, 517, None),
                                                      (2, 16, 64, 1, 40, None), (3, 18, 300, 257, 1, None),
                                                      (4, 12, 200, 70, 90, 2.5)])
@pytest.mark.parametrize("cstep", ["copies", "direct", "brick", "brick_chunk64"])
def test_ragged_shapes_match_oracle(gpu_lib, seed, N, npx, nrot, ndata, qr, cstep):
    # random pixel positions in a ball of radius N/2 - 2 spread each 64-pixel group
    # beyond the rotation-major compression's local box (global-atomic path) and over
    # many bricks; qr = 2.5 keeps them inside one box (local-box path).  c-step forms:
    # rotation-major with per-XCD grid copies or direct atomics, brick-major with the
    # default work items or 64-visit ones (several items per brick).
    from gpu_helpers import geometry, pack, run_steps, upload_counts

    t = tiny_problem(seed, grid_n=N, n_pix=npx, n_rot=nrot, n_data=ndata, photons=200.0, q_radius=qr)
    q, quat = _inputs_f32(t["q"], t["quat"])
    geo = geometry(N, q, t["mask"], quat, t["log_w"], ndata)
    if cstep.startswith("brick"):
        geo.use_brick_scatter(chunk=64 if cstep == "brick_chunk64" else 0)
    K = pack(geo, upload_counts(t["counts"]))
    g = run_steps(geo, t["model"], K, grid_copies=cstep == "copies")
    o = _oracle(t["model"], t["counts"], q, t["mask"], quat, t["log_w"], N)
    _check_all(g, o, t["mask"], f"seed{seed} c-step {cstep}")


@pytest.mark.parametrize("brick", [False, True])
def test_frame_chunks_accumulate_before_division(gpu_lib, brick):
    from gpu_helpers import geometry, pack, rel_l2, run_steps, upload_counts

    t = tiny_problem(5, grid_n=20, n_pix=400, n_rot=200, n_data=700, photons=150.0)
    q, quat = _inputs_f32(t["q"], t["quat"])
    geo = geometry(20, q, t["mask"], quat, t["log_w"], 700)
    if brick:
        geo.use_brick_scatter()
    chunks = []
    for s in range(0, 700, 256):
        g = geo.with_frames(min(256, 700 - s))
        chunks.append((g, pack(g, upload_counts(t["counts"][s:s + 256])), s))
    r = run_steps(geo, t["model"], None, frame_chunks=chunks)
    o = _oracle(t["model"], t["counts"], q, t["mask"], quat, t["log_w"], 20)
    assert rel_l2(r["model"], o["model"]) <= MODEL_TOL
    assert np.max(np.abs(r["P"] - o["P"])) <= P_TOL
    assert abs(r["loglik"] - o["loglik"]) <= 1e-6 * abs(o["loglik"])


def test_empty_frame_set_keeps_model(gpu_lib):
    from gpu_helpers import geometry, pack, run_steps

    t = tiny_problem(6, grid_n=12, n_pix=50, n_rot=10, n_data=0)
    q, quat = _inputs_f32(t["q"], t["quat"])
    geo = geometry(12, q, t["mask"], quat, t["log_w"], 0)
    import torch

    K = pack(geo, torch.zeros(1, dtype=torch.uint16, device="cuda"))
    g = run_steps(geo, t["model"], K)
    np.testing.assert_array_equal(g["model"], np.asarray(t["model"], np.float32).astype(np.float64))
    assert math.isnan(g["loglik"])
    assert np.all(g["den"] == 0)


@pytest.mark.parametrize("brick", [False, True])
def test_single_rotation_mean_frame_on_gpu(gpu_lib, brick):
    # identity rotation, flat detector on integer voxels: the touched voxels are
    # exactly the mean frame (closed form of the method)
    from gpu_helpers import geometry, pack, run_steps, upload_counts

    N = 16
    u = np.arange(-4, 5)
    X, Y = np.meshgrid(u, u, indexing="ij")
    q = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    mask = np.ones(q.shape[0], np.uint8)
    mask[7] = 0
    K = np.random.default_rng(3).poisson(5.0, size=(37, q.shape[0])).astype(np.uint16)
    K[:, mask == 0] = 0
    geo = geometry(N, q, mask, np.array([[1.0, 0, 0, 0]]), np.array([0.0]), 37)
    if brick:
        geo.use_brick_scatter()
    g = run_steps(geo, np.ones(N ** 3), pack(geo, upload_counts(K)))
    l = ((X.ravel() + 8) * N + (Y.ravel() + 8)) * N + 8
    v = mask.astype(bool)
    np.testing.assert_allclose(g["model"][l[v]], K.mean(axis=0)[v], rtol=2e-7)
    np.testing.assert_allclose(g["P"], 1.0)


def _shard_run(geo, model, K, n):
    import torch

    ps, ds = geo.pix_stride, geo.data_stride
    c = torch.empty(ps, dtype=torch.float64, device="cuda")
    slices = E.slices_tensor(geo)
    S = torch.empty(geo.n_rot, dtype=torch.float64, device="cuda")
    E.emc_expand(geo, model, c, slices, S)
    G = torch.empty(geo.n_rot * ds, dtype=torch.float32, device="cuda")
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    E.emc_loglik(geo, K, slices, None, c, G, b)
    stats = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    E.emc_responsibilities(geo, G, S, b, E.EMC_RESP_PARTIAL, stats)
    return dict(G=G, S=S, b=b, stats=stats)


def test_virtual_rotation_shards_equal_unsharded(gpu_lib):
    """Four rotation shares on one GPU, statistics combined on the host (Section 3.2)."""
    import torch

    from gpu_helpers import geometry, pack, upload_counts

    t = tiny_problem(8, grid_n=20, n_pix=300, n_rot=400, n_data=150, photons=200.0)
    q, quat = _inputs_f32(t["q"], t["quat"])
    n = 150
    geo_full = geometry(20, q, t["mask"], quat, t["log_w"], n)
    Kd = pack(geo_full, upload_counts(t["counts"]))
    model = torch.as_tensor(t["model"], dtype=torch.float32, device="cuda")
    full = _shard_run(geo_full, model, Kd, n)
    ds = geo_full.data_stride
    P_full = torch.empty(400 * ds, dtype=torch.float32, device="cuda")
    L_full = torch.empty(n, dtype=torch.float64, device="cuda")
    rho_full = torch.empty(400, dtype=torch.float64, device="cuda")
    E.emc_responsibilities(geo_full, full["G"], full["S"], full["b"], E.EMC_RESP_FINALIZE, full["stats"],
                           P_full, L_full, rho_full)
    bounds = [0, 90, 200, 333, 400]
    shards = []
    for a, z in zip(bounds[:-1], bounds[1:]):
        geo = geometry(20, q, t["mask"], quat[a:z], t["log_w"][a:z], n)
        shards.append((geo, _shard_run(geo, model, Kd, n)))
    # host combination of the per-frame statistics (what an all-reduce would carry)
    st = np.stack([s["stats"].cpu().numpy().reshape(n, 2) for _, s in shards])
    m = st[:, :, 0].max(0)
    s = (st[:, :, 1] * np.exp(st[:, :, 0] - m[None, :])).sum(0)
    glob = torch.as_tensor(np.stack([m, s], 1).reshape(-1), device="cuda")
    P_parts, rho_parts = [], []
    for geo, o in shards:
        P = torch.empty(geo.n_rot * ds, dtype=torch.float32, device="cuda")
        L = torch.empty(n, dtype=torch.float64, device="cuda")
        rho = torch.empty(geo.n_rot, dtype=torch.float64, device="cuda")
        E.emc_responsibilities(geo, o["G"], o["S"], o["b"], E.EMC_RESP_FINALIZE, glob, P, L, rho)
        P_parts.append(P.view(geo.n_rot, ds)[:, :n].cpu().numpy())
        rho_parts.append(rho.cpu().numpy())
        # each share centres its own slices, so the FP32 contractions round differently
        np.testing.assert_allclose(L.cpu().numpy(), L_full.cpu().numpy(), rtol=1e-6)
    P_sh = np.concatenate(P_parts, axis=0)
    P_un = P_full.view(400, ds)[:, :n].cpu().numpy()
    np.testing.assert_allclose(P_sh, P_un, rtol=1e-4, atol=1e-5)
    np.testing.assert_allclose(P_sh.sum(0), 1.0, atol=1e-5)
    np.testing.assert_allclose(np.concatenate(rho_parts), rho_full.cpu().numpy(), rtol=1e-4, atol=1e-5)


@pytest.mark.parametrize("precision", [E.EMC_PREC_FP32, E.EMC_PREC_BF16])
@pytest.mark.parametrize("brick", [False, True])
def test_iterate_entry_point_equals_steps(gpu_lib, cfg1, precision, brick):
    import torch

    from gpu_helpers import geometry, pack, run_steps, upload_counts

    inp = cfg1
    q, quat = _inputs_f32(inp.q, inp.quat)
    geo = geometry(32, q, inp.mask, quat, inp.log_w, inp.wl.n_data, precision)
    if brick:
        geo.use_brick_scatter()
    K = pack(geo, upload_counts(inp.counts))
    steps = run_steps(geo, inp.model_start, K)
    ws = torch.empty(E.emc_workspace_bytes(geo), dtype=torch.uint8, device="cuda")
    m_in = torch.as_tensor(inp.model_start, dtype=torch.float32, device="cuda")
    m_out = torch.empty_like(m_in)
    ll = torch.empty(1, dtype=torch.float64, device="cuda")
    P = torch.empty(geo.n_rot * geo.data_stride, dtype=geo.p_dtype, device="cuda")
    E.emc_iterate(geo, m_in, K, m_out, ll, P_out=P, ws=ws)
    torch.cuda.synchronize()
    np.testing.assert_allclose(m_out.double().cpu().numpy(), steps["model"], rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(P.view(geo.n_rot, -1)[:, :geo.n_data].double().cpu().numpy(), steps["P"], atol=1e-6)
    assert abs(ll.item() - steps["loglik"]) <= 1e-9 * abs(steps["loglik"])


# ------------------------------------------------------------------------------- BF16 form
@pytest.mark.parametrize("start", ["random_smooth", "true_model"])
def test_bf16_config1_within_mixed_tolerance(gpu_lib, cfg1, start):
    from gpu_helpers import (geometry, pack, q_rel_err, rel_l2, run_steps, top1_agreement, top1_same_precision,
                             top1_strict, upload_counts)

    inp = cfg1
    model = inp.model_start if start == "random_smooth" else inp.model_true
    q, quat = _inputs_f32(inp.q, inp.quat)
    geo = geometry(32, q, inp.mask, quat, inp.log_w, inp.wl.n_data, E.EMC_PREC_BF16)
    K = pack(geo, upload_counts(inp.counts))
    g = run_steps(geo, model, K)
    o = _oracle(model, inp.counts, q, inp.mask, quat, inp.log_w, 32)
    _check_expand(g, o, inp.mask, 2e-4)           # hi + lo keeps ~16 significant bits of the row maximum
    errs = dict(Q=q_rel_err(g["Q"], o["Q"]), P=float(np.max(np.abs(g["P"] - o["P"]))),
                L=abs(g["loglik"] - o["loglik"]) / abs(o["loglik"]), model=rel_l2(g["model"], o["model"]),
                top1=top1_same_precision(g["P"], o["P"]), top1_tie_aware=top1_agreement(g["P"], o["P"]),
                top1_strict=top1_strict(g["P"], o["P"]))
    print(f"\n[bf16 {start}] errors vs FP64 oracle: {errs}")
    assert errs["model"] <= MIXED_MODEL_TOL, errs
    assert errs["top1"] >= MIXED_TOP1, errs
    assert g["P_pad_max"] == 0
    np.testing.assert_allclose(g["P"].sum(0), 1.0, atol=1e-2)


def test_bf16_ragged_within_mixed_tolerance(gpu_lib):
    from gpu_helpers import geometry, pack, rel_l2, run_steps, top1_same_precision, upload_counts

    t = tiny_problem(9, grid_n=24, n_pix=529, n_rot=300, n_data=333, photons=200.0)
    q, quat = _inputs_f32(t["q"], t["quat"])
    geo = geometry(24, q, t["mask"], quat, t["log_w"], 333, E.EMC_PREC_BF16)
    g = run_steps(geo, t["model"], pack(geo, upload_counts(t["counts"])))
    o = _oracle(t["model"], t["counts"], q, t["mask"], quat, t["log_w"], 24)
    assert rel_l2(g["model"], o["model"]) <= MIXED_MODEL_TOL
    assert top1_same_precision(g["P"], o["P"]) >= MIXED_TOP1


def test_bf16_pack_rejects_counts_above_256(gpu_lib):
    from gpu_helpers import geometry, upload_counts

    t = tiny_problem(10, grid_n=12, n_pix=64, n_rot=4, n_data=8)
    t["mask"][:] = 1
    counts = t["counts"].copy()
    counts[3, 5] = 257
    geo = geometry(12, t["q"], t["mask"], t["quat"], t["log_w"], 8, E.EMC_PREC_BF16)
    with pytest.raises(E.EmcError) as e:
        E.emc_pack_frames(geo, upload_counts(counts), E.frames_tensor(geo))
    assert e.value.status == E.EMC_ERR_RANGE
    counts[3, 5] = 256
    E.emc_pack_frames(geo, upload_counts(counts), E.frames_tensor(geo))   # 256 is exact
