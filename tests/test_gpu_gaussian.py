"""Gaussian noise model with fluence on the GPU (FP32 form) against the FP64 oracle.

Tolerances (the FP32 form's): responsibilities max-abs <= 1e-3; updated model,
fluence update and log-evidence relative error <= 1e-5 (the contraction runs in
FP32 MFMA on centred slices, everything after it in FP64)."""
import numpy as np
import pytest

from emc_inputs import tiny_problem
from oracle import gauss_oracle as GO
from paper_1409_4256_amd import emc as E

pytestmark = pytest.mark.gpu

P_TOL, REL_TOL = 1e-3, 1e-5


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _run_gpu(geo, model, K, sigma, phi_in=None):
    """One GPU iteration; phi_in None: fluence from the model (first iteration)."""
    import torch

    n, ds = geo.n_data, geo.data_stride
    phi = torch.ones(max(1, geo.n_rot * ds), dtype=torch.float32, device="cuda")
    if phi_in is not None:
        phi.view(geo.n_rot, ds)[:, :n] = torch.as_tensor(np.asarray(phi_in, np.float32), device="cuda")
    m_in = torch.as_tensor(np.asarray(model, np.float32), device="cuda")
    m_out = torch.empty_like(m_in)
    ll = torch.empty(1, dtype=torch.float64, device="cuda")
    P = torch.empty(max(1, geo.n_rot * ds), dtype=torch.float32, device="cuda")
    ws = torch.empty(E.emc_gaussian_workspace_bytes(geo), dtype=torch.uint8, device="cuda")
    E.emc_iterate_gaussian(geo, sigma, m_in, K, phi, phi_in is None, m_out, ll, P_out=P, ws=ws)
    torch.cuda.synchronize()
    return dict(model=m_out.double().cpu().numpy(), loglik=ll.item(),
                P=P[:geo.n_rot * ds].view(geo.n_rot, ds)[:, :n].double().cpu().numpy(),
                phi=phi[:geo.n_rot * ds].view(geo.n_rot, ds)[:, :n].double().cpu().numpy(),
                phi_pad=phi[:geo.n_rot * ds].view(geo.n_rot, ds)[:, n:].cpu().numpy())


def _check(g, o, tag):
    from gpu_helpers import rel_l2

    dP = np.max(np.abs(g["P"] - o["P"]))
    em = rel_l2(g["model"], o["model"])
    ephi = np.max(np.abs(g["phi"] - o["phi"]) / np.abs(o["phi"]))
    print(f"\n[gaussian {tag}] mean max_j P {o['P'].max(axis=0).mean():.3f}; "
          f"P max-abs {dP:.2e}, model rel L2 {em:.2e}, phi max rel {ephi:.2e}, "
          f"loglik {g['loglik']:.6f} (oracle {o['loglik']:.6f})")
    assert dP <= P_TOL, (tag, dP)
    assert em <= REL_TOL, (tag, em)
    assert ephi <= REL_TOL, (tag, ephi)
    assert abs(g["loglik"] - o["loglik"]) <= REL_TOL * abs(o["loglik"]), tag
    assert np.all(g["phi_pad"] == 1.0)


@pytest.mark.parametrize("seed,N,npx,nrot,ndata,sigma,brick", [
    (0, 20, 300, 200, 300, 1.0, False),
    (1, 16, 257, 129, 517, 2.0, False),      # ragged pixel and frame counts
    (2, 24, 400, 300, 200, 1.5, True),       # brick-major c-step
    (3, 20, 300, 200, 300, 8.0, False),      # broad posteriors (large sigma)
])
def test_two_iterations_match_oracle(gpu_lib, seed, N, npx, nrot, ndata, sigma, brick):
    from gpu_helpers import geometry, pack, upload_counts

    t = tiny_problem(seed, grid_n=N, n_pix=npx, n_rot=nrot, n_data=ndata, photons=200.0)
    q, quat = _f32(t["q"]), _f32(t["quat"])
    print(f"[gaussian] seed {seed} N {N} npx {npx} nrot {nrot} ndata {ndata} sigma {sigma} brick {brick}",
          flush=True)
    geo = geometry(N, q, t["mask"], quat, t["log_w"], ndata)
    if brick:
        geo.use_brick_scatter(chunk=64)
    K = pack(geo, upload_counts(t["counts"]))
    model = _f32(t["model"])
    # iteration 1: fluence from the model's own slices
    o1 = GO.iterate(model, t["counts"], q, t["mask"], quat, t["log_w"], N, sigma)
    g1 = _run_gpu(geo, model, K, sigma)
    _check(g1, o1, f"seed{seed} it1")
    # iteration 2 from the oracle's model and fluence (rounded to FP32 on both sides)
    m2, phi2 = _f32(o1["model"]), _f32(o1["phi"])
    o2 = GO.iterate(m2, t["counts"], q, t["mask"], quat, t["log_w"], N, sigma, phi=phi2)
    g2 = _run_gpu(geo, m2, K, sigma, phi_in=phi2)
    _check(g2, o2, f"seed{seed} it2")


def test_single_identity_rotation_closed_form_on_gpu(gpu_lib):
    """One identity rotation, detector on integer voxels: P = 1 and the touched voxels
    hold the fluence-corrected mean frame."""
    from gpu_helpers import geometry, pack, upload_counts

    N = 16
    u = np.arange(-4, 5)
    X, Y = np.meshgrid(u, u, indexing="ij")
    q = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    mask = np.ones(q.shape[0], np.uint8)
    mask[7] = 0
    rng = np.random.default_rng(3)
    K = rng.poisson(5.0, size=(37, q.shape[0])).astype(np.uint16)
    K[:, mask == 0] = 0
    phi = _f32(rng.uniform(0.5, 2.0, size=(1, 37)))
    geo = geometry(N, q, mask, np.array([[1.0, 0, 0, 0]]), np.array([0.0]), 37)
    g = _run_gpu(geo, np.ones(N ** 3), pack(geo, upload_counts(K)), 1.0, phi_in=phi)
    l = ((X.ravel() + 8) * N + (Y.ravel() + 8)) * N + 8
    v = mask.astype(bool)
    np.testing.assert_allclose(g["P"], 1.0)
    np.testing.assert_allclose(g["model"][l[v]], (K / phi[0][:, None]).mean(axis=0)[v], rtol=2e-6)


def test_bf16_form_is_refused(gpu_lib):
    import torch

    from gpu_helpers import geometry

    t = tiny_problem(4, grid_n=12, n_pix=50, n_rot=10, n_data=5)
    geo = geometry(12, t["q"], t["mask"], t["quat"], t["log_w"], 5, E.EMC_PREC_BF16)
    m = torch.ones(12 ** 3, dtype=torch.float32, device="cuda")
    ws = torch.empty(E.emc_gaussian_workspace_bytes(geo), dtype=torch.uint8, device="cuda")
    with pytest.raises(E.EmcError) as e:
        E.emc_iterate_gaussian(geo, 1.0, m, torch.zeros(E.emc_frames_bytes(geo), dtype=torch.uint8, device="cuda"),
                               torch.ones(10 * 256, device="cuda"), True, m.clone(),
                               torch.empty(1, dtype=torch.float64, device="cuda"), ws=ws)
    assert e.value.status == E.EMC_ERR_UNSUPPORTED
