"""emc_iterate_noalloc (the library's static device buffer as workspace) against
emc_iterate with a caller workspace: same problem, same inputs, two calls in a
row on one GPU, the second with a smaller problem (grid, pixels, rotations and
frames all smaller), both precisions and both c-step forms.

The two entry points run the same kernels; only the c-step's FP64 atomics may
add in another order, so the models agree to far below the FP32 form's model
tolerance (relative L2 1e-5) and the responsibilities are identical."""
import numpy as np
import pytest

from emc_inputs import tiny_problem

pytestmark = pytest.mark.gpu

CASES = [  # (seed, grid_n, n_pix, n_rot, n_data): the second call is smaller in every size
    (31, 24, 529, 300, 333),
    (32, 16, 130, 90, 70),
]


def _run(emc, t, prec, brick, noalloc):
    import torch

    dev = "cuda"
    n_data = t["counts"].shape[0]
    geo = emc.Geometry(t["grid_n"], torch.as_tensor(t["q"]), torch.as_tensor(t["mask"]),
                       torch.as_tensor(t["quat"]), torch.as_tensor(t["log_w"]), n_data, prec)
    if brick:
        geo.use_brick_scatter()
    K = emc.frames_tensor(geo)
    emc.emc_pack_frames(geo, torch.from_numpy(t["counts"]).to(dev), K)
    m_in = torch.as_tensor(t["model"], dtype=torch.float32, device=dev)
    m_out = torch.full_like(m_in, float("nan"))
    ll = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    P = torch.full((geo.n_rot * geo.data_stride,), float("nan"), dtype=geo.p_dtype, device=dev)
    if noalloc:
        emc.emc_iterate_noalloc(geo, m_in, K, m_out, ll, P_out=P)
    else:
        ws = torch.empty(emc.emc_workspace_bytes(geo), dtype=torch.uint8, device=dev)
        emc.emc_iterate(geo, m_in, K, m_out, ll, P_out=P, ws=ws)
    torch.cuda.synchronize()
    return (m_out.double().cpu().numpy(), ll.item(),
            P.view(geo.n_rot, geo.data_stride)[:, :n_data].double().cpu().numpy())


@pytest.mark.parametrize("brick", [False, True])
@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_equals_iterate_on_two_calls(gpu_lib, prec, brick):
    emc = gpu_lib
    for seed, n, npix, nrot, nd in CASES:
        print(f"[noalloc] prec {prec} brick {brick} case {seed}: N={n} n_pix={npix} n_rot={nrot} n_data={nd}",
              flush=True)
        t = tiny_problem(seed, grid_n=n, n_pix=npix, n_rot=nrot, n_data=nd, photons=200.0)
        m_ref, ll_ref, P_ref = _run(emc, t, prec, brick, noalloc=False)
        m, ll, P = _run(emc, t, prec, brick, noalloc=True)
        assert np.all(np.isfinite(m)) and np.isfinite(ll) and np.all(np.isfinite(P))
        err = np.linalg.norm(m - m_ref) / np.linalg.norm(m_ref)
        print(f"[noalloc]   model rel L2 {err:.2e}, loglik {ll:.9f} vs {ll_ref:.9f}, "
              f"P max-abs {np.max(np.abs(P - P_ref)):.1e}", flush=True)
        assert err <= 1e-7
        assert abs(ll - ll_ref) <= 1e-12 * abs(ll_ref)
        np.testing.assert_array_equal(P, P_ref)
