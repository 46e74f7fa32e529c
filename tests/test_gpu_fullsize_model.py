"""The whole iteration's model update (eq. 2.4, 2.9, 2.11-2.12) at the full 128^3 grid
and all 25000 rotations of the 128x128-detector workload, on a 1000-frame share of its
frames (the FP64 oracle cannot hold 100000 frames at every rotation): the GPU's FP32 and
BF16 forms against the oracle's iteration, whose sums over rotations run a chunk of
rotations at a time in plain C (oracle/native.py).

Tolerances: FP32 form model relative L2 <= 1e-5 and mean log-evidence relative
<= 1e-6; BF16 form model relative L2 <= 1e-3."""
import numpy as np
import pytest

from emc_inputs import WORKLOADS, make_inputs, scaled

pytestmark = pytest.mark.gpu

N_FRAMES = 1000


@pytest.fixture(scope="module")
def problem(gpu_lib):
    import time

    import torch

    from oracle import native as ON

    wl = scaled(WORKLOADS[2], n_data=N_FRAMES)
    print(f"\n[fullsize model] inputs: 128^3, {wl.n_rot} rotations, {wl.n_data} frames", flush=True)
    inp = make_inputs(wl, device="cuda", with_truth=False)
    q = np.asarray(inp.q, np.float32).astype(np.float64)
    quat = np.asarray(inp.quat, np.float32).astype(np.float64)
    model = np.asarray(inp.model_start, np.float32).astype(np.float64)
    K = inp.counts.view(torch.int16).to(torch.int32).cpu().numpy()
    t0 = time.perf_counter()
    o = ON.iterate_chunked(model, K, q, inp.mask, quat, inp.log_w, wl.grid_n)
    print(f"[fullsize model] oracle iteration in {time.perf_counter() - t0:.1f} s", flush=True)
    return inp, o


@pytest.mark.parametrize("prec", [0, 1])
def test_model_update_at_full_rotation_count_matches_oracle(problem, gpu_lib, prec):
    import torch

    from gpu_helpers import rel_l2

    emc = gpu_lib
    inp, o = problem
    wl = inp.wl
    geo = emc.Geometry(wl.grid_n, torch.as_tensor(inp.q), torch.as_tensor(inp.mask), torch.as_tensor(inp.quat),
                       torch.as_tensor(inp.log_w), wl.n_data, prec)
    geo.use_brick_scatter()
    K = emc.frames_tensor(geo)
    emc.emc_pack_frames(geo, inp.counts, K)
    ws = torch.empty(emc.emc_workspace_bytes(geo), dtype=torch.uint8, device="cuda")
    m_in = torch.as_tensor(inp.model_start, dtype=torch.float32, device="cuda")
    m_out = torch.empty_like(m_in)
    ll = torch.empty(1, dtype=torch.float64, device="cuda")
    emc.emc_iterate(geo, m_in, K, m_out, ll, ws=ws)
    torch.cuda.synchronize()
    err = rel_l2(m_out.double().cpu().numpy(), o["model"])
    lerr = abs(ll.item() - o["loglik"]) / abs(o["loglik"])
    print(f"\n[fullsize model] {'bf16' if prec else 'fp32'}: model rel L2 vs oracle {err:.2e}, mean log-evidence "
          f"rel {lerr:.2e}", flush=True)
    if prec == 0:
        assert err <= 1e-5 and lerr <= 1e-6
    else:
        assert err <= 1e-3 and lerr <= 1e-4
