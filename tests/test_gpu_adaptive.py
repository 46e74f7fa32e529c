"""Adaptive EMC on 600-cell rotation sets (Section 3.4, eq. (2.7), eq. (3.1)) on the GPU.

* One iteration on the refinement-2 set (420 rotations, prior weights that are
  not uniform) matches the FP64 oracle to the FP32 form's tolerances.
* The driver follows eq. (3.1) step by step: every change of d is the rule's
  answer to the two log-evidences before it, and each iteration runs on the
  Mrot(d) rotations of its level.
"""
import numpy as np
import pytest

import oracle as O
from emc_inputs import WORKLOADS, make_inputs, tiny_problem
from paper_1409_4256_amd import emc as E
from paper_1409_4256_amd import rotations as R

pytestmark = pytest.mark.gpu


def test_600cell_set_iteration_matches_oracle(gpu_lib):
    from gpu_helpers import geometry, pack, rel_l2, run_steps, upload_counts

    t = tiny_problem(21, grid_n=20, n_pix=300, n_rot=1, n_data=300, photons=200.0)
    quat, log_w = R.rotation_set(2)
    q = np.asarray(t["q"], np.float32).astype(np.float64)
    quat32 = np.asarray(quat, np.float32).astype(np.float64)
    print(f"[adaptive] oracle parity on the d = 2 set ({len(quat)} rotations)", flush=True)
    geo = geometry(20, q, t["mask"], quat32, log_w, 300)
    geo.use_brick_scatter()
    g = run_steps(geo, t["model"], pack(geo, upload_counts(t["counts"])))
    o = O.iterate(np.asarray(t["model"], np.float32).astype(np.float64), t["counts"], q, t["mask"], quat32, log_w, 20)
    assert np.max(np.abs(g["P"] - o["P"])) <= 1e-3
    assert rel_l2(g["model"], o["model"]) <= 1e-5
    assert abs(g["loglik"] - o["loglik"]) <= 1e-6 * abs(o["loglik"])


@pytest.fixture(scope="module")
def small_inputs(gpu_lib):
    print("[adaptive] inputs: 32^3 grid, 32x32 detector, 1000 frames", flush=True)
    return make_inputs(WORKLOADS[1], device="cuda", with_truth=False)


@pytest.mark.parametrize("tol,d_start,d_max", [(0.05, 2, 4), (1e9, 1, 3)])
def test_driver_follows_the_refinement_rule(gpu_lib, small_inputs, tol, d_start, d_max):
    import torch

    from paper_1409_4256_amd.adaptive import AdaptiveEMC

    inp = small_inputs
    counts = inp.counts if isinstance(inp.counts, torch.Tensor) else torch.as_tensor(inp.counts)
    run = AdaptiveEMC(32, inp.q, inp.mask, counts.cuda(), d_start, d_max, precision=E.EMC_PREC_FP32, tol=tol)
    model = torch.as_tensor(inp.model_start, dtype=torch.float32, device="cuda")
    out = run.run(model, 8)
    h = run.history
    print("\n[adaptive] " + "; ".join(f"it {i}: d {d} ({n} rot) L {L:.3f} {ms:.1f} ms" for i, d, n, L, ms, _ in h))
    assert len(h) == 8 and torch.isfinite(out).all().item()
    d, L_prev = d_start, None
    for i, d_i, n_i, L_i, _, _ in h:
        assert d_i == d and n_i == R.mrot(d)
        assert np.isfinite(L_i)
        d = R.next_refinement(L_prev, L_i, d, d_max, tol)
        L_prev = L_i
    if tol > 1.0:   # the rule fires from the second iteration on: one level per iteration up to d_max
        assert [x[1] for x in h] == [1, 1, 2, 3, 3, 3, 3, 3]
