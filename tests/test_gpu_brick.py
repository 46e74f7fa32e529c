"""Brick-major c-step (eq. (2.12) with the loop nest turned round) on the GPU.

The plan's visit lists are index work: they must equal, brick by brick, the set
a brute-force CPU pass finds (every (rotation, 64-pixel group) whose used pixels
put a trilinear corner inside the brick).  The sums must equal the
rotation-major c-step's up to FP64 rounding order and the oracle's to the FP32
form's tolerance, also where corners leave the grid and bricks are partial."""
import numpy as np
import pytest

import oracle as O
from emc_inputs import tiny_problem
from paper_1409_4256_amd import emc as E

pytestmark = pytest.mark.gpu

B = 16


def _rot(quat):
    """Rotation matrices of unit-normalised quaternions (w, x, y, z), active."""
    w, x, y, z = (quat[:, k] for k in range(4))
    n = w * w + x * x + y * y + z * z
    s = 2.0 / n
    return np.stack([
        np.stack([1 - s * (y * y + z * z), s * (x * y - w * z), s * (x * z + w * y)], -1),
        np.stack([s * (x * y + w * z), 1 - s * (x * x + z * z), s * (y * z - w * x)], -1),
        np.stack([s * (x * z - w * y), s * (y * z + w * x), 1 - s * (x * x + y * y)], -1)], 1)


def _brute_visits(q, mask, quat, N):
    """{brick: sorted array of j * n_groups + t} by brute force over every pixel."""
    nb = -(-N // B)
    G = -(-len(q) // 64)
    used = np.flatnonzero(mask)
    R = _rot(quat)
    out = {}
    for j in range(len(quat)):
        p = q[used] @ R[j].T + 0.5 * N
        b = np.floor(p).astype(np.int64)
        for d in range(8):
            c = b + np.array([d >> 2, (d >> 1) & 1, d & 1])
            ok = np.all((c >= 0) & (c < N), axis=1)
            cb = c[ok] // B
            bricks = (cb[:, 0] * nb + cb[:, 1]) * nb + cb[:, 2]
            for br, t in set(zip(bricks.tolist(), (used[ok] // 64).tolist())):
                out.setdefault(br, set()).add(j * G + t)
    return {k: np.array(sorted(v)) for k, v in out.items()}


def _plan_lists(geo, plan):
    """{brick: sorted visits} and the items, read back from the plan's buffer."""
    import torch

    buf = geo.scatter_buf
    base = buf.data_ptr()
    vis = buf[plan.visits - base:plan.visits - base + 4 * plan.n_visits].view(torch.int32).cpu().numpy()
    items = buf[plan.items - base:plan.items - base + 16 * plan.n_items].view(torch.int32).cpu().numpy()
    items = items.reshape(-1, 4)
    lists = {}
    for br, a, z, _ in items:
        lists.setdefault(int(br), []).append(vis[a:z])
    return {k: np.sort(np.concatenate(v)) for k, v in lists.items()}, items


@pytest.mark.parametrize("seed,N,npx,nrot,qr,chunk", [
    (0, 40, 700, 60, None, 0),      # partial bricks (40 = 2 * 16 + 8), groups spread over the ball
    (1, 24, 300, 90, 30.0, 64),     # pixels beyond the grid: corners clipped, some groups reach nothing
    (2, 16, 130, 40, 2.5, 64),      # compact groups, a single brick, ragged last group
])
def test_plan_lists_equal_brute_force(gpu_lib, seed, N, npx, nrot, qr, chunk):
    from gpu_helpers import geometry

    t = tiny_problem(seed, grid_n=N, n_pix=npx, n_rot=nrot, n_data=1, q_radius=qr)
    q = np.asarray(t["q"], np.float32).astype(np.float64)
    quat = np.asarray(t["quat"], np.float32).astype(np.float64)
    geo = geometry(N, q, t["mask"], quat, t["log_w"], 1)
    plan = geo.use_brick_scatter(chunk=chunk)
    print(f"[brick plan] seed {seed} N {N} npx {npx} nrot {nrot} visits {plan.n_visits} items {plan.n_items}",
          flush=True)
    got, items = _plan_lists(geo, plan)
    ref = _brute_visits(q, t["mask"], quat, N)
    assert sorted(got) == sorted(ref)
    for k in ref:
        np.testing.assert_array_equal(got[k], ref[k])
    assert plan.n_visits == sum(len(v) for v in ref.values())
    # items tile [0, n_visits) without overlap, at most `chunk` visits each
    spans = sorted((int(a), int(z)) for _, a, z, _ in items)
    assert spans[0][0] == 0 and spans[-1][1] == plan.n_visits
    assert all(s[1] == n[0] for s, n in zip(spans[:-1], spans[1:]))
    assert all(0 < z - a <= plan.chunk for a, z in spans)
    assert plan.chunk == (chunk or 2048)
    assert plan.n_bricks == (-(-N // B)) ** 3


@pytest.mark.parametrize("seed,N,npx,nrot,ndata,qr", [(3, 40, 600, 120, 150, None), (4, 24, 300, 90, 80, 30.0)])
def test_brick_sums_equal_rotation_major(gpu_lib, seed, N, npx, nrot, ndata, qr):
    """Same num/den as the rotation-major c-step (FP64, summation order aside) and
    the oracle's; qr = 30 puts pixels beyond the grid (clipped corners)."""
    from gpu_helpers import geometry, pack, rel_l2, run_steps, upload_counts

    t = tiny_problem(seed, grid_n=N, n_pix=npx, n_rot=nrot, n_data=ndata, photons=200.0, q_radius=qr)
    q = np.asarray(t["q"], np.float32).astype(np.float64)
    quat = np.asarray(t["quat"], np.float32).astype(np.float64)
    print(f"[brick sums] seed {seed} N {N} npx {npx} nrot {nrot} ndata {ndata}", flush=True)
    geo = geometry(N, q, t["mask"], quat, t["log_w"], ndata)
    K = pack(geo, upload_counts(t["counts"]))
    rot = run_steps(geo, t["model"], K, grid_copies=False)
    geo_b = geometry(N, q, t["mask"], quat, t["log_w"], ndata)
    geo_b.use_brick_scatter(chunk=64)
    brk = run_steps(geo_b, t["model"], pack(geo_b, upload_counts(t["counts"])))
    for k in ("num", "den"):
        assert rel_l2(brk[k], rot[k]) <= 1e-12, (k, rel_l2(brk[k], rot[k]))
    np.testing.assert_array_equal(brk["den"] == 0, rot["den"] == 0)
    o = O.iterate(np.asarray(t["model"], np.float32).astype(np.float64), t["counts"], q, t["mask"], quat,
                  t["log_w"], N)
    assert rel_l2(brk["num"], o["num"]) <= 1e-5 and rel_l2(brk["den"], o["den"]) <= 1e-5
    assert rel_l2(brk["model"], o["model"]) <= 1e-5


def test_plan_of_another_geometry_is_refused(gpu_lib):
    import torch

    from gpu_helpers import geometry

    t = tiny_problem(5, grid_n=20, n_pix=200, n_rot=30, n_data=10)
    geo = geometry(20, t["q"], t["mask"], t["quat"], t["log_w"], 0)
    geo.use_brick_scatter()
    other = geometry(20, t["q"], t["mask"], t["quat"], t["log_w"], 0)   # same values, other buffers
    other.pb.scatter = geo.pb.scatter
    num = torch.empty(20 ** 3, dtype=torch.float64, device="cuda")
    den = torch.empty_like(num)
    E.emc_compress(geo, None, None, None, None, num, den)               # its own geometry: accepted
    with pytest.raises(E.EmcError) as e:
        E.emc_compress(other, None, None, None, None, num, den)
    assert e.value.status == E.EMC_ERR_INVALID_ARG and "another geometry" in e.value.message
