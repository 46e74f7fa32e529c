"""Pins of the proposal-network oracle against library routines and finite differences."""
import numpy as np
import pytest
import torch

from oracle import cnn_oracle as C


def _small_params(rng, n_cells=7):
    p = C.init_params(rng, n_cells)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.1
    return p


def test_conv_forward_matches_torch_conv2d():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 5, 16, 16))
    w = rng.standard_normal((4, 5, 3, 3))
    b = rng.standard_normal(4)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b),
                                     stride=2, padding=1).numpy()
    np.testing.assert_allclose(C.conv_forward(x, w, b), ref, rtol=1e-12, atol=1e-12)


def test_conv_backward_matches_torch_autograd():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 3, 8, 8))
    w = rng.standard_normal((5, 3, 3, 3))
    b = rng.standard_normal(5)
    dout = rng.standard_normal((2, 5, 4, 4))
    xt, wt, bt = (torch.from_numpy(a).requires_grad_() for a in (x, w, b))
    torch.nn.functional.conv2d(xt, wt, bt, stride=2, padding=1).backward(torch.from_numpy(dout))
    dx, dw, db = C.conv_backward(x, w, dout)
    np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(dw, wt.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_network_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    p = _small_params(rng)
    x = np.abs(rng.standard_normal((2, 1, 64, 64)))
    T = rng.dirichlet(np.ones(7), size=2)
    z, acts = C.forward(p, x)
    g = C.backward(p, acts, z, T)
    h = 1e-6
    for key in ("w0", "b0", "w2", "b3", "wf", "bf"):
        flat = p[key].reshape(-1)
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = C.loss(C.forward(p, x)[0], T)
            flat[idx] = old - h
            lm = C.loss(C.forward(p, x)[0], T)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[key].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (key, idx, fd, an)


def test_softmax_cross_entropy_gradient_closed_form():
    rng = np.random.default_rng(4)
    z = rng.standard_normal((3, 6))
    T = rng.dirichlet(np.ones(6), size=3)
    zt = torch.from_numpy(z).requires_grad_()
    (-(torch.from_numpy(T) * torch.log_softmax(zt, 1)).sum() / 3).backward()
    sm = np.exp(C.log_softmax(z))
    np.testing.assert_allclose(zt.grad.numpy(), (sm - T) / 3, rtol=1e-12)


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    p = {"a": rng.standard_normal((3, 4)), "b": rng.standard_normal(5)}
    pt = [torch.from_numpy(p[k].copy()).requires_grad_() for k in ("a", "b")]
    opt = torch.optim.Adam(pt, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    state = {}
    for step in range(3):
        g = {"a": rng.standard_normal((3, 4)), "b": rng.standard_normal(5)}
        for t, k in zip(pt, ("a", "b")):
            t.grad = torch.from_numpy(g[k].copy())
        opt.step()
        C.adam_step(p, g, state, lr=1e-2)
    np.testing.assert_allclose(p["a"], pt[0].detach().numpy(), rtol=1e-12)
    np.testing.assert_allclose(p["b"], pt[1].detach().numpy(), rtol=1e-12)


def test_bin_log_sums_two_by_two_blocks():
    from emc_inputs import WORKLOADS, detector_mask, pixel_order, proposal_bins

    wl = WORKLOADS[2]
    rng = np.random.default_rng(6)
    order = pixel_order(wl.det_n)
    mask = detector_mask(wl)
    img = rng.poisson(0.5, size=(2, wl.det_n, wl.det_n)).astype(np.float64)     # row-major detector
    counts = img.reshape(2, -1)[:, order] * mask[None, :]
    x = C.bin_log(counts, proposal_bins(wl.det_n, mask))
    m2 = np.zeros(wl.det_n * wl.det_n)
    m2[order] = mask
    ref = (img * m2.reshape(wl.det_n, wl.det_n)).reshape(2, 64, 2, 64, 2).sum(axis=(2, 4))
    np.testing.assert_allclose(x[:, 0], np.log1p(ref), rtol=1e-14)


def test_cell_targets_and_assignment():
    rng = np.random.default_rng(7)
    P = rng.dirichlet(np.ones(10), size=4).T          # [j][k]
    cell_of = np.array([0, 2, 2, 1, 0, 1, 1, 2, 0, 0])
    T = C.cell_targets(P, cell_of, 3)
    np.testing.assert_allclose(T.sum(1), 1.0)
    np.testing.assert_allclose(T[:, 2], P[[1, 2, 7]].sum(0))
    q = np.array([[1.0, 0, 0, 0], [0, 1.0, 0, 0]])
    coarse = np.array([[0, -1.0, 0, 0], [0.9, 0.1, 0, 0]])
    assert list(C.assign_cells(q, coarse)) == [1, 0]   # -q is the same rotation


def test_topk_ties_prefer_lower_index():
    z = np.array([[1.0, 3.0, 3.0, 0.5, 3.0]])
    assert list(C.topk_cells(z, 3)[0]) == [1, 2, 4]


def test_topk_equals_repeated_selection():
    # an independent definition: k rounds of "the largest remaining value, the lowest
    # index among equals", on rows with many ties (values drawn from a few levels)
    g = np.random.default_rng(8)
    z = g.integers(0, 6, size=(40, 30)).astype(np.float64) + 0.25 * (g.random((40, 30)) < 0.1)
    k = 9
    got = C.topk_cells(z, k)
    for r in range(z.shape[0]):
        left, ref = list(range(z.shape[1])), []
        for _ in range(k):
            best = left[0]
            for c in left[1:]:
                if z[r, c] > z[r, best]:
                    best = c
            ref.append(best)
            left.remove(best)
        assert list(got[r]) == ref
