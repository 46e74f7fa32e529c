"""Plain FP64 reference of the learned orientation proposal -- test infrastructure only.

The proposal network reads a frame and scores the cells of a coarse rotation
grid; it is trained on the responsibilities of full EMC iterations (summed
over the fine rotations of each cell) and only narrows the E-step's search,
whose full form stays the fallback and the measure of recall.  The paper has no
such network: this oracle fixes the network the GPU path implements.

Network (NCHW, float64 here):
  x = log(1 + 2x2-binned frame), 1 x 64 x 64 (masked pixels contribute 0)
  4 x [conv 3x3, stride 2, zero padding 1, bias, ReLU]: 1->32->64->128->128
      channels, 64^2 -> 32^2 -> 16^2 -> 8^2 -> 4^2
  flatten (c, y, x) -> 2048 -> linear -> n_cells logits
Loss: soft-target cross entropy, -(1/B) sum_k sum_c T_kc log softmax(z_k)_c.
Optimiser: Adam (bias-corrected moments).

parity pinned: tests/test_cnn_oracle_pins.py (torch conv2d, central finite
differences, closed-form softmax gradient, torch Adam).
"""
from __future__ import annotations

import numpy as np

CHANNELS = (1, 32, 64, 128, 128)
IMAGE = 64


def init_params(rng: np.random.Generator, n_cells: int):
    """He-normal weights, zero biases.  Returns a dict of float64 arrays."""
    p = {}
    for l in range(4):
        ci, co = CHANNELS[l], CHANNELS[l + 1]
        p[f"w{l}"] = rng.standard_normal((co, ci, 3, 3)) * np.sqrt(2.0 / (ci * 9))
        p[f"b{l}"] = np.zeros(co)
    fan = CHANNELS[-1] * (IMAGE // 16) ** 2
    p["wf"] = rng.standard_normal((n_cells, fan)) * np.sqrt(2.0 / fan)
    p["bf"] = np.zeros(n_cells)
    return p


def bin_log(counts: np.ndarray, bin_index: np.ndarray) -> np.ndarray:
    """x[k] = log1p of the per-bin sums of frame k; bin_index[i] in [0, 64*64) or -1."""
    K = np.asarray(counts, dtype=np.float64)
    x = np.zeros((K.shape[0], IMAGE * IMAGE))
    use = bin_index >= 0
    for k in range(K.shape[0]):
        x[k] = np.bincount(bin_index[use], weights=K[k, use], minlength=IMAGE * IMAGE)
    return np.log1p(x).reshape(-1, 1, IMAGE, IMAGE)


def conv_forward(x, w, b):
    """out[n, o, y, x] = b[o] + sum_{c, dy, dx} w[o, c, dy, dx] xp[n, c, 2y + dy, 2x + dx],
    xp = x zero-padded by one on each side."""
    n, c, h, _ = x.shape
    oh = h // 2
    xp = np.zeros((n, c, h + 2, h + 2))
    xp[:, :, 1:-1, 1:-1] = x
    out = np.zeros((n, w.shape[0], oh, oh)) + b[None, :, None, None]
    for dy in range(3):
        for dx in range(3):
            patch = xp[:, :, dy:dy + 2 * oh:2, dx:dx + 2 * oh:2]          # [n, c, oh, oh]
            out += np.einsum("ncyx,oc->noyx", patch, w[:, :, dy, dx])
    return out


def conv_backward(x, w, dout):
    """Gradients of conv_forward: (dx, dw, db)."""
    n, c, h, _ = x.shape
    oh = h // 2
    xp = np.zeros((n, c, h + 2, h + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for dy in range(3):
        for dx in range(3):
            patch = xp[:, :, dy:dy + 2 * oh:2, dx:dx + 2 * oh:2]
            dw[:, :, dy, dx] = np.einsum("noyx,ncyx->oc", dout, patch)
            dxp[:, :, dy:dy + 2 * oh:2, dx:dx + 2 * oh:2] += np.einsum("noyx,oc->ncyx", dout, w[:, :, dy, dx])
    return dxp[:, :, 1:-1, 1:-1], dw, dout.sum(axis=(0, 2, 3))


def forward(p, x):
    """Returns (logits [B][n_cells], cache for backward)."""
    acts = [x]
    h = x
    for l in range(4):
        h = np.maximum(conv_forward(h, p[f"w{l}"], p[f"b{l}"]), 0.0)
        acts.append(h)
    flat = h.reshape(h.shape[0], -1)
    z = flat @ p["wf"].T + p["bf"]
    return z, acts


def log_softmax(z):
    m = z.max(axis=1, keepdims=True)
    return z - m - np.log(np.exp(z - m).sum(axis=1, keepdims=True))


def loss(z, T):
    return float(-(T * log_softmax(z)).sum() / z.shape[0])


def backward(p, acts, z, T):
    """Gradients of loss(forward(p, x), T) with respect to every parameter."""
    B = z.shape[0]
    sm = np.exp(log_softmax(z))
    dz = (sm * T.sum(axis=1, keepdims=True) - T) / B
    h = acts[-1]
    flat = h.reshape(B, -1)
    g = {"wf": dz.T @ flat, "bf": dz.sum(axis=0)}
    dh = (dz @ p["wf"]).reshape(h.shape)
    for l in range(3, -1, -1):
        dh = dh * (acts[l + 1] > 0)                       # ReLU
        dx, g[f"w{l}"], g[f"b{l}"] = conv_backward(acts[l], p[f"w{l}"], dh)
        dh = dx
    return g


def adam_step(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update; `state` holds t and the first and second moments."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m *= b1
        m += (1 - b1) * g[k]
        v *= b2
        v += (1 - b2) * g[k] * g[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] -= lr * mh / (np.sqrt(vh) + eps)


def cell_targets(P: np.ndarray, cell_of: np.ndarray, n_cells: int) -> np.ndarray:
    """T[k][c] = sum over fine rotations j of cell c of P[j][k]."""
    T = np.zeros((P.shape[1], n_cells))
    np.add.at(T.T, cell_of, P)
    return T


def assign_cells(quat: np.ndarray, coarse: np.ndarray) -> np.ndarray:
    """Coarse cell of each fine rotation: the coarse quaternion of largest |<q, q_c>|
    (q and -q are the same rotation); the lowest index wins ties."""
    qn = quat / np.linalg.norm(quat, axis=1, keepdims=True)
    cn = coarse / np.linalg.norm(coarse, axis=1, keepdims=True)
    return np.argmax(np.abs(qn @ cn.T), axis=1)


def topk_cells(z: np.ndarray, k: int) -> np.ndarray:
    """Indices of the k largest logits of each row, largest first; ties -> lower index."""
    order = np.argsort(-z, axis=1, kind="stable")
    return order[:, :k]
