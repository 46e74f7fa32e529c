"""Seeded synthetic inputs for the EMC iteration.

This module builds the problem statement the method starts from (photon-count
frames, detector pixel coordinates and mask, a rotation set with prior weights,
a starting model), with the shapes and statistics of the paper's workloads
(binned 64x64 / 128x128 detectors with a grid of Mpix^{3/2} voxels, sparse
Poisson photon counts; Section 4.1, Table 4.1).  It serves both the FP64
oracle and the GPU path and deliberately holds none of the method's
arithmetic: no interpolation, no likelihood, no normalisation, no
compression.  Patterns are sampled from the exact structure factor of a
random arrangement of Gaussian atoms evaluated at the rotated pixel
coordinates, never from the grid.

Randomness: ``numpy.random.Generator(PCG64(SeedSequence([1409, cfg, stream])))``
with one stream per purpose (see ``STREAMS``); Poisson photon sampling uses a
torch generator seeded from stream 3 (so large workloads can be drawn on the
device the data will live on).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

STREAMS = {
    "atoms": 0,
    "rotations": 1,
    "orientations": 2,
    "photons": 3,
    "mask": 4,
    "start": 5,
    "coarse": 6,
    "audit": 7,
    "cnn": 8,
}

ATOM_SIGMA_NM = 0.1  # Gaussian atoms of width 1 Angstrom


def rng(cfg: int, stream: str) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([1409, cfg, STREAMS[stream]])))


@dataclasses.dataclass(frozen=True)
class Workload:
    """Sizes and physics of one synthetic workload (lengths in nm, px/D in m)."""

    cfg: int
    name: str
    grid_n: int          # N: model is N^3 voxels
    det_n: int           # detector is det_n x det_n pixels
    n_rot: int           # Mrot: rotations in this share
    n_data: int          # Mdata: frames
    photons: float       # mean photons per frame
    n_atoms: int
    radius_nm: float
    mask: str            # "center3" | "random5"
    n_iter: int = 1
    px_m: float = 600e-6
    dist_m: float = 0.1
    lam_nm: float = 1.0
    pool: int = 4096     # distinct true orientations the frames are drawn from

    @property
    def n_pix(self) -> int:
        return self.det_n * self.det_n


WORKLOADS = {
    # 32^3 grid, 32x32 detector, 1000 rotations, 1000 frames at ~500 photons
    1: Workload(1, "emc32_r1000_d1000", 32, 32, 1000, 1000, 500.0, 200, 2.0, "center3", 1, pool=1000),
    # one GPU's share at 128^3: 128x128 detector, 25000 rotations, 100000 frames at ~2000 photons
    2: Workload(2, "emc128_r25000_d100000", 128, 128, 25000, 100000, 2000.0, 2000, 6.0, "random5", 5),
    # 160^3, 100000 rotations, 500000 frames at ~1000 photons (streamed in 50000-frame chunks)
    5: Workload(5, "emc160_r100000_d500000", 160, 128, 100000, 500000, 1000.0, 3000,
                6.0 * 1.5 ** (1.0 / 3.0), "random5", 10),
}


def scaled(base: Workload, **kw) -> Workload:
    """A smaller workload with the same physics (for tests that must finish fast)."""
    return dataclasses.replace(base, **kw)


# ----------------------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------------------
TILE = 8


def pixel_order(n: int, tile: int = TILE) -> np.ndarray:
    """Order of the detector's pixels in the pixel list: tile x tile blocks, blocks
    row-major, pixels row-major inside a block (partial blocks at the edges).
    Entry p is the row-major index u*n + v of list position p.  Spatially compact
    groups of 64 consecutive pixels let the compression accumulate locally."""
    out = []
    for tu in range(0, n, tile):
        for tv in range(0, n, tile):
            for u in range(tu, min(tu + tile, n)):
                for v in range(tv, min(tv + tile, n)):
                    out.append(u * n + v)
    return np.asarray(out, dtype=np.int64)


def proposal_bins(n: int, mask: np.ndarray, image: int = 64) -> np.ndarray:
    """Bin of each listed pixel in the proposal network's image (image x image,
    row-major), -1 for masked pixels; the detector is reduced by n // image
    along each axis (2 x 2 sum-binning for a 128 x 128 detector)."""
    f = max(1, n // image)
    order = pixel_order(n)
    u, v = order // n, order % n
    b = (u // f) * image + (v // f)
    b = np.where((u // f < image) & (v // f < image), b, -1)
    return np.where(np.asarray(mask) > 0, b, -1).astype(np.int32)


def detector_q(wl: Workload):
    """Pixel scattering vectors on the Ewald sphere, in voxel units.

    Pixel (u, v) sits at x = (u - n/2) px, y = (v - n/2) px at distance D; its
    scattering vector is q = (x/r, y/r, D/r - 1)/lambda with r = |(x, y, D)|, so
    |q| = 2 sin(theta)/lambda.  The voxel spacing puts the detector corner at
    N/2 - 2 voxels, so every rotated pixel keeps two voxels of margin.
    Returns (q_vox [n_pix][3] float64 in pixel_order, dq_per_voxel_nm^-1).
    """
    n = wl.det_n
    x = (np.arange(n) - n / 2) * wl.px_m
    X, Y = np.meshgrid(x, x, indexing="ij")
    r = np.sqrt(X * X + Y * Y + wl.dist_m ** 2)
    q = np.stack([X / r, Y / r, wl.dist_m / r - 1.0], axis=-1) / wl.lam_nm
    q = q.reshape(-1, 3)[pixel_order(n)]
    dq = float(np.linalg.norm(q, axis=1).max() / (wl.grid_n / 2 - 2))
    return q / dq, dq


def detector_mask(wl: Workload) -> np.ndarray:
    """1 = pixel used, 0 = missing/saturated pixel (in pixel-list order)."""
    n = wl.det_n
    m = np.ones((n, n), dtype=np.uint8)
    if wl.mask == "center3":
        c = n // 2
        m[c - 1:c + 2, c - 1:c + 2] = 0
    elif wl.mask == "random5":
        k = int(round(0.05 * n * n))
        off = rng(wl.cfg, "mask").choice(n * n, size=k, replace=False)
        m.reshape(-1)[off] = 0
    elif wl.mask != "none":
        raise ValueError(wl.mask)
    return m.reshape(-1)[pixel_order(n)]


def shoemake_quaternions(g: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random unit quaternions (w, x, y, z) by Shoemake's subgroup method."""
    u1, u2, u3 = g.random(n), g.random(n), g.random(n)
    a, b = np.sqrt(u1), np.sqrt(1.0 - u1)
    return np.stack([a * np.cos(2 * np.pi * u3), b * np.sin(2 * np.pi * u2),
                     b * np.cos(2 * np.pi * u2), a * np.sin(2 * np.pi * u3)], axis=1)


def rotation_set(wl: Workload):
    """Method rotation set: Shoemake quaternions with equal prior weights 1/Mrot."""
    quat = shoemake_quaternions(rng(wl.cfg, "rotations"), wl.n_rot)
    log_w = np.full(wl.n_rot, -math.log(wl.n_rot))
    return quat, log_w


def atoms(wl: Workload) -> np.ndarray:
    """Atom centres uniform in a ball of the workload's radius (nm)."""
    g = rng(wl.cfg, "atoms")
    d = g.standard_normal((wl.n_atoms, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = wl.radius_nm * g.random(wl.n_atoms) ** (1.0 / 3.0)
    return d * r[:, None]


# ----------------------------------------------------------------------------------------
# diffraction physics (exact structure factor; no grid interpolation)
# ----------------------------------------------------------------------------------------
def _intensity_torch(qphys, atom_pos, device, chunk=1 << 16):
    """|F(q)|^2 exp(-4 pi^2 sigma^2 |q|^2) of Gaussian atoms, q in nm^-1, [n][3] -> [n]."""
    import torch

    qt = torch.as_tensor(qphys, dtype=torch.float64, device=device)
    at = torch.as_tensor(atom_pos, dtype=torch.float64, device=device).T.contiguous()
    out = torch.empty(qt.shape[0], dtype=torch.float64, device=device)
    for s in range(0, qt.shape[0], chunk):
        ph = (2.0 * math.pi) * (qt[s:s + chunk] @ at)
        re = torch.cos(ph).sum(dim=1)
        im = torch.sin(ph).sum(dim=1)
        q2 = (qt[s:s + chunk] ** 2).sum(dim=1)
        out[s:s + chunk] = (re * re + im * im) * torch.exp(-4.0 * math.pi ** 2 * ATOM_SIGMA_NM ** 2 * q2)
    return out


def true_orientations(wl: Workload, n: int) -> np.ndarray:
    """Rotation matrices of the frames' true orientations (continuous, uniform)."""
    from scipy.spatial.transform import Rotation

    return Rotation.random(n, random_state=rng(wl.cfg, "orientations")).as_matrix()


@dataclasses.dataclass
class Inputs:
    wl: Workload
    q: np.ndarray            # [n_pix][3] float64 voxel units
    mask: np.ndarray         # [n_pix] uint8
    quat: np.ndarray         # [n_rot][4] float64 (w, x, y, z)
    log_w: np.ndarray        # [n_rot] float64
    counts: object           # [n_data][n_pix] uint16 (numpy, or torch tensor on `device`)
    model_start: np.ndarray  # [N^3] float64, random-smooth start
    model_true: Optional[np.ndarray]  # [N^3] float64 scaled intensity on the grid (small grids only)
    alpha: float
    truth_index: np.ndarray  # [n_data] int: pool orientation of each frame


def make_inputs(wl: Workload, device: str = "cpu", with_truth: bool = True) -> Inputs:
    """Build every input of workload `wl`.  Heavy physics runs on `device` (torch)."""
    import torch
    from scipy.ndimage import gaussian_filter

    q_vox, dq = detector_q(wl)
    mask = detector_mask(wl)
    quat, log_w = rotation_set(wl)
    apos = atoms(wl)
    valid = np.flatnonzero(mask)

    pool = min(wl.pool, wl.n_data)
    Rt = true_orientations(wl, pool)
    # physical scattering vectors of the rotated valid pixels for every pool orientation
    qp = q_vox[valid] * dq                                   # [nv][3]
    rot_q = np.einsum("tab,ib->tia", Rt, qp).reshape(-1, 3)   # [pool*nv][3]
    inten = _intensity_torch(rot_q, apos, device).reshape(pool, valid.size)
    alpha = wl.photons / float(inten.sum(dim=1).mean())
    lam_pool = (alpha * inten).to(torch.float32)

    g_idx = rng(wl.cfg, "orientations")
    g_idx.random(16)  # decorrelate from the orientation draw
    truth = g_idx.integers(0, pool, size=wl.n_data) if pool < wl.n_data else np.arange(wl.n_data)

    tg = torch.Generator(device=device)
    tg.manual_seed(int(rng(wl.cfg, "photons").integers(0, 2 ** 62)))
    counts = torch.zeros((wl.n_data, wl.n_pix), dtype=torch.uint16, device=device)
    vt = torch.as_tensor(valid, device=device)
    tt = torch.as_tensor(truth, device=device)
    step = max(1, (1 << 26) // max(1, valid.size))
    for s in range(0, wl.n_data, step):
        lam = lam_pool[tt[s:s + step]]
        k = torch.poisson(lam, generator=tg)
        blk = torch.zeros((k.shape[0], wl.n_pix), dtype=torch.float32, device=device)
        blk[:, vt] = k
        counts[s:s + step] = blk.to(torch.uint16)
    if device == "cpu":
        counts = counts.numpy()

    N = wl.grid_n
    model_true = None
    if with_truth:
        ax = (np.arange(N) - N / 2) * dq
        X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
        grid_q = np.stack([X, Y, Z], axis=-1).reshape(-1, 3)
        model_true = alpha * _intensity_torch(grid_q, apos, device).cpu().numpy()

    # random-smooth start: blurred uniform noise, scaled to the mean photon count per valid pixel
    noise = rng(wl.cfg, "start").random((N, N, N))
    sm = gaussian_filter(noise, sigma=2.0, mode="wrap")
    ax = np.arange(N) - N / 2
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    ball = (X * X + Y * Y + Z * Z) <= (N / 2 - 2) ** 2
    model_start = (sm * (wl.photons / valid.size / sm[ball].mean())).reshape(-1)

    return Inputs(wl, q_vox, mask, quat, log_w, counts, model_start, model_true, alpha,
                  np.asarray(truth))


def tiny_problem(seed: int, grid_n: int, n_pix: int, n_rot: int, n_data: int,
                 q_radius: Optional[float] = None, photons: float = 30.0):
    """Unstructured random problem for brute-force checks on tiny sizes.

    Pixel coordinates are uniform in a ball of radius `q_radius` (default
    N/2 - 2), frames are Poisson draws around a random positive level, the
    model is random positive.  Returns a dict of float64/uint16 numpy arrays.
    """
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([1409, 100, seed])))
    rad = (grid_n / 2 - 2) if q_radius is None else q_radius
    d = g.standard_normal((n_pix, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    q = d * (rad * g.random(n_pix) ** (1.0 / 3.0))[:, None]
    mask = (g.random(n_pix) > 0.15).astype(np.uint8)
    if mask.sum() == 0:
        mask[0] = 1
    quat = shoemake_quaternions(g, n_rot)
    lw = g.random(n_rot) + 0.5
    log_w = np.log(lw / lw.sum())
    model = g.gamma(2.0, photons / max(1, n_pix) / 2.0, size=grid_n ** 3) + 1e-3
    lam = g.gamma(1.0, photons / max(1, n_pix), size=(n_data, n_pix))
    counts = (g.poisson(lam) * mask[None, :]).astype(np.uint16)
    return dict(q=q, mask=mask, quat=quat, log_w=log_w, model=model, counts=counts, grid_n=grid_n)
