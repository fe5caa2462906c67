"""Seeded generators for the five SPI-shaped workloads (see package doc).

Workload shapes follow the paper's setting (section IV-A: 128x128 images of a
protein, model orientations drawn from a fixed set; section II-A/B: M model
images, N experimental images) scaled to one GPU:

==  =====  ======  ========  ==========  ========  =======
id  N^3    atoms   detector  references  images    photons
==  =====  ======  ========  ==========  ========  =======
1   33^3   100     64x64     1,000       256       50
2   65^3   200     128x128   10,000      2,048     20
3   33^3   100     64x64     50,000      2,048     50
4   65^3   200     128x128   (assigned)  4,096     20
5   129^3  500     256x256   100,000     16,384    5
==  =====  ======  ========  ==========  ========  =======

Workload 3 reuses workload 1's molecule, model, detector and streams (so its
first 256 images and first 1,000 references equal workload 1's); workload 4
reuses workload 2's streams and adds a complex perturbation and weights.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Roles of the independent random streams of one workload.
ROLE = dict(molecule=0, image_quats=1, ref_quats=2, poisson=3, weights=4,
            perturbation=5, fd_voxels=6, points=7, model=8)


@dataclass(frozen=True)
class Config:
    cid: int            # workload id
    seed_id: int        # whose random streams it uses
    n_model: int        # N (odd): model grid is N^3 modes {-h..h}^3
    n_atoms: int
    n_det: int          # detector is n_det x n_det pixels
    n_refs: int         # reference (model) orientations M
    n_images: int       # experimental images
    photons: float      # mean photons per pixel
    complex_model: bool = False
    chunk: int = 0      # orientation chunk for streaming (0: no chunking)

    @property
    def n_pix(self) -> int:
        return self.n_det * self.n_det


CONFIGS = {
    1: Config(1, 1, 33, 100, 64, 1_000, 256, 50.0),
    2: Config(2, 2, 65, 200, 128, 10_000, 2_048, 20.0),
    3: Config(3, 1, 33, 100, 64, 50_000, 2_048, 50.0),
    4: Config(4, 2, 65, 200, 128, 10_000, 4_096, 20.0, complex_model=True),
    5: Config(5, 5, 129, 500, 256, 100_000, 16_384, 5.0, chunk=8_192),
}


def config(cid: int) -> Config:
    return CONFIGS[cid]


def rng(seed_id: int, role: str) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([seed_id, ROLE[role]]))


def molecule(cfg: Config) -> np.ndarray:
    """Scatterer positions in voxel units, uniform in a ball of radius
    0.3 * N/2 (the box [-1,1]^3 scaled to N voxels), shape (n_atoms, 3)."""
    g = rng(cfg.seed_id, "molecule")
    d = g.standard_normal((cfg.n_atoms, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = 0.3 * (cfg.n_model / 2.0) * g.random(cfg.n_atoms) ** (1.0 / 3.0)
    return d * r[:, None]


def intensity_model(cfg: Config, sigma: float = 0.5):
    """Model coefficients of a molecule's diffraction intensity.

    The molecule's structure factor with a Gaussian form factor of width
    ``sigma`` voxels, F(q) = sum_a exp(-i q.x_a) exp(-sigma^2 |q|^2 / 2), is
    sampled on the grid q_j = 2 pi j / N, j in {-h..h}^3, and squared,
    I_j = |F(q_j)|^2.  The coefficients m_k, k in {-h..h}^3, are the inverse
    DFT of I (the sampled autocorrelation), so that the trigonometric
    polynomial sum_k m_k exp(i k.q) reproduces I_j at every q_j.  m is real
    and even; it is returned symmetrised in float64 with I (both shape N^3,
    C order, index i <-> mode i - h).
    """
    N = cfg.n_model
    h = (N - 1) // 2
    j = np.arange(-h, h + 1)
    q1 = 2.0 * np.pi * j / N
    xa = molecule(cfg)
    # exp(-i q.x) factorises over the three axes.
    e0 = np.exp(-1j * np.outer(xa[:, 0], q1))
    e1 = np.exp(-1j * np.outer(xa[:, 1], q1))
    e2 = np.exp(-1j * np.outer(xa[:, 2], q1))
    F = np.einsum("ai,aj,ak->ijk", e0, e1, e2, optimize=True)
    qq = q1[:, None, None] ** 2 + q1[None, :, None] ** 2 + q1[None, None, :] ** 2
    F *= np.exp(-0.5 * sigma * sigma * qq)
    I = (F.real ** 2 + F.imag ** 2)
    # m_k = N^-3 sum_j I_j exp(-2 pi i j.k / N), centred indices on both sides.
    mk = np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(I))) / N ** 3
    m = mk.real
    m = 0.5 * (m + m[::-1, ::-1, ::-1])
    return m, I


def detector_q(n_det: int, q_max: float = 0.9 * np.pi) -> np.ndarray:
    """Ewald-sphere points of a flat n_det x n_det detector, shape (P, 3).

    Pixel (r, c) (index p = r*n + c) sits at (c - (n-1)/2, r - (n-1)/2, 2n)
    in pixel pitches from the sample; its scattered direction s_hat minus the
    beam direction (0, 0, 1) is the momentum transfer up to the factor
    2 pi / lambda, which is fixed here by scaling the corner pixel to
    |q| = q_max (0.9 of the grid's Nyquist pi by default).
    """
    n = n_det
    c = np.arange(n) - (n - 1) / 2.0
    Y, X = np.meshgrid(c, c, indexing="ij")
    Z = np.full_like(X, 2.0 * n)
    v = np.stack([X, Y, Z], axis=-1).reshape(-1, 3)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    v[:, 2] -= 1.0
    return v * (q_max / np.linalg.norm(v, axis=1).max())


def quaternions(cfg: Config, role: str, n: int) -> np.ndarray:
    """n unit quaternions (w, x, y, z), uniform on SO(3): four i.i.d. normals
    normalised.  ``role`` is "image_quats" or "ref_quats"."""
    g = rng(cfg.seed_id, role)
    q = g.standard_normal((n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def poisson_counts(cfg: Config, lam: np.ndarray) -> np.ndarray:
    """Poisson photon counts with means ``lam`` (row-major image order),
    returned as float32."""
    g = rng(cfg.seed_id, "poisson")
    return g.poisson(np.asarray(lam, dtype=np.float64)).astype(np.float32)


def photon_scale(noiseless: np.ndarray, photons: float) -> float:
    """Scale that brings the mean of unscaled noiseless images to ``photons``
    per pixel (folded into the model, so slices and images share a scale)."""
    return float(photons / np.mean(noiseless, dtype=np.float64))


def pixel_weights(cfg: Config, n_images: int, n_pix: int) -> np.ndarray:
    """Per-pixel weights uniform in [0.5, 1), float32 (n_images, n_pix)."""
    g = rng(cfg.seed_id, "weights")
    return (0.5 + 0.5 * g.random((n_images, n_pix))).astype(np.float32)


def complex_perturbation(cfg: Config, m: np.ndarray) -> np.ndarray:
    """m + 0.1 rms(m) (g1 + i g2)/sqrt 2 with g1, g2 i.i.d. N(0,1)."""
    g = rng(cfg.seed_id, "perturbation")
    g1 = g.standard_normal(m.shape)
    g2 = g.standard_normal(m.shape)
    rms = math.sqrt(float(np.mean(m * m)))
    return m + 0.1 * rms * (g1 + 1j * g2) / math.sqrt(2.0)


def fd_voxels(cfg: Config, count: int) -> np.ndarray:
    """``count`` distinct flat voxel indices of the N^3 model grid."""
    g = rng(cfg.seed_id, "fd_voxels")
    return np.sort(g.choice(cfg.n_model ** 3, size=count, replace=False))


def random_points(seed: int, n: int, radius: float | None = None) -> np.ndarray:
    """n points uniform in the cube [-pi, pi)^3, or in the ball of the given
    radius if ``radius`` is set; float64 (n, 3)."""
    g = rng(seed, "points")
    if radius is None:
        return g.uniform(-np.pi, np.pi, size=(n, 3))
    d = g.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d * (radius * g.random(n) ** (1.0 / 3.0))[:, None]


def random_model(seed: int, n_model: int, complex_model: bool = False) -> np.ndarray:
    """White-spectrum model coefficients, N(0,1) per mode (complex if asked)."""
    g = rng(seed, "model")
    shape = (n_model,) * 3
    m = g.standard_normal(shape)
    if complex_model:
        m = m + 1j * g.standard_normal(shape)
    return m
