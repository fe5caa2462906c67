"""Shared helpers of the GPU parity tests (inputs from synth, expected
values from the oracle only; no input is ever produced by the library under
test)."""
import functools

import numpy as np
import torch

import synth
from oracle import geometry, nufft

DEV = "cuda:0"


def rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def gpu(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).to(DEV).contiguous()


def host(t):
    return t.detach().cpu().numpy()


@functools.lru_cache(maxsize=None)
def model(cid: int):
    m, _ = synth.intensity_model(synth.config(cid))
    return m


@functools.lru_cache(maxsize=None)
def detector(n: int):
    return synth.detector_q(n)


def f32(x):
    """The float32 value both sides start from, as float64."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def oracle_slices(m, quats, det, real=True, w=6):
    """Oracle slices at float32-rounded inputs (M, P)."""
    q = f32(quats)
    d = f32(det)
    x = geometry.slice_points(q, d).reshape(-1, 3)
    s = nufft.nufft2(m, x, w=w, real=real)
    return s.reshape(len(q), len(d))


def molecule_slices(cid: int, quats, det, sigma: float = 0.5):
    """Matcher inputs made without the library: the diffraction intensity of
    the workload's molecule, |F(x)|^2 with the structure factor and Gaussian
    form factor the model is built from (F(x) = sum_a exp(-i x.x_a)
    exp(-sigma^2 |x|^2 / 2)), evaluated directly at the rotated detector
    points x = R(q) q_p (the oracle's rotation).  float64 arithmetic through
    torch on the device; returns float32 (len(quats), len(det)) on DEV."""
    cfg = synth.config(cid)
    xaT = torch.from_numpy(np.ascontiguousarray(synth.molecule(cfg).T)).to(DEV)        # (3, A)
    Rt = torch.from_numpy(np.ascontiguousarray(
        geometry.quat_to_R(f32(quats)).transpose(0, 2, 1))).to(DEV)                  # (n, 3, 3)
    d = torch.from_numpy(f32(det)).to(DEV)                                            # (P, 3)
    n, P = Rt.shape[0], d.shape[0]
    chunk = max(1, int(1.3e8 // (P * xaT.shape[1])))   # about 1 GB of phases at a time
    out = torch.empty((n, P), dtype=torch.float32, device=DEV)
    for c0 in range(0, n, chunk):
        x = torch.matmul(d, Rt[c0:c0 + chunk])          # (c, P, 3): rows R q_p
        ph = torch.matmul(x, xaT)                       # (c, P, A)
        fr, fi = torch.cos(ph).sum(-1), torch.sin(ph).sum(-1)
        env = torch.exp(-sigma * sigma * (x * x).sum(-1))
        out[c0:c0 + chunk] = ((fr * fr + fi * fi) * env).float()
    return out
