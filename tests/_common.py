"""Shared helpers of the GPU parity tests (inputs from synth, expected
values from the oracle only)."""
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
