"""Orientations: unit quaternions to rotation matrices, and slice points.

Slicing (section II-A) evaluates the model at the detector's Ewald-sphere
points rotated by each orientation of a fixed set.  Reading: quaternions are
(w, x, y, z), Hamilton convention, renormalised; point x_{m,p} = R(q_m) q_p
with R acting on column vectors.

TEST INFRASTRUCTURE ONLY (see package docstring).
"""
from __future__ import annotations

import numpy as np


def quat_to_R(quats) -> np.ndarray:
    """Rotation matrices (M, 3, 3) of quaternions (M, 4) = (w, x, y, z)."""
    q = np.asarray(quats, dtype=np.float64).reshape(-1, 4)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def slice_points(quats, det_q) -> np.ndarray:
    """Points x_{m,p} = R(q_m) q_p, shape (M, P, 3), float64."""
    R = quat_to_R(quats)
    q = np.asarray(det_q, dtype=np.float64).reshape(-1, 3)
    return np.einsum("mij,pj->mpi", R, q)
