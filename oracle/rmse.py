"""Localisation error measure of Section 4, eq. (20).  Test infrastructure
only: see the package docstring.

Each estimated direction s is first mapped to what the array can resolve:
f_1 maps to the half circle of the linear array (elevation only,
g(s) = atan2(s_z, sqrt(s_x^2 + s_y^2)), f_1(s) = [cos g, 0, sin g]); f_2
folds onto the upper half-sphere of the planar array ([s_x, s_y, |s_z|]);
f_3 is the identity (3-D array).  RMSE_alpha is the distance between the
power-weighted mean of the mapped estimates and the mapped true direction:
|| sum_f f(s_f) Y_f / sum_f Y_f - f(s_0) ||_2."""
from __future__ import annotations

import numpy as np


def doa_map(s: np.ndarray, alpha: int) -> np.ndarray:
    """f_alpha of Section 4 on directions s [..., 3]."""
    s = np.asarray(s, dtype=np.float64)
    if alpha == 1:
        g = np.arctan2(s[..., 2], np.sqrt(s[..., 0] ** 2 + s[..., 1] ** 2))
        return np.stack([np.cos(g), np.zeros_like(g), np.sin(g)], axis=-1)
    if alpha == 2:
        return np.stack([s[..., 0], s[..., 1], np.abs(s[..., 2])], axis=-1)
    if alpha == 3:
        return s.copy()
    raise ValueError("alpha is 1, 2 or 3")


def rmse_alpha(s_est: np.ndarray, Y: np.ndarray, s0: np.ndarray, alpha: int) -> float:
    """Eq. (20) for estimates s_est [F, 3] with powers Y [F] and true
    direction s0 [3]."""
    Y = np.asarray(Y, dtype=np.float64)
    m = (doa_map(s_est, alpha) * Y[:, None]).sum(axis=0) / Y.sum()
    return float(np.linalg.norm(m - doa_map(s0, alpha)))
