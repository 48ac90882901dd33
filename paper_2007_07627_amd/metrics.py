"""Evaluation metrics reported next to registration results."""
from __future__ import annotations

import numpy as np


def rmse(T_gt, T, P):
    """RMSE between the ground-truth and computed alignment over the source
    points (eq. mse, Sec. 4.2), in FP64."""
    P = np.asarray(P, np.float64)
    Tg = np.asarray(T_gt, np.float64)
    Tc = np.asarray(T, np.float64)
    a = P @ Tg[:3, :3].T + Tg[:3, 3]
    b = P @ Tc[:3, :3].T + Tc[:3, 3]
    return float(np.sqrt(np.mean(np.sum((a - b) ** 2, axis=1))))


def rotation_error_rad(Ta, Tb):
    """Angle of Ra^T Rb."""
    Ra = np.asarray(Ta)[:3, :3]
    Rb = np.asarray(Tb)[:3, :3]
    c = (np.trace(Ra.T @ Rb) - 1.0) / 2.0
    s = np.linalg.norm(np.array([(Ra.T @ Rb)[2, 1] - (Ra.T @ Rb)[1, 2],
                                 (Ra.T @ Rb)[0, 2] - (Ra.T @ Rb)[2, 0],
                                 (Ra.T @ Rb)[1, 0] - (Ra.T @ Rb)[0, 1]])) / 2.0
    return float(np.arctan2(s, np.clip(c, -1.0, 1.0)))


def translation_error(Ta, Tb):
    return float(np.linalg.norm(np.asarray(Ta)[:3, 3] - np.asarray(Tb)[:3, 3]))
