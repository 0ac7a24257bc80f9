"""Helpers shared by the GPU tests (no arithmetic of the method here)."""
import numpy as np


def angles(a, b):
    """Angle (rad) between corresponding unit vectors of a and b,
    atan2(|a x b|, a.b), which stays accurate for small angles and for
    vectors whose norm is 1 only to FP32 rounding."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    cr = np.linalg.norm(np.cross(a, b), axis=1)
    dt = (a * b).sum(axis=1)
    return np.arctan2(cr, dt)


def max_angle(a, b):
    """Largest of angles(a, b)."""
    return float(angles(a, b).max())


def mean_angle(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    cr = np.linalg.norm(np.cross(a, b), axis=1)
    dt = (a * b).sum(axis=1)
    return float(np.arctan2(cr, dt).mean())
