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


def parity_report(label, S, S_ref, m=None, m_ref=None, E=None, E_ref=None):
    """Print one line with the measured differences of a run against the
    oracle (max and mean angle, largest |dm|, largest |dE| / |E|) and
    return them as a dict (None where an input is missing)."""
    out = {"max": max_angle(S, S_ref), "mean": mean_angle(S, S_ref), "dm": None, "dE": None}
    if m is not None:
        out["dm"] = float(np.abs(np.asarray(m) - np.asarray(m_ref)).max())
    if E is not None:
        E_ref = np.asarray(E_ref)
        out["dE"] = float((np.abs(np.asarray(E) - E_ref) / np.abs(E_ref).max()).max())
    fmt = lambda v: "-" if v is None else f"{v:.2e}"
    print(f"\nPARITY {label}: max angle {fmt(out['max'])} mean angle {fmt(out['mean'])} "
          f"|dm| {fmt(out['dm'])} |dE|/|E| {fmt(out['dE'])}", flush=True)
    return out
