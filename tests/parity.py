"""Comparison helpers for GPU-vs-oracle parity (test infrastructure)."""
import numpy as np


def rel_fro(a, b) -> float:
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def dilate(mask: np.ndarray, r: int) -> np.ndarray:
    out = mask.copy()
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            out |= np.roll(np.roll(mask, dy, axis=0), dx, axis=1)
    return out


def pd_db_error(pd_gpu, pd_or, tube_mask):
    """Max / p99 / p99.9 of |10 log10(PD_gpu / PD_oracle)| over pixels above the
    noise floor: floor = median oracle PD outside the vessels dilated by 2 px,
    'above' = PD_oracle >= 2 x floor."""
    pd_or = np.asarray(pd_or, dtype=np.float64)
    pd_gpu = np.asarray(pd_gpu, dtype=np.float64)
    bg = ~dilate(tube_mask, 2)
    floor = np.median(pd_or[bg]) if np.any(bg) else np.median(pd_or)
    sel = pd_or >= 2.0 * floor
    err = np.abs(10.0 * np.log10(np.maximum(pd_gpu[sel], 1e-300) / pd_or[sel]))
    if err.size == 0:
        return 0.0, 0.0, 0.0, 0
    return float(err.max()), float(np.percentile(err, 99)), float(np.percentile(err, 99.9)), int(sel.sum())


def knee_tie(curv: np.ndarray, k_a: int, k_b: int, rtol: float = 1e-9) -> bool:
    """Two cut indices are a tie when the curvature at both agrees within rtol."""
    a, b = curv[k_a - 1], curv[k_b - 1]
    return abs(a - b) <= rtol * max(abs(a), abs(b))
