"""Helpers for the GPU parity tests (no method arithmetic here)."""
import numpy as np


def rel_err(a, b):
    """sqrt(sum |a - b|^2) / sqrt(sum |b|^2): the relative (RMS) error over all particles."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt(np.sum(b * b))
    return float(np.sqrt(np.sum((a - b) ** 2)) / den) if den > 0 else float(np.sqrt(np.sum(a * a)))


def pp_err(a, b):
    """Largest per-particle error max_i |a_i - b_i| / max(|b_i|, RMS_j |b_j|): each
    particle's error against its own force, floored at the RMS force (a particle whose
    pair forces nearly cancel has no meaningful relative error of its own)."""
    a = np.asarray(a, dtype=np.float64).reshape(-1, 3)
    b = np.asarray(b, dtype=np.float64).reshape(-1, 3)
    d = np.linalg.norm(a - b, axis=1)
    m = np.linalg.norm(b, axis=1)
    rms = np.sqrt(np.mean(m * m)) if m.size else 0.0
    floor = np.maximum(m, rms)
    if not np.any(floor > 0):
        return float(d.max()) if d.size else 0.0
    return float(np.max(d / np.where(floor > 0, floor, 1.0)))


# Per-particle tolerances (pp_err).  FP64: the same 1e-10 as the norm.  Mixed: each
# pair force is rounded to FP32 (2^-24 relative), a particle sums about 20 of them,
# and near contact single pair forces reach tens of times the RMS force, so one
# particle's error may reach 2^-24 x 20 x 50 = 6e-5 of the RMS force; 1e-4 bounds it.
PP_FP64_TOL = 1e-10
PP_MIXED_TOL = 1e-4


def check_forces(F, F0, rms_tol, pp_tol, label=""):
    """Assert both the relative RMS error and the per-particle error; return them."""
    e, q = rel_err(F, F0), pp_err(F, F0)
    print(f"{label}: rms {e:.3e}  per-particle {q:.3e}")
    assert e < rms_tol, (label, e)
    assert q < pp_tol, (label, q)
    return e, q


def to_np(t):
    return t.detach().cpu().numpy()


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
