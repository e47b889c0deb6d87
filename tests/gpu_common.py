"""Helpers for the GPU parity tests (no method arithmetic here)."""
import numpy as np


def rel_err(a, b):
    """sqrt(sum |a - b|^2) / sqrt(sum |b|^2): the relative (RMS) error over all particles."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt(np.sum(b * b))
    return float(np.sqrt(np.sum((a - b) ** 2)) / den) if den > 0 else float(np.sqrt(np.sum(a * a)))


def to_np(t):
    return t.detach().cpu().numpy()


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
