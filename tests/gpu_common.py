"""Helpers shared by the GPU parity tests: device transfer and error metrics."""
import numpy as np


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t):
    return t.detach().cpu().numpy()


def rel_err(got, ref) -> float:
    """Global relative error ||got - ref|| / ||ref|| (||ref|| = 0: absolute)."""
    d = np.linalg.norm((np.asarray(got) - np.asarray(ref)).ravel())
    n = np.linalg.norm(np.asarray(ref).ravel())
    return float(d / n) if n > 0 else float(d)


def max_rel_err(got, ref) -> float:
    """Largest elementwise deviation relative to the largest reference entry."""
    ref = np.asarray(ref)
    scale = np.max(np.abs(ref))
    return float(np.max(np.abs(np.asarray(got) - ref)) / (scale if scale > 0 else 1.0))


def link_errors(got, ref):
    """Per-link relative Frobenius error of eq. (8): (median, 99th percentile, max)."""
    num = np.sqrt(np.sum(np.abs(got - ref) ** 2, axis=(-2, -1))).ravel()
    den = np.sqrt(np.sum(np.abs(ref) ** 2, axis=(-2, -1))).ravel()
    e = num / np.where(den > 0, den, 1.0)
    return float(np.median(e)), float(np.quantile(e, 0.99)), float(np.max(e))
