"""Helpers for GPU parity tests (no arithmetic of the method)."""
import numpy as np


def rel_maxnorm(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def gather_rows(band, rows, b=0):
    """[len(rows), S] host array of selected rows of a device band [batch, S, ld]."""
    import torch

    idx = torch.as_tensor(np.asarray(rows, dtype=np.int64), device=band.device)
    return band[b].index_select(1, idx).T.double().cpu().numpy()
