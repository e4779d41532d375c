"""Helpers shared by the GPU parity tests (inputs and comparisons only)."""
import numpy as np
import scipy.sparse as sp


def csr_dense(m: sp.spmatrix) -> np.ndarray:
    return sp.csr_matrix(m).toarray()


def max_abs_diff(a: sp.spmatrix, b: sp.spmatrix) -> float:
    d = (sp.csr_matrix(a) - sp.csr_matrix(b))
    return float(np.abs(d.data).max()) if d.nnz else 0.0


def support_mismatch(gpu: sp.spmatrix, ref: sp.spmatrix):
    """Entries in the support of exactly one of the two matrices."""
    g = sp.csr_matrix(gpu).copy()
    r = sp.csr_matrix(ref).copy()
    g.data[:] = 1.0
    r.data[:] = 1.0
    d = (g - r).tocoo()
    keep = d.data != 0
    return list(zip(d.row[keep].tolist(), d.col[keep].tolist()))


def threshold_band(prev: sp.spmatrix, G: np.ndarray, tau: float, lam1: float, i: int, j: int) -> float:
    """| |omega_ij - tau G_ij| / tau - lam1 |: distance of an entry from the threshold."""
    z = sp.csr_matrix(prev)[i, j] - tau * G[i, j]
    return abs(abs(z) / tau - lam1)
