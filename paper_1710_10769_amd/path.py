"""Tuning lambda1 to a target sparsity and scoring support recovery.

Section 4 chooses the tuning parameters so that estimates reach a given
average degree (the degree of the true graph, or the sparsity of a competing
estimate), and scores the recovered sparsity pattern against the true
precision matrix by positive predictive value and false discovery rate
(Table 1).  The solves run on the GPU through ``Solver``; the search and the
scoring are host logic.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.sparse as sp


def average_degree(omega: sp.spmatrix) -> float:
    """Off-diagonal stored entries per row (both triangles counted once per row)."""
    om = sp.csr_matrix(omega)
    off = om.nnz - int(np.count_nonzero(om.diagonal()))
    return off / om.shape[0]


def support_recovery(estimate: sp.spmatrix, truth: sp.spmatrix) -> dict:
    """PPV and FDR of the estimated off-diagonal support against the true one.

    An edge is an unordered pair i < j with a nonzero entry.  PPV = TP / (TP + FP),
    FDR = FP / (TP + FP) = 1 - PPV (both 0 when nothing is estimated); recall is
    TP / (TP + FN).
    """
    def edges(m):
        u = sp.triu(sp.csr_matrix(m), k=1).tocoo()
        keep = u.data != 0
        return set(zip(u.row[keep].tolist(), u.col[keep].tolist()))
    e, t = edges(estimate), edges(truth)
    tp = len(e & t)
    fp = len(e - t)
    fn = len(t - e)
    est = tp + fp
    return {"tp": tp, "fp": fp, "fn": fn,
            "ppv": tp / est if est else 0.0,
            "fdr": fp / est if est else 0.0,
            "recall": tp / (tp + fn) if tp + fn else 0.0}


@dataclasses.dataclass
class SearchResult:
    lam1: float
    degree: float
    iters: int
    omega: sp.csr_matrix
    history: List[tuple]


def lambda1_for_degree(solver, target_degree: float, lam2: float, lo: float = 0.0,
                       hi: float = 1.0, tol: float = 1e-5, max_iter: int = 200,
                       steps: int = 14, rel_tol: float = 0.02) -> SearchResult:
    """Bisection on lambda1 (the estimated degree falls as lambda1 grows) until the
    average degree is within ``rel_tol`` of the target or ``steps`` solves are done.
    Every solve starts from Omega = I.  ``solver`` already holds the data."""
    history = []
    best: Optional[SearchResult] = None
    a, b = lo, hi
    for _ in range(steps):
        lam1 = 0.5 * (a + b)
        solver.reset()
        info = solver.solve(lam1, lam2, tol, max_iter)
        om = solver.get_omega_scipy()
        deg = average_degree(om)
        history.append((lam1, deg, info.iters))
        cand = SearchResult(lam1, deg, info.iters, om, history)
        if best is None or abs(deg - target_degree) < abs(best.degree - target_degree):
            best = cand
        if abs(deg - target_degree) <= rel_tol * max(target_degree, 1e-12):
            break
        if deg > target_degree:
            a = lam1
        else:
            b = lam1
    best.history = history
    return best


def multisection_round(lo: float, hi: float, k: int):
    """The k probes of one round: evenly spaced strictly inside (lo, hi)."""
    return [lo + (hi - lo) * (j + 1) / (k + 1) for j in range(k)]


def next_bracket(lo: float, hi: float, lams, degrees, target: float):
    """The degree falls as lambda1 grows: the new bracket runs from the last probe whose
    degree is above the target to the first one at or below it (or the old ends)."""
    i = next((j for j, d in enumerate(degrees) if d <= target), len(degrees))
    return (lams[i - 1] if i > 0 else lo), (lams[i] if i < len(lams) else hi)


def lambda1_for_degree_batched(X, target_degree: float, lam2: float, lo: float = 0.0,
                               hi: float = 1.0, probes: int = 8, rounds: int = 6,
                               rel_tol: float = 0.02, tol: float = 1e-5, max_iter: int = 200,
                               precision: str = "fp32") -> SearchResult:
    """Multisection on lambda1 through the batched path: every round solves ``probes``
    lambda1 values of the bracket at once (one batch of one instance, each from
    Omega = I), keeps the sub-bracket where the degree crosses the target, and stops
    once a probe's average degree is within ``rel_tol`` of the target or after
    ``rounds`` rounds.  X: (n, p) CUDA tensor (float32, or float64 for FP64)."""
    from ._lib import Batch
    p = X.shape[1]
    history = []
    best: Optional[SearchResult] = None
    a, b = lo, hi
    for _ in range(rounds):
        lams = multisection_round(a, b, probes)
        bt = Batch([X], lams, precision=precision)
        iters, _, _ = bt.solve(lam2, tol, max_iter)
        degs = []
        for j, lam1 in enumerate(lams):
            r, c, v = bt.get_omega(0, j)
            om = sp.csr_matrix((v.cpu().numpy(), c.cpu().numpy(), r.cpu().numpy()), shape=(p, p))
            deg = average_degree(om)
            degs.append(deg)
            history.append((lam1, deg, iters[j]))
            if best is None or abs(deg - target_degree) < abs(best.degree - target_degree):
                best = SearchResult(lam1, deg, iters[j], om, history)
        bt.close()
        if abs(best.degree - target_degree) <= rel_tol * max(target_degree, 1e-12):
            break
        a, b = next_bracket(a, b, lams, degs, target_degree)
    best.history = history
    return best


def scale_for_lambda_grid(max_offdiag_s: float, lam1_top: float, lam2: float) -> float:
    """Factor c for data whose sample covariance S has unit diagonal, such that the
    estimate from c^2 S turns diagonal exactly at lambda1 = lam1_top for this lambda2.

    With unit diagonal, Omega = D (d_i = 1 / sqrt(c^2 + lambda2)) is optimal iff every
    |G_ij(D)| = c^2 |s_ij| d <= lambda1 (the KKT conditions at a diagonal point), so the
    threshold is c^2 m / sqrt(c^2 + lambda2) with m = max_{i != j} |s_ij|; solving
    c^2 m / sqrt(c^2 + lambda2) = lam1_top for u = c^2 gives
    m^2 u^2 - lam1_top^2 u - lam1_top^2 lambda2 = 0.  By the scaling identity of the
    objective, c only selects which part of the lambda path a fixed grid samples.
    """
    m, a, b = float(max_offdiag_s), float(lam1_top), float(lam2)
    if not (m > 0 and a > 0 and b >= 0):
        raise ValueError("need max_offdiag_s > 0, lam1_top > 0, lam2 >= 0")
    u = (a * a + (a ** 4 + 4.0 * m * m * a * a * b) ** 0.5) / (2.0 * m * m)
    return u ** 0.5
