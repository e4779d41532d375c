"""Closed forms and optimality checks of the CONCORD / PseudoNet problem.

TEST INFRASTRUCTURE ONLY.

* diagonal_solution: the minimiser when every off-diagonal entry is zero at the
  optimum, omega_ii = 1/sqrt(s_ii + lam2) (stationarity of
  -log w + (s_ii + lam2) w^2 / 2).
* lambda1_max: the smallest lam1 for which that diagonal matrix is optimal,
  max_{i != j} |s_ij| (d_i + d_j) / 2 with d_i = 1/sqrt(s_ii + lam2) (the
  off-diagonal gradient at diag(d) is s_ij (d_i + d_j) / 2 and the
  subgradient condition asks it to stay within [-lam1, lam1]).
* kkt_residual: how far a candidate Omega is from the optimality conditions
  of F = f + lam1 ||Omega_X||_1: G_ii = 0, G_ij = -lam1 sign(omega_ij) on the
  support, |G_ij| <= lam1 off it.  The gradient here is written from the
  definition of f directly (S Omega + Omega S)/2 etc.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def diagonal_solution(S: np.ndarray, lam2: float) -> np.ndarray:
    return 1.0 / np.sqrt(np.diag(S) + lam2)


def lambda1_max(S: np.ndarray, lam2: float) -> float:
    d = diagonal_solution(S, lam2)
    A = np.abs(S) * (d[:, None] + d[None, :]) * 0.5
    np.fill_diagonal(A, 0.0)
    return float(A.max()) if A.size > 1 else 0.0


def kkt_residual(omega, S: np.ndarray, lam1: float, lam2: float) -> float:
    Om = omega.toarray() if sp.issparse(omega) else np.asarray(omega, dtype=np.float64)
    G = 0.5 * (S @ Om + Om @ S) + lam2 * Om
    G[np.diag_indices_from(G)] -= 1.0 / np.diag(Om)
    p = Om.shape[0]
    off = ~np.eye(p, dtype=bool)
    on = (Om != 0) & off
    zero = (Om == 0) & off
    r_diag = np.abs(np.diag(G)).max()
    r_on = np.abs(G[on] + lam1 * np.sign(Om[on])).max() if on.any() else 0.0
    r_off = np.maximum(np.abs(G[zero]) - lam1, 0.0).max() if zero.any() else 0.0
    return float(max(r_diag, r_on, r_off))
