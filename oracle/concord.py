"""Plain FP64 proximal-gradient solver for the CONCORD / PseudoNet objective.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Objective (the half-scaled reading of eq. (1), whose exact gradient is the one
Algorithm 1 computes in its gradient step):

    f(Omega) = -sum_i log omega_ii + 1/2 tr(Omega S Omega) + lam2/2 ||Omega||_F^2
    F(Omega) = f(Omega) + lam1 * sum_{i != j} |omega_ij|

Eq. (1) writes -log det(Omega_D^2) + tr(Omega S Omega); its gradient would be
twice Algorithm 1's G.  Taking f as above makes the gradient, the smooth value
and the sufficient-decrease test of Algorithm 1 mutually consistent; it is eq.
(1) at (2*lam1, 2*lam2), halved.

Ω is a scipy CSR matrix (both triangles stored, diagonal always present); G,
W and the prox argument are dense, exactly as Algorithm 1 writes them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
import scipy.sparse as sp


# --------------------------------------------------------------------------
# Elementwise pieces
# --------------------------------------------------------------------------

def soft_threshold(z: np.ndarray, alpha: float) -> np.ndarray:
    """Eq. (2): z - a if z > a; z + a if z < -a; 0 otherwise (|z| = a gives 0)."""
    z = np.asarray(z, dtype=np.float64)
    return np.where(z > alpha, z - alpha, np.where(z < -alpha, z + alpha, 0.0))


def prox_step(omega: sp.csr_matrix, G: np.ndarray, tau: float, lam1: float) -> sp.csr_matrix:
    """Algorithm 1, soft-threshold step: S_{tau*lam1}(Omega - tau*G).

    The l1 penalty of eq. (1) covers only the off-diagonal part Omega_X, so the
    threshold is applied off the diagonal and the diagonal takes the plain
    gradient step.  Exact zeros are dropped from the returned CSR.
    """
    Z = omega.toarray() - tau * G
    d = np.diag(Z).copy()
    P = soft_threshold(Z, tau * lam1)
    np.fill_diagonal(P, d)
    out = sp.csr_matrix(P)
    out.eliminate_zeros()
    out.sort_indices()
    return out


def sample_covariance(X: np.ndarray) -> np.ndarray:
    """Algorithm 1 / Algorithm 2, once: S = X^T X / n."""
    X = np.asarray(X, dtype=np.float64)
    return (X.T @ X) / X.shape[0]


def penalty(omega: sp.csr_matrix, lam1: float) -> float:
    """lam1 * sum over off-diagonal entries of |omega_ij| (eq. (1), Omega_X)."""
    coo = omega.tocoo()
    off = coo.row != coo.col
    return lam1 * float(np.abs(coo.data[off]).sum())


def _diag(omega: sp.csr_matrix) -> np.ndarray:
    return np.asarray(omega.diagonal(), dtype=np.float64)


# --------------------------------------------------------------------------
# The products of Algorithm 2 (Cov) and Algorithm 3 (Obs)
# --------------------------------------------------------------------------

def _products(omega: sp.csr_matrix, variant: str, S: Optional[np.ndarray],
              X: Optional[np.ndarray]):
    """W = Omega S and the quadratic trace tr(Omega S Omega).

    Cov (Algorithm 2): W = Omega S; tr(Omega S Omega) = sum(W o Omega)
    (trace of a product of symmetric matrices as an elementwise sum, Section 3).
    Obs (Algorithm 3): Y = Omega X^T, W = Y X / n, tr(Omega S Omega) = ||Y||_F^2 / n.
    The 1/n is placed on W and on ||Y||^2 (the text puts it on Y; Algorithm 3
    puts it on ||Y||^2); both give W = Omega S.
    """
    if variant == "cov":
        W = np.asarray(omega @ S)
        quad = float(np.sum(W * omega.toarray()))
        return W, quad, None
    if variant == "obs":
        n = X.shape[0]
        Y = np.asarray(omega @ X.T)
        W = (Y @ X) / n
        quad = float(np.sum(Y * Y)) / n
        return W, quad, Y
    raise ValueError(f"unknown variant {variant!r}")


def smooth_objective(omega: sp.csr_matrix, lam2: float, variant: str = "cov",
                     S: Optional[np.ndarray] = None, X: Optional[np.ndarray] = None) -> float:
    """f(Omega) of the module docstring, via the variant's own products."""
    d = _diag(omega)
    if np.any(d <= 0):
        return math.inf
    _, quad, _ = _products(omega, variant, S, X)
    fro2 = float(np.sum(omega.data ** 2))
    return -float(np.sum(np.log(d))) + 0.5 * quad + 0.5 * lam2 * fro2


def gradient(W: np.ndarray, omega: sp.csr_matrix, lam2: float) -> np.ndarray:
    """Algorithm 1 gradient: G = -(Omega_D)^{-1} + 1/2 (W + W^T) + lam2 * Omega.

    W + W^T is formed so G_ij and G_ji are bitwise equal (iterates stay exactly
    symmetric).
    """
    G = 0.5 * (W + W.T)
    G = G + lam2 * omega.toarray()
    G[np.diag_indices_from(G)] -= 1.0 / _diag(omega)
    return G


def test_difference_terms(omega: sp.csr_matrix, omega_plus: sp.csr_matrix, variant: str,
                          lam2: float, S=None, X=None):
    """Terms of the sufficient-decrease test in exact difference form.

    With Delta = Omega+ - Omega and x_i = Delta_ii / omega_ii,
        f(Omega+) - f(Omega) - <G, Delta>
          = sum_i [x_i - log1p(x_i)] + 1/2 tr(Delta S Delta) + lam2/2 ||Delta||^2
    (the cross terms cancel against <1/2(Omega S + S Omega), Delta>), so the
    test of Algorithm 1 reads  lhs <= ||Delta||^2 / (2 tau).
    Returns (lhs, ||Delta||_F^2).  Every term of lhs is >= 0.
    """
    D = (omega_plus - omega).tocsr()
    x = np.asarray(D.diagonal()) / _diag(omega)
    logterm = float(np.sum(x - np.log1p(x)))
    if variant == "cov":
        quad = float(np.sum(np.asarray(D @ S) * D.toarray()))
    else:
        DX = np.asarray(D @ X.T)
        quad = float(np.sum(DX * DX)) / X.shape[0]
    dd = float(np.sum(D.data ** 2))
    return logterm + 0.5 * quad + 0.5 * lam2 * dd, dd


# --------------------------------------------------------------------------
# The outer loop
# --------------------------------------------------------------------------

@dataclasses.dataclass
class IterRecord:
    k: int            # iterations completed after this step
    tau: float        # accepted step size
    trials: int       # number of step sizes tried (1 = tau accepted at 1)
    f: float          # smooth value at the accepted iterate
    F: float          # full objective at the accepted iterate
    nnz: int          # stored entries of the accepted iterate (incl. diagonal)
    delta_fro: float  # ||Omega^{k+1} - Omega^k||_F
    lhs: float = 0.0  # difference-form left side at the accepted step
    rhs: float = 0.0  # ||Delta||^2 / (2 tau)


@dataclasses.dataclass
class SolveResult:
    omega: sp.csr_matrix
    log: List[IterRecord]
    F0: float
    f0: float
    status: str                 # "converged", "max_iter", "fixed", "linesearch"
    iterates: Optional[List[sp.csr_matrix]] = None
    last_G: Optional[np.ndarray] = None
    last_tau: Optional[float] = None
    last_omega_prev: Optional[sp.csr_matrix] = None


def solve(lam1: float, lam2: float, variant: str = "cov", X: Optional[np.ndarray] = None,
          S: Optional[np.ndarray] = None, tol: float = 1e-5, max_iter: int = 200,
          fixed_iters: Optional[int] = None, tau_replay: Optional[Sequence[int]] = None,
          max_backtracks: int = 60, omega_init: Optional[sp.spmatrix] = None,
          check_literal: bool = True, record_iterates: bool = False) -> SolveResult:
    """Algorithm 1 in the Cov (Algorithm 2) or Obs (Algorithm 3) form, FP64.

    Per iteration: products W (and Y), gradient G, smooth value f; then the
    backtracking search tau = 1, 1/2, 1/4, ... (restarted at 1 every iteration)
    of prox step and sufficient-decrease test.  A trial whose diagonal is not
    positive is rejected (f is +inf there).  The test is decided in its exact
    difference form; when ``check_literal`` the paper's literal form (recompute
    the products at Omega+, compare f values) is evaluated too and must agree
    whenever its margin exceeds 1e-10 * max(1, |f|).  The test accepts on <=.

    Stopping: after each accepted step, stop when |F_new - F_old| < tol*|F_old|
    or when ``max_iter`` steps are done; ``fixed_iters`` runs exactly that many.

    ``tau_replay[k]`` (number of trials, 1-based) replaces the search at
    iteration k: tau = 2^-(trials-1) is accepted without testing.
    """
    if variant not in ("cov", "obs"):
        raise ValueError(variant)
    if lam1 < 0 or lam2 < 0:
        raise ValueError("lambda must be >= 0")
    if variant == "cov" and S is None:
        S = sample_covariance(X)
    if variant == "obs" and X is None:
        raise ValueError("Obs needs X")
    if X is not None:
        X = np.asarray(X, dtype=np.float64)
    p = S.shape[0] if S is not None else X.shape[1]
    omega = sp.identity(p, format="csr", dtype=np.float64) if omega_init is None \
        else sp.csr_matrix(omega_init, dtype=np.float64)
    omega.sort_indices()

    W, quad, _ = _products(omega, variant, S, X)
    f = -float(np.sum(np.log(_diag(omega)))) + 0.5 * quad + 0.5 * lam2 * float(np.sum(omega.data ** 2))
    F = f + penalty(omega, lam1)
    f0, F0 = f, F
    log: List[IterRecord] = []
    iterates = [omega] if record_iterates else None
    n_iter = fixed_iters if fixed_iters is not None else max_iter
    status = "fixed" if fixed_iters is not None else "max_iter"
    last_G = last_tau = last_prev = None

    for k in range(n_iter):
        G = gradient(W, omega, lam2)
        accepted = None
        forced = tau_replay[k] if tau_replay is not None else None
        trials = 0
        tau = 1.0
        while trials < max_backtracks + 1:
            trials += 1
            cand = prox_step(omega, G, tau, lam1)
            dpos = np.all(_diag(cand) > 0)
            if forced is not None:
                if trials < forced:
                    tau *= 0.5
                    continue
                if not dpos:
                    raise RuntimeError("replayed step leaves the domain")
                lhs, dd = test_difference_terms(omega, cand, variant, lam2, S, X)
                accepted = (cand, lhs, dd)
                break
            if not dpos:
                tau *= 0.5
                continue
            lhs, dd = test_difference_terms(omega, cand, variant, lam2, S, X)
            rhs = dd / (2.0 * tau)
            ok = lhs <= rhs
            if check_literal:
                f_plus = smooth_objective(cand, lam2, variant, S, X)
                Dm = (cand - omega).toarray()
                lit_rhs = f + float(np.sum(G * Dm)) + rhs
                margin = lit_rhs - f_plus
                if abs(margin) > 1e-10 * max(1.0, abs(f)):
                    if (margin >= 0) != ok:
                        raise AssertionError(
                            f"literal and difference tests disagree at k={k} tau={tau}: "
                            f"margin={margin} lhs={lhs} rhs={rhs}")
            if ok:
                accepted = (cand, lhs, dd)
                break
            tau *= 0.5
        if accepted is None:
            status = "linesearch"
            break
        cand, lhs, dd = accepted
        last_G, last_tau, last_prev = G, tau, omega
        omega = cand
        W, quad, _ = _products(omega, variant, S, X)
        f = -float(np.sum(np.log(_diag(omega)))) + 0.5 * quad + 0.5 * lam2 * float(np.sum(omega.data ** 2))
        F_new = f + penalty(omega, lam1)
        log.append(IterRecord(k=k + 1, tau=tau, trials=trials, f=f, F=F_new, nnz=omega.nnz,
                              delta_fro=math.sqrt(dd), lhs=lhs, rhs=dd / (2.0 * tau)))
        if record_iterates:
            iterates.append(omega)
        F_old, F = F, F_new
        if fixed_iters is None and abs(F_new - F_old) < tol * abs(F_old):
            status = "converged"
            break
    return SolveResult(omega=omega, log=log, F0=F0, f0=f0, status=status, iterates=iterates,
                       last_G=last_G, last_tau=last_tau, last_omega_prev=last_prev)


# --------------------------------------------------------------------------
# Differentiation form: value and gradients of the smooth part
# --------------------------------------------------------------------------

def smooth_value_and_grads(omega: sp.spmatrix, X: np.ndarray, lam2: float):
    """f(Omega; X) in the Obs form and its gradients, FP64.

    f = -sum log omega_ii + ||Omega X^T||_F^2 / (2n) + lam2/2 ||Omega||_F^2.
    Returns (f, G, dX) where G is the gradient over symmetric matrices (the
    same G as Algorithm 1's gradient step) as a dense array, and
    dX = d f / d X = (Omega Y)^T / n with Y = Omega X^T (n x p).
    """
    omega = sp.csr_matrix(omega, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    Y = np.asarray(omega @ X.T)
    d = _diag(omega)
    f = -float(np.sum(np.log(d))) + float(np.sum(Y * Y)) / (2 * n) \
        + 0.5 * lam2 * float(np.sum(omega.data ** 2))
    W = (Y @ X) / n
    G = gradient(W, omega, lam2)
    dX = np.asarray(omega @ Y).T / n
    return f, G, dX


def smooth_value_and_sampled_grads(omega: sp.spmatrix, X: np.ndarray, lam2: float,
                                   entries, x_cols):
    """As smooth_value_and_grads, for large p: f, G at the listed (i, j) entries and
    the listed columns of dX, each computed one by one from Y = Omega X^T.

    G_ij = (Y_i . X^T_j + Y_j . X^T_i) / (2n) + lam2 omega_ij - [i == j] / omega_ii
    (half the sum of (Omega S)_ij and (Omega S)_ji, written with S = X^T X / n);
    dX[:, j] = (sum_k omega_jk Y_k) / n.
    """
    omega = sp.csr_matrix(omega, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    Xt = X.T
    Y = np.asarray(omega @ Xt)
    d = _diag(omega)
    f = -float(np.sum(np.log(d))) + float(np.sum(Y * Y)) / (2 * n) \
        + 0.5 * lam2 * float(np.sum(omega.data ** 2))
    G = []
    for (i, j) in entries:
        w = omega[i, j]
        g = (float(Y[i] @ Xt[j]) + float(Y[j] @ Xt[i])) / (2 * n) + lam2 * w
        if i == j:
            g -= 1.0 / w
        G.append(g)
    dX = []
    for j in x_cols:
        row = omega.getrow(j)
        acc = np.zeros(n)
        for k, v in zip(row.indices, row.data):
            acc += v * Y[k]
        dX.append(acc / n)
    return f, np.array(G), np.array(dX).T


# --------------------------------------------------------------------------
# Tuning lambda1 to a target average degree (Section 4) and support recovery (Table 1)
# --------------------------------------------------------------------------

def lambda1_search(X: np.ndarray, target_degree: float, lam2: float, lo: float, hi: float,
                   probes: int, rounds: int, rel_tol: float, tol: float = 1e-5,
                   max_iter: int = 200, variant: str = "cov"):
    """Multisection search for the lambda1 whose estimate has the target average degree
    (off-diagonal stored entries per row), written out plainly: each round solves
    (Algorithm 1, from Omega = I) at `probes` lambda1 values evenly spaced strictly
    inside the bracket; the bracket becomes the two probes around the first one whose
    degree is at or below the target (the degree falls as lambda1 grows); the search
    stops when the probe closest to the target so far (the first such probe on ties) is
    within rel_tol of it, or after `rounds` rounds.
    Returns (best lambda1, its degree, its estimate, [(lambda1, degree, iterations)])."""
    p = X.shape[1]
    history = []
    best = None
    a, b = lo, hi
    for _ in range(rounds):
        lams = [a + (b - a) * (j + 1) / (probes + 1) for j in range(probes)]
        degs = []
        for lam1 in lams:
            r = solve(lam1, lam2, variant, X=X, tol=tol, max_iter=max_iter, check_literal=False)
            deg = (r.omega.nnz - int(np.count_nonzero(r.omega.diagonal()))) / p
            degs.append(deg)
            history.append((lam1, deg, len(r.log)))
            if best is None or abs(deg - target_degree) < abs(best[1] - target_degree):
                best = (lam1, deg, r.omega)
        if abs(best[1] - target_degree) <= rel_tol * max(target_degree, 1e-12):
            break
        i = 0
        while i < len(degs) and degs[i] > target_degree:
            i += 1
        a, b = (lams[i - 1] if i > 0 else a), (lams[i] if i < len(lams) else b)
    return best[0], best[1], best[2], history


def edge_scores(estimate: sp.spmatrix, truth: sp.spmatrix):
    """Positive predictive value and false discovery rate of the estimated edges (unordered
    pairs i < j with a nonzero entry) against the true ones: PPV = TP/(TP+FP),
    FDR = FP/(TP+FP) (both 0 for an empty estimate)."""
    def edges(m):
        u = sp.triu(sp.csr_matrix(m), k=1).tocoo()
        return {(int(i), int(j)) for i, j, v in zip(u.row, u.col, u.data) if v != 0}
    e, t = edges(estimate), edges(truth)
    tp, fp = len(e & t), len(e - t)
    return (tp / (tp + fp), fp / (tp + fp)) if tp + fp else (0.0, 0.0)
