"""Exact minimiser of the CONCORD / PseudoNet objective for p <= 3.

TEST INFRASTRUCTURE ONLY.  Written independently of ``oracle.concord``: it
shares no function with it, and it never uses the gradient formula of
Algorithm 1.  It pins the oracle's converged result.

Method (sign-pattern enumeration):
  theta = (omega_11..omega_pp, omega_ij for i<j), Omega(theta) symmetric.
  F(theta) = -sum log theta_d + q(theta) + 2*lam1*sum_{i<j} |theta_ij|, where
  q(theta) = 1/2 tr(Omega S Omega) + lam2/2 ||Omega||_F^2 is a quadratic form
  in theta.  Its Hessian and linear term are read off by evaluating q at unit
  vectors (exact for a quadratic).  For every sign pattern sigma in
  {-1,0,+1}^{p(p-1)/2} the entries with sigma=0 are fixed at zero and
  |theta_ij| is replaced by sigma_ij*theta_ij; the resulting smooth, strictly
  convex function is minimised by damped Newton on theta_d > 0.  Solutions
  whose signs agree with sigma are feasible; the smallest F among them is the
  global minimum.
"""
from __future__ import annotations

import itertools

import numpy as np


def _omega_from_theta(theta, p):
    Om = np.zeros((p, p))
    Om[np.diag_indices(p)] = theta[:p]
    iu = np.triu_indices(p, 1)
    Om[iu] = theta[p:]
    Om[(iu[1], iu[0])] = theta[p:]
    return Om


def _q(theta, S, lam2, p):
    Om = _omega_from_theta(theta, p)
    return 0.5 * np.trace(Om @ S @ Om) + 0.5 * lam2 * np.sum(Om * Om)


def objective(theta, S, lam1, lam2):
    p = S.shape[0]
    d = theta[:p]
    if np.any(d <= 0):
        return np.inf
    return -np.sum(np.log(d)) + _q(theta, S, lam2, p) + 2.0 * lam1 * np.sum(np.abs(theta[p:]))


def minimise(S: np.ndarray, lam1: float, lam2: float, newton_iters: int = 200):
    """Return (Omega_hat dense, F_min) for p <= 3."""
    S = np.asarray(S, dtype=np.float64)
    p = S.shape[0]
    if p > 3:
        raise ValueError("brute force is for p <= 3")
    m = p * (p - 1) // 2
    dim = p + m
    zero = np.zeros(dim)
    q0 = _q(zero, S, lam2, p)
    E = np.eye(dim)
    qe = np.array([_q(E[a], S, lam2, p) for a in range(dim)])
    H = np.empty((dim, dim))
    for a in range(dim):
        for b in range(dim):
            H[a, b] = _q(E[a] + E[b], S, lam2, p) - qe[a] - qe[b] + q0
    lin = qe - q0 - 0.5 * np.diag(H)

    best = (None, np.inf)
    for sigma in itertools.product((-1, 0, 1), repeat=m):
        sigma = np.array(sigma, dtype=np.float64)
        free = np.concatenate([np.ones(p, bool), sigma != 0])
        idx = np.flatnonzero(free)
        c = lin.copy()
        c[p:] += 2.0 * lam1 * sigma
        Hs = H[np.ix_(idx, idx)]
        cs = c[idx]
        nd = p

        def h(t):
            if np.any(t[:nd] <= 0):
                return np.inf
            return -np.sum(np.log(t[:nd])) + 0.5 * t @ Hs @ t + cs @ t

        t = np.zeros(idx.size)
        t[:nd] = 1.0
        for _ in range(newton_iters):
            g = Hs @ t + cs
            g[:nd] -= 1.0 / t[:nd]
            Hh = Hs.copy()
            Hh[np.arange(nd), np.arange(nd)] += 1.0 / t[:nd] ** 2
            step = np.linalg.solve(Hh, g)
            s = 1.0
            h0 = h(t)
            while True:
                tn = t - s * step
                if np.all(tn[:nd] > 0) and h(tn) <= h0 - 1e-4 * s * (g @ step):
                    break
                s *= 0.5
                if s < 1e-30:
                    tn = t
                    break
            t = tn
            if np.max(np.abs(s * step)) < 1e-15:
                break
        theta = np.zeros(dim)
        theta[idx] = t
        off = theta[p:]
        ok = np.all((sigma == 0) | (sigma * off > 0))
        if not ok:
            continue
        Fv = objective(theta, S, lam1, lam2)
        if Fv < best[1]:
            best = (theta, Fv)
    theta, Fv = best
    return _omega_from_theta(theta, p), Fv
