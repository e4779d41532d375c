"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a printed
definition, a closed form, brute force, optimality conditions, an identity the
paper states, finite differences, or a metamorphic relation.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import datagen
import oracle
from oracle import brute, checks
from oracle import concord as oc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _small_X(p, n, seed, deg=3):
    rng = _rng(seed)
    om = datagen.random_omega0(p, min(deg, p - 1), rng) if p > 2 else datagen.chain_omega0(p)
    return datagen.sample_cholesky(om, n, rng)


# ---------------------------------------------------------------- eq. (2)

def test_soft_threshold_golden():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "soft_threshold_eq2.txt"))
            if l.strip() and not l.startswith("#")]
    for z, a, e in rows:
        got = float(oc.soft_threshold(np.array([float(z)]), float(a))[0])
        assert abs(got - float(e)) < 1e-15, (z, a, got, e)


def test_prox_leaves_diagonal_unthresholded():
    om = sp.identity(3, format="csr") * 0.2
    G = np.full((3, 3), 0.05)
    out = oc.prox_step(sp.csr_matrix(om), G, 1.0, 1.0).toarray()
    # off-diagonal: S_1(-0.05) = 0; diagonal: 0.2 - 0.05 = 0.15 (no threshold)
    assert np.allclose(np.diag(out), 0.15)
    assert np.count_nonzero(out - np.diag(np.diag(out))) == 0


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("variant", ["cov", "obs"])
def test_diagonal_S_closed_form(variant):
    # X with orthogonal columns -> S diagonal; minimiser omega_ii = 1/sqrt(s_ii + lam2)
    rng = _rng(7)
    n, p = 40, 12
    Q, _ = np.linalg.qr(rng.standard_normal((n, p)))
    scales = rng.uniform(0.5, 2.0, p)
    X = Q * scales * math.sqrt(n)
    S = oc.sample_covariance(X)
    assert np.abs(S - np.diag(np.diag(S))).max() < 1e-12
    lam2 = 0.1
    res = oc.solve(0.05, lam2, variant, X=X, tol=0.0, max_iter=3000, check_literal=False)
    want = 1.0 / np.sqrt(np.diag(S) + lam2)
    Om = res.omega.toarray()
    assert np.abs(np.diag(Om) - want).max() < 1e-7
    assert np.abs(Om - np.diag(np.diag(Om))).max() == 0.0


def test_lambda1_max_closed_form():
    X = _small_X(15, 60, 11)
    S = oc.sample_covariance(X)
    lam2 = 0.1
    lmax = checks.lambda1_max(S, lam2)
    d = checks.diagonal_solution(S, lam2)
    res = oc.solve(lmax * 1.0001, lam2, "cov", S=S, tol=0.0, max_iter=3000, check_literal=False)
    Om = res.omega.toarray()
    assert np.abs(Om - np.diag(np.diag(Om))).max() == 0.0
    assert np.abs(np.diag(Om) - d).max() < 1e-7
    # just below lambda1_max at least one off-diagonal entry must enter
    res2 = oc.solve(lmax * 0.9, lam2, "cov", S=S, tol=1e-12, max_iter=5000)
    assert res2.omega.nnz > 15


# ------------------------------------------------------------- brute force

@pytest.mark.parametrize("p,seed,lam1", [(2, 1, 0.05), (2, 2, 0.5), (3, 3, 0.1), (3, 4, 0.02),
                                         (3, 5, 0.3)])
def test_bruteforce_small_p(p, seed, lam1):
    rng = _rng(seed)
    X = rng.standard_normal((20, p)) @ rng.standard_normal((p, p))
    S = oc.sample_covariance(X)
    lam2 = 0.1
    Om_bf, F_bf = brute.minimise(S, lam1, lam2)
    res = oc.solve(lam1, lam2, "cov", S=S, tol=0.0, max_iter=4000, check_literal=False)
    Om = res.omega.toarray()
    assert np.abs(Om - Om_bf).max() < 1e-6, (Om, Om_bf)
    F_or = res.log[-1].F if res.log else res.F0
    assert F_or >= F_bf - 1e-9
    assert abs(F_or - F_bf) < 1e-8


# ----------------------------------------------------- iteration invariants

@pytest.fixture(scope="module")
def run30():
    X = _small_X(30, 50, 21, deg=4)
    res = oc.solve(0.15, 0.1, "cov", X=X, tol=1e-12, max_iter=400, record_iterates=True)
    return X, res


def test_monotone_and_symmetric(run30):
    X, res = run30
    Fs = [res.F0] + [r.F for r in res.log]
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(Fs, Fs[1:]))
    for it in res.iterates:
        d = (it - it.T)
        assert d.nnz == 0 or np.abs(d.data).max() == 0.0
        assert np.all(it.diagonal() > 0)
    for r in res.log:
        assert r.lhs <= r.rhs


def test_kkt_at_convergence(run30):
    X, res = run30
    S = oc.sample_covariance(X)
    assert res.status == "converged"
    # tol 1e-12 on relative F change leaves a KKT residual well below 1e-4
    assert checks.kkt_residual(res.omega, S, 0.15, 0.1) < 1e-4
    tight = oc.solve(0.15, 0.1, "cov", X=X, tol=0.0, max_iter=3000, check_literal=False)
    assert checks.kkt_residual(tight.omega, S, 0.15, 0.1) < 1e-8


def test_cov_equals_obs():
    X = _small_X(25, 40, 31, deg=4)
    a = oc.solve(0.1, 0.05, "cov", X=X, tol=1e-9, max_iter=100, record_iterates=True)
    b = oc.solve(0.1, 0.05, "obs", X=X, tol=1e-9, max_iter=100, record_iterates=True)
    assert [r.trials for r in a.log] == [r.trials for r in b.log]
    for A, B in zip(a.iterates, b.iterates):
        assert np.abs((A - B).toarray()).max() < 1e-12


def test_difference_form_identity():
    # f(Omega+) - f(Omega) - <G, Delta> equals the difference-form left side
    X = _small_X(20, 30, 41, deg=3)
    S = oc.sample_covariance(X)
    rng = _rng(42)
    om = sp.identity(20, format="csr") * 1.3
    W = np.asarray(om @ S)
    G = oc.gradient(W, om, 0.2)
    for tau in (1.0, 0.25, 0.01):
        cand = oc.prox_step(sp.csr_matrix(om), G + 0.01 * (lambda A: A + A.T)(rng.standard_normal((20, 20))),
                            tau, 0.05)
        if np.any(cand.diagonal() <= 0):
            continue
        lhs, dd = oc.test_difference_terms(om, cand, "cov", 0.2, S=S)
        f0 = oc.smooth_objective(om, 0.2, "cov", S=S)
        f1 = oc.smooth_objective(cand, 0.2, "cov", S=S)
        lin = float(np.sum(G * (cand - om).toarray()))
        assert abs((f1 - f0 - lin) - lhs) < 1e-12 * max(1.0, abs(f0))


def test_replay_reproduces_run(run30):
    X, res = run30
    trials = [r.trials for r in res.log]
    rep = oc.solve(0.15, 0.1, "cov", X=X, fixed_iters=len(trials), tau_replay=trials,
                   record_iterates=True, check_literal=False)
    for A, B in zip(res.iterates, rep.iterates):
        assert np.abs((A - B).toarray()).max() == 0.0


# -------------------------------------------------------------- metamorphic

def test_scaling_identity():
    # Omega_hat(c^2 S; lam1, lam2) = Omega_hat(S; lam1/c, lam2/c^2) / c
    X = _small_X(12, 40, 51, deg=3)
    c = 1.7
    lam1, lam2 = 0.2, 0.1
    a = oc.solve(lam1, lam2, "cov", X=c * X, tol=0.0, max_iter=2000, check_literal=False)
    b = oc.solve(lam1 / c, lam2 / c ** 2, "cov", X=X, tol=0.0, max_iter=2000, check_literal=False)
    assert np.abs(a.omega.toarray() - b.omega.toarray() / c).max() < 1e-6


def test_permutation_equivariance():
    X = _small_X(14, 40, 61, deg=3)
    perm = _rng(62).permutation(14)
    a = oc.solve(0.15, 0.1, "cov", X=X, tol=0.0, max_iter=2000, check_literal=False)
    b = oc.solve(0.15, 0.1, "cov", X=X[:, perm], tol=0.0, max_iter=2000, check_literal=False)
    A = a.omega.toarray()[np.ix_(perm, perm)]
    assert np.abs(A - b.omega.toarray()).max() < 1e-6


# ------------------------------------------------------- differentiation form

def test_smooth_gradients_finite_differences():
    rng = _rng(71)
    p, n = 9, 15
    X = rng.standard_normal((n, p))
    om0 = datagen.random_omega0(p, 3, rng)
    lam2 = 0.1
    f, G, dX = oc.smooth_value_and_grads(om0, X, lam2)
    # f agrees with the Cov form of the same objective
    S = oc.sample_covariance(X)
    assert abs(f - oc.smooth_objective(sp.csr_matrix(om0), lam2, "cov", S=S)) < 1e-12
    h = 1e-6
    D = om0.toarray()
    for (i, j) in [(0, 0), (3, 3), (0, 1), (2, 7), (5, 8)]:
        E = np.zeros((p, p))
        E[i, j] += 1.0
        if i != j:
            E[j, i] += 1.0
        fp = oc.smooth_value_and_grads(sp.csr_matrix(D + h * E), X, lam2)[0]
        fm = oc.smooth_value_and_grads(sp.csr_matrix(D - h * E), X, lam2)[0]
        fd = (fp - fm) / (2 * h)
        want = G[i, j] * (2.0 if i != j else 1.0)
        assert abs(fd - want) < 1e-6 * max(1.0, abs(want)), (i, j, fd, want)
    for (a, b) in [(0, 0), (4, 2), (14, 8)]:
        Xp = X.copy(); Xp[a, b] += h
        Xm = X.copy(); Xm[a, b] -= h
        fd = (oc.smooth_value_and_grads(om0, Xp, lam2)[0] - oc.smooth_value_and_grads(om0, Xm, lam2)[0]) / (2 * h)
        assert abs(fd - dX[a, b]) < 1e-6 * max(1.0, abs(fd))


# ------------------------------------------- planted mistakes must be caught

def test_planted_gradient_mistake_is_caught(monkeypatch):
    """A dropped lam2 term in the gradient must break the diagonal closed form."""
    real = oc.gradient

    def wrong(W, omega, lam2):
        return real(W, omega, 0.0)

    monkeypatch.setattr(oc, "gradient", wrong)
    rng = _rng(7)
    n, p = 40, 6
    Q, _ = np.linalg.qr(rng.standard_normal((n, p)))
    X = Q * math.sqrt(n)
    S = oc.sample_covariance(X)
    res = oc.solve(0.05, 0.5, "cov", X=X, tol=1e-14, max_iter=3000, check_literal=False)
    want = 1.0 / np.sqrt(np.diag(S) + 0.5)
    assert np.abs(res.omega.diagonal() - want).max() > 1e-3


def test_planted_threshold_mistake_is_caught(monkeypatch):
    """Thresholding the diagonal too (eq. (2) over all i, j) contradicts the closed form."""
    def wrong(omega, G, tau, lam1):
        Z = omega.toarray() - tau * G
        out = sp.csr_matrix(oc.soft_threshold(Z, tau * lam1))
        out.eliminate_zeros()
        return out

    monkeypatch.setattr(oc, "prox_step", wrong)
    rng = _rng(8)
    n, p = 40, 6
    Q, _ = np.linalg.qr(rng.standard_normal((n, p)))
    X = Q * math.sqrt(n)
    S = oc.sample_covariance(X)
    res = oc.solve(0.2, 0.1, "cov", X=X, tol=1e-14, max_iter=3000, check_literal=False)
    want = 1.0 / np.sqrt(np.diag(S) + 0.1)
    assert np.abs(res.omega.diagonal() - want).max() > 1e-3


def test_s1_cov_obs_rule_golden():
    # Section S.1 criterion evaluated from its own formula, against the printed thresholds.
    rows = [l.split() for l in open(os.path.join(GOLDEN, "cov_obs_rule_s1.txt"))
            if l.strip() and not l.startswith("#")]
    for r_obs, t, pct in rows:
        r_obs, t, pct = float(r_obs), float(t), float(pct)
        thr = r_obs / (1 - r_obs) / t * 100
        assert abs(thr - pct) < 0.05 + 1e-12, (r_obs, thr, pct)


def test_sampled_grads_match_dense():
    rng = _rng(81)
    p, n = 30, 12
    X = rng.standard_normal((n, p))
    om = datagen.random_omega0(p, 4, rng)
    f, G, dX = oc.smooth_value_and_grads(om, X, 0.1)
    ent = [(0, 0), (3, 7), (7, 3), (29, 29), (5, 11)]
    f2, g2, dx2 = oc.smooth_value_and_sampled_grads(om, X, 0.1, ent, [0, 4, 29])
    assert abs(f - f2) < 1e-12
    assert np.allclose(g2, [G[i, j] for i, j in ent], atol=1e-12)
    assert np.allclose(dx2, dX[:, [0, 4, 29]], atol=1e-12)
