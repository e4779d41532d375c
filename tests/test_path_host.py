"""Host logic of the lambda1 search and support scoring (no GPU)."""
import numpy as np
import scipy.sparse as sp

from paper_1710_10769_amd.path import average_degree, support_recovery


def test_support_recovery_counts():
    truth = sp.csr_matrix(np.array([[2, 1, 0, 0], [1, 2, 1, 0], [0, 1, 2, 1], [0, 0, 1, 2]], float))
    est = sp.csr_matrix(np.array([[2, 1, 0, 1], [1, 2, 0, 0], [0, 0, 2, 1], [1, 0, 1, 2]], float))
    r = support_recovery(est, truth)
    # estimated edges {01, 03, 23}; true {01, 12, 23}
    assert (r["tp"], r["fp"], r["fn"]) == (2, 1, 1)
    assert abs(r["ppv"] - 2 / 3) < 1e-15 and abs(r["fdr"] - 1 / 3) < 1e-15
    assert abs(r["ppv"] + r["fdr"] - 1) < 1e-15
    assert support_recovery(sp.identity(4), truth)["ppv"] == 0.0


def test_average_degree():
    m = sp.csr_matrix(np.array([[1, 1, 0], [1, 1, 1], [0, 1, 1]], float))
    assert average_degree(m) == 4 / 3


def test_scale_for_lambda_grid_hits_the_threshold():
    from paper_1710_10769_amd.path import scale_for_lambda_grid
    for m, a, b in [(0.6, 0.8, 0.1), (0.3, 0.72, 0.49), (0.9, 0.5, 0.0)]:
        c = scale_for_lambda_grid(m, a, b)
        # threshold of the scaled problem: c^2 m / sqrt(c^2 + lambda2)
        assert abs(c * c * m / (c * c + b) ** 0.5 - a) < 1e-12


def test_scale_for_lambda_grid_matches_the_diagonal_optimum():
    """At the computed scale the oracle's lambda1_max closed form equals the target."""
    import numpy as np
    from oracle import checks
    from paper_1710_10769_amd.path import scale_for_lambda_grid
    rng = np.random.Generator(np.random.PCG64(3))
    X = rng.standard_normal((50, 6))
    X = (X - X.mean(0)) / X.std(0)
    S = X.T @ X / 50
    m = np.abs(S - np.diag(np.diag(S))).max()
    c = scale_for_lambda_grid(m, 0.8, 0.1)
    assert abs(checks.lambda1_max(c * c * S, 0.1) - 0.8) < 1e-12


def test_oracle_multisection_probes_and_selection():
    """One round of three probes at 0.1, 0.2, 0.3 with the target set to the degree the
    oracle reaches at 0.2 returns exactly that lambda1 and degree."""
    import datagen
    from oracle import concord as oc
    rng = np.random.Generator(np.random.PCG64(9))
    om0 = datagen.random_omega0(30, 4, rng)
    X = datagen.sample_cholesky(om0, 60, rng)
    r = oc.solve(0.2, 0.1, "cov", X=X, tol=1e-5, max_iter=200, check_literal=False)
    target = (r.omega.nnz - 30) / 30
    lam, deg, om, hist = oc.lambda1_search(X, target, 0.1, lo=0.0, hi=0.4, probes=3, rounds=1,
                                           rel_tol=0.0)
    assert [h[0] for h in hist] == [0.1, 0.2, 0.30000000000000004] or \
        [round(h[0], 12) for h in hist] == [0.1, 0.2, 0.3]
    assert lam == 0.2 and deg == target
    assert hist[0][1] >= hist[1][1] >= hist[2][1]   # the degree falls as lambda1 grows


def test_next_bracket():
    from paper_1710_10769_amd.path import multisection_round, next_bracket
    lams = multisection_round(0.0, 1.0, 4)
    assert lams == [0.2, 0.4, 0.6, 0.8]
    assert next_bracket(0.0, 1.0, lams, [9, 7, 5, 3], 6) == (0.4, 0.6)
    assert next_bracket(0.0, 1.0, lams, [5, 4, 3, 2], 6) == (0.0, 0.2)
    assert next_bracket(0.0, 1.0, lams, [9, 8, 7, 7], 6) == (0.8, 1.0)
