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
