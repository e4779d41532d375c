"""lambda1 search to a target degree and support recovery on the GPU."""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


def test_lambda1_search_hits_target_degree():
    import torch
    from paper_1710_10769_amd import Solver
    from paper_1710_10769_amd.path import lambda1_for_degree, support_recovery
    rng = np.random.Generator(np.random.PCG64(77))
    p, n, deg = 400, 800, 6
    om0 = datagen.random_omega0(p, deg, rng)
    X = datagen.sample_cholesky(om0, n, rng)
    print(f"[case] lambda1 search p={p} n={n} target degree {deg}", flush=True)
    s = Solver(p, n, variant="cov", precision="fp32")
    s.set_data(torch.from_numpy(X.astype(np.float32)).cuda())
    res = lambda1_for_degree(s, float(deg), 0.1, lo=0.0, hi=1.0, rel_tol=0.05)
    assert abs(res.degree - deg) <= 0.05 * deg, res.history
    rec = support_recovery(res.omega, om0)
    # n = 2p samples of a degree-6 graph: well above chance (an estimate of the same
    # size drawn at random would score PPV ~ deg / (p - 1) = 0.015)
    assert rec["ppv"] > 0.5 and rec["recall"] > 0.5, rec
    assert abs(rec["ppv"] + rec["fdr"] - 1.0) < 1e-12
    s.close()
