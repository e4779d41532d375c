"""lambda1 search to a target degree and support recovery on the GPU: the batched
multisection against the oracle's own search (same bracket, probes and stop rule) in
FP64, and the single-handle bisection in FP32."""
import numpy as np
import pytest

import datagen
from oracle import concord as oc

pytestmark = pytest.mark.gpu


def test_batched_search_equals_oracle_search_fp64():
    import torch
    from paper_1710_10769_amd.path import lambda1_for_degree_batched, support_recovery
    rng = np.random.Generator(np.random.PCG64(78))
    p, n, deg = 200, 400, 6
    om0 = datagen.random_omega0(p, deg, rng)
    X = datagen.sample_cholesky(om0, n, rng)
    kw = dict(lo=0.0, hi=0.6, probes=6, rounds=4, rel_tol=0.01, tol=1e-5, max_iter=200)
    print(f"[case] batched lambda1 search fp64 p={p} n={n} target degree {deg}", flush=True)
    res = lambda1_for_degree_batched(torch.from_numpy(X).cuda(), float(deg), 0.1,
                                     precision="fp64", **kw)
    lam_o, deg_o, om_o, hist_o = oc.lambda1_search(X, float(deg), 0.1, **kw)
    print("[case] gpu", res.history, "\n[case] oracle", hist_o, flush=True)
    assert [h[:2] for h in res.history] == [h[:2] for h in hist_o]
    assert [h[2] for h in res.history] == [h[2] for h in hist_o]   # iterations too
    assert (res.lam1, res.degree) == (lam_o, deg_o)
    rec = support_recovery(res.omega, om0)
    ppv_o, fdr_o = oc.edge_scores(om_o, om0)
    assert (rec["ppv"], rec["fdr"]) == (ppv_o, fdr_o)
    assert abs(res.degree - deg) <= 0.1 * deg


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
