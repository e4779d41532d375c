"""Batched lambda path (Cov, FP32 products, FP64 reductions): every (instance,
lambda1) solve equals the same solve run alone, and one instance is checked
against the FP64 oracle."""
import numpy as np
import pytest

import datagen
from oracle import concord as oc
from tests.gpu_common import max_abs_diff

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("workers", [None, "1"])
def test_batch_matches_single_solves_and_oracle(workers, monkeypatch):
    """With one worker every instance of a shape after the first reuses that
    worker's handle; the results must not depend on it."""
    import torch
    from paper_1710_10769_amd import Batch, Solver
    assert torch.cuda.is_available()
    if workers:
        monkeypatch.setenv("CONCORD_BATCH_WORKERS", workers)
    l1s, lam2 = datagen.lambda_path_c4()
    inst = datagen.c4_instances(count=6, scale=0.05)   # p in {50, 100, 200, 400}
    print("[case] batch 6 instances, workers", workers, "p =", [p for p, _, _ in inst],
          flush=True)
    assert len({p for p, _, _ in inst}) < len(inst), "some shape must repeat"
    Xs = [torch.from_numpy(X.astype(np.float32)).cuda() for _, X, _ in inst]
    b = Batch(Xs, l1s)
    iters, Fs, rc = b.solve(lam2, 1e-5, 200)
    assert rc >= 0
    for i, (p, X, _) in enumerate(inst):
        for l, lam1 in enumerate(l1s):
            r, c, v = b.get_omega(i, l)
            s = Solver(p, X.shape[0], variant="cov", precision="fp32")
            s.set_data(Xs[i])
            si = s.solve(lam1, lam2, 1e-5, 200)
            assert si.iters == iters[i * len(l1s) + l]
            om1 = s.get_omega_scipy()
            import scipy.sparse as sp
            om2 = sp.csr_matrix((v.cpu().numpy(), c.cpu().numpy(), r.cpu().numpy()), shape=(p, p))
            assert max_abs_diff(om1, om2) == 0.0
            s.close()
    # instance 1 at lambda1[0] against the oracle (converged solutions)
    p, X, _ = inst[1]
    X64 = X.astype(np.float32).astype(np.float64)
    ref = oc.solve(l1s[0], lam2, "cov", X=X64, tol=1e-5, max_iter=200, check_literal=False)
    r, c, v = b.get_omega(1, 0)
    import scipy.sparse as sp
    om = sp.csr_matrix((v.cpu().numpy(), c.cpu().numpy(), r.cpu().numpy()), shape=(p, p))
    assert max_abs_diff(om, ref.omega) <= 1e-3 * np.abs(ref.omega.data).max()
    b.close()
