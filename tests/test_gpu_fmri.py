"""fMRI-shaped Cov workload (spatial kNN blocks) on the GPU against the oracle.

The recipe of the p = 91,282 workload at a reduced size (blocks and n scaled down),
with the data scaled so that the paper's lambda1 grid samples the non-trivial part
of the path; iterates replayed step by step against the FP64 oracle (FP32 form)."""
import numpy as np
import pytest

import datagen
from oracle import concord as oc
from tests.gpu_common import check_support, max_abs_diff, oracle_grad_fn

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lam1", [0.52, 0.64])
def test_fmri_shaped_cov_replay(lam1):
    import torch
    from paper_1710_10769_amd import Solver
    from paper_1710_10769_amd.path import scale_for_lambda_grid
    w = datagen.make_workload("c6_fmri_cov_p91282", p=1200, n=240)
    X = w.X
    S = X.T @ X / w.n
    m = np.abs(S - np.diag(np.diag(S))).max()
    X = (X * scale_for_lambda_grid(m, 0.80, 0.10)).astype(np.float32).astype(np.float64)
    p, n, lam2, iters = w.p, w.n, 0.10, 8
    print(f"[case] fmri-shaped cov fp32 p={p} n={n} lam1={lam1}", flush=True)
    ref = oc.solve(lam1, lam2, "cov", X=X, fixed_iters=iters, record_iterates=True,
                   check_literal=False)
    assert max(r.nnz for r in ref.log) > p, "case must grow the support"
    s = Solver(p, n, variant="cov", precision="fp32")
    s.set_data(torch.from_numpy(X.astype(np.float32)).cuda())
    prev = s.get_omega_scipy()
    for it, rec in enumerate(ref.log):
        info = s.step_replay(lam1, lam2, rec.trials)
        got, want = s.get_omega_scipy(), ref.iterates[it + 1]
        err = max_abs_diff(got, want)
        assert err <= 1e-4 * np.abs(want.data).max(), (it, err)
        check_support(f"fmri lam1={lam1} it={it}", "fp32", lam1, rec.tau, got, want, prev,
                      ref.iterates[it], s.get_candidates_scipy(),
                      oracle_grad_fn(ref.iterates[it], X, lam2))
        prev = got
        assert abs(info.F - rec.F) <= 1e-5 * abs(rec.F)
    s.close()
