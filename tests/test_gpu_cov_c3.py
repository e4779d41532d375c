"""Cov form at its full size (p = 16,384, n = 4,096, random degree 8): the first
two iterations with the oracle's step sizes replayed, in each precision form,
compared with the FP64 oracle element by element."""
import numpy as np
import pytest

import datagen
from oracle import concord as oc
from tests.gpu_common import check_support, max_abs_diff, oracle_grad_fn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c3():
    import torch
    assert torch.cuda.is_available()
    print("[case] c3 generating p=16384 n=4096 seed=3", flush=True)
    w = datagen.make_workload("c3_cov_p16384", backend="torch", device="cuda")
    X = w.X.astype(np.float32).astype(np.float64)   # every form reads the same values
    print("[case] c3 oracle: S and two iterations", flush=True)
    S = oc.sample_covariance(X)
    ref = oc.solve(w.lam1, w.lam2, "cov", S=S, fixed_iters=2, record_iterates=True,
                   check_literal=False)
    return w, X, ref


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_c3_two_iterations(c3, precision):
    import torch
    from paper_1710_10769_amd import Solver
    w, X, ref = c3
    print(f"[case] c3 {precision} replay {[r.trials for r in ref.log]}", flush=True)
    s = Solver(w.p, w.n, variant="cov", precision=precision)
    s.set_data(torch.from_numpy(X).to("cuda", torch.float64 if precision == "fp64" else torch.float32))
    prev = s.get_omega_scipy()
    for it, rec in enumerate(ref.log):
        info = s.step_replay(w.lam1, w.lam2, rec.trials)
        got = s.get_omega_scipy()
        want = ref.iterates[it + 1]
        err = max_abs_diff(got, want)
        scale = np.abs(want.data).max()
        tol = 1e-6 if precision == "fp64" else 1e-4 * scale
        assert err <= tol, (it, err, tol)
        check_support(f"c3 it={it}", precision, w.lam1, rec.tau, got, want, prev,
                      ref.iterates[it], s.get_candidates_scipy(),
                      oracle_grad_fn(ref.iterates[it], X, w.lam2))
        prev = got
        assert abs(info.F - rec.F) <= (1e-9 if precision == "fp64" else 1e-5) * abs(rec.F)
        assert info.nnz > w.p
    s.close()
