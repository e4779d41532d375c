"""Batched lambda path (Cov; every solve of the batch on the device at once).

Every (instance, lambda1) solve of the batch equals the same solve run alone on the
single solver (bitwise), and every one is checked against the FP64 oracle: the single
solve, stepped one iteration at a time, takes the oracle's step sizes and stops at the
oracle's iteration, and the final iterate is within 1e-4 * max|Omega| of the oracle's.
Graph replay, the number of iterations per replay, candidate-capacity regrowth and
the FP64 form give the same iterates."""
import numpy as np
import pytest
import scipy.sparse as sp

import datagen
from oracle import concord as oc
from tests.gpu_common import max_abs_diff

pytestmark = pytest.mark.gpu


def _csr(r, c, v, p):
    return sp.csr_matrix((v.cpu().numpy(), c.cpu().numpy(), r.cpu().numpy()), shape=(p, p))


def _single(p, X, lam1, lam2, tol, max_iter, precision="fp32"):
    from paper_1710_10769_amd import Solver
    s = Solver(p, X.shape[0], variant="cov", precision=precision)
    s.set_data(X)
    si = s.solve(lam1, lam2, tol, max_iter)
    return s, si


@pytest.mark.timeout(900)
def test_batch_matches_single_solves_and_oracle():
    import torch
    from paper_1710_10769_amd import Batch
    assert torch.cuda.is_available()
    l1s, lam2 = datagen.lambda_path_c4()
    tol, max_iter = 1e-5, 200
    inst = datagen.c4_instances(count=6, scale=0.25)   # p in {250, 500, 1000, 2000}
    ps = [p for p, _, _ in inst]
    print("[case] batch 6 instances x 3 lambda1, p =", ps, flush=True)
    assert max(ps) >= 1000 and len(set(ps)) < len(ps), "sizes must reach 1000 and repeat"
    Xs = [torch.from_numpy(X.astype(np.float32)).cuda() for _, X, _ in inst]
    b = Batch(Xs, l1s)
    iters, Fs, rc = b.solve(lam2, tol, max_iter)
    st = b.stats()
    print("[case] batch stats", st, "iterations", iters, flush=True)
    assert rc >= 0
    # device-side control: one host synchronisation per replay of 4 iterations
    assert st["host_syncs"] == st["launches"] <= -(-max(iters) // 4) + 1
    for i, (p, X, _) in enumerate(inst):
        X64 = X.astype(np.float32).astype(np.float64)
        for l, lam1 in enumerate(l1s):
            print(f"[case] instance {i} p={p} lam1={lam1}", flush=True)
            got = _csr(*b.get_omega(i, l), p)
            s, si = _single(p, Xs[i], lam1, lam2, tol, max_iter)
            assert si.iters == iters[i * len(l1s) + l]
            assert Fs[i * len(l1s) + l] == si.F
            assert max_abs_diff(s.get_omega_scipy(), got) == 0.0   # batch == single, bitwise
            ref = oc.solve(lam1, lam2, "cov", X=X64, tol=tol, max_iter=max_iter,
                           check_literal=False)
            s.reset()
            trials = [s.step(lam1, lam2).n_trials for _ in ref.log]
            assert trials == [r.trials for r in ref.log], (i, l, trials)
            assert si.iters == len(ref.log)
            scale = np.abs(ref.omega.data).max()
            err = max_abs_diff(got, ref.omega)
            print(f"[case] instance {i} lam1={lam1} iters={si.iters} err/scale={err / scale:.2e}",
                  flush=True)
            assert err <= 1e-4 * scale, (i, l, err, scale)
            s.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64", "bf16x3"])
def test_batch_graph_modes_and_regrowth(precision):
    """lambda1 small enough that the candidate sets outgrow their first capacity (the
    host regrows between replays); direct launches, one iteration per replay and four
    give the same iterates, equal to the single solver's (in every precision form: the
    BF16 split forms S from hi/lo planes and stores it as hi/lo pairs, as the single
    solver does)."""
    import torch
    from paper_1710_10769_amd import Batch
    dt = torch.float64 if precision == "fp64" else torch.float32
    inst = datagen.c4_instances(count=3, sizes=(300, 520, 700), scale=1.0)
    l1s, lam2 = [0.05, 0.2], 0.1
    Xs = [torch.from_numpy(X).to("cuda", dt) for _, X, _ in inst]
    runs = []
    for mode in ((True, 4), (True, 1), (False, 3)):
        print(f"[case] batch {precision} graph={mode[0]} iters_per_launch={mode[1]}", flush=True)
        b = Batch(Xs, l1s, precision=precision, use_graph=mode[0], iters_per_launch=mode[1])
        iters, Fs, rc = b.solve(lam2, 1e-6, 60)
        st = b.stats()
        assert st["regrows"] > 0, st
        runs.append((iters, Fs, [[_csr(*b.get_omega(i, l), p) for l in range(len(l1s))]
                                 for i, (p, _, _) in enumerate(inst)]))
        b.close()
    for r in runs[1:]:
        assert r[0] == runs[0][0] and r[1] == runs[0][1]
        for a_, b_ in zip(r[2], runs[0][2]):
            for x, y in zip(a_, b_):
                assert max_abs_diff(x, y) == 0.0
    for i, (p, _, _) in enumerate(inst):
        for l, lam1 in enumerate(l1s):
            s, si = _single(p, Xs[i], lam1, lam2, 1e-6, 60, precision)
            assert si.iters == runs[0][0][i * len(l1s) + l]
            assert max_abs_diff(s.get_omega_scipy(), runs[0][2][i][l]) == 0.0
            s.close()
