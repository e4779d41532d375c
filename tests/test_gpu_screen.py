"""The Cov refresh's exact tile screening (GPU, through the C-ABI).

The refresh skips the S loads of a pair of 64 x 64 tiles when a bound on |M_ij| over
the pair is at most lambda1; the candidate words of a skipped pair are provably empty.
These tests build a banded covariance (large entries near the diagonal, tiny ones
elsewhere), so most pairs are skipped, and check
  * the number of pairs that loaded S against the bound recomputed on the host, and
  * the candidate count of a step from Omega = I against the dense count
    |{(i, j) : i == j or |S_ij| > lambda1}| (at Omega = I, M = S), with lambda1 placed
    away from every |S_ij| so the count does not depend on rounding.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _banded_cov(p, seed):
    """Exactly symmetric S: rho^|i-j| within distance 3, +-1e-3 noise elsewhere."""
    rng = np.random.default_rng(seed)
    noise = rng.uniform(-1e-3, 1e-3, size=(p, p))
    S = (noise + noise.T) * 0.5
    i = np.arange(p)
    d = np.abs(i[:, None] - i[None, :])
    near = d <= 3
    S[near] = (0.6 ** d)[near]
    return S


def _tile_max(S):
    p = S.shape[0]
    T = (p + 63) // 64
    A = np.zeros((T * 64, T * 64))
    A[:p, :p] = np.abs(S)
    return A.reshape(T, 64, T, 64).max(axis=(1, 3))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("p", [700, 1000])
def test_screen_stats_match_host_bound_at_identity(precision, p):
    import torch
    from paper_1710_10769_amd import Solver
    _say(f"screen stats {precision} p={p} seed=11")
    S = _banded_cov(p, 11)
    dt = torch.float64 if precision == "fp64" else torch.float32
    Sd = S if precision == "fp64" else S.astype(np.float32).astype(np.float64)
    lam1 = 0.3
    s = Solver(p, 1, variant="cov", precision=precision)
    s.set_covariance(torch.from_numpy(np.ascontiguousarray(S)).to("cuda", dt))
    pairs, active = s.refresh_screen_stats(lam1)
    s.close()
    T = (p + 63) // 64
    assert pairs == T * (T + 1) // 2
    # at Omega = I: bound(I, J) = (smax[I, J] + smax[J, I]) / 2 = smax[I, J]; the kernel
    # widens by 1.01 + 3 * 2^-23 (one nonzero per row) and skips when <= threshold
    sm = _tile_max(Sd)
    widen = 1.01 + 3 * 2.0 ** -23
    iu = np.triu_indices(T, 1)
    b = sm[iu] * widen
    thr = lam1 if precision == "fp64" else float(np.float32(lam1))
    if precision == "fp32" and thr > lam1:
        thr = float(np.nextafter(np.float32(lam1), np.float32(0)))
    # rounding of the bound itself may move a pair sitting exactly at the threshold
    lo = int((b > thr * (1 + 1e-9)).sum()) + T
    hi = int((b > thr * (1 - 1e-9)).sum()) + T
    assert lo <= active <= hi, (active, lo, hi)
    assert active < pairs   # the banded S must actually be screened


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_screened_step_keeps_every_candidate(precision):
    import torch
    from paper_1710_10769_amd import Solver
    p = 1000
    _say(f"screened candidates {precision} p={p} seed=12")
    S = _banded_cov(p, 12)
    Sd = S if precision == "fp64" else S.astype(np.float32).astype(np.float64)
    # lambda1 between 0.6^2 = 0.36 and 0.6 = 0.6: the |i - j| = 1 entries pass, the rest fail
    lam1 = 0.45
    a = np.abs(Sd)
    assert np.min(np.abs(a - lam1)) > 1e-3
    dense = int(((a > lam1) | np.eye(p, dtype=bool)).sum())
    dt = torch.float64 if precision == "fp64" else torch.float32
    s = Solver(p, 1, variant="cov", precision=precision)
    s.set_covariance(torch.from_numpy(np.ascontiguousarray(S)).to("cuda", dt))
    info = s.step(lam1, 0.1)
    pairs, active = s.refresh_screen_stats(lam1)
    s.close()
    assert info.n_candidates == dense
    assert active < pairs


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("source", ["banded_S", "random_X"])
def test_screening_does_not_change_the_solve(precision, source):
    """Screened and unscreened refreshes give bitwise the same iterates."""
    import torch
    import datagen
    from paper_1710_10769_amd import Solver
    p = 1000 if source == "banded_S" else 900
    _say(f"screen on/off {precision} {source} p={p}")
    dt = torch.float64 if precision == "fp64" else torch.float32
    if source == "banded_S":
        # (a supplied S is held in FP32 by the BF16-split form as well)
        data = torch.from_numpy(np.ascontiguousarray(_banded_cov(p, 13))).to("cuda", dt)
        lam1, lam2, n = 0.45, 0.1, 1
    else:
        w = datagen.make_workload("c3_cov_p16384", p=p, n=400)
        data = torch.from_numpy(np.ascontiguousarray(w.X)).to("cuda", dt)
        lam1, lam2, n = w.lam1, w.lam2, 400
    out = []
    for screen in (True, False):
        s = Solver(p, n, variant="cov", precision=precision, screen=screen)
        if source == "banded_S":
            s.set_covariance(data)
        else:
            s.set_data(data)
        # step by step, with a lambda1 change in the middle: the candidate counts must match
        # too (stale candidate words of screened-out tiles would show up as extra candidates)
        seq = [lam1] * 8 + [lam1 * 1.3] * 4 + [lam1] * 4
        steps = [s.step(l1, lam2) for l1 in seq]
        info = s.solve(lam1, lam2, 1e-7, 40)
        om = s.get_omega_scipy()
        out.append(([(i.tau, i.F, i.nnz, i.n_candidates) for i in steps], info.iters, info.F,
                     info.nnz, om))
        s.close()
    (t0, i0, F0, z0, o0), (t1, i1, F1, z1, o1) = out
    assert t0 == t1
    assert (i0, z0) == (i1, z1)
    assert F0 == F1
    assert np.array_equal(o0.indptr, o1.indptr) and np.array_equal(o0.indices, o1.indices)
    assert np.array_equal(o0.data, o1.data)
