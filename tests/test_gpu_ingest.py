"""Data ingest on the GPU: the transpose into the library layout (16-byte and
element-wise forms) and the non-finite check it carries."""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def _say(*a):
    print("[case]", *a, flush=True)


def _omega(s):
    o = s.get_omega_scipy()
    o.sort_indices()
    return o


@pytest.mark.parametrize("variant,precision", [("obs", "fp32"), ("obs", "bf16x3"),
                                               ("cov", "fp32")])
def test_aligned_and_unaligned_ingest_agree(variant, precision):
    """The same X given 16-byte aligned (vector transpose) and as a view one column
    in (element-wise transpose) gives bitwise the same iterates."""
    torch = _torch()
    from paper_1710_10769_amd import Solver
    p, n = 203, 130   # ragged in both tile dimensions and in groups of 4
    _say(f"ingest {variant} {precision} p={p} n={n} seed=2")
    w = datagen.make_workload("c2_obs_p20000", p=p, n=n)
    X = torch.from_numpy(w.X.astype(np.float32)).cuda()
    wide = torch.zeros((n, p + 1), dtype=torch.float32, device="cuda")
    wide[:, 1:] = X
    Xv = wide[:, 1:]                      # data pointer 4 bytes past a 16-byte boundary
    assert Xv.data_ptr() % 16 != 0 and X.data_ptr() % 16 == 0
    out = []
    for data in (X, Xv):
        s = Solver(p, n, variant=variant, precision=precision)
        s.set_data(data)
        for _ in range(3):
            s.step(0.2, 0.1)
        out.append((_omega(s), s.objective(0.2, 0.1)))
        s.close()
    (a, fa), (b, fb) = out
    assert a.nnz == b.nnz and np.array_equal(a.indices, b.indices)
    assert np.array_equal(a.data, b.data)
    assert fa == fb


def test_nonfinite_x_leaves_no_data_then_recovers():
    torch = _torch()
    from paper_1710_10769_amd import Solver
    from paper_1710_10769_amd._lib import ConcordError, ENONFINITE, ENODATA
    p, n = 150, 90
    _say(f"ingest non-finite X obs fp32 p={p} n={n} seed=2")
    w = datagen.make_workload("c2_obs_p20000", p=p, n=n)
    X = torch.from_numpy(w.X.astype(np.float32)).cuda()
    bad = X.clone()
    bad[n - 1, p - 1] = float("nan")      # last element: the ragged corner tile
    ref = Solver(p, n, variant="obs", precision="fp32")
    ref.set_data(X)
    ref.step(0.2, 0.1)
    s = Solver(p, n, variant="obs", precision="fp32")
    s.set_data(X)
    with pytest.raises(ConcordError) as e:
        s.set_data(bad)
    assert e.value.code == ENONFINITE
    with pytest.raises(ConcordError) as e:
        s.step(0.2, 0.1)
    assert e.value.code == ENODATA
    bad[n - 1, p - 1] = float("inf")
    bad[0, 0] = 1.0
    with pytest.raises(ConcordError) as e:
        s.set_data(bad)
    assert e.value.code == ENONFINITE
    s.set_data(X)
    s.step(0.2, 0.1)
    a, b = _omega(s), _omega(ref)
    assert np.array_equal(a.indices, b.indices) and np.array_equal(a.data, b.data)
    s.close()
    ref.close()


def test_nonfinite_s_keeps_previous_data():
    torch = _torch()
    from paper_1710_10769_amd import Solver
    from paper_1710_10769_amd._lib import ConcordError, ENONFINITE
    p, n = 150, 90
    _say(f"ingest non-finite S cov fp64 p={p} n={n} seed=3")
    w = datagen.make_workload("c3_cov_p16384", p=p, n=n)
    S = torch.from_numpy(w.X.T @ w.X / n).cuda()
    bad = S.clone()
    bad[3, 7] = float("nan")
    ref = Solver(p, n, variant="cov", precision="fp64")
    ref.set_covariance(S)
    ref.step(0.3, 0.1)
    s = Solver(p, n, variant="cov", precision="fp64")
    s.set_covariance(S)
    with pytest.raises(ConcordError) as e:
        s.set_covariance(bad)
    assert e.value.code == ENONFINITE
    s.step(0.3, 0.1)
    a, b = _omega(s), _omega(ref)
    assert np.array_equal(a.indices, b.indices) and np.array_equal(a.data, b.data)
    s.close()
    ref.close()
