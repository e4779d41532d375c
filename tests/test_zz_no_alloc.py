"""concord_smooth_value_noalloc (the entry point that allocates nothing) against
concord_smooth_value on a handle: same iterate, same data, two calls in a row with
the second problem smaller, in both precision forms; plus its argument checks."""
import ctypes

import numpy as np
import pytest
import scipy.sparse as sp

import datagen

pytestmark = pytest.mark.gpu


def _case(p, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    om0 = datagen.random_omega0(p, 8, rng)
    X = datagen.sample_cholesky(om0, n, rng)
    om = sp.csr_matrix(datagen.perturb_symmetric(om0, rng, 0.1))
    om.sort_indices()
    return om, X


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_equals_handle_twice(precision):
    import torch
    from paper_1710_10769_amd import Solver, _lib
    dt = torch.float64 if precision == "fp64" else torch.float32
    code = _lib.F64 if precision == "fp64" else _lib.F32
    lam2 = 0.1
    # the second call is smaller than the first; n = 201 leaves a ragged last chunk and
    # the padded leading dimension of the first call is not the row length
    for p, n, pad, seed in ((1500, 700, 8, 61), (333, 201, 3, 62)):
        print(f"[case] noalloc {precision} p={p} n={n} seed={seed}", flush=True)
        om, X = _case(p, n, seed)
        Xd = torch.from_numpy(X).to("cuda", dt)
        rp = torch.from_numpy(om.indptr.astype(np.int64)).cuda()
        cl = torch.from_numpy(om.indices.astype(np.int32)).cuda()
        v = torch.from_numpy(om.data.copy()).cuda()
        s = Solver(p, n, variant="obs", precision=precision)
        s.set_data(Xd)
        s.set_omega(rp, cl, v)
        f_handle = s.smooth_value(lam2)
        s.close()
        vw = 2 if precision == "fp64" else 4
        ldx = -(-(n + pad) // vw) * vw
        Xt = torch.zeros((p, ldx), dtype=dt, device="cuda")
        Xt[:, :n] = Xd.t()
        f_out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        _lib.concord_smooth_value_noalloc(p, n, Xt.data_ptr(), ldx, code, om.nnz, rp.data_ptr(),
                                          cl.data_ptr(), v.data_ptr(), lam2, f_out.data_ptr(),
                                          torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        f_na = float(f_out.item())
        print(f"[case] handle {f_handle!r} noalloc {f_na!r}", flush=True)
        assert f_na == f_handle


def test_noalloc_rejects_bad_arguments():
    """Checked before any launch: sizes, alignment, leading dimension, lambda2, and a
    problem larger than the per-device array."""
    from paper_1710_10769_amd import _lib
    lib = _lib.load()
    fn = lib.concord_smooth_value_noalloc
    good = dict(p=10, n=8, Xt=256, ldx=8, dtype=_lib.F32, nnz=10, rp=512, cl=1024, v=2048,
                lam2=0.1, f=4096)

    def call(**kw):
        a = dict(good, **kw)
        return fn(a["p"], a["n"], a["Xt"], a["ldx"], a["dtype"], a["nnz"], a["rp"], a["cl"],
                  a["v"], a["lam2"], a["f"], None)
    assert call(p=0) == _lib.EINVAL
    assert call(ldx=6) == _lib.EINVAL          # < n
    assert call(ldx=10) == _lib.EINVAL         # not a multiple of 4 (F32)
    assert call(Xt=260) == _lib.EINVAL         # not 16-byte aligned
    assert call(dtype=7) == _lib.EINVAL
    assert call(lam2=-1.0) == _lib.EINVAL
    assert call(f=0) == _lib.EINVAL
    assert call(nnz=5) == _lib.EINVAL          # fewer entries than the diagonal
    assert call(p=2_000_000, nnz=2_000_000) == _lib.EINVAL   # beyond CONCORD_NOALLOC_SCRATCH_BYTES
