"""Differentiation form on the GPU: forward f(Omega; X), backward d f/d Omega
(on the stored entries) and d f/d X, against the FP64 oracle and finite
differences."""
import numpy as np
import pytest
import scipy.sparse as sp

import datagen
from oracle import concord as oc

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def _say(*a):
    print("[case]", *a, flush=True)


def _csr_tensors(torch, om, dtype):
    om = sp.csr_matrix(om)
    om.sort_indices()
    return (torch.from_numpy(om.indptr.astype(np.int64)).cuda(),
            torch.from_numpy(om.indices.astype(np.int32)).cuda(),
            torch.from_numpy(om.data.copy()).to("cuda", dtype))


def _case(p, n, seed, deg=20):
    rng = np.random.Generator(np.random.PCG64(seed))
    om0 = datagen.random_omega0(p, deg, rng)
    X = datagen.sample_cholesky(om0, n, rng)
    om = datagen.perturb_symmetric(om0, rng, 0.1)
    return om0, om, X


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_forward_backward_vs_oracle_p500(precision):
    torch = _torch()
    from paper_1710_10769_amd import Solver
    from paper_1710_10769_amd.autograd import concord_smooth
    p, n, lam2 = 500, 250, 0.1
    _say(f"autograd {precision} p={p} n={n} seed=55")
    _, om, X = _case(p, n, 55)
    if precision == "fp32":
        X = X.astype(np.float32).astype(np.float64)
    dt = torch.float64 if precision == "fp64" else torch.float32
    f_ref, G_ref, dX_ref = oc.smooth_value_and_grads(om, X, lam2)
    s = Solver(p, n, variant="obs", precision=precision)
    rp, cl, v = _csr_tensors(torch, om, dt)
    v.requires_grad_(True)
    Xt = torch.from_numpy(X).to("cuda", dt).requires_grad_(True)
    f = concord_smooth(v, Xt, rp, cl, lam2, s)
    f.backward()
    tol = 1e-10 if precision == "fp64" else 2e-5
    assert abs(f.item() - f_ref) <= tol * abs(f_ref)
    omc = sp.csr_matrix(om)
    rows = np.repeat(np.arange(p), np.diff(omc.indptr))
    g_ref = G_ref[rows, omc.indices]
    g = v.grad.double().cpu().numpy()
    assert np.abs(g - g_ref).max() <= tol * np.abs(g_ref).max() * (1 if precision == "fp64" else 5)
    dx = Xt.grad.double().cpu().numpy()
    assert np.abs(dx - dX_ref).max() <= tol * np.abs(dX_ref).max() * (1 if precision == "fp64" else 5)
    s.close()


@pytest.mark.parametrize("precision,n,deg", [("fp64", 700, 90), ("fp32", 1100, 70),
                                              ("fp32", 300, 90)])
def test_backward_long_rows_vs_oracle(precision, n, deg):
    """Rows with more than 64 stored entries (the pair walk takes them 64 at a time)
    and, for n past one column block of the row pass (FP64 n > 512, FP32 n > 1024),
    the per-block partial sums."""
    torch = _torch()
    from paper_1710_10769_amd import Solver
    from paper_1710_10769_amd.autograd import concord_smooth
    p, lam2 = 300, 0.1
    _say(f"autograd long rows {precision} p={p} n={n} deg={deg} seed=56")
    _, om, X = _case(p, n, 56, deg=deg)
    assert np.diff(sp.csr_matrix(om).indptr).max() > 64
    if precision == "fp32":
        X = X.astype(np.float32).astype(np.float64)
    dt = torch.float64 if precision == "fp64" else torch.float32
    f_ref, G_ref, dX_ref = oc.smooth_value_and_grads(om, X, lam2)
    s = Solver(p, n, variant="obs", precision=precision)
    rp, cl, v = _csr_tensors(torch, om, dt)
    v.requires_grad_(True)
    Xt = torch.from_numpy(X).to("cuda", dt).requires_grad_(True)
    f = concord_smooth(v, Xt, rp, cl, lam2, s)
    f.backward()
    tol = 1e-10 if precision == "fp64" else 1e-4
    omc = sp.csr_matrix(om)
    rows = np.repeat(np.arange(p), np.diff(omc.indptr))
    g_ref = G_ref[rows, omc.indices]
    g = v.grad.double().cpu().numpy()
    assert np.abs(g - g_ref).max() <= tol * np.abs(g_ref).max()
    dx = Xt.grad.double().cpu().numpy()
    assert np.abs(dx - dX_ref).max() <= tol * np.abs(dX_ref).max()
    s.close()


@pytest.mark.parametrize("precision,n,deg", [("fp32", 1000, 20), ("fp64", 400, 90)])
def test_both_gradients_in_one_pass_equal_separate_passes(precision, n, deg):
    """Asking for both gradients takes the one row pass (each row Y_j gathered once for
    both); its outputs equal those of asking for one at a time bitwise (d f / d X alone
    is the plain SpMM Omega Y, whose FMA order the row pass keeps)."""
    torch = _torch()
    from paper_1710_10769_amd import Solver
    p, lam2 = 333, 0.1
    _say(f"autograd fused vs separate {precision} p={p} n={n} deg={deg} seed=58")
    _, om, X = _case(p, n, 58, deg=deg)
    dt = torch.float64 if precision == "fp64" else torch.float32
    s = Solver(p, n, variant="obs", precision=precision)
    rp, cl, v = _csr_tensors(torch, om, dt)
    s.set_data(torch.from_numpy(X).to("cuda", dt))
    s.set_omega(rp, cl, v)
    g_both, x_both = s.gradient(lam2, want_omega=True, want_x=True, dtype=dt)
    g_only, _ = s.gradient(lam2, want_omega=True, want_x=False, dtype=dt)
    _, x_only = s.gradient(lam2, want_omega=False, want_x=True, dtype=dt)
    assert torch.equal(g_both, g_only) and torch.equal(x_both, x_only)
    s.close()


def test_forward_stores_no_y_and_backward_returns_its_buffers():
    """The forward reduces ||Omega X^T||^2 without forming Y in memory; the backward
    recomputes Y in buffers of its own call and returns them (allocator bridge counts)."""
    torch = _torch()
    from paper_1710_10769_amd import Solver, TorchAllocator
    from paper_1710_10769_amd.autograd import concord_smooth
    p, n, lam2 = 400, 300, 0.1
    _say(f"autograd buffers fp32 p={p} n={n} seed=59")
    _, om, X = _case(p, n, 59, deg=10)
    alloc = TorchAllocator(torch.cuda.current_device())
    s = Solver(p, n, variant="obs", precision="fp32", allocator=alloc)
    rp, cl, v = _csr_tensors(torch, om, torch.float32)
    v.requires_grad_(True)
    x = torch.from_numpy(X).to("cuda", torch.float32).requires_grad_(True)
    f = concord_smooth(v, x, rp, cl, lam2, s)
    live_after_forward = dict(alloc.live)
    dense = (-(-p // 256) * 256) * (-(-n // 64) * 64) * 4   # rows padded to 256, K to 64
    # the handle holds X^T in its dense layout and no second such buffer for Y
    assert sum(1 for b in live_after_forward.values() if b == dense) == 1
    n_before = alloc.n_alloc
    f.backward()
    assert alloc.n_alloc == n_before + 1            # one block: Y, Omega Y and the halves d_ij
    assert alloc.live == live_after_forward         # all of them returned
    f_ref, G_ref, dX_ref = oc.smooth_value_and_grads(om, X.astype(np.float32).astype(np.float64),
                                                     lam2)
    assert abs(f.item() - f_ref) <= 2e-5 * abs(f_ref)
    dx = x.grad.double().cpu().numpy()
    assert np.abs(dx - dX_ref).max() <= 1e-4 * np.abs(dX_ref).max()
    s.close()


def test_incoming_gradient_scales_outputs():
    """backward of c * f returns c times the gradients of f (the unit case skips the
    multiply; any other incoming gradient takes it)."""
    torch = _torch()
    from paper_1710_10769_amd import Solver
    from paper_1710_10769_amd.autograd import concord_smooth
    p, n, lam2 = 203, 120, 0.1   # p % 4 != 0: d f / d X leaves by the element-wise transpose
    _say(f"autograd incoming gradient fp32 p={p} n={n} seed=57")
    _, om, X = _case(p, n, 57, deg=10)
    s = Solver(p, n, variant="obs", precision="fp32")
    rp, cl, v0 = _csr_tensors(torch, om, torch.float32)
    X0 = torch.from_numpy(X).to("cuda", torch.float32)
    grads = []
    for c in (1.0, 2.5):
        v = v0.clone().requires_grad_(True)
        x = X0.clone().requires_grad_(True)
        (c * concord_smooth(v, x, rp, cl, lam2, s)).backward()
        grads.append((v.grad.clone(), x.grad.clone()))
    (gv1, gx1), (gv2, gx2) = grads
    c = torch.tensor(2.5, dtype=torch.float32, device="cuda")
    assert torch.equal(gv2, c * gv1) and torch.equal(gx2, c * gx1)
    f_ref, G_ref, dX_ref = oc.smooth_value_and_grads(om, X.astype(np.float32).astype(np.float64),
                                                     lam2)
    dx = gx1.double().cpu().numpy()
    assert np.abs(dx - dX_ref).max() <= 1e-4 * np.abs(dX_ref).max()
    s.close()


def test_finite_differences_fp64_p500():
    """Symmetric directions on the stored pattern and random directions in X,
    evaluated with the GPU's own forward (central differences)."""
    torch = _torch()
    from paper_1710_10769_amd import Solver
    from paper_1710_10769_amd.autograd import concord_smooth
    p, n, lam2 = 500, 250, 0.1
    _say(f"finite differences fp64 p={p} n={n}")
    _, om, X = _case(p, n, 55)
    s = Solver(p, n, variant="obs", precision="fp64")
    rp, cl, v = _csr_tensors(torch, om, torch.float64)
    Xt = torch.from_numpy(X).cuda()
    v1 = v.clone().requires_grad_(True)
    X1 = Xt.clone().requires_grad_(True)
    concord_smooth(v1, X1, rp, cl, lam2, s).backward()
    gv, gx = v1.grad, X1.grad
    rng = np.random.Generator(np.random.PCG64(5))
    omc = sp.csr_matrix(om)
    for t in range(3):
        # symmetric direction on the pattern
        D = datagen.perturb_symmetric(omc, rng, 1.0) - omc
        D = sp.csr_matrix(D)
        D.sort_indices()
        dvals = np.asarray(D[np.repeat(np.arange(p), np.diff(omc.indptr)), omc.indices]).ravel()
        dv = torch.from_numpy(dvals).cuda()
        h = 1e-6
        fp = concord_smooth(v + h * dv, Xt, rp, cl, lam2, s).item()
        fm = concord_smooth(v - h * dv, Xt, rp, cl, lam2, s).item()
        fd = (fp - fm) / (2 * h)
        an = float((gv * dv).sum())
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (t, fd, an)
        V = torch.from_numpy(rng.standard_normal((n, p))).cuda()
        fp = concord_smooth(v, Xt + h * V, rp, cl, lam2, s).item()
        fm = concord_smooth(v, Xt - h * V, rp, cl, lam2, s).item()
        fd = (fp - fm) / (2 * h)
        an = float((gx * V).sum())
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (t, fd, an)
    s.close()


def test_gradcheck_small():
    torch = _torch()
    from paper_1710_10769_amd import Solver
    from paper_1710_10769_amd.autograd import concord_smooth
    p, n, lam2 = 24, 12, 0.1
    _say(f"gradcheck fp64 p={p} n={n}")
    _, om, X = _case(p, n, 56, deg=4)
    s = Solver(p, n, variant="obs", precision="fp64")
    rp, cl, v = _csr_tensors(torch, om, torch.float64)
    Xt = torch.from_numpy(X).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: concord_smooth(v, x, rp, cl, lam2, s), (Xt,),
                                     eps=1e-6, atol=1e-7, rtol=1e-6)
    # values through a symmetric parametrisation: u holds each upper entry once
    omc = sp.csr_matrix(om)
    rows = np.repeat(np.arange(p), np.diff(omc.indptr))
    cols = omc.indices
    up = rows <= cols
    key = {(int(i), int(j)): k for k, (i, j) in enumerate(zip(rows[up], cols[up]))}
    idx = torch.tensor([key[(min(i, j), max(i, j))] for i, j in zip(rows, cols)]).cuda()
    u = v[torch.from_numpy(np.flatnonzero(up)).cuda()].clone().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda uu: concord_smooth(uu[idx], Xt.detach(), rp, cl, lam2, s),
                                     (u,), eps=1e-6, atol=1e-7, rtol=1e-6)
    s.close()


def test_c5_full_size_sampled():
    """p = 200,000, n = 1,000, FP32: f, sampled G entries and sampled columns of
    d f/d X against the oracle computing them one by one."""
    torch = _torch()
    from paper_1710_10769_amd import Solver
    from paper_1710_10769_amd.autograd import concord_smooth
    _say("c5 full size p=200000 n=1000 deg=20 seed=5: generating (B B^T + CG on the GPU)")
    w = datagen.make_workload("c5_grad_p200000", backend="torch", device="cuda")
    p, n, lam2 = w.p, w.n, w.lam2
    rng = np.random.Generator(np.random.PCG64(505))
    om = datagen.perturb_symmetric(w.omega0, rng, 0.1)
    X = w.X.astype(np.float32).astype(np.float64)
    _say("c5 full size: GPU forward/backward")
    s = Solver(p, n, variant="obs", precision="fp32")
    rp, cl, v = _csr_tensors(torch, om, torch.float32)
    v.requires_grad_(True)
    Xt = torch.from_numpy(X.astype(np.float32)).cuda().requires_grad_(True)
    f = concord_smooth(v, Xt, rp, cl, lam2, s)
    f.backward()
    omc = sp.csr_matrix(om)
    rows = np.repeat(np.arange(p), np.diff(omc.indptr))
    pick = rng.choice(omc.nnz, size=400, replace=False)
    ent = [(int(rows[k]), int(omc.indices[k])) for k in pick]
    ent += [(i, i) for i in rng.choice(p, size=50, replace=False)]
    diag_pos = [omc.indptr[i] + int(np.flatnonzero(omc.indices[omc.indptr[i]:omc.indptr[i + 1]] == i)[0])
                for i, _ in ent[400:]]
    cols = rng.choice(p, size=20, replace=False)
    _say("c5 full size: oracle (sampled)")
    f_ref, g_ref, dx_ref = oc.smooth_value_and_sampled_grads(om, X, lam2, ent, cols)
    assert abs(f.item() - f_ref) <= 1e-5 * abs(f_ref)
    g = v.grad.double().cpu().numpy()
    got = np.concatenate([g[pick], g[diag_pos]])
    assert np.abs(got - g_ref).max() <= 1e-4 * np.abs(g_ref).max()
    dx = Xt.grad.double().cpu().numpy()[:, cols]
    assert np.abs(dx - dx_ref).max() <= 1e-4 * np.abs(dx_ref).max()
    s.close()
