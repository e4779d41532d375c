"""Seeded synthetic inputs for the CONCORD / PseudoNet proximal-gradient solver.

This module only draws inputs. It holds none of the solver's arithmetic, so the
FP64 oracle (``oracle/``) and the HIP path can both take their inputs from it
without sharing any of the method.

Workloads follow the synthetic recipe of the paper (Section 4, first paragraph):
a banded "chain" or a random, strictly diagonally dominant true precision
matrix Omega0, and Gaussian samples whose rows are N(0, Omega0^{-1}).

Draw order for every workload, from one ``numpy.random.Generator(PCG64(seed))``:
edges -> signs -> magnitudes -> normals Z (n x p, row-major).

Two exact samplers are provided:

* Cholesky: Omega0 = L L^T, X = Z L^{-1}  (rows have covariance Omega0^{-1}).
* B B^T + CG (for p too large for a dense factor): with the diagonal equal to
  the row abs-sum plus delta, Omega0 = B B^T for a sparse B with one column per
  edge plus one per vertex; x = Omega0^{-1} B z with z ~ N(0, I) has covariance
  Omega0^{-1}.  The solve is conjugate gradients to a 1e-13 relative residual.
"""
from __future__ import annotations

import dataclasses
import os
from typing import Optional

import numpy as np
import scipy.sparse as sp

__all__ = [
    "chain_omega0",
    "random_omega0",
    "sample_cholesky",
    "sample_bbt_cg",
    "standardize_columns",
    "Workload",
    "make_workload",
    "WORKLOADS",
    "c4_instances",
    "spatial_omega0",
    "FMRI_BLOCKS",
    "FMRI_LAMBDA1",
    "FMRI_LAMBDA2",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def chain_omega0(p: int, diag: float = 1.0, off: float = 0.4) -> sp.csr_matrix:
    """Tridiagonal chain-graph precision matrix (banded Omega0, Section 4)."""
    if p < 1:
        raise ValueError("p must be >= 1")
    main = np.full(p, diag)
    offd = np.full(max(p - 1, 0), off)
    return sp.diags([offd, main, offd], [-1, 0, 1], shape=(p, p), format="csr")


def _random_pairs(p: int, m: int, rng: np.random.Generator) -> tuple[np.ndarray, np.ndarray]:
    """Exactly m distinct unordered pairs i<j, uniform, in order of first draw."""
    max_pairs = p * (p - 1) // 2
    if m > max_pairs:
        raise ValueError(f"cannot draw {m} distinct pairs from p={p}")
    codes = np.empty(0, dtype=np.int64)
    while codes.size < m:
        need = m - codes.size
        k = max(64, int(need * 1.25) + 16)
        a = rng.integers(0, p, size=k, dtype=np.int64)
        b = rng.integers(0, p, size=k, dtype=np.int64)
        keep = a != b
        a, b = a[keep], b[keep]
        lo = np.minimum(a, b)
        hi = np.maximum(a, b)
        new = lo * p + hi
        allc = np.concatenate([codes, new])
        _, first = np.unique(allc, return_index=True)
        first.sort()
        codes = allc[first][:m]
    return codes // p, codes % p


def random_omega0(p: int, deg: float, rng: np.random.Generator,
                  lo: float = 0.1, hi: float = 0.3, delta: float = 0.1) -> sp.csr_matrix:
    """Random strictly diagonally dominant Omega0 with average off-diagonal degree ``deg``.

    p*deg/2 distinct pairs; |value| ~ U[lo, hi]; sign +-1 with probability 1/2;
    diagonal = row abs-sum + delta.
    """
    m = int(round(p * deg / 2))
    i, j = _random_pairs(p, m, rng)
    signs = np.where(rng.random(m) < 0.5, -1.0, 1.0)
    mags = rng.uniform(lo, hi, size=m)
    v = signs * mags
    rows = np.concatenate([i, j])
    cols = np.concatenate([j, i])
    vals = np.concatenate([v, v])
    off = sp.csr_matrix((vals, (rows, cols)), shape=(p, p))
    d = np.asarray(abs(off).sum(axis=1)).ravel() + delta
    om = (off + sp.diags(d)).tocsr()
    om.sort_indices()
    return om


def sample_cholesky(omega0: sp.spmatrix, n: int, rng: np.random.Generator,
                    backend: str = "numpy", device: Optional[str] = None) -> np.ndarray:
    """n rows ~ N(0, Omega0^{-1}) via the dense Cholesky factor of Omega0 (FP64).

    The normals always come from ``rng`` (host).  The dense factor and the
    triangular solve run in NumPy/SciPy, or in torch on ``device`` (plumbing
    only, for large p); both are FP64 and agree to rounding.
    """
    p = omega0.shape[0]
    z = rng.standard_normal((n, p))
    dense = omega0.toarray()
    if backend == "torch":
        try:
            return _cholesky_torch(dense, z, n, p, device)
        except RuntimeError:
            pass   # device linear algebra unavailable: same factor and solve on the host
    import scipy.linalg as sla
    L = sla.cholesky(dense, lower=True)
    xt = sla.solve_triangular(L.T, z.T, lower=False)
    return np.ascontiguousarray(xt.T)


def _cholesky_torch(dense, z, n, p, device):
    if True:
        import torch
        dev = torch.device(device or "cpu")
        A = torch.from_numpy(dense).to(dev)
        L = torch.linalg.cholesky(A)
        U = L.T.contiguous()
        del A, L
        # X = Z L^{-1}  <=>  X^T = L^{-T} Z^T, solved for blocks of right-hand sides
        x = np.empty((n, p))
        for c0 in range(0, n, 512):
            c1 = min(n, c0 + 512)
            Zt = torch.from_numpy(np.ascontiguousarray(z[c0:c1].T)).to(dev)
            x[c0:c1] = torch.linalg.solve_triangular(U, Zt, upper=True).T.cpu().numpy()
            del Zt
        del U
        return x


def _bbt_factor(omega0: sp.csr_matrix) -> sp.csr_matrix:
    """Sparse B with B B^T = Omega0 for a matrix whose diagonal dominates.

    Each edge e=(i,j) with value a contributes sqrt|a| (e_i + sign(a) e_j); the
    vertex columns carry sqrt(omega_ii - sum_j |omega_ij|).
    """
    coo = sp.triu(omega0, k=1).tocoo()
    p = omega0.shape[0]
    E = coo.nnz
    a = coo.data
    s = np.sqrt(np.abs(a))
    rows = np.concatenate([coo.row, coo.col])
    cols = np.concatenate([np.arange(E), np.arange(E)])
    vals = np.concatenate([s, np.sign(a) * s])
    absrow = np.asarray(abs(omega0 - sp.diags(omega0.diagonal())).sum(axis=1)).ravel()
    slack = omega0.diagonal() - absrow
    if np.any(slack < 0):
        raise ValueError("Omega0 is not diagonally dominant; B B^T sampler needs slack >= 0")
    rows = np.concatenate([rows, np.arange(p)])
    cols = np.concatenate([cols, E + np.arange(p)])
    vals = np.concatenate([vals, np.sqrt(slack)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(p, E + p))


def sample_bbt_cg(omega0: sp.spmatrix, n: int, rng: np.random.Generator,
                  rtol: float = 1e-13, chunk: int = 64, backend: str = "numpy",
                  device: Optional[str] = None, max_iter: int = 2000) -> np.ndarray:
    """n rows ~ N(0, Omega0^{-1}) without a dense factor (B B^T + CG).

    Samples are processed in column chunks of ``chunk`` right-hand sides; the
    normals for chunk c are the rows c*chunk.. of an (n x (E+p)) standard-normal
    matrix drawn row by row, so the result does not depend on ``chunk``.
    """
    om = sp.csr_matrix(omega0)
    B = _bbt_factor(om)
    p, q = B.shape
    out = np.empty((n, p))
    if backend == "torch":
        import torch
        dev = torch.device(device or "cpu")
        Bt = torch.sparse_csr_tensor(torch.from_numpy(B.indptr.astype(np.int64)),
                                     torch.from_numpy(B.indices.astype(np.int64)),
                                     torch.from_numpy(B.data), size=B.shape,
                                     dtype=torch.float64).to(dev)
        At = torch.sparse_csr_tensor(torch.from_numpy(om.indptr.astype(np.int64)),
                                     torch.from_numpy(om.indices.astype(np.int64)),
                                     torch.from_numpy(om.data), size=om.shape,
                                     dtype=torch.float64).to(dev)
        mv = lambda M, v: M @ v  # noqa: E731
        to = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
        back = lambda t: t.cpu().numpy()  # noqa: E731
        dot = lambda a, b: (a * b).sum(dim=0)  # noqa: E731
        Bm, Am = Bt, At
    else:
        mv = lambda M, v: M @ v  # noqa: E731
        to = lambda a: a  # noqa: E731
        back = lambda a: a  # noqa: E731
        dot = lambda a, b: np.einsum("ij,ij->j", a, b)  # noqa: E731
        Bm, Am = B, om
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        z = rng.standard_normal((c1 - c0, q))
        b = mv(Bm, to(np.ascontiguousarray(z.T)))
        x = b * 0.0
        r = b.clone() if backend == "torch" else b.copy()
        d = r.clone() if backend == "torch" else r.copy()
        rr = dot(r, r)
        bnorm2 = rr.clone() if backend == "torch" else rr.copy()
        for _ in range(max_iter):
            Ad = mv(Am, d)
            alpha = rr / dot(d, Ad)
            x = x + d * alpha
            r = r - Ad * alpha
            rr_new = dot(r, r)
            if float((rr_new / bnorm2).max()) < rtol * rtol:
                break
            d = r + d * (rr_new / rr)
            rr = rr_new
        out[c0:c1] = back(x).T
    return out


# fMRI-shaped stand-in (Section 5; Section S.3.1): p = 91,282 coordinates, the left
# hemisphere's 29,696 given by the paper, the right hemisphere taken of the same size
# and the remaining 31,890 as a third (volume) block; the estimates the paper shows are
# block diagonal by hemisphere with spatially nearest coordinates linked.
FMRI_BLOCKS = (("sphere", 29696), ("sphere", 29696), ("ball", 31890))
FMRI_LAMBDA1 = (0.48, 0.5, 0.52, 0.54, 0.57, 0.59, 0.61, 0.64, 0.67, 0.69, 0.72)
FMRI_LAMBDA2 = (0.10, 0.13, 0.16, 0.2, 0.25, 0.31, 0.39, 0.49)


def _sphere_points(m: int) -> np.ndarray:
    """m nearly evenly spaced points on the unit sphere (golden-angle spiral)."""
    t = np.arange(m) + 0.5
    polar = np.arccos(1.0 - 2.0 * t / m)
    azim = np.pi * (1.0 + 5.0 ** 0.5) * t
    return np.c_[np.cos(azim) * np.sin(polar), np.sin(azim) * np.sin(polar), np.cos(polar)]


def _ball_points(m: int, rng: np.random.Generator) -> np.ndarray:
    """m points uniform in the unit ball (radius by inverse CDF, direction Gaussian)."""
    g = rng.standard_normal((m, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return g * rng.random(m)[:, None] ** (1.0 / 3.0)


def _knn_pairs(pts: np.ndarray, k: int) -> tuple[np.ndarray, np.ndarray]:
    """Unordered pairs i<j with j among the k nearest points of i or i among those of j."""
    from scipy.spatial import cKDTree
    m = len(pts)
    _, idx = cKDTree(pts).query(pts, k + 1)
    r = np.repeat(np.arange(m, dtype=np.int64), k)
    c = idx[:, 1:].ravel().astype(np.int64)
    keep = r != c
    r, c = r[keep], c[keep]
    codes = np.unique(np.minimum(r, c) * m + np.maximum(r, c))
    return codes // m, codes % m


def spatial_omega0(blocks, k: int, rng: np.random.Generator, lo: float = 0.1, hi: float = 0.3,
                   delta: float = 0.1) -> sp.csr_matrix:
    """Block-diagonal Omega0 with k-nearest-neighbour graphs on points in space.

    Each block is ("sphere", m) (points on a sphere) or ("ball", m) (points in a ball);
    blocks are independent.  Every edge gets -U[lo, hi] (a positive partial correlation
    between neighbours, like a spatially smooth signal); diagonal = row abs-sum + delta.
    """
    rows, cols, vals = [], [], []
    base = 0
    for kind, m in blocks:
        pts = _sphere_points(m) if kind == "sphere" else _ball_points(m, rng)
        i, j = _knn_pairs(pts, k)
        v = -rng.uniform(lo, hi, size=i.size)
        rows += [i + base, j + base]
        cols += [j + base, i + base]
        vals += [v, v]
        base += m
    off = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                        shape=(base, base))
    d = np.asarray(abs(off).sum(axis=1)).ravel() + delta
    om = (off + sp.diags(d)).tocsr()
    om.sort_indices()
    return om


def fmri_blocks(scale: float = 1.0):
    """FMRI_BLOCKS with every block size multiplied by ``scale`` (at least 16 each)."""
    return tuple((kind, max(16, int(round(m * scale)))) for kind, m in FMRI_BLOCKS)


def standardize_columns(X: np.ndarray) -> np.ndarray:
    """Centre each column and divide by its population standard deviation (1/n)."""
    mu = X.mean(axis=0, keepdims=True)
    Xc = X - mu
    sd = np.sqrt((Xc * Xc).mean(axis=0, keepdims=True))
    sd[sd == 0] = 1.0
    return Xc / sd


@dataclasses.dataclass
class Workload:
    """One synthetic problem: X (n x p, FP64), the true Omega0, and solver settings."""
    name: str
    X: np.ndarray
    omega0: sp.csr_matrix
    lam1: float
    lam2: float
    variant: str          # "cov" or "obs"
    tol: float
    max_iter: int
    fixed_iters: Optional[int] = None
    seed: int = 0

    @property
    def p(self) -> int:
        return self.X.shape[1]

    @property
    def n(self) -> int:
        return self.X.shape[0]


# Recipes of the five workloads (sizes, graphs, penalties, stopping rules).
WORKLOADS = {
    # Cov, FP64, p=200, n=100, chain graph, Cholesky sampler.
    "c1_cov_fp64_p200": dict(p=200, n=100, graph="chain", seed=1, lam1=0.3, lam2=0.1,
                             variant="cov", tol=1e-5, max_iter=200),
    # Obs, p=20,000, n=5,000, random degree 10, standardised columns, 100 iterations.
    "c2_obs_p20000": dict(p=20000, n=5000, graph="random", deg=10, seed=2, lam1=0.4,
                          lam2=0.05, variant="obs", tol=0.0, max_iter=100, fixed_iters=100,
                          standardize=True),
    # Cov, p=16,384, n=4,096, random degree 8.
    "c3_cov_p16384": dict(p=16384, n=4096, graph="random", deg=8, seed=3, lam1=0.3,
                          lam2=0.1, variant="cov", tol=1e-5, max_iter=200),
    # Differentiation form, Obs, p=200,000, n=1,000, random degree 20, B B^T + CG sampler.
    "c5_grad_p200000": dict(p=200000, n=1000, graph="random", deg=20, seed=5, lam1=0.0,
                            lam2=0.1, variant="obs", tol=0.0, max_iter=0, sampler="cg"),
    # fMRI-shaped Cov stand-in (Section 5): three spatial kNN blocks (k = 6), n = 5,142,
    # B B^T + CG sampler, standardised columns; lambda grid FMRI_LAMBDA1 x FMRI_LAMBDA2.
    "c6_fmri_cov_p91282": dict(p=91282, n=5142, graph="spatial", knn=6, seed=6,
                               lam1=0.48, lam2=0.10, variant="cov", tol=1e-5, max_iter=200,
                               sampler="cg", cg_chunk=512, standardize=True),
    # Finite-difference size of the differentiation form.
    "c5_fd_p500": dict(p=500, n=250, graph="random", deg=20, seed=55, lam1=0.0, lam2=0.1,
                       variant="obs", tol=0.0, max_iter=0),
}


def make_workload(name: str, p: Optional[int] = None, n: Optional[int] = None,
                  backend: str = "numpy", device: Optional[str] = None, **over) -> Workload:
    """Build a named workload; ``p``/``n`` override the size (same recipe, smaller shape)."""
    r = dict(WORKLOADS[name])
    r.update(over)
    if p is not None:
        r["p"] = p
    if n is not None:
        r["n"] = n
    rng = _rng(r["seed"])
    if r["graph"] == "chain":
        om = chain_omega0(r["p"])
    elif r["graph"] == "spatial":
        # p overrides scale the three blocks proportionally
        om = spatial_omega0(fmri_blocks(r["p"] / 91282.0), r["knn"], rng)
    else:
        om = random_omega0(r["p"], r["deg"], rng)
    sampler = r.get("sampler", "cholesky")
    if sampler == "cg":
        X = sample_bbt_cg(om, r["n"], rng, backend=backend, device=device,
                          chunk=r.get("cg_chunk", 64))
    else:
        X = sample_cholesky(om, r["n"], rng, backend=backend, device=device)
    if r.get("standardize"):
        X = standardize_columns(X)
    return Workload(name=name, X=X, omega0=om, lam1=r["lam1"], lam2=r["lam2"],
                    variant=r["variant"], tol=r["tol"], max_iter=r["max_iter"],
                    fixed_iters=r.get("fixed_iters"), seed=r["seed"])


def c4_instances(count: int = 48, sizes=(1000, 2000, 4000, 8000), scale: float = 1.0,
                 backend: str = "numpy", device: Optional[str] = None):
    """The batched lambda-path workload: ``count`` instances of uneven p.

    Instance i uses seed 400+i; p ~ U{sizes} (scaled by ``scale`` for small
    test runs); n = p/2; even i chain graph, odd i random degree 6.
    Returns a list of (p, X, omega0).
    """
    out = []
    for i in range(count):
        rng = _rng(400 + i)
        p = int(sizes[int(rng.integers(0, len(sizes)))] * scale)
        p = max(p, 8)
        n = max(p // 2, 2)
        if i % 2 == 0:
            om = chain_omega0(p)
        else:
            om = random_omega0(p, 6, rng)
        X = sample_cholesky(om, n, rng, backend=backend, device=device)
        out.append((p, X, om))
    return out


def lambda_path_c4():
    """lambda1 values of the batched path and its lambda2."""
    return (0.2, 0.3, 0.5), 0.1


def env_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def perturb_symmetric(omega: sp.spmatrix, rng: np.random.Generator, scale: float = 0.1):
    """Omega with every stored value scaled by (1 + scale*U(-1, 1)), the same factor
    for (i, j) and (j, i), so the result stays symmetric with the same pattern."""
    om = sp.csr_matrix(omega, dtype=np.float64).copy()
    coo = sp.triu(om).tocoo()
    fac = 1.0 + scale * rng.uniform(-1.0, 1.0, size=coo.nnz)
    up = sp.csr_matrix((coo.data * fac, (coo.row, coo.col)), shape=om.shape)
    low = sp.triu(up, k=1).T
    out = (up + low).tocsr()
    out.sort_indices()
    return out
