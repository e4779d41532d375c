"""The seeded input generators: structure, exactness and reproducibility."""
import numpy as np
import scipy.sparse as sp

import datagen


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def test_random_omega0_structure():
    om = datagen.random_omega0(500, 10, _rng(3))
    assert (om - om.T).nnz == 0 or abs(om - om.T).max() == 0
    off = om - sp.diags(om.diagonal())
    assert off.nnz == 500 * 10  # exactly p*deg/2 pairs, both triangles
    v = np.abs(off.data)
    assert v.min() >= 0.1 and v.max() <= 0.3
    rows = np.asarray(abs(off).sum(axis=1)).ravel()
    assert np.allclose(om.diagonal() - rows, 0.1)


def test_chain_omega0():
    om = datagen.chain_omega0(6).toarray()
    assert np.allclose(np.diag(om), 1.0) and np.allclose(np.diag(om, 1), 0.4)
    assert np.count_nonzero(om) == 6 + 2 * 5


def test_seed_reproducible():
    a = datagen.make_workload("c1_cov_fp64_p200")
    b = datagen.make_workload("c1_cov_fp64_p200")
    assert np.array_equal(a.X, b.X)
    c = datagen.make_workload("c2_obs_p20000", p=300, n=80)
    d = datagen.make_workload("c2_obs_p20000", p=300, n=80)
    assert np.array_equal(c.X, d.X)
    assert np.allclose(c.X.mean(axis=0), 0, atol=1e-12)
    assert np.allclose((c.X ** 2).mean(axis=0), 1.0)


def test_bbt_factor_exact():
    om = datagen.random_omega0(300, 8, _rng(5))
    B = datagen._bbt_factor(om)
    assert abs(B @ B.T - om).max() < 1e-14


def test_samplers_have_covariance_inverse_omega():
    om = datagen.random_omega0(20, 4, _rng(9))
    inv = np.linalg.inv(om.toarray())
    for X in (datagen.sample_cholesky(om, 40000, _rng(10)),
              datagen.sample_bbt_cg(om, 40000, _rng(11), chunk=5000)):
        C = X.T @ X / X.shape[0]
        assert np.abs(C - inv).max() < 0.05 * np.abs(inv).max()


def test_cg_sampler_solves_exactly():
    # x = Omega0^{-1} B z: check the residual of the linear system for one chunk
    om = datagen.random_omega0(200, 20, _rng(12))
    X = datagen.sample_bbt_cg(om, 3, _rng(13), chunk=3)
    rng = _rng(13)
    B = datagen._bbt_factor(om)
    z = rng.standard_normal((3, B.shape[1]))
    b = B @ z.T
    r = om @ X.T - b
    assert np.abs(r).max() < 1e-10 * np.abs(b).max()


def test_spatial_omega0_blocks_and_dominance():
    blocks = (("sphere", 300), ("sphere", 300), ("ball", 320))
    om = datagen.spatial_omega0(blocks, 6, datagen._rng(6))
    p = 920
    assert om.shape == (p, p)
    assert abs(om - om.T).max() == 0
    A = om.toarray()
    off = A - np.diag(np.diag(A))
    # strictly diagonally dominant with margin 0.1, every coupling negative in [-0.3, -0.1]
    assert np.allclose(np.diag(A), np.abs(off).sum(1) + 0.1)
    nz = off[off != 0]
    assert (nz <= -0.1).all() and (nz >= -0.3).all()
    # no edge between blocks; every vertex has at least its k nearest neighbours
    bounds = np.cumsum([0, 300, 300, 320])
    for b in range(3):
        for c in range(3):
            if b != c:
                assert not off[bounds[b]:bounds[b + 1], bounds[c]:bounds[c + 1]].any()
    assert ((off != 0).sum(1) >= 6).all()


def test_spatial_omega0_is_seeded():
    blocks = (("sphere", 100), ("ball", 120))
    a = datagen.spatial_omega0(blocks, 4, datagen._rng(9))
    b = datagen.spatial_omega0(blocks, 4, datagen._rng(9))
    assert (a != b).nnz == 0


def test_fmri_shape_matches_the_paper():
    assert sum(m for _, m in datagen.FMRI_BLOCKS) == 91282
    assert datagen.FMRI_BLOCKS[0][1] == 29696
    assert len(datagen.FMRI_LAMBDA1) == 11 and len(datagen.FMRI_LAMBDA2) == 8
