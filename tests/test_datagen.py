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
