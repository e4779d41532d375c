"""The C-ABI library loads on the CPU and exports every symbol the header declares.

Error paths that are decided before any GPU work (argument validation) are
exercised here too; nothing below launches a kernel.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "concord.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(concord_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1710_10769_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import paper_1710_10769_amd.build as b
        b.build()
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    from paper_1710_10769_amd import _lib
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTED) | {"concord_config_init"}


def test_version_and_null_handles(lib):
    from paper_1710_10769_amd import _lib
    assert "gfx950" in _lib.concord_version()
    assert lib.concord_last_error(None) == b"null handle"
    lib.concord_destroy(None)
    lib.concord_batch_destroy(None)
    si = _lib.concord_step_info()
    assert lib.concord_step(None, 0.1, 0.1, ctypes.byref(si)) == _lib.EINVAL
    assert lib.concord_solve(None, 0.1, 0.1, 1e-5, 10, None) == _lib.EINVAL
    assert lib.concord_reset(None) == _lib.EINVAL
    nnz = ctypes.c_int64()
    assert lib.concord_get_omega(None, ctypes.byref(nnz), None, None, None, 0) == _lib.EINVAL
    assert lib.concord_contraction_variant(None, None, 0) == _lib.EINVAL
    assert lib.concord_refresh_screen_stats(None, 0.1, None, None) == _lib.EINVAL


def test_config_defaults(lib):
    from paper_1710_10769_amd import _lib
    cfg = _lib.concord_config_init()
    assert (cfg.variant, cfg.precision, cfg.device) == (_lib.COV, _lib.FP64, -1)
    assert (cfg.max_backtracks, cfg.trial_batch) == (60, 8)
    assert ctypes.sizeof(_lib.concord_config) == 96
    assert cfg.no_screen == 0
    assert (cfg.tau0, cfg.shrink) == (1.0, 0.5)
    assert not cfg.alloc_fn and not cfg.free_fn and not cfg.alloc_user


@pytest.mark.parametrize("field,value", [("p", 0), ("variant", 7), ("variant", -1), ("precision", 9),
                                         ("trial_batch", 0), ("trial_batch", 9),
                                         ("max_backtracks", -1), ("n", -3), ("tau0", 0.0),
                                         ("tau0", float("inf")), ("shrink", 1.0),
                                         ("shrink", 0.0)])
def test_create_rejects_bad_config(lib, field, value):
    from paper_1710_10769_amd import _lib
    cfg = _lib.concord_config_init()
    cfg.p, cfg.n, cfg.variant = 10, 5, _lib.OBS
    setattr(cfg, field, value)
    h = ctypes.c_void_p()
    assert lib.concord_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.EINVAL
    assert not h.value


def test_allocator_bridge_needs_both_callbacks(lib):
    """alloc_fn without free_fn (or the reverse) is rejected before any device work."""
    from paper_1710_10769_amd import _lib
    keep = _lib.ALLOC_FN(lambda user, n, s: None), _lib.FREE_FN(lambda user, p, n, s: None)
    for which in (0, 1):
        cfg = _lib.concord_config_init()
        cfg.p, cfg.n, cfg.variant = 10, 5, _lib.OBS
        if which == 0:
            cfg.alloc_fn = keep[0]
        else:
            cfg.free_fn = keep[1]
        h = ctypes.c_void_p()
        assert lib.concord_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.EINVAL
        assert not h.value


def test_candidates_need_a_handle(lib):
    from paper_1710_10769_amd import _lib
    nnz = ctypes.c_int64()
    assert lib.concord_get_candidates(None, ctypes.byref(nnz), None, None, None, None) == _lib.EINVAL


def test_obs_and_auto_need_n(lib):
    from paper_1710_10769_amd import _lib
    for v in (_lib.OBS, _lib.AUTO):
        cfg = _lib.concord_config_init()
        cfg.p, cfg.n, cfg.variant = 10, 0, v
        h = ctypes.c_void_p()
        assert lib.concord_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.EINVAL
    assert lib.concord_variant_of(None) == _lib.EINVAL


def test_batch_create_rejects_bad_args(lib):
    from paper_1710_10769_amd import _lib
    h = ctypes.c_void_p()
    l1 = (ctypes.c_double * 1)(-1.0)
    ps = (ctypes.c_int64 * 1)(10)
    assert lib.concord_batch_create(None, 1, ps, ps, None, ps, 1, l1, ctypes.byref(h)) == _lib.EINVAL
    assert lib.concord_batch_create(None, 0, ps, ps, None, ps, 1, l1, ctypes.byref(h)) == _lib.EINVAL
    cfg = _lib.concord_batch_config()
    lib.concord_batch_config_init(ctypes.byref(cfg))
    assert (cfg.precision, cfg.trial_batch, cfg.iters_per_launch, cfg.use_graph) == (_lib.FP32, 8, 4, 1)
    X = (ctypes.c_void_p * 1)(4096)
    l1 = (ctypes.c_double * 1)(0.2)
    for field, value in (("precision", 3), ("iters_per_launch", 0), ("trial_batch", 9),
                         ("shrink", 1.5)):
        bad = _lib.concord_batch_config()
        lib.concord_batch_config_init(ctypes.byref(bad))
        setattr(bad, field, value)
        assert lib.concord_batch_create(ctypes.byref(bad), 1, ps, ps, X, ps, 1, l1,
                                        ctypes.byref(h)) == _lib.EINVAL
        assert not h.value


def test_missing_library_fails_loudly(tmp_path):
    from paper_1710_10769_amd import _lib
    saved = _lib._lib
    try:
        _lib._lib = None
        with pytest.raises(RuntimeError, match="not built"):
            _lib.load(str(tmp_path / "nope.so"))
    finally:
        _lib._lib = saved


def test_suggest_variant_lemma_3_1_rule(lib):
    """The flop rule reproduces Section S.1's printed thresholds: with t = 10 and
    many iterations, Cov has fewer flops while r_nnz < r_obs / (1 - r_obs) / t."""
    from paper_1710_10769_amd import _lib
    p, t, s = 20000, 10.0, 1e6
    for r_obs, pct in ((0.01, 0.1), (0.10, 1.1), (0.25, 3.3)):
        n = int(r_obs * p)
        thr = r_obs / (1 - r_obs) / t          # relaxed form (S.2)
        below = _lib.concord_suggest_variant(p, n, 0.9 * thr * p, t, s)
        above = _lib.concord_suggest_variant(p, n, 1.1 * thr * p, t, s)
        assert below["paper_choice"] == "cov" and above["paper_choice"] == "obs", (r_obs, below, above)
        assert abs(thr * 100 - pct) < 0.05


def test_suggest_variant_time_model(lib):
    from paper_1710_10769_amd import _lib
    # the benchmark workload (p 20k, n 5k, nearly diagonal): Cov's streaming passes win,
    # even priced without screening
    e = _lib.concord_suggest_variant(20000, 5000, 1.0, 3.0, 100, "bf16x3")
    assert e["choice"] == "cov" and e["cov_seconds"] < e["obs_seconds"] / 3
    # the model's terms: S once, then per iteration the kept S tiles and the words (Cov);
    # the contraction and its dense result and Y (Obs)
    p, n, s, R, B = 1000.0, 200.0, 30.0, 100e12, 2000e9
    e = _lib.concord_suggest_variant(1000, 200, 5.0, 3.0, s, "fp32", R / 1e12, B / 1e9, 0.25)
    assert abs(e["cov_seconds"] - (n * p * p / R + s * (0.25 * p * p * 4 + 0.25 * p * p) / B)) < 1e-15
    assert abs(e["obs_seconds"] - s * (2 * n * p * p / R + (2 * p * p * 4 + 2 * p * n * 4) / B)) < 1e-15
    # screening lowers only Cov's price
    e1 = _lib.concord_suggest_variant(1000, 200, 5.0, 3.0, s, "fp32", 100.0, 2000.0, 1.0)
    assert e1["cov_seconds"] > e["cov_seconds"] and e1["obs_seconds"] == e["obs_seconds"]
    # Obs stores its dense contraction result every iteration and forms 2np^2 flops where
    # Cov forms S once with np^2: priced this way Cov wins at every shape, although the
    # flop rule of Lemma 3.1 picks Obs for few samples and many iterations
    for (p_, n_, s_) in ((20000, 5000, 100), (20000, 8, 30), (200000, 100, 50), (500, 400, 1)):
        e = _lib.concord_suggest_variant(p_, n_, 5.0, 3.0, s_, "fp32", 1.0, 8000.0)
        assert e["choice"] == "cov" and e["cov_seconds"] < e["obs_seconds"], (p_, n_, s_)
    e = _lib.concord_suggest_variant(20000, 100, 50.0, 3.0, 30, "bf16x3")
    assert e["paper_choice"] == "obs" and e["choice"] == "cov"
    # flop counts are Lemma 3.1's
    p, n, d, t, s = 1000, 200, 5.0, 4.0, 30.0
    e = _lib.concord_suggest_variant(p, n, d, t, s, "fp32")
    assert e["cov_flops"] == 2 * n * p * p + 2 * d * p * p * (s * t + 1)
    assert e["obs_flops"] == 2 * n * p * p * s + 2 * d * n * p * (s * t + 1)
    with pytest.raises(_lib.ConcordError):
        _lib.concord_suggest_variant(0, 10, 1.0, 1.0, 1.0)
