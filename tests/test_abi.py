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
    assert ctypes.sizeof(_lib.concord_config) == 56
    assert cfg.no_screen == 0


@pytest.mark.parametrize("field,value", [("p", 0), ("variant", 7), ("precision", 9),
                                         ("trial_batch", 0), ("trial_batch", 9),
                                         ("max_backtracks", -1), ("n", -3)])
def test_create_rejects_bad_config(lib, field, value):
    from paper_1710_10769_amd import _lib
    cfg = _lib.concord_config_init()
    cfg.p, cfg.n, cfg.variant = 10, 5, _lib.OBS
    setattr(cfg, field, value)
    h = ctypes.c_void_p()
    assert lib.concord_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.EINVAL
    assert not h.value


def test_obs_needs_n(lib):
    from paper_1710_10769_amd import _lib
    cfg = _lib.concord_config_init()
    cfg.p, cfg.n, cfg.variant = 10, 0, _lib.OBS
    h = ctypes.c_void_p()
    assert lib.concord_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.EINVAL


def test_batch_create_rejects_bad_args(lib):
    from paper_1710_10769_amd import _lib
    h = ctypes.c_void_p()
    l1 = (ctypes.c_double * 1)(-1.0)
    ps = (ctypes.c_int64 * 1)(10)
    assert lib.concord_batch_create(1, ps, ps, None, ps, 1, l1, None, ctypes.byref(h)) == _lib.EINVAL
    assert lib.concord_batch_create(0, ps, ps, None, ps, 1, l1, None, ctypes.byref(h)) == _lib.EINVAL


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
    # the benchmark workload (p 20k, n 5k, nearly diagonal): Cov's streaming passes win
    e = _lib.concord_suggest_variant(20000, 5000, 1.0, 3.0, 100, "bf16x3")
    assert e["choice"] == "cov" and e["cov_seconds"] < e["obs_seconds"] / 3
    # very wide p, few samples, dense iterates: Obs
    e = _lib.concord_suggest_variant(200000, 100, 50.0, 3.0, 50, "bf16x3")
    assert e["choice"] == "obs"
    # flop counts are Lemma 3.1's
    p, n, d, t, s = 1000, 200, 5.0, 4.0, 30.0
    e = _lib.concord_suggest_variant(p, n, d, t, s, "fp32")
    assert e["cov_flops"] == 2 * n * p * p + 2 * d * p * p * (s * t + 1)
    assert e["obs_flops"] == 2 * n * p * p * s + 2 * d * n * p * (s * t + 1)
    with pytest.raises(_lib.ConcordError):
        _lib.concord_suggest_variant(0, 10, 1.0, 1.0, 1.0)
