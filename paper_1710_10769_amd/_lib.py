"""ctypes binding of libconcord (include/concord.h).

Argument marshalling only: every step of the iteration runs in the HIP
kernels of the library.  The module-level functions carry the C names; the
``Solver`` class wraps a handle for torch tensors (device memory and the
current HIP stream come from PyTorch).

The library must have been built (``python -m paper_1710_10769_amd.build``);
importing a function of this module without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libconcord.so")

OK, WMAXITER = 0, 1
EINVAL, ENOMEM, EHIP, ENOTPD, ENONFINITE, ELINESEARCH, ENODATA = -1, -2, -3, -4, -5, -6, -7
COV, OBS, AUTO = 0, 1, 2
FP64, FP32, BF16X3 = 0, 1, 2
F64, F32 = 0, 1
DATA_X, DATA_S = 0, 1
GRAD_MASKED, GRAD_DENSE = 0, 1

_CODES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EHIP: "EHIP", ENOTPD: "ENOTPD",
          ENONFINITE: "ENONFINITE", ELINESEARCH: "ELINESEARCH", ENODATA: "ENODATA"}

_VARIANTS = {"cov": COV, "obs": OBS, "auto": AUTO}
_PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}


class ConcordError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


# allocator bridge: void* alloc(void* user, size_t bytes, void* stream);
#                   void free(void* user, void* ptr, size_t bytes, void* stream)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                           ctypes.c_void_p)


class concord_config(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int64), ("n", ctypes.c_int64), ("variant", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("device", ctypes.c_int32), ("max_backtracks", ctypes.c_int32),
                ("trial_batch", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("no_screen", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tau0", ctypes.c_double), ("shrink", ctypes.c_double),
                ("alloc_fn", ALLOC_FN), ("free_fn", FREE_FN), ("alloc_user", ctypes.c_void_p)]


class concord_step_info(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("tau", ctypes.c_double), ("n_trials", ctypes.c_int32),
                ("n_batches", ctypes.c_int32), ("f", ctypes.c_double), ("F", ctypes.c_double),
                ("nnz", ctypes.c_int64), ("delta_fro", ctypes.c_double),
                ("n_candidates", ctypes.c_int64), ("lhs", ctypes.c_double),
                ("rhs", ctypes.c_double)]


class concord_profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 8), ("launches", ctypes.c_int64 * 8)]


PROF_CLASSES = ("dense", "spmm", "cand", "trial", "emit", "refresh")


class concord_variant_estimate(ctypes.Structure):
    _fields_ = [("paper_choice", ctypes.c_int32), ("choice", ctypes.c_int32),
                ("cov_flops", ctypes.c_double), ("obs_flops", ctypes.c_double),
                ("cov_seconds", ctypes.c_double), ("obs_seconds", ctypes.c_double)]


class concord_batch_config(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("device", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("max_backtracks", ctypes.c_int32),
                ("trial_batch", ctypes.c_int32), ("tau0", ctypes.c_double),
                ("shrink", ctypes.c_double), ("iters_per_launch", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("alloc_fn", ALLOC_FN), ("free_fn", FREE_FN),
                ("alloc_user", ctypes.c_void_p)]


class concord_batch_stats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("host_syncs", ctypes.c_int64),
                ("iterations_launched", ctypes.c_int64), ("regrows", ctypes.c_int64),
                ("s_ms", ctypes.c_double), ("iterate_ms", ctypes.c_double)]


class concord_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("f", ctypes.c_double), ("F", ctypes.c_double),
                ("nnz", ctypes.c_int64), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None

_P = ctypes.c_void_p
_I32, _I64, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_SIGS = {
    "concord_config_init": (None, [ctypes.POINTER(concord_config)]),
    "concord_create": (_I32, [ctypes.POINTER(concord_config), ctypes.POINTER(_P)]),
    "concord_set_data": (_I32, [_P, _I32, _P, _I32, _I64, _I64, _I64]),
    "concord_set_omega": (_I32, [_P, _I64, _P, _P, _P, _I32]),
    "concord_reset": (_I32, [_P]),
    "concord_step": (_I32, [_P, _D, _D, ctypes.POINTER(concord_step_info)]),
    "concord_step_replay": (_I32, [_P, _D, _D, _I32, ctypes.POINTER(concord_step_info)]),
    "concord_solve": (_I32, [_P, _D, _D, _D, _I64, ctypes.POINTER(concord_solve_info)]),
    "concord_objective": (_I32, [_P, _D, _D, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "concord_get_omega": (_I32, [_P, ctypes.POINTER(_I64), _P, _P, _P, _I32]),
    "concord_get_candidates": (_I32, [_P, ctypes.POINTER(_I64), _P, _P, _P, _P]),
    "concord_iterations": (_I64, [_P]),
    "concord_smooth_value": (_I32, [_P, _D, ctypes.POINTER(_D)]),
    "concord_gradient": (_I32, [_P, _D, _I32, _P, _P, _I32]),
    "concord_smooth_value_noalloc": (_I32, [_I64, _I64, _P, _I64, _I32, _I64, _P, _P, _P, _D, _P,
                                            _P]),
    "concord_batch_config_init": (None, [ctypes.POINTER(concord_batch_config)]),
    "concord_batch_create": (_I32, [ctypes.POINTER(concord_batch_config), _I32,
                                    ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_P),
                                    ctypes.POINTER(_I64), _I32, ctypes.POINTER(_D),
                                    ctypes.POINTER(_P)]),
    "concord_batch_solve": (_I32, [_P, _D, _D, _I64, ctypes.POINTER(_I64), ctypes.POINTER(_D),
                                   ctypes.POINTER(_I32)]),
    "concord_batch_stats_get": (_I32, [_P, ctypes.POINTER(concord_batch_stats)]),
    "concord_batch_get_omega": (_I32, [_P, _I32, _I32, ctypes.POINTER(_I64), _P, _P, _P]),
    "concord_batch_last_error": (ctypes.c_char_p, [_P]),
    "concord_batch_destroy": (None, [_P]),
    "concord_suggest_variant": (_I32, [_I64, _I64, _D, _D, _D, _I32, _D, _D, _D, ctypes.c_void_p]),
    "concord_measure_rates": (_I32, [_I32, _I32, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "concord_variant_of": (_I32, [_P]),
    "concord_set_profiling": (_I32, [_P, _I32]),
    "concord_get_profile": (_I32, [_P, ctypes.c_void_p]),
    "concord_contraction_variant": (_I32, [_P, ctypes.c_char_p, _I32]),
    "concord_refresh_screen_stats": (_I32, [_P, _D, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "concord_last_error": (ctypes.c_char_p, [_P]),
    "concord_destroy": (None, [_P]),
    "concord_version": (ctypes.c_char_p, []),
}
EXPORTED = tuple(_SIGS)


def load(path: str = LIB_PATH):
    """Load libconcord.so and set every signature.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libconcord.so not built at {path}; run python -m paper_1710_10769_amd.build")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, handle=None, batch=False) -> int:
    if rc < 0:
        msg = ""
        if handle is not None:
            fn = load().concord_batch_last_error if batch else load().concord_last_error
            msg = (fn(handle) or b"").decode()
        raise ConcordError(rc, msg)
    return rc


# ---- the C entry points under their own names ------------------------------------

def concord_version() -> str:
    return load().concord_version().decode()


def concord_config_init() -> concord_config:
    cfg = concord_config()
    load().concord_config_init(ctypes.byref(cfg))
    return cfg


def concord_create(cfg: concord_config) -> int:
    h = ctypes.c_void_p()
    _check(load().concord_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def concord_destroy(h) -> None:
    load().concord_destroy(h)


def concord_last_error(h) -> str:
    return (load().concord_last_error(h) or b"").decode()


def concord_set_data(h, kind: int, ptr: int, dtype: int, rows: int, cols: int, ld: int) -> int:
    return _check(load().concord_set_data(h, kind, ptr, dtype, rows, cols, ld), h)


def concord_set_omega(h, nnz: int, rowptr: int, col: int, val: int, dtype: int) -> int:
    return _check(load().concord_set_omega(h, nnz, rowptr, col, val, dtype), h)


def concord_reset(h) -> int:
    return _check(load().concord_reset(h), h)


@dataclasses.dataclass
class StepInfo:
    k: int
    tau: float
    n_trials: int
    n_batches: int
    f: float
    F: float
    nnz: int
    delta_fro: float
    n_candidates: int
    lhs: float
    rhs: float


def _step_info(si: concord_step_info) -> StepInfo:
    return StepInfo(**{k: getattr(si, k) for k, _ in concord_step_info._fields_})


def concord_step(h, lam1: float, lam2: float) -> StepInfo:
    si = concord_step_info()
    _check(load().concord_step(h, lam1, lam2, ctypes.byref(si)), h)
    return _step_info(si)


def concord_step_replay(h, lam1: float, lam2: float, trials: int) -> StepInfo:
    si = concord_step_info()
    _check(load().concord_step_replay(h, lam1, lam2, trials, ctypes.byref(si)), h)
    return _step_info(si)


@dataclasses.dataclass
class SolveInfo:
    iters: int
    f: float
    F: float
    nnz: int
    status: int


def concord_solve(h, lam1: float, lam2: float, tol: float, max_iter: int) -> SolveInfo:
    si = concord_solve_info()
    rc = _check(load().concord_solve(h, lam1, lam2, tol, max_iter, ctypes.byref(si)), h)
    return SolveInfo(si.iters, si.f, si.F, si.nnz, rc)


def concord_objective(h, lam1: float, lam2: float) -> Tuple[float, float]:
    f, F = ctypes.c_double(), ctypes.c_double()
    _check(load().concord_objective(h, lam1, lam2, ctypes.byref(f), ctypes.byref(F)), h)
    return f.value, F.value


def concord_get_omega(h, rowptr: int = 0, col: int = 0, val: int = 0, dtype: int = F64) -> int:
    nnz = ctypes.c_int64()
    _check(load().concord_get_omega(h, ctypes.byref(nnz), rowptr or None, col or None,
                                    val or None, dtype), h)
    return nnz.value


def concord_get_candidates(h, rowptr: int = 0, col: int = 0, omega: int = 0,
                           grad: int = 0) -> int:
    nnz = ctypes.c_int64()
    _check(load().concord_get_candidates(h, ctypes.byref(nnz), rowptr or None, col or None,
                                         omega or None, grad or None), h)
    return nnz.value


def concord_suggest_variant(p: int, n: int, d: float, t: float, s: float,
                            precision: str = "bf16x3", dense_tflops: float = 0.0,
                            hbm_gbps: float = 0.0, screen_fraction: float = 1.0) -> dict:
    """Product form for a problem (Lemma 3.1 flop rule and the library's time model)."""
    est = concord_variant_estimate()
    _check(load().concord_suggest_variant(p, n, d, t, s, _PRECISIONS[precision], dense_tflops,
                                          hbm_gbps, screen_fraction, ctypes.byref(est)))
    names = {COV: "cov", OBS: "obs"}
    return {"paper_choice": names[est.paper_choice], "choice": names[est.choice],
            "cov_flops": est.cov_flops, "obs_flops": est.obs_flops,
            "cov_seconds": est.cov_seconds, "obs_seconds": est.obs_seconds}


def concord_measure_rates(device: int = -1, precision: str = "bf16x3") -> Tuple[float, float]:
    """(dense contraction TFLOP/s, device copy GB/s) measured on the device (cached)."""
    d, h = ctypes.c_double(), ctypes.c_double()
    _check(load().concord_measure_rates(device, _PRECISIONS[precision], ctypes.byref(d),
                                        ctypes.byref(h)))
    return d.value, h.value


def concord_variant_of(h) -> str:
    v = load().concord_variant_of(h)
    if v < 0:
        _check(v, h)
    return {COV: "cov", OBS: "obs"}[v]


def concord_set_profiling(h, on: bool) -> int:
    return _check(load().concord_set_profiling(h, 1 if on else 0), h)


def concord_get_profile(h) -> dict:
    pr = concord_profile()
    _check(load().concord_get_profile(h, ctypes.byref(pr)), h)
    return {name: (pr.ms[i], pr.launches[i]) for i, name in enumerate(PROF_CLASSES)}


def concord_contraction_variant(h) -> Tuple[int, str]:
    """(index, name) of the contraction tile variant the autotuner picked (-1 if untuned)."""
    buf = ctypes.create_string_buffer(64)
    v = load().concord_contraction_variant(h, buf, 64)
    if v < -1:
        _check(v, h)
    return v, buf.value.decode()


def concord_refresh_screen_stats(h, lam1: float) -> Tuple[int, int]:
    """(tile pairs, pairs that loaded S) of one Cov refresh at the current iterate."""
    pairs, active = _I64(0), _I64(0)
    _check(load().concord_refresh_screen_stats(h, lam1, ctypes.byref(pairs), ctypes.byref(active)), h)
    return int(pairs.value), int(active.value)


def concord_iterations(h) -> int:
    return load().concord_iterations(h)


def concord_smooth_value(h, lam2: float) -> float:
    f = ctypes.c_double()
    _check(load().concord_smooth_value(h, lam2, ctypes.byref(f)), h)
    return f.value


def concord_smooth_value_noalloc(p: int, n: int, Xt: int, ldx: int, dtype: int, nnz: int,
                                 rowptr: int, col: int, val: int, lam2: float, f_out: int,
                                 stream: Optional[int] = None) -> int:
    """Handle-less smooth value into the device double at f_out; allocates nothing."""
    return _check(load().concord_smooth_value_noalloc(p, n, Xt, ldx, dtype, nnz, rowptr, col, val,
                                                      lam2, f_out, stream))


def concord_gradient(h, lam2: float, mode: int, dOmega: int, dX: int, dtype: int) -> int:
    return _check(load().concord_gradient(h, lam2, mode, dOmega or None, dX or None, dtype), h)


# ---- torch-facing wrapper --------------------------------------------------------

def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _stream_ptr(stream) -> Optional[int]:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream or None


class TorchAllocator:
    """Allocator bridge to PyTorch's caching allocator: the library's device
    workspace comes from torch.cuda.caching_allocator_alloc on the handle's
    stream and goes back through caching_allocator_delete (the library has
    synchronised that stream first).  `fail_after` (tests) makes the bridge
    return NULL once that many blocks have been handed out."""

    def __init__(self, device: int, fail_after: Optional[int] = None):
        self.device = device
        self.fail_after = fail_after
        self.live = {}
        self.n_alloc = 0
        self.n_free = 0
        self.alloc_fn = ALLOC_FN(self._alloc)
        self.free_fn = FREE_FN(self._free)

    def _alloc(self, user, nbytes, stream):
        torch = _torch()
        if self.fail_after is not None and self.n_alloc >= self.fail_after:
            return None
        try:
            ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, stream or 0)
        except Exception:   # out of memory: the library reports ENOMEM
            return None
        self.live[ptr] = int(nbytes)
        self.n_alloc += 1
        return ptr

    def _free(self, user, ptr, nbytes, stream):
        if ptr in self.live:
            del self.live[ptr]
            self.n_free += 1
            try:
                _torch().cuda.caching_allocator_delete(ptr)
            except Exception:   # interpreter shutdown: torch's allocator is gone already
                pass

    def install(self, cfg: "concord_config") -> None:
        cfg.alloc_fn = self.alloc_fn
        cfg.free_fn = self.free_fn
        cfg.alloc_user = None


class Solver:
    """One CONCORD problem on the current GPU (a library handle)."""

    def __init__(self, p: int, n: int, variant: str = "obs", precision: str = "fp32",
                 stream=None, device: Optional[int] = None, trial_batch: int = 8,
                 max_backtracks: int = 60, use_graph: bool = False, screen: bool = True,
                 tau0: float = 1.0, shrink: float = 0.5, allocator="torch"):
        """allocator: "torch" (default) routes the library's device workspace through
        PyTorch's caching allocator, None lets the library use hipMalloc, or a
        TorchAllocator instance."""
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library needs a gfx950 device")
        cfg = concord_config_init()
        cfg.p, cfg.n = p, n
        cfg.variant = _VARIANTS[variant]
        cfg.precision = _PRECISIONS[precision]
        cfg.stream = _stream_ptr(stream)
        cfg.device = torch.cuda.current_device() if device is None else device
        cfg.trial_batch = trial_batch
        cfg.max_backtracks = max_backtracks
        cfg.use_graph = 1 if use_graph else 0
        cfg.no_screen = 0 if screen else 1
        cfg.tau0, cfg.shrink = tau0, shrink
        if allocator == "torch":
            allocator = TorchAllocator(cfg.device)
        self._alloc = allocator   # keeps the callbacks alive as long as the handle
        if allocator is not None:
            allocator.install(cfg)
        self.p, self.n, self.precision = p, n, precision
        self.device = torch.device("cuda", cfg.device)
        self._h = concord_create(cfg)
        self.variant = concord_variant_of(self._h)   # the form an "auto" handle picked
        self._keep = None

    def close(self):
        if getattr(self, "_h", None):
            concord_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_data(self, X) -> None:
        """X: (n, p) CUDA tensor, float32 or float64, row-major (any row stride)."""
        assert X.is_cuda and X.dim() == 2 and X.stride(1) == 1
        concord_set_data(self._h, DATA_X, X.data_ptr(), _dtype_code(X), X.shape[0], X.shape[1],
                         X.stride(0))

    def set_covariance(self, S) -> None:
        assert S.is_cuda and S.dim() == 2 and S.stride(1) == 1
        concord_set_data(self._h, DATA_S, S.data_ptr(), _dtype_code(S), S.shape[0], S.shape[1],
                         S.stride(0))

    def set_omega(self, rowptr, col, val) -> None:
        torch = _torch()
        rowptr = rowptr.to(self.device, torch.int64).contiguous()
        col = col.to(self.device, torch.int32).contiguous()
        val = val.to(self.device).contiguous()
        concord_set_omega(self._h, col.numel(), rowptr.data_ptr(), col.data_ptr(), val.data_ptr(),
                          _dtype_code(val))

    def reset(self) -> None:
        concord_reset(self._h)

    def step(self, lam1: float, lam2: float) -> StepInfo:
        return concord_step(self._h, lam1, lam2)

    def step_replay(self, lam1: float, lam2: float, trials: int) -> StepInfo:
        return concord_step_replay(self._h, lam1, lam2, trials)

    def solve(self, lam1: float, lam2: float, tol: float = 1e-5, max_iter: int = 200) -> SolveInfo:
        return concord_solve(self._h, lam1, lam2, tol, max_iter)

    def objective(self, lam1: float, lam2: float) -> Tuple[float, float]:
        return concord_objective(self._h, lam1, lam2)

    def set_profiling(self, on: bool = True) -> None:
        concord_set_profiling(self._h, on)

    def profile(self) -> dict:
        """{class: (milliseconds, launch groups)} since profiling was switched on."""
        return concord_get_profile(self._h)

    def contraction_variant(self) -> Tuple[int, str]:
        """(index, name) of the dense-contraction tile variant in use (-1 if untuned)."""
        return concord_contraction_variant(self._h)

    def refresh_screen_stats(self, lam1: float) -> Tuple[int, int]:
        """(tile pairs, pairs that loaded S) of the Cov refresh at the current iterate
        for lam1: the exact screening skips the others."""
        return concord_refresh_screen_stats(self._h, lam1)

    @property
    def iterations(self) -> int:
        return concord_iterations(self._h)

    def nnz(self) -> int:
        """Stored entries of the current iterate."""
        return concord_get_omega(self._h)

    def get_omega(self, dtype=None):
        """Current iterate as CUDA tensors (rowptr int64, col int32, val)."""
        torch = _torch()
        dtype = dtype or torch.float64
        nnz = concord_get_omega(self._h)
        rowptr = torch.empty(self.p + 1, dtype=torch.int64, device=self.device)
        col = torch.empty(max(nnz, 1), dtype=torch.int32, device=self.device)
        val = torch.empty(max(nnz, 1), dtype=dtype, device=self.device)
        concord_get_omega(self._h, rowptr.data_ptr(), col.data_ptr(), val.data_ptr(),
                          F64 if dtype == torch.float64 else F32)
        return rowptr, col[:nnz], val[:nnz]

    def get_candidates(self):
        """Candidate set of the last step and the gradient on it: CUDA tensors
        (rowptr int64, col int32, omega float64, grad float64)."""
        torch = _torch()
        nnz = concord_get_candidates(self._h)
        rowptr = torch.empty(self.p + 1, dtype=torch.int64, device=self.device)
        col = torch.empty(max(nnz, 1), dtype=torch.int32, device=self.device)
        om = torch.empty(max(nnz, 1), dtype=torch.float64, device=self.device)
        gr = torch.empty(max(nnz, 1), dtype=torch.float64, device=self.device)
        concord_get_candidates(self._h, rowptr.data_ptr(), col.data_ptr(), om.data_ptr(),
                               gr.data_ptr())
        return rowptr, col[:nnz], om[:nnz], gr[:nnz]

    def get_candidates_scipy(self):
        """(omega, grad) of the last step's candidate set as SciPy CSR matrices."""
        import numpy as np
        import scipy.sparse as sp
        r, c, o, g = self.get_candidates()
        r, c = r.cpu().numpy(), c.cpu().numpy().astype(np.int64)
        shape = (self.p, self.p)
        return (sp.csr_matrix((o.cpu().numpy(), c, r), shape=shape),
                sp.csr_matrix((g.cpu().numpy(), c, r), shape=shape))

    def get_omega_scipy(self):
        import numpy as np
        import scipy.sparse as sp
        r, c, v = self.get_omega()
        return sp.csr_matrix((v.cpu().numpy(), c.cpu().numpy().astype(np.int64),
                              r.cpu().numpy()), shape=(self.p, self.p))

    def smooth_value(self, lam2: float) -> float:
        return concord_smooth_value(self._h, lam2)

    def gradient(self, lam2: float, mode: str = "masked", want_omega=True, want_x=True,
                 dtype=None):
        torch = _torch()
        dtype = dtype or torch.float32
        nnz = concord_get_omega(self._h)
        dOm = None
        if want_omega:
            dOm = torch.empty(nnz if mode == "masked" else (self.p, self.p), dtype=dtype,
                              device=self.device)
        dX = torch.empty((self.n, self.p), dtype=dtype, device=self.device) if want_x else None
        concord_gradient(self._h, lam2, GRAD_MASKED if mode == "masked" else GRAD_DENSE,
                         dOm.data_ptr() if dOm is not None else 0,
                         dX.data_ptr() if dX is not None else 0,
                         F64 if dtype == torch.float64 else F32)
        return dOm, dX


class Batch:
    """Many independent Cov problems solved over one lambda1 path at once on the GPU
    (the batched form of the C-ABI): every (instance, lambda1) solve runs from Omega = I
    with concord_solve's stopping rule, in launches shared by all solves."""

    def __init__(self, Xs, lambda1s, stream=None, precision: str = "fp32",
                 iters_per_launch: int = 4, use_graph: bool = True, trial_batch: int = 8,
                 max_backtracks: int = 60, tau0: float = 1.0, shrink: float = 0.5,
                 allocator="torch"):
        torch = _torch()
        self.count = len(Xs)
        self._Xs = [x.contiguous() for x in Xs]
        want = torch.float64 if precision == "fp64" else torch.float32
        for x in self._Xs:
            assert x.dtype == want and x.is_cuda and x.dim() == 2
        ps = (ctypes.c_int64 * self.count)(*[x.shape[1] for x in self._Xs])
        ns = (ctypes.c_int64 * self.count)(*[x.shape[0] for x in self._Xs])
        lds = (ctypes.c_int64 * self.count)(*[x.stride(0) for x in self._Xs])
        ptrs = (ctypes.c_void_p * self.count)(*[x.data_ptr() for x in self._Xs])
        self.lambda1s = list(lambda1s)
        l1 = (ctypes.c_double * len(self.lambda1s))(*self.lambda1s)
        cfg = concord_batch_config()
        load().concord_batch_config_init(ctypes.byref(cfg))
        cfg.precision = _PRECISIONS[precision]
        cfg.device = self._Xs[0].device.index
        cfg.stream = _stream_ptr(stream)
        cfg.iters_per_launch = iters_per_launch
        cfg.use_graph = 1 if use_graph else 0
        cfg.trial_batch, cfg.max_backtracks = trial_batch, max_backtracks
        cfg.tau0, cfg.shrink = tau0, shrink
        if allocator == "torch":
            allocator = TorchAllocator(cfg.device)
        self._alloc = allocator
        if allocator is not None:
            allocator.install(cfg)
        h = ctypes.c_void_p()
        _check(load().concord_batch_create(ctypes.byref(cfg), self.count, ps, ns, ptrs, lds,
                                           len(self.lambda1s), l1, ctypes.byref(h)))
        self._h = h.value
        self.ps = [x.shape[1] for x in self._Xs]
        self.device = self._Xs[0].device

    def solve(self, lam2: float, tol: float, max_iter: int):
        """(iterations, F, status) per solve s = instance * len(lambda1s) + l, and the
        call's status."""
        m = self.count * len(self.lambda1s)
        iters = (ctypes.c_int64 * m)()
        Fs = (ctypes.c_double * m)()
        st = (ctypes.c_int32 * m)()
        rc = load().concord_batch_solve(self._h, lam2, tol, max_iter, iters, Fs, st)
        _check(rc, self._h, batch=True)
        self.status = list(st)
        return list(iters), list(Fs), rc

    def stats(self) -> dict:
        s = concord_batch_stats()
        _check(load().concord_batch_stats_get(self._h, ctypes.byref(s)), self._h, batch=True)
        return {k: getattr(s, k) for k, _ in concord_batch_stats._fields_}

    def get_omega(self, instance: int, l1_index: int):
        torch = _torch()
        nnz = ctypes.c_int64()
        _check(load().concord_batch_get_omega(self._h, instance, l1_index, ctypes.byref(nnz),
                                              None, None, None), self._h, batch=True)
        p = self.ps[instance]
        rowptr = torch.empty(p + 1, dtype=torch.int64, device=self.device)
        col = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=self.device)
        val = torch.empty(max(nnz.value, 1), dtype=torch.float64, device=self.device)
        _check(load().concord_batch_get_omega(self._h, instance, l1_index, ctypes.byref(nnz),
                                              rowptr.data_ptr(), col.data_ptr(), val.data_ptr()),
               self._h, batch=True)
        return rowptr, col[:nnz.value], val[:nnz.value]

    def close(self):
        if getattr(self, "_h", None):
            load().concord_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
