"""Thin ctypes binding of libcgs (include/cgs.h).

Argument marshalling only: every function here converts NumPy arrays to
pointers, calls the C entry point of the same name and turns a non-zero
status into :class:`CgsError`.  All computation runs in the HIP library.
The library must have been built (``python -m paper_2102_05297_amd.build``);
importing this module without it raises ``ImportError``.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcgs.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2102_05297_amd.build`")
_lib = C.CDLL(_LIB_PATH)

# ----------------------------------------------------------------- constants
OK, EINVAL, ENOMEM, EDEVICE, EEMPTY, ESTATE, ERANGE = 0, -1, -2, -3, -4, -5, -6
KIND_CODES = {"DIV": 0, "DIV2": 1, "PROD_LE": 2, "PROD3_LE": 3, "PROD_GE": 4, "LE": 5}
MAX_PARAMS, MAX_RADIX, MAX_COUNTERS, MAX_TREES, MAX_DEPTH = 32, 16, 64, 64, 14
MAX_RADIUS, MAX_NEIGHBOURS = 3, 65536
NO_PROFILE = (1 << 64) - 1

# The C-ABI function names, for symbol checks.
EXPORTS = (
    "cgs_last_error", "cgs_version", "cgs_default_params", "cgs_default_expert_params",
    "cgs_synchronize", "cgs_space_create", "cgs_space_info", "cgs_space_decode",
    "cgs_space_valid_index", "cgs_space_copy_valid", "cgs_space_copy_mask", "cgs_space_destroy",
    "cgs_model_load_forest", "cgs_model_info", "cgs_model_refresh", "cgs_model_copy_predictions",
    "cgs_model_copy_leaf_ids", "cgs_model_destroy", "cgs_session_create", "cgs_search_step",
    "cgs_sample_next", "cgs_session_step_info", "cgs_session_kernel_times", "cgs_mark_explored", "cgs_session_copy_scores",
    "cgs_session_copy_weights", "cgs_session_copy_explored", "cgs_session_destroy",
    "cgs_sample_weights", "cgs_expert_system", "cgs_mlp_param_count", "cgs_model_load_mlp",
    "cgs_mlp_train", "cgs_mlp_gradients", "cgs_mlp_forward", "cgs_mlp_copy_params",
    "cgs_batch_create", "cgs_batch_step", "cgs_batch_step_time", "cgs_batch_autotune",
    "cgs_batch_set_schedule", "cgs_batch_destroy", "cgs_model_rmse",
    "cgs_model_gather_predictions", "cgs_search_step_neighbourhood",
    "cgs_session_copy_neighbourhood", "cgs_model_fit_tree", "cgs_model_forest_shape",
    "cgs_model_copy_forest", "cgs_poly_design", "cgs_model_fit_poly", "cgs_poly_shape",
    "cgs_poly_copy_coefficients", "cgs_model_load_predictions", "cgs_default_tuning_opts",
    "cgs_tuning_run", "cgs_batch_draw", "cgs_tuning_run_batch", "cgs_search_run",
    "cgs_default_online_opts", "cgs_online_run", "cgs_sample_weights_noalloc",
)


class CgsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.cgs_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {status}: {msg}")


# ----------------------------------------------------------------- structs
class cgs_constraint(C.Structure):
    _fields_ = [("kind", C.c_int32), ("a", C.c_int32), ("b", C.c_int32), ("c", C.c_int32),
                ("bound", C.c_int64)]


class cgs_params(C.Structure):
    _fields_ = [("gamma", C.c_float), ("w_min", C.c_float), ("block_log2", C.c_int32),
                ("timing", C.c_int32)]


class cgs_expert_params(C.Structure):
    _fields_ = [("inst_reaction", C.c_double), ("volta", C.c_int32), ("reserved", C.c_int32),
                ("cores", C.c_double), ("threads", C.c_double)]


class cgs_step_info(C.Structure):
    _fields_ = [("n_unexplored", C.c_uint64), ("total_weight", C.c_uint64), ("s_min", C.c_float),
                ("s_max", C.c_float), ("device_ms", C.c_float), ("n_active", C.c_int32)]


class cgs_mlp_desc(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("hidden", C.c_int32), ("n_out", C.c_int32),
                ("reserved", C.c_int32)]


class cgs_train_opts(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("batch", C.c_int32), ("steps", C.c_int32)]


class cgs_batch_schedule(C.Structure):
    _fields_ = [("score_grid", C.c_int32), ("weight_grid", C.c_int32), ("use_graph", C.c_int32),
                ("variant", C.c_int32)]


class cgs_tree_fit_report(C.Structure):
    _fields_ = [("depth", C.c_int32), ("max_depth", C.c_int32), ("min_leaf", C.c_int32),
                ("n_counters", C.c_int32), ("n_train", C.c_uint64), ("n_test", C.c_uint64),
                ("n_split", C.c_uint32), ("fit_ms", C.c_float),
                ("scale_log2", C.c_int32 * 64), ("abs_err", C.c_uint64 * 15),
                ("sq_err", (C.c_uint64 * 2) * 15)]


class cgs_tuning_opts(C.Structure):
    _fields_ = [("draws", C.c_int32), ("stop_at_well", C.c_int32), ("max_tests", C.c_uint64),
                ("well_factor", C.c_double)]


class cgs_online_opts(C.Structure):
    _fields_ = [("retrain_every", C.c_int32), ("train_steps", C.c_int32), ("batch", C.c_int32),
                ("reserved", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("threshold", C.c_double)]


class cgs_poly_fit_report(C.Structure):
    _fields_ = [("n_subspaces", C.c_int32), ("n_terms", C.c_int32), ("order", C.c_int32),
                ("n_counters", C.c_int32), ("n_points", C.c_uint64), ("fit_ms", C.c_float),
                ("eval_ms", C.c_float), ("pivot_clamped", C.c_int32), ("reserved", C.c_int32)]


_p = C.c_void_p
_u64 = C.c_uint64
_i32 = C.c_int32
_ptr = C.POINTER


def _sig(name, args, res=C.c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_lib.cgs_last_error.argtypes = []
_lib.cgs_last_error.restype = C.c_char_p
_sig("cgs_version", [])
_sig("cgs_default_params", [_ptr(cgs_params)], None)
_sig("cgs_default_expert_params", [_ptr(cgs_expert_params)], None)
_sig("cgs_synchronize", [_p])
_sig("cgs_space_create", [C.c_int, _p, _p, C.c_int, _p, _p, _ptr(_p)])
_sig("cgs_space_info", [_p, _ptr(_u64), _ptr(_u64)])
_sig("cgs_space_decode", [_p, _u64, _p])
_sig("cgs_space_valid_index", [_p, _u64, _ptr(C.c_int64)])
_sig("cgs_space_copy_valid", [_p, _u64, _u64, _p])
_sig("cgs_space_copy_mask", [_p, _p, _u64])
_sig("cgs_space_destroy", [_p], None)
_sig("cgs_model_load_forest", [_p, C.c_int, C.c_int, C.c_int, _p, _p, _p, _ptr(_p)])
_sig("cgs_model_info", [_p, _ptr(C.c_int), _ptr(C.c_float)])
_sig("cgs_model_refresh", [_p])
_sig("cgs_model_copy_predictions", [_p, _u64, _u64, _p])
_sig("cgs_model_copy_leaf_ids", [_p, _u64, _u64, _p])
_sig("cgs_model_rmse", [_p, _p, _p, _u64, _ptr(C.c_double)])
_sig("cgs_model_gather_predictions", [_p, _p, _u64, _p])
_sig("cgs_model_destroy", [_p], None)
_sig("cgs_model_fit_tree", [_p, _u64, C.c_int, _p, _p, _p, C.c_int, C.c_int, _ptr(_p),
                            _ptr(cgs_tree_fit_report)])
_sig("cgs_model_forest_shape", [_p, _ptr(C.c_int), _ptr(C.c_int)])
_sig("cgs_model_copy_forest", [_p, _p, _p, _p])
_sig("cgs_poly_design", [_p, _u64, _p, _ptr(_u64)])
_sig("cgs_model_fit_poly", [_p, _u64, C.c_int, _p, _p, C.c_int, _ptr(_p),
                            _ptr(cgs_poly_fit_report)])
_sig("cgs_poly_shape", [_p, _ptr(C.c_int), _ptr(C.c_int)])
_sig("cgs_poly_copy_coefficients", [_p, _p])
_sig("cgs_model_load_predictions", [_p, C.c_int, _p, _ptr(_p)])
_sig("cgs_default_tuning_opts", [_ptr(cgs_tuning_opts)], None)
_sig("cgs_tuning_run", [_p, _p, _p, _p, _ptr(cgs_expert_params), _p, _u64, _ptr(cgs_tuning_opts),
                        _u64, _p, _p, _ptr(_u64), _ptr(_u64)])
_sig("cgs_session_create", [_p, _ptr(cgs_params), _ptr(_p)])
_sig("cgs_search_run", [_p, _p, C.c_int, _p, _p, _p, _p, _p, _p])
_sig("cgs_search_step", [_p, _p, _u64, _p, _p, _ptr(cgs_expert_params)])
_sig("cgs_default_online_opts", [_ptr(cgs_online_opts)], None)
_sig("cgs_online_run", [_p, _p, _p, C.c_int, _p, _p, _p, _u64, _p, _p, _u64, _p, _p,
                        _ptr(cgs_online_opts), _p, _p, _p, _p, _p, _p])
_sig("cgs_search_step_neighbourhood", [_p, _p, _u64, C.c_int, _p, _p, _ptr(cgs_expert_params)])
_sig("cgs_session_copy_neighbourhood", [_p, _u64, _p, _p, _p, _ptr(_u64)])
_sig("cgs_sample_next", [_p, _u64, _ptr(_u64), _ptr(_u64)])
_sig("cgs_session_step_info", [_p, _ptr(cgs_step_info)])
_sig("cgs_session_kernel_times", [_p, _p, _p])
_sig("cgs_mark_explored", [_p, _u64])
_sig("cgs_session_copy_scores", [_p, _u64, _u64, _p])
_sig("cgs_session_copy_weights", [_p, _u64, _u64, _p])
_sig("cgs_session_copy_explored", [_p, _p, _u64])
_sig("cgs_session_destroy", [_p], None)
_sig("cgs_sample_weights", [_p, _p, _u64, _p, C.c_int, _p])
_sig("cgs_sample_weights_noalloc", [_p, _p, _u64, _p, C.c_int, _p])
_sig("cgs_expert_system", [_p, _ptr(cgs_expert_params), _p, _p, _ptr(C.c_double)])
_sig("cgs_mlp_param_count", [_ptr(cgs_mlp_desc)], C.c_uint64)
_sig("cgs_model_load_mlp", [_p, _ptr(cgs_mlp_desc), _p, _ptr(_p)])
_sig("cgs_mlp_train", [_p, _p, _p, _u64, _p, _ptr(cgs_train_opts), _p])
_sig("cgs_mlp_gradients", [_p, _p, _p, C.c_uint32, _p, _p])
_sig("cgs_mlp_forward", [_p, _p, C.c_uint32, _p])
_sig("cgs_mlp_copy_params", [_p, _p, _u64])
_sig("cgs_batch_create", [C.c_int, _p, _p, _ptr(cgs_batch_schedule), _ptr(_p)])
_sig("cgs_batch_step", [_p, _p, _p, _p, _p, _p, _p])
_sig("cgs_batch_step_time", [_p, _ptr(C.c_float)])
_sig("cgs_batch_draw", [_p, _p, _p, _p, _p])
_sig("cgs_tuning_run_batch", [_p, _p, _p, _ptr(cgs_expert_params), _p, _u64, _ptr(cgs_tuning_opts),
                              _u64, _p, _p, _p, _p])
_sig("cgs_batch_autotune", [_p, C.c_char_p, _ptr(cgs_batch_schedule)])
_sig("cgs_batch_set_schedule", [_p, _ptr(cgs_batch_schedule)])
_sig("cgs_batch_destroy", [_p], None)


def _check(st: int, where: str) -> None:
    if st != OK:
        raise CgsError(st, where)


def _arr(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _ptrof(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def library_path() -> str:
    return _LIB_PATH


def cgs_version() -> int:
    return int(_lib.cgs_version())


def cgs_default_params() -> cgs_params:
    p = cgs_params()
    _lib.cgs_default_params(C.byref(p))
    return p


def cgs_default_online_opts(**kw) -> cgs_online_opts:
    """Online-retraining settings: retrain every 20 steps with 500 Adam steps
    of 256 pairs (lr 1e-3), surrogate kept while its RMSE is <= 0.05;
    keyword arguments override fields."""
    o = cgs_online_opts()
    _lib.cgs_default_online_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def cgs_default_expert_params() -> cgs_expert_params:
    p = cgs_expert_params()
    _lib.cgs_default_expert_params(C.byref(p))
    return p


def cgs_expert_system(pc, expert: Optional[cgs_expert_params] = None):
    """Returns (B[18], delta[24], delta_threads), float64."""
    pc = _arr(pc, np.float64)
    B = np.zeros(18)
    d = np.zeros(24)
    dt = C.c_double(0.0)
    _check(_lib.cgs_expert_system(_ptrof(pc), C.byref(expert) if expert else None, _ptrof(B),
                                  _ptrof(d), C.byref(dt)), "cgs_expert_system")
    return B, d, dt.value


# ----------------------------------------------------------------- handles
class Space:
    """A tuning space on the device (cgs_space)."""

    def __init__(self, radix: Sequence[int], values: Sequence[Sequence[int]],
                 constraints: Sequence = (), stream: Optional[int] = None):
        r = _arr(radix, np.int32)
        v = _arr([x for tab in values for x in tab], np.int64)
        cons = (cgs_constraint * max(1, len(constraints)))()
        for i, (kind, a, b, c, bound) in enumerate(constraints):
            cons[i] = cgs_constraint(KIND_CODES[kind] if isinstance(kind, str) else int(kind),
                                     int(a), int(b), int(c), int(bound))
        h = C.c_void_p()
        _check(_lib.cgs_space_create(len(r), _ptrof(r), _ptrof(v), len(constraints), cons,
                                     C.c_void_p(stream) if stream else None, C.byref(h)),
               "cgs_space_create")
        self.h = h
        self.radix = [int(x) for x in r]
        n_raw, n_valid = _u64(), _u64()
        _check(_lib.cgs_space_info(h, C.byref(n_raw), C.byref(n_valid)), "cgs_space_info")
        self.n_raw, self.n_valid = int(n_raw.value), int(n_valid.value)

    @classmethod
    def from_spec(cls, spec, stream=None) -> "Space":
        return cls(spec.radix, spec.values, spec.constraints, stream)

    def decode(self, raw: int) -> np.ndarray:
        out = np.zeros(len(self.radix), dtype=np.int32)
        _check(_lib.cgs_space_decode(self.h, int(raw), _ptrof(out)), "cgs_space_decode")
        return out

    def valid_index(self, raw: int) -> int:
        out = C.c_int64()
        _check(_lib.cgs_space_valid_index(self.h, int(raw), C.byref(out)), "cgs_space_valid_index")
        return int(out.value)

    def copy_valid(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        count = self.n_valid - first if count is None else count
        out = np.zeros(count, dtype=np.uint32)
        _check(_lib.cgs_space_copy_valid(self.h, first, count, _ptrof(out)), "cgs_space_copy_valid")
        return out

    def copy_mask(self) -> np.ndarray:
        n = (self.n_raw + 31) // 32
        out = np.zeros(n, dtype=np.uint32)
        _check(_lib.cgs_space_copy_mask(self.h, _ptrof(out), n), "cgs_space_copy_mask")
        return out

    def synchronize(self) -> None:
        _check(_lib.cgs_synchronize(self.h), "cgs_synchronize")

    def sample_weights(self, q, uniforms) -> np.ndarray:
        q = _arr(q, np.uint32)
        u = _arr(uniforms, np.uint64)
        picks = np.full(len(u), -1, dtype=np.int64)
        _check(_lib.cgs_sample_weights(self.h, _ptrof(q), len(q), _ptrof(u), len(u),
                                       _ptrof(picks)), "cgs_sample_weights")
        return picks

    def sample_weights_noalloc(self, q, uniforms) -> np.ndarray:
        """sample_weights through the entry point that allocates no device
        memory (at most 2^22 weights)."""
        q = _arr(q, np.uint32)
        u = _arr(uniforms, np.uint64)
        picks = np.full(len(u), -1, dtype=np.int64)
        _check(_lib.cgs_sample_weights_noalloc(self.h, _ptrof(q), len(q), _ptrof(u), len(u),
                                               _ptrof(picks)), "cgs_sample_weights_noalloc")
        return picks

    def close(self) -> None:
        if getattr(self, "h", None):
            _lib.cgs_space_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class _Model:
    """Common part of the model handles (cgs_model)."""
    h = None
    space: "Space"
    n_counters: int

    def eval_ms(self) -> float:
        n = C.c_int()
        ms = C.c_float()
        _check(_lib.cgs_model_info(self.h, C.byref(n), C.byref(ms)), "cgs_model_info")
        return float(ms.value)

    def refresh(self) -> None:
        _check(_lib.cgs_model_refresh(self.h), "cgs_model_refresh")

    def copy_predictions(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        count = self.space.n_valid - first if count is None else count
        out = np.zeros((count, self.n_counters), dtype=np.float32)
        _check(_lib.cgs_model_copy_predictions(self.h, first, count, _ptrof(out)),
               "cgs_model_copy_predictions")
        return out

    def gather_predictions(self, valid_idx) -> np.ndarray:
        """Predictions [n][C] of the listed valid indices."""
        idx = _arr(valid_idx, np.uint32)
        out = np.zeros((len(idx), self.n_counters), dtype=np.float32)
        _check(_lib.cgs_model_gather_predictions(self.h, _ptrof(idx), len(idx), _ptrof(out)),
               "cgs_model_gather_predictions")
        return out

    def rmse(self, other: "_Model", sample) -> float:
        """RMS difference of the two models' predictions over valid indices."""
        smp = _arr(sample, np.uint32)
        out = C.c_double()
        _check(_lib.cgs_model_rmse(self.h, other.h, _ptrof(smp), len(smp), C.byref(out)),
               "cgs_model_rmse")
        return float(out.value)

    def close(self) -> None:
        if getattr(self, "h", None):
            _lib.cgs_model_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class ForestModel(_Model):
    """A regression forest and its cached predictions (cgs_model)."""

    def __init__(self, space: Space, feat, thr, leaves):
        leaves = _arr(leaves, np.float32)
        T, L, Cn = leaves.shape
        depth = int(L).bit_length() - 1
        feat = _arr(feat, np.uint8)
        thr = _arr(thr, np.uint8)
        h = C.c_void_p()
        _check(_lib.cgs_model_load_forest(space.h, T, depth, Cn, _ptrof(feat), _ptrof(thr),
                                          _ptrof(leaves), C.byref(h)), "cgs_model_load_forest")
        self.h, self.space = h, space
        self.n_trees, self.depth, self.n_counters = T, depth, Cn

    @classmethod
    def from_spec(cls, space: Space, forest) -> "ForestModel":
        return cls(space, forest.feat, forest.thr, forest.leaves)

    @classmethod
    def fit(cls, space: Space, points, targets, keys, max_depth: int, min_leaf: int = 1):
        """Fit one regression tree on measured pairs (cgs_model_fit_tree):
        points = valid indices [n], targets [n][C], keys = 64-bit random
        numbers [n] that choose the training half.  Returns (model, report)."""
        pts = _arr(points, np.uint32)
        y = _arr(targets, np.float32)
        if y.ndim != 2 or len(y) != len(pts):
            raise ValueError("targets must be [n][C] with one row per point")
        ks = _arr(keys, np.uint64)
        if len(ks) != len(pts):
            raise ValueError("one key per point")
        rep = cgs_tree_fit_report()
        h = C.c_void_p()
        _check(_lib.cgs_model_fit_tree(space.h, len(pts), y.shape[1], _ptrof(pts), _ptrof(y),
                                       _ptrof(ks), int(max_depth), int(min_leaf), C.byref(h),
                                       C.byref(rep)), "cgs_model_fit_tree")
        m = cls.__new__(cls)
        m.h, m.space = h, space
        m.n_trees, m.depth, m.n_counters = 1, int(rep.depth), int(y.shape[1])
        D = int(max_depth)
        report = {
            "depth": int(rep.depth), "n_train": int(rep.n_train), "n_test": int(rep.n_test),
            "n_split": int(rep.n_split), "fit_ms": float(rep.fit_ms),
            "scale_log2": [int(v) for v in rep.scale_log2[: y.shape[1]]],
            "abs_err": [int(v) for v in rep.abs_err[: D + 1]],
            "sq_err": [int(rep.sq_err[d][0]) | (int(rep.sq_err[d][1]) << 64) for d in range(D + 1)],
        }
        return m, report

    def copy_forest(self):
        """(feat, thr, leaves) in the layout of the constructor."""
        T, D = C.c_int(), C.c_int()
        _check(_lib.cgs_model_forest_shape(self.h, C.byref(T), C.byref(D)), "cgs_model_forest_shape")
        n_int = (1 << D.value) - 1
        feat = np.zeros((T.value, n_int), dtype=np.uint8)
        thr = np.zeros((T.value, n_int), dtype=np.uint8)
        leaves = np.zeros((T.value, 1 << D.value, self.n_counters), dtype=np.float32)
        _check(_lib.cgs_model_copy_forest(self.h, _ptrof(feat), _ptrof(thr), _ptrof(leaves)),
               "cgs_model_copy_forest")
        return feat, thr, leaves

    def copy_leaf_ids(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        count = self.space.n_valid - first if count is None else count
        out = np.zeros((self.n_trees, count), dtype=np.uint16)
        _check(_lib.cgs_model_copy_leaf_ids(self.h, first, count, _ptrof(out)),
               "cgs_model_copy_leaf_ids")
        return out


class PolyModel(_Model):
    """Least-squares polynomial counter models per binary subspace
    (cgs_model_fit_poly)."""

    def __init__(self, space: Space, points, targets, order: int):
        pts = _arr(points, np.uint32)
        y = _arr(targets, np.float32)
        if y.ndim != 2 or len(y) != len(pts):
            raise ValueError("targets must be [n][C] with one row per point")
        rep = cgs_poly_fit_report()
        h = C.c_void_p()
        _check(_lib.cgs_model_fit_poly(space.h, len(pts), y.shape[1], _ptrof(pts), _ptrof(y),
                                       int(order), C.byref(h), C.byref(rep)), "cgs_model_fit_poly")
        self.h, self.space = h, space
        self.n_counters, self.order = int(y.shape[1]), int(order)
        self.report = {k: getattr(rep, k) for k, _ in cgs_poly_fit_report._fields_}

    @staticmethod
    def design(space: Space) -> np.ndarray:
        """Valid indices of the design configurations (cgs_poly_design)."""
        n = C.c_uint64()
        out = np.zeros(max(1, space.n_valid), dtype=np.uint32)
        _check(_lib.cgs_poly_design(space.h, len(out), _ptrof(out), C.byref(n)), "cgs_poly_design")
        return out[: n.value].copy()

    def coefficients(self) -> np.ndarray:
        """float64 [subspaces][terms][counters]."""
        S, T = C.c_int(), C.c_int()
        _check(_lib.cgs_poly_shape(self.h, C.byref(S), C.byref(T)), "cgs_poly_shape")
        out = np.zeros((S.value, T.value, self.n_counters), dtype=np.float64)
        _check(_lib.cgs_poly_copy_coefficients(self.h, _ptrof(out)), "cgs_poly_copy_coefficients")
        return out


class TableModel(_Model):
    """Predictions given by the caller, [n_valid][C] (cgs_model_load_predictions)."""

    def __init__(self, space: Space, predictions):
        pred = _arr(predictions, np.float32)
        if pred.ndim != 2 or len(pred) != space.n_valid:
            raise ValueError("predictions must be [n_valid][C]")
        h = C.c_void_p()
        _check(_lib.cgs_model_load_predictions(space.h, pred.shape[1], _ptrof(pred), C.byref(h)),
               "cgs_model_load_predictions")
        self.h, self.space, self.n_counters = h, space, int(pred.shape[1])


def mlp_flatten(params) -> np.ndarray:
    """[W1, b1, W2, b2, W3, b3] -> the library's fp32 parameter vector."""
    return np.concatenate([np.asarray(p, dtype=np.float32).ravel() for p in params])


class MLPModel(_Model):
    """The perceptron surrogate (cgs_model): F -> H -> H -> C."""

    def __init__(self, space: Space, params):
        W1, b1, W2, b2, W3, b3 = params
        H, F = np.shape(W1)
        Cn = np.shape(W3)[0]
        self.desc = cgs_mlp_desc(int(F), int(H), int(Cn), 0)
        flat = mlp_flatten(params)
        if flat.size != int(_lib.cgs_mlp_param_count(C.byref(self.desc))):
            raise ValueError("parameter shapes do not match the perceptron layout")
        h = C.c_void_p()
        _check(_lib.cgs_model_load_mlp(space.h, C.byref(self.desc), _ptrof(flat), C.byref(h)),
               "cgs_model_load_mlp")
        self.h, self.space = h, space
        self.F, self.H, self.n_counters = int(F), int(H), int(Cn)
        self.n_params = flat.size

    def train(self, cfg_raw, targets, batch_idx, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """Adam steps over the rows of batch_idx [steps][batch]; returns the losses."""
        cfg = _arr(cfg_raw, np.uint32)
        tg = _arr(targets, np.float32)
        bi = _arr(batch_idx, np.int32)
        steps, batch = bi.shape
        opts = cgs_train_opts(lr, beta1, beta2, eps, batch, steps)
        losses = np.zeros(max(steps, 1), dtype=np.float32)
        _check(_lib.cgs_mlp_train(self.h, _ptrof(cfg), _ptrof(tg), len(cfg), _ptrof(bi),
                                  C.byref(opts), _ptrof(losses)), "cgs_mlp_train")
        return losses[:steps]

    def gradients(self, cfg_raw, targets):
        cfg = _arr(cfg_raw, np.uint32)
        tg = _arr(targets, np.float32)
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = C.c_float()
        _check(_lib.cgs_mlp_gradients(self.h, _ptrof(cfg), _ptrof(tg), len(cfg), _ptrof(g),
                                      C.byref(loss)), "cgs_mlp_gradients")
        return g, float(loss.value)

    def forward(self, cfg_raw) -> np.ndarray:
        cfg = _arr(cfg_raw, np.uint32)
        y = np.zeros((len(cfg), self.n_counters), dtype=np.float32)
        _check(_lib.cgs_mlp_forward(self.h, _ptrof(cfg), len(cfg), _ptrof(y)), "cgs_mlp_forward")
        return y

    def copy_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(_lib.cgs_mlp_copy_params(self.h, _ptrof(out), self.n_params),
               "cgs_mlp_copy_params")
        return out

    def unflatten(self, flat):
        F, H, Cn = self.F, self.H, self.n_counters
        sizes = [(H, F), (H,), (H, H), (H,), (Cn, H), (Cn,)]
        out, o = [], 0
        for shp in sizes:
            n = int(np.prod(shp))
            out.append(np.asarray(flat[o:o + n]).reshape(shp))
            o += n
        return out


class Session:
    """One search over a space (cgs_session)."""

    def __init__(self, space: Space, params: Optional[cgs_params] = None):
        h = C.c_void_p()
        _check(_lib.cgs_session_create(space.h, C.byref(params) if params else None, C.byref(h)),
               "cgs_session_create")
        self.h, self.space = h, space

    def search_step(self, model, profile_raw: int, delta=None, measured=None,
                    expert: Optional[cgs_expert_params] = None) -> None:
        d = None if delta is None else _arr(delta, np.float32)
        m = None if measured is None else _arr(measured, np.float64)
        _check(_lib.cgs_search_step(self.h, model.h, int(profile_raw), _ptrof(d), _ptrof(m),
                                    C.byref(expert) if expert else None), "cgs_search_step")

    def search_step_neighbourhood(self, model, profile_raw: int, radius: int, delta=None,
                                  measured=None, expert: Optional[cgs_expert_params] = None) -> None:
        d = None if delta is None else _arr(delta, np.float32)
        m = None if measured is None else _arr(measured, np.float64)
        _check(_lib.cgs_search_step_neighbourhood(self.h, model.h, int(profile_raw), int(radius),
                                                  _ptrof(d), _ptrof(m),
                                                  C.byref(expert) if expert else None),
               "cgs_search_step_neighbourhood")

    def copy_neighbourhood(self):
        """(valid indices, scores, quantised weights) of the last restricted
        step's candidates, in candidate order."""
        n = _u64()
        cap = MAX_NEIGHBOURS
        idx = np.zeros(cap, dtype=np.uint32)
        sc = np.zeros(cap, dtype=np.float32)
        q = np.zeros(cap, dtype=np.uint32)
        _check(_lib.cgs_session_copy_neighbourhood(self.h, cap, _ptrof(idx), _ptrof(sc), _ptrof(q),
                                                   C.byref(n)), "cgs_session_copy_neighbourhood")
        k = int(n.value)
        return idx[:k].copy(), sc[:k].copy(), q[:k].copy()

    def sample_next(self, u64: int):
        """(raw index, valid index) of the drawn configuration; None when exhausted."""
        raw, valid = _u64(), _u64()
        st = _lib.cgs_sample_next(self.h, int(u64), C.byref(raw), C.byref(valid))
        if st == EEMPTY:
            return None
        _check(st, "cgs_sample_next")
        return int(raw.value), int(valid.value)

    def search_run(self, model, measured, experts, uniforms):
        """The uniform start and len(measured) profiled steps, one draw each,
        in the library (cgs_search_run): (raw[n + 1], valid[n + 1],
        step wall times in microseconds [n])."""
        pc = _arr(measured, np.float64).reshape(-1, 24)
        n = pc.shape[0]
        if len(experts) != n:
            raise ValueError("one expert-parameter set per step")
        eps = (cgs_expert_params * max(n, 1))(*experts)
        us = _arr(uniforms, np.uint64)
        if len(us) < n + 1:
            raise ValueError("n_steps + 1 random numbers needed")
        raw = np.zeros(n + 1, dtype=np.uint64)
        val = np.zeros(n + 1, dtype=np.uint64)
        t_us = np.zeros(max(n, 1), dtype=np.float64)
        _check(_lib.cgs_search_run(self.h, model.h, n, _ptrof(pc), C.cast(eps, C.c_void_p),
                                   _ptrof(us), _ptrof(raw), _ptrof(val), _ptrof(t_us)),
               "cgs_search_run")
        return raw, val, t_us[:n]

    def online_run(self, tree, mlp, deltas, uniforms, noise, seed_cfg, seed_targets, val_sample,
                   batch_u64=None, opts: Optional[cgs_online_opts] = None):
        """A search with the perceptron surrogate retrained online and the tree
        as fallback, in the library (cgs_online_run).  deltas [n][C],
        uniforms [n + 1], noise [n + 1][C]; batch_u64 [windows - 1][steps]
        [batch] 64-bit numbers choosing the training rows.  Returns a dict:
        raw / valid picks, per-window RMSE and model, step and retrain times."""
        o = opts if opts is not None else cgs_default_online_opts()
        d = _arr(deltas, np.float32)
        n = d.shape[0]
        Cn = tree.n_counters
        d = d.reshape(n, Cn)
        us = _arr(uniforms, np.uint64)
        nz = _arr(noise, np.float32).reshape(-1, Cn)
        if len(us) < n + 1 or nz.shape[0] < n + 1:
            raise ValueError("n_steps + 1 uniforms and noise rows needed")
        cfg = _arr(seed_cfg, np.uint32)
        tg = _arr(seed_targets, np.float32).reshape(len(cfg), Cn)
        val = _arr(val_sample, np.uint32)
        W = 1 + n // o.retrain_every
        bu = None
        if batch_u64 is not None:
            bu = _arr(batch_u64, np.uint64)
            if bu.size < (W - 1) * o.train_steps * o.batch:
                raise ValueError("batch_u64 needs (windows - 1) * train_steps * batch numbers")
        raw = np.zeros(n + 1, np.uint64)
        valid = np.zeros(n + 1, np.uint64)
        rmse = np.zeros(W, np.float64)
        use = np.zeros(W, np.int32)
        step_us = np.zeros(max(n, 1), np.float64)
        retrain_ms = np.zeros(max(W - 1, 1), np.float64)
        st = _lib.cgs_online_run(self.h, tree.h, mlp.h, n, _ptrof(d), _ptrof(us), _ptrof(nz),
                                 len(cfg), _ptrof(cfg), _ptrof(tg), len(val), _ptrof(val),
                                 _ptrof(bu), C.byref(o), _ptrof(raw), _ptrof(valid),
                                 _ptrof(rmse), _ptrof(use), _ptrof(step_us), _ptrof(retrain_ms))
        done = int((raw != np.uint64(2 ** 64 - 1)).sum())
        if st != EEMPTY:
            _check(st, "cgs_online_run")
        return {"raw": raw[:done], "picks": [int(x) for x in valid[:done]],
                "windows": [{"step": w * o.retrain_every, "rmse": float(rmse[w]),
                             "model": "mlp" if use[w] == 1 else "tree"}
                            for w in range(W) if use[w] >= 0],
                "step_us": step_us[:max(done - 1, 0)],
                "retrain_ms": retrain_ms[:W - 1]}

    def tuning_run(self, model, runtime, counters, uniforms, draws: int = 5,
                   max_tests: Optional[int] = None, stop_at_well: bool = True,
                   well_factor: float = 1.1, expert: Optional["cgs_expert_params"] = None):
        """Alg. 1 on tables of measured runtimes [n_valid] and counters
        [n_valid][24] (cgs_tuning_run): (tested valid indices, profiled flags,
        tests to the first well-performing configuration, 0 if none)."""
        rt = _arr(runtime, np.float32)
        pc = _arr(counters, np.float64)
        us = _arr(uniforms, np.uint64)
        cap = int(max_tests if max_tests is not None else len(us) + 1)
        opts = cgs_tuning_opts(int(draws), 1 if stop_at_well else 0, cap, float(well_factor))
        ep = expert if expert is not None else cgs_default_expert_params()
        tested = np.zeros(cap, dtype=np.uint64)
        prof = np.zeros(cap, dtype=np.uint8)
        nt, tw = _u64(), _u64()
        _check(_lib.cgs_tuning_run(self.h, model.h, _ptrof(rt), _ptrof(pc), C.byref(ep), _ptrof(us),
                                   len(us), C.byref(opts), cap, _ptrof(tested), _ptrof(prof),
                                   C.byref(nt), C.byref(tw)), "cgs_tuning_run")
        n = int(nt.value)
        return tested[:n].astype(np.int64), prof[:n].astype(bool), int(tw.value)

    def step_info(self) -> cgs_step_info:
        info = cgs_step_info()
        _check(_lib.cgs_session_step_info(self.h, C.byref(info)), "cgs_session_step_info")
        return info

    def kernel_times(self):
        """(total ms[4], launches[4]): score pass, weight pass, draws, reserved."""
        ms = np.zeros(4, dtype=np.float64)
        n = np.zeros(4, dtype=np.uint64)
        _check(_lib.cgs_session_kernel_times(self.h, _ptrof(ms), _ptrof(n)),
               "cgs_session_kernel_times")
        return ms, n

    def mark_explored(self, raw: int) -> None:
        _check(_lib.cgs_mark_explored(self.h, int(raw)), "cgs_mark_explored")

    def copy_scores(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        count = self.space.n_valid - first if count is None else count
        out = np.zeros(count, dtype=np.float32)
        _check(_lib.cgs_session_copy_scores(self.h, first, count, _ptrof(out)),
               "cgs_session_copy_scores")
        return out

    def copy_weights(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        count = self.space.n_valid - first if count is None else count
        out = np.zeros(count, dtype=np.uint32)
        _check(_lib.cgs_session_copy_weights(self.h, first, count, _ptrof(out)),
               "cgs_session_copy_weights")
        return out

    def copy_explored(self) -> np.ndarray:
        n = (self.space.n_valid + 31) // 32
        out = np.zeros(n, dtype=np.uint32)
        _check(_lib.cgs_session_copy_explored(self.h, _ptrof(out), n), "cgs_session_copy_explored")
        return out

    def close(self) -> None:
        if getattr(self, "h", None):
            _lib.cgs_session_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Batch:
    """Independent sessions stepped together (cgs_batch)."""

    def __init__(self, sessions, models, schedule: Optional[cgs_batch_schedule] = None):
        n = len(sessions)
        hs = (C.c_void_p * n)(*[x.h for x in sessions])
        hm = (C.c_void_p * n)(*[x.h for x in models])
        h = C.c_void_p()
        _check(_lib.cgs_batch_create(n, hs, hm, C.byref(schedule) if schedule else None,
                                     C.byref(h)), "cgs_batch_create")
        self.h, self.sessions, self.models, self.n = h, list(sessions), list(models), n

    def step(self, profiles, deltas, uniforms):
        """(raw[n], valid[n], status[n]); raw/valid are 2^64-1 where status != 0."""
        pr = _arr([int(p) for p in profiles], np.uint64)
        d = None if deltas is None else _arr(np.concatenate([np.ravel(x) for x in deltas]), np.float32)
        u = _arr(uniforms, np.uint64)
        raw = np.zeros(self.n, dtype=np.uint64)
        val = np.zeros(self.n, dtype=np.uint64)
        st = np.zeros(self.n, dtype=np.int32)
        _check(_lib.cgs_batch_step(self.h, _ptrof(pr), _ptrof(d), _ptrof(u), _ptrof(raw),
                                   _ptrof(val), _ptrof(st)), "cgs_batch_step")
        return raw, val, st

    def draw(self, uniforms):
        """One more draw in every session from its last batch step's weights
        (cgs_batch_draw): (raw[n], valid[n], status[n])."""
        u = _arr(uniforms, np.uint64)
        raw = np.zeros(self.n, dtype=np.uint64)
        val = np.zeros(self.n, dtype=np.uint64)
        st = np.zeros(self.n, dtype=np.int32)
        _check(_lib.cgs_batch_draw(self.h, _ptrof(u), _ptrof(raw), _ptrof(val), _ptrof(st)),
               "cgs_batch_draw")
        return raw, val, st

    def tuning_run(self, runtime, counters, uniforms, draws: int = 5,
                   max_tests: Optional[int] = None, stop_at_well: bool = True,
                   well_factor: float = 1.1, expert: Optional["cgs_expert_params"] = None):
        """Alg. 1 for every session at once (cgs_tuning_run_batch); uniforms
        [n][k] are run i's random numbers.  Per run: (tested valid indices,
        profiled flags, tests to the first well-performing configuration)."""
        rt = _arr(runtime, np.float32)
        pc = _arr(counters, np.float64)
        us = _arr(uniforms, np.uint64)
        if us.ndim != 2 or us.shape[0] != self.n:
            raise ValueError("uniforms must be [n_sessions][k]")
        cap = int(max_tests if max_tests is not None else us.shape[1] + 1)
        opts = cgs_tuning_opts(int(draws), 1 if stop_at_well else 0, cap, float(well_factor))
        ep = expert if expert is not None else cgs_default_expert_params()
        tested = np.zeros((self.n, cap), dtype=np.uint64)
        prof = np.zeros((self.n, cap), dtype=np.uint8)
        nt = np.zeros(self.n, dtype=np.uint64)
        tw = np.zeros(self.n, dtype=np.uint64)
        _check(_lib.cgs_tuning_run_batch(self.h, _ptrof(rt), _ptrof(pc), C.byref(ep), _ptrof(us),
                                         us.shape[1], C.byref(opts), cap, _ptrof(tested),
                                         _ptrof(prof), _ptrof(nt), _ptrof(tw)),
               "cgs_tuning_run_batch")
        return [(tested[i, :int(nt[i])].astype(np.int64), prof[i, :int(nt[i])].astype(bool),
                 int(tw[i])) for i in range(self.n)]

    def step_ms(self) -> float:
        ms = C.c_float()
        _check(_lib.cgs_batch_step_time(self.h, C.byref(ms)), "cgs_batch_step_time")
        return float(ms.value)

    def autotune(self, cache_path: Optional[str] = None) -> cgs_batch_schedule:
        sched = cgs_batch_schedule()
        _check(_lib.cgs_batch_autotune(self.h, cache_path.encode() if cache_path else None,
                                       C.byref(sched)), "cgs_batch_autotune")
        return sched

    def set_schedule(self, sched: cgs_batch_schedule) -> None:
        _check(_lib.cgs_batch_set_schedule(self.h, C.byref(sched)), "cgs_batch_set_schedule")

    def close(self) -> None:
        if getattr(self, "h", None):
            _lib.cgs_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()
