"""ctypes binding of ``libadmm_hip.so`` (C ABI in ``include/admm.h``).

Argument marshalling only: every step of the ADMM iteration runs in the
library's HIP kernels.  The library must have been built in-tree
(``paper_1603_02526_amd/build.py``); loading fails loudly otherwise, and
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libadmm_hip.so")

OK, E_ARG, E_STATE, E_NUMERIC, E_HIP, E_OOM, E_NO_DEVICE, E_UNSUPPORTED = range(8)
STATUS_NAMES = {0: "OK", 1: "E_ARG", 2: "E_STATE", 3: "E_NUMERIC", 4: "E_HIP",
                5: "E_OOM", 6: "E_NO_DEVICE", 7: "E_UNSUPPORTED"}

KIND = dict(nonoverlap=1, wall=2, radius=3, quad=4, box=5, hinge=6, l2=7,
            lindyn=8, lindyn0=9, minerr=10, equal=11, margin=12)
FP32, FP64 = 0, 1
OPT_PAIR_ROWS, OPT_DRIVER, OPT_PAIR_STATE, OPT_GRAPH_BLOCK, OPT_THREE_WEIGHT, OPT_ZLIST = 1, 2, 3, 4, 5, 6
ZLIST_AUTO, ZLIST_ZMAJOR = 0, 1
DRIVER_AUTO, DRIVER_LAUNCHES, DRIVER_RESIDENT, DRIVER_GRAPH = 0, 1, 2, 3
PAIR_STATE_AUTO, PAIR_STATE_DENSE = 0, 1


class AdmmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class GraphInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "n_vars", "n_scalars", "n_factors", "n_edges", "n_slots", "n_buckets",
        "n_pair_tiles", "n_contributions", "state_bytes",
        "algo_bytes_per_iter", "layout_bytes_per_iter")] + [
        ("precision", ctypes.c_int32), ("alpha_is_one", ctypes.c_int32),
        ("driver", ctypes.c_int32), ("resident_lds_bytes", ctypes.c_int32),
        ("sparse_pair_state", ctypes.c_int32), ("three_weight", ctypes.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None

I32P = ctypes.POINTER(ctypes.c_int32)
DP = ctypes.POINTER(ctypes.c_double)
VP = ctypes.c_void_p


def _sig(L, name, res, args):
    f = getattr(L, name)
    f.restype = res
    f.argtypes = args


def lib():
    """Load the in-tree HIP library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python paper_1603_02526_amd/build.py` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        st = ctypes.c_int
        _sig(L, "admm_last_error", ctypes.c_char_p, [])
        _sig(L, "admm_abi_version", ctypes.c_int32, [])
        _sig(L, "admm_graph_create", st, [ctypes.c_int32, I32P, ctypes.c_int32,
                                          ctypes.POINTER(VP)])
        _sig(L, "admm_graph_add_factors", st, [VP, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.c_int32, I32P, DP,
                                               ctypes.c_int32, ctypes.c_int32])
        _sig(L, "admm_graph_set_rho", st, [VP, ctypes.c_double])
        _sig(L, "admm_graph_set_alpha", st, [VP, ctypes.c_double])
        _sig(L, "admm_graph_set_group_rho", st, [VP, ctypes.c_int32, ctypes.c_double])
        _sig(L, "admm_graph_set_group_alpha", st, [VP, ctypes.c_int32, ctypes.c_double])
        _sig(L, "admm_graph_finalize", st, [VP, ctypes.c_int32])
        _sig(L, "admm_graph_set_option", st, [VP, ctypes.c_int32, ctypes.c_int64])
        _sig(L, "admm_graph_info_get", st, [VP, ctypes.POINTER(GraphInfo)])
        _sig(L, "admm_set_state", st, [VP, DP, DP, VP])
        _sig(L, "admm_run", st, [VP, ctypes.c_int32, VP])
        _sig(L, "admm_run_profiled", st, [VP, ctypes.c_int32, VP, DP, DP])
        _sig(L, "admm_get_z", st, [VP, DP, VP])
        _sig(L, "admm_get_u", st, [VP, DP, VP])
        _sig(L, "admm_get_x", st, [VP, DP, VP])
        _sig(L, "admm_get_residuals", st, [VP, DP, DP, VP])
        _sig(L, "admm_z_device_ptr", st, [VP, ctypes.POINTER(VP)])
        _sig(L, "admm_graph_destroy", st, [VP])
        _lib = L
    return _lib


def check(status: int):
    if status != OK:
        raise AdmmError(status, lib().admm_last_error().decode())


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(I32P)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(DP)


def _stream(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream or None
    return int(stream.cuda_stream) or None   # a torch.cuda.Stream


class Graph:
    """A factor graph on one GPU (paper Sec. II-III)."""

    def __init__(self, var_dims, precision: int = FP32):
        d, dp = _i32(var_dims)
        h = VP()
        check(lib().admm_graph_create(len(d), dp, int(precision), ctypes.byref(h)))
        self._h = h
        self.precision = precision
        self.n_scalars = int(d.sum())
        self.n_slots = 0
        self.var_dims = d

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.admm_graph_destroy(h)
            self._h = None

    def add_factors(self, kind: str, var_ids, params=None, shared=False):
        v, vp = _i32(var_ids)
        if v.ndim == 1:
            v = v[:, None]
            v, vp = _i32(v)
        n, arity = v.shape
        p = np.zeros(0) if params is None else np.asarray(params, dtype=np.float64)
        plen = int(p.shape[-1]) if p.size else 0
        p, pp = _f64(p if p.size else np.zeros(1))
        check(lib().admm_graph_add_factors(self._h, KIND[kind], n, arity, vp,
                                           pp, plen, 1 if shared else 0))
        self.n_slots += int(self.var_dims[v].sum())

    def set_rho(self, rho: float):
        check(lib().admm_graph_set_rho(self._h, float(rho)))

    def set_group_rho(self, group: int, rho: float):
        """rho of the edges of the group-th add_factors call."""
        check(lib().admm_graph_set_group_rho(self._h, int(group), float(rho)))

    def set_group_alpha(self, group: int, alpha: float):
        """alpha of the edges of the group-th add_factors call."""
        check(lib().admm_graph_set_group_alpha(self._h, int(group), float(alpha)))

    def set_alpha(self, alpha: float):
        check(lib().admm_graph_set_alpha(self._h, float(alpha)))

    def set_option(self, option: int, value: int):
        check(lib().admm_graph_set_option(self._h, int(option), int(value)))

    def finalize(self, device: int = 0):
        check(lib().admm_graph_finalize(self._h, int(device)))

    def info(self) -> dict:
        inf = GraphInfo()
        check(lib().admm_graph_info_get(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def set_state(self, z, u=None, stream=None):
        z, zp = _f64(z)
        assert z.shape == (self.n_scalars,)
        if u is None:
            check(lib().admm_set_state(self._h, zp, None, _stream(stream)))
        else:
            u, up = _f64(u)
            assert u.shape == (self.n_slots,)
            check(lib().admm_set_state(self._h, zp, up, _stream(stream)))

    def run(self, iters: int, stream=None):
        check(lib().admm_run(self._h, int(iters), _stream(stream)))

    def run_profiled(self, iters: int, stream=None) -> Tuple[float, float]:
        xm, zm = ctypes.c_double(), ctypes.c_double()
        check(lib().admm_run_profiled(self._h, int(iters), _stream(stream),
                                      ctypes.byref(xm), ctypes.byref(zm)))
        return xm.value, zm.value

    def _get(self, fn, n, stream):
        out = np.zeros(n)
        check(fn(self._h, out.ctypes.data_as(DP), _stream(stream)))
        return out

    def z(self, stream=None) -> np.ndarray:
        return self._get(lib().admm_get_z, self.n_scalars, stream)

    def u(self, stream=None) -> np.ndarray:
        return self._get(lib().admm_get_u, self.n_slots, stream)

    def x(self, stream=None) -> np.ndarray:
        return self._get(lib().admm_get_x, self.n_slots, stream)

    def residuals(self, stream=None) -> Tuple[float, float]:
        r, s = ctypes.c_double(), ctypes.c_double()
        check(lib().admm_get_residuals(self._h, ctypes.byref(r), ctypes.byref(s),
                                       _stream(stream)))
        return r.value, s.value

    def z_device_ptr(self) -> int:
        p = VP()
        check(lib().admm_z_device_ptr(self._h, ctypes.byref(p)))
        return int(p.value or 0)

    @classmethod
    def from_problem(cls, problem, precision: int = FP32, device: Optional[int] = 0,
                     rho: Optional[float] = None, alpha: Optional[float] = None,
                     pair_rows: int = 0, driver: int = DRIVER_AUTO,
                     pair_state: int = PAIR_STATE_AUTO, graph_block: int = 0,
                     three_weight: bool = False, zlist: int = ZLIST_AUTO):
        """Build from an object with var_dims, groups (kind, var_ids, params,
        shared), rho, alpha and z0.  device=None skips finalize."""
        g = cls(problem.var_dims, precision)
        for i, grp in enumerate(problem.groups):
            g.add_factors(grp.kind, grp.var_ids, grp.params, grp.shared)
            if getattr(grp, "rho", None) is not None:
                g.set_group_rho(i, grp.rho)
            if getattr(grp, "alpha", None) is not None:
                g.set_group_alpha(i, grp.alpha)
        g.set_rho(problem.rho if rho is None else rho)
        g.set_alpha(problem.alpha if alpha is None else alpha)
        if pair_rows:
            g.set_option(OPT_PAIR_ROWS, pair_rows)
        if driver != DRIVER_AUTO:
            g.set_option(OPT_DRIVER, driver)
        if pair_state != PAIR_STATE_AUTO:
            g.set_option(OPT_PAIR_STATE, pair_state)
        if graph_block:
            g.set_option(OPT_GRAPH_BLOCK, graph_block)
        if three_weight:
            g.set_option(OPT_THREE_WEIGHT, 1)
        if zlist:
            g.set_option(OPT_ZLIST, zlist)
        if device is not None:
            g.finalize(device)
            g.set_state(problem.z0)
        return g
