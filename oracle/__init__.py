"""CPU oracle for ADMM on a factor graph (test infrastructure only).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its Python
binding) never imports, links or executes anything here.

``admm_oracle.cpp`` is a plain serial FP64 implementation of the paper's
Algorithm 2 (Sec. II) and of the appendix's proximal operators; this
module loads it with ctypes and adds the FP64 objective evaluations used
to compare final results (packing area term, SVM primal objective, MPC
stage cost), written directly from the problem definitions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "admm_oracle.cpp")

KIND = dict(nonoverlap=1, wall=2, radius=3, quad=4, box=5, hinge=6, l2=7,
            lindyn=8, lindyn0=9, minerr=10, equal=11, margin=12)


LIB_OMP_PATH = os.path.join(HERE, "liboracle_omp.so")


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (-O2, no fast-math): the serial library
    and the same source with OpenMP (multi-core timing; identical results)."""
    for path, extra in ((LIB_PATH, []), (LIB_OMP_PATH, ["-fopenmp"])):
        if force or not os.path.exists(path) or \
                os.path.getmtime(path) < os.path.getmtime(SRC):
            tmp = path + f".tmp{os.getpid()}"
            subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared",
                                   "-fno-fast-math", "-ffp-contract=off", *extra,
                                   SRC, "-o", tmp])
            os.replace(tmp, path)
    return LIB_PATH


_libs = {}


def lib(openmp: bool = False):
    """The serial oracle library, or its OpenMP build (threads from
    OMP_NUM_THREADS)."""
    L = _libs.get(openmp)
    if L is None:
        build()
        L = ctypes.CDLL(LIB_OMP_PATH if openmp else LIB_PATH)
        vp, ip, dp, lp = (ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                          ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(ctypes.c_long))
        L.orc_graph_create.restype = vp
        L.orc_graph_create.argtypes = [ctypes.c_int, ip]
        L.orc_graph_destroy.argtypes = [vp]
        L.orc_add_factors.restype = ctypes.c_int
        L.orc_add_factors.argtypes = [vp, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ip, dp, ctypes.c_int,
                                      ctypes.c_int]
        L.orc_set_params.argtypes = [vp, ctypes.c_double, ctypes.c_double]
        L.orc_num_slots.restype = ctypes.c_long
        L.orc_num_slots.argtypes = [vp]
        L.orc_num_z.restype = ctypes.c_long
        L.orc_num_z.argtypes = [vp]
        L.orc_set_state.argtypes = [vp, dp, dp]
        L.orc_run.restype = ctypes.c_int
        L.orc_run.argtypes = [vp, ctypes.c_int, ctypes.c_double]
        L.orc_run_region.restype = ctypes.c_int
        L.orc_run_region.argtypes = [vp, ctypes.c_int, ctypes.c_double]
        for nm in ("orc_get_z", "orc_get_u", "orc_get_x", "orc_get_m"):
            getattr(L, nm).argtypes = [vp, dp]
        L.orc_get_slot_z.argtypes = [vp, lp]
        L.orc_residuals.argtypes = [vp, dp, dp]
        L.orc_prox.restype = ctypes.c_int
        L.orc_prox.argtypes = [ctypes.c_int, ctypes.c_int, ip, dp,
                               ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_twa.argtypes = [vp, ctypes.c_int]
        L.orc_set_zu.argtypes = [vp, dp, dp]
        L.orc_run_noisy.restype = ctypes.c_int
        L.orc_run_noisy.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_ulonglong]
        L.orc_get_wr.argtypes = [vp, dp]
        L.orc_prox_free.restype = ctypes.c_int
        L.orc_prox_free.argtypes = [ctypes.c_int, dp, dp, dp, dp]
        L.orc_set_factor_weights.restype = ctypes.c_int
        L.orc_set_factor_weights.argtypes = [vp, ctypes.c_long, ctypes.c_long,
                                             ctypes.c_double, ctypes.c_double]
        _libs[openmp] = L
    return L


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def prox(kind: str, dims, params, rho: float, nv) -> np.ndarray:
    """Apply one proximal operator to the concatenated edge vector ``nv``."""
    dims = np.ascontiguousarray(dims, dtype=np.int32)
    params = np.ascontiguousarray(params, dtype=np.float64).ravel()
    nv = np.ascontiguousarray(nv, dtype=np.float64).ravel()
    out = np.zeros_like(nv)
    rc = lib().orc_prox(KIND[kind], len(dims), _ip(dims), _dp(params),
                        len(params), float(rho), _dp(nv), _dp(out))
    if rc != 0:
        raise ValueError(f"oracle prox {kind} rejected its arguments ({rc})")
    return out


def prox_free(kind: str, params, wl, nv) -> np.ndarray:
    """Three-weight variant: the non-overlap or wall prox with received
    weights ``wl`` per slot, at least one of them zero."""
    params = np.ascontiguousarray(params if params is not None else [0.0], dtype=np.float64)
    wl = np.ascontiguousarray(wl, dtype=np.float64).ravel()
    nv = np.ascontiguousarray(nv, dtype=np.float64).ravel()
    out = np.zeros_like(nv)
    if lib().orc_prox_free(KIND[kind], _dp(params), _dp(wl), _dp(nv), _dp(out)) != 0:
        raise ValueError(f"no three-weight prox for {kind}")
    return out


class OracleGraph:
    """Algorithm 2 in FP64 on a ``workloads.Problem``."""

    def __init__(self, problem, rho: Optional[float] = None,
                 alpha: Optional[float] = None, openmp: bool = False, twa: bool = False):
        L = self._L = lib(openmp)
        dims = np.ascontiguousarray(problem.var_dims, dtype=np.int32)
        self._h = L.orc_graph_create(len(dims), _ip(dims))
        first = 0
        for g in problem.groups:
            vid = np.ascontiguousarray(g.var_ids, dtype=np.int32)
            par = np.ascontiguousarray(g.params, dtype=np.float64)
            if par.size == 0:
                par = np.zeros(1)
            rc = L.orc_add_factors(self._h, KIND[g.kind], g.n, g.arity,
                                   _ip(vid), _dp(par), g.param_len,
                                   1 if g.shared else 0)
            if rc != 0:
                raise ValueError("oracle: bad factor group")
            grho, galpha = getattr(g, "rho", None), getattr(g, "alpha", None)
            if grho is not None or galpha is not None:
                L.orc_set_factor_weights(self._h, first, g.n, float(grho or 0.0),
                                         float(galpha or 0.0))
            first += g.n
        L.orc_set_params(self._h, float(problem.rho if rho is None else rho),
                         float(problem.alpha if alpha is None else alpha))
        self.n_slots = int(L.orc_num_slots(self._h))
        self.n_z = int(L.orc_num_z(self._h))
        self.twa = bool(twa)
        L.orc_set_twa(self._h, 1 if twa else 0)
        self.set_state(problem.z0)

    def __del__(self):
        if getattr(self, "_h", None) and getattr(self, "_L", None) is not None:
            self._L.orc_graph_destroy(self._h)
            self._h = None

    def set_state(self, z, u=None):
        z = np.ascontiguousarray(z, dtype=np.float64)
        assert z.shape == (self.n_z,)
        if u is not None:
            u = np.ascontiguousarray(u, dtype=np.float64)
            assert u.shape == (self.n_slots,)
            self._L.orc_set_state(self._h, _dp(z), _dp(u))
        else:
            self._L.orc_set_state(self._h, _dp(z), None)

    def replace_zu(self, z, u):
        """Overwrite z and u of a running iteration, keeping the rest of its
        state (the three-weight variant's received weights)."""
        z = np.ascontiguousarray(z, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        assert z.shape == (self.n_z,) and u.shape == (self.n_slots,)
        self._L.orc_set_zu(self._h, _dp(z), _dp(u))

    def run(self, iters: int, tol: float = 0.0, region: bool = False) -> int:
        """Run Algorithm 2; region=True uses the one-parallel-region loop
        structure (the paper's second CPU scheme) instead of one parallel
        region per update.  Both give the same results bit for bit."""
        fn = self._L.orc_run_region if region else self._L.orc_run
        done = int(fn(self._h, int(iters), float(tol)))
        if done < 0:
            raise ValueError("the one-region scheme runs plain Algorithm 2 only")
        return done

    def run_noisy(self, iters: int, eps: float, seed: int) -> int:
        """Algorithm 2 with relative noise eps injected into z and u before
        every iteration (a model of a lower precision's rounding, to measure
        how far rounding alone moves a trajectory)."""
        done = int(self._L.orc_run_noisy(self._h, int(iters), float(eps), int(seed)))
        if done < 0:
            raise ValueError("noisy runs are plain Algorithm 2 only")
        return done

    @property
    def wr(self) -> np.ndarray:
        """Three-weight variant: the weight each factor sent on each edge slot
        in the last x-update (0 or the edge's rho)."""
        return self._get(self._L.orc_get_wr, self.n_slots)

    def _get(self, fn, n):
        out = np.zeros(n)
        fn(self._h, _dp(out))
        return out

    @property
    def z(self) -> np.ndarray:
        return self._get(self._L.orc_get_z, self.n_z)

    @property
    def u(self) -> np.ndarray:
        return self._get(self._L.orc_get_u, self.n_slots)

    @property
    def x(self) -> np.ndarray:
        return self._get(self._L.orc_get_x, self.n_slots)

    @property
    def m(self) -> np.ndarray:
        return self._get(self._L.orc_get_m, self.n_slots)

    @property
    def slot_z(self) -> np.ndarray:
        out = np.zeros(self.n_slots, dtype=np.int64)
        self._L.orc_get_slot_z(self._h,
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_long)))
        return out

    def residuals(self) -> Tuple[float, float]:
        r, s = ctypes.c_double(), ctypes.c_double()
        self._L.orc_residuals(self._h, ctypes.byref(r), ctypes.byref(s))
        return r.value, s.value


# ---------------------------------------------------------------------------
# Objectives, evaluated in FP64 from z (problem definitions, Sec. V).
# ---------------------------------------------------------------------------

def packing_objective(problem, z) -> dict:
    """-gamma/2 sum r_i^2 plus feasibility measures of a packing."""
    z = np.asarray(z, dtype=np.float64)
    c = np.stack([z[0::3], z[1::3]], axis=1)
    r = z[2::3]
    gamma = problem.meta["gamma"]
    out = dict(objective=-0.5 * gamma * float(np.sum(r * r)),
               area=float(np.pi * np.sum(r * r)))
    N = len(r)
    worst = 0.0
    for i in range(N - 1):
        d = np.sqrt(np.sum((c[i + 1:] - c[i]) ** 2, axis=1))
        worst = max(worst, float(np.max(r[i] + r[i + 1:] - d, initial=0.0)))
    for Q, V in problem.meta["walls"]:
        g = r - ((c[:, 0] - V[0]) * Q[0] + (c[:, 1] - V[1]) * Q[1])
        worst = max(worst, float(np.max(g, initial=0.0)))
    worst = max(worst, float(np.max(-r, initial=0.0)))
    out["max_violation"] = worst
    return out


def svm_objective(problem, z) -> float:
    """1/2 lambda |w|^2 + C sum_i max(0, 1 - y_i (w.a_i + b))."""
    z = np.asarray(z, dtype=np.float64)
    d = problem.meta["d"]
    w, b = z[:d], z[d]
    a, y, C = problem.meta["a"], problem.meta["y"], problem.meta["C"]
    hinge = np.maximum(0.0, 1.0 - y * (a @ w + b))
    return float(0.5 * problem.meta["l2_weight"] * w @ w + C * hinge.sum())


def mpc_objective(inst, z) -> dict:
    """Stage cost 1/2 sum (x^T Q x + u^T R u) over z laid out per step as
    (u_t, x_{t+1}), plus the largest dynamics and box violations."""
    z = np.asarray(z, dtype=np.float64)
    T, n, m = inst.T, inst.n, inst.m
    blk = z.reshape(T, n + m)
    U = blk[:, :m]
    X = blk[:, m:]
    cost = 0.5 * float(np.sum(X * X * inst.q[None, :]) +
                       np.sum(U * U * inst.r[None, :]))
    xprev = np.vstack([inst.x0[None, :], X[:-1]])
    dyn = X - (xprev @ inst.A.T + U @ inst.B.T)
    box = np.max(np.abs(U)) - inst.u_box if inst.u_box > 0 else 0.0
    return dict(cost=cost, dyn_violation=float(np.max(np.abs(dyn))),
                box_violation=float(max(0.0, box)))
