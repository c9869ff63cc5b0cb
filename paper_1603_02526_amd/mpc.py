"""ctypes binding of the batched MPC solver (``admm_mpc_batch_*`` in
``include/admm.h``).  Device arrays are torch tensors (float32 / int32 on
the batch's device); every computation runs in the HIP library."""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np

from .admm import check, lib, _stream

VP = ctypes.c_void_p
I32P = ctypes.POINTER(ctypes.c_int32)
DP = ctypes.POINTER(ctypes.c_double)
I64P = ctypes.POINTER(ctypes.c_int64)
FP = ctypes.POINTER(ctypes.c_float)

_sigs_done = False


def _setup():
    global _sigs_done
    if _sigs_done:
        return lib()
    L = lib()
    st = ctypes.c_int
    L.admm_mpc_batch_create.restype = st
    L.admm_mpc_batch_create.argtypes = [ctypes.c_int32, I32P, I32P, I32P, DP, DP, DP, DP, DP,
                                        ctypes.c_double, ctypes.c_int32, ctypes.POINTER(VP)]
    L.admm_mpc_batch_sizes.restype = st
    L.admm_mpc_batch_sizes.argtypes = [VP, I64P, I64P, I64P]
    L.admm_mpc_batch_solve.restype = st
    L.admm_mpc_batch_solve.argtypes = [VP, VP, VP, ctypes.c_int32, ctypes.c_float,
                                       ctypes.c_int32, VP, VP, VP]
    L.admm_mpc_batch_solve_state.restype = st
    L.admm_mpc_batch_solve_state.argtypes = [VP, VP, VP, VP, ctypes.c_float, ctypes.c_int32,
                                             VP, VP, VP, VP]
    L.admm_mpc_batch_shift.restype = st
    L.admm_mpc_batch_shift.argtypes = [VP, VP, VP, VP, VP, VP, VP, VP, VP]
    L.admm_mpc_batch_dual_complete.restype = st
    L.admm_mpc_batch_dual_complete.argtypes = [VP, VP, VP, VP]
    L.admm_mpc_batch_set_plan.restype = st
    L.admm_mpc_batch_set_plan.argtypes = [VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.admm_mpc_batch_get_plan.restype = st
    L.admm_mpc_batch_get_plan.argtypes = [VP, I32P, I32P, I32P, I32P]
    L.admm_mpc_batch_tune.restype = st
    L.admm_mpc_batch_tune.argtypes = [VP, VP, ctypes.c_float, ctypes.c_int32, VP, VP,
                                      ctypes.c_int32, FP, ctypes.c_int32, I32P, VP]
    L.admm_mpc_batch_destroy.restype = st
    L.admm_mpc_batch_destroy.argtypes = [VP]
    _sigs_done = True
    return L


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    assert t.is_contiguous()
    return t.data_ptr()


class MPCBatch:
    """A batch of MPC instances resident on one GPU (objects with T, n, m,
    A, B, q, r, u_box, as produced by ``workloads.mpc_batch``)."""

    def __init__(self, instances: Sequence, rho: float = 1.0, device: int = 0):
        L = _setup()
        self.instances = list(instances)
        N = len(self.instances)
        T = np.array([i.T for i in self.instances], np.int32)
        n = np.array([i.n for i in self.instances], np.int32)
        m = np.array([i.m for i in self.instances], np.int32)
        A = np.concatenate([np.asarray(i.A, np.float64).ravel() for i in self.instances])
        B = np.concatenate([np.asarray(i.B, np.float64).ravel() for i in self.instances])
        q = np.concatenate([np.asarray(i.q, np.float64).ravel() for i in self.instances])
        r = np.concatenate([np.asarray(i.r, np.float64).ravel() for i in self.instances])
        ub = np.array([i.u_box for i in self.instances], np.float64)
        h = VP()
        check(L.admm_mpc_batch_create(N, T.ctypes.data_as(I32P), n.ctypes.data_as(I32P),
                                      m.ctypes.data_as(I32P), A.ctypes.data_as(DP),
                                      B.ctypes.data_as(DP), q.ctypes.data_as(DP),
                                      r.ctypes.data_as(DP), ub.ctypes.data_as(DP),
                                      float(rho), int(device), ctypes.byref(h)))
        self._h = h
        self.device = device
        self.rho = rho
        zt, ut, xt = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(L.admm_mpc_batch_sizes(h, ctypes.byref(zt), ctypes.byref(ut), ctypes.byref(xt)))
        self.z_total, self.u_total, self.x0_total = zt.value, ut.value, xt.value
        self.n_inst = N
        k = (n + m).astype(np.int64)
        self.z_off = np.concatenate([[0], np.cumsum(T * k)])[:-1]
        self.x0_off = np.concatenate([[0], np.cumsum(n.astype(np.int64))])[:-1]
        self.u_off = np.concatenate([[0], np.cumsum(3 * T * k)])[:-1]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                lib().admm_mpc_batch_destroy(h)
            except Exception:
                pass
            self._h = None

    def solve(self, x0, z_out, iters_out, z_init=None, dual: bool = False,
              tol: float = 1e-4, max_iter: int = 10000, stream=None):
        check(_setup().admm_mpc_batch_solve(self._h, _ptr(x0), _ptr(z_init), 1 if dual else 0,
                                            float(tol), int(max_iter), _ptr(z_out),
                                            _ptr(iters_out), _stream(stream)))

    def solve_state(self, x0, z_out, iters_out, z_init=None, u_init=None, u_out=None,
                    tol: float = 1e-4, max_iter: int = 10000, stream=None):
        """Solve from (z_init, u_init) and return the final duals in u_out."""
        check(_setup().admm_mpc_batch_solve_state(self._h, _ptr(x0), _ptr(z_init), _ptr(u_init),
                                                  float(tol), int(max_iter), _ptr(z_out),
                                                  _ptr(u_out), _ptr(iters_out), _stream(stream)))

    def shift(self, x0, z, x0_next, z_next=None, u=None, u_next=None, w=None, stream=None):
        """One receding-horizon step: x0_next = A x0 + B u_0 + w, and the
        trajectory (and duals) moved one step forward."""
        check(_setup().admm_mpc_batch_shift(self._h, _ptr(x0), _ptr(z), _ptr(u), _ptr(w),
                                            _ptr(x0_next), _ptr(z_next), _ptr(u_next),
                                            _stream(stream)))

    def dual_complete(self, z, u_out, stream=None):
        check(_setup().admm_mpc_batch_dual_complete(self._h, _ptr(z), _ptr(u_out),
                                                    _stream(stream)))

    def set_plan(self, pack1: int = 4, order: int = 1, grid: int = 0):
        check(_setup().admm_mpc_batch_set_plan(self._h, pack1, order, grid))

    def plan(self):
        v = [ctypes.c_int32() for _ in range(4)]
        check(_setup().admm_mpc_batch_get_plan(self._h, *[ctypes.byref(x) for x in v]))
        return dict(pack1=v[0].value, order=v[1].value, grid=v[2].value, resident=v[3].value)

    def tune(self, x0, z_scratch, iters_scratch, tol=1e-4, max_iter=10000, reps=2,
             stream=None) -> List[float]:
        times = (ctypes.c_float * 64)()
        nc = ctypes.c_int32()
        check(_setup().admm_mpc_batch_tune(self._h, _ptr(x0), float(tol), int(max_iter),
                                           _ptr(z_scratch), _ptr(iters_scratch), int(reps),
                                           times, 64, ctypes.byref(nc), _stream(stream)))
        return [times[i] for i in range(nc.value)]

    # host-side layout helpers (no arithmetic of the method)
    def pack_x0(self, x0_list) -> np.ndarray:
        return np.concatenate([np.asarray(x, np.float32).ravel() for x in x0_list])

    def split_z(self, z) -> list:
        z = np.asarray(z)
        out = []
        for i, inst in enumerate(self.instances):
            o = self.z_off[i]
            out.append(z[o:o + inst.T * (inst.n + inst.m)])
        return out
