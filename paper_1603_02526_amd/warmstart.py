"""Learned warm start for batched MPC.

For one fixed system (A, B, T, Q, R, box) an MLP maps the initial state x0
to the initial trajectory z0 of the ADMM.  The network is trained on the GPU
(library kernels) on solutions the batched ADMM solver itself produces from
x0 ~ N(0, I).  At solve time the predicted z0 is completed with the duals
that would make it a fixed point (dual completion), and the ADMM residual
decides when the solve is done, so a poor prediction costs iterations, never
accuracy; the cold start (z0 = 0, u0 = 0) stays available.

Only device memory and streams come from torch; every computation (ADMM,
dual completion, network forward/backward/Adam) is a library kernel.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Optional

import numpy as np

from . import mlp as MLPm
from . import mpc as MPCm


@dataclasses.dataclass
class System:
    A: np.ndarray
    B: np.ndarray
    T: int
    q: np.ndarray
    r: np.ndarray
    u_box: float = 1.0

    @property
    def n(self):
        return self.A.shape[0]

    @property
    def m(self):
        return self.B.shape[1]

    @property
    def z_dim(self):
        return self.T * (self.n + self.m)


class _Inst:
    """Instance record for MPCBatch (the system repeated; x0 comes per solve)."""

    def __init__(self, s: System):
        self.T, self.n, self.m = s.T, s.n, s.m
        self.A, self.B, self.q, self.r, self.u_box = s.A, s.B, s.q, s.r, s.u_box
        self.x0 = np.zeros(s.n)


class WarmStart:
    """Batched solver + MLP for one system.  ``batch`` instances per launch."""

    def __init__(self, system: System, batch: int = 4096, hidden: int = 256,
                 device: int = 0, init_seed: int = 0):
        import torch
        self.torch = torch
        self.sys = system
        self.batch = batch
        self.dev = torch.device("cuda", device)
        self.solver = MPCm.MPCBatch([_Inst(system)] * batch, rho=1.0, device=device)
        self.net = MLPm.MLP(system.n, hidden, system.z_dim, max_batch=batch, device=device)
        self.net.set_params(MLPm.init_params(system.n, hidden, system.z_dim, init_seed))
        self.z = torch.zeros(self.solver.z_total, dtype=torch.float32, device=self.dev)
        self.z0 = torch.zeros(self.solver.z_total, dtype=torch.float32, device=self.dev)
        self.iters = torch.zeros(batch, dtype=torch.int32, device=self.dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.dev)

    # ------------------------------------------------------------------
    def generate(self, n_samples: int, seed: int, tol: float = 1e-5, max_iter: int = 20000):
        """Cold-solve n_samples (rounded up to whole batches) x0 ~ N(0, I):
        returns device tensors X [N, n] and Z [N, z_dim]."""
        torch = self.torch
        nb = (n_samples + self.batch - 1) // self.batch
        N = nb * self.batch
        rng = np.random.default_rng(seed)
        X = torch.tensor(rng.standard_normal((N, self.sys.n)).astype(np.float32), device=self.dev)
        Z = torch.empty((N, self.sys.z_dim), dtype=torch.float32, device=self.dev)
        for b in range(nb):
            xb = X[b * self.batch:(b + 1) * self.batch].contiguous()
            zb = Z[b * self.batch:(b + 1) * self.batch]
            self.solver.solve(xb.view(-1), zb.view(-1), self.iters, tol=tol, max_iter=max_iter)
        torch.cuda.synchronize()
        return X, Z

    def train(self, X, Z, epochs: int, lr: float = 1e-3, lr_final: Optional[float] = None,
              warmup: int = 200):
        """Fit the network's fixed output affine to the targets' per-output
        mean and spread, then run Adam on contiguous minibatches of the
        (already i.i.d.) samples.  The learning rate rises linearly over the
        first `warmup` steps, then decays geometrically to lr_final.
        Returns the normalised loss of the last minibatch of each epoch."""
        torch = self.torch
        self.net.fit_output_scaling(Z, sd_min=1e-4)
        N = X.shape[0]
        steps_per_epoch = N // self.batch
        total = epochs * steps_per_epoch
        lr_final = lr if lr_final is None else lr_final
        hist = []
        k = 0
        for e in range(epochs):
            for s in range(steps_per_epoch):
                o = ((s + e * 7) % steps_per_epoch) * self.batch
                if k < warmup:
                    cur = lr * (k + 1) / warmup
                else:
                    cur = lr * (lr_final / lr) ** ((k - warmup) / max(1, total - warmup - 1))
                self.net.train_step(X[o:o + self.batch], Z[o:o + self.batch], cur, self.loss)
                k += 1
            torch.cuda.synchronize()
            hist.append(float(self.loss.item()))
        return hist

    # ------------------------------------------------------------------
    def solve(self, x0, mode: str, tol: float = 1e-4, max_iter: int = 20000):
        """x0: device [batch, n].  mode: 'cold', 'warm_z' (z0 from the MLP,
        u0 = 0) or 'warm' (z0 from the MLP plus dual completion).  Returns
        (z, iters) device tensors; the caller synchronises."""
        if mode == "cold":
            self.solver.solve(x0.view(-1), self.z, self.iters, tol=tol, max_iter=max_iter)
        else:
            self.net.forward(x0, self.z0.view(self.batch, -1))
            self.solver.solve(x0.view(-1), self.z, self.iters, z_init=self.z0,
                              dual=(mode == "warm"), tol=tol, max_iter=max_iter)
        return self.z, self.iters

    def timed(self, x0, mode: str, reps: int = 3, tol: float = 1e-4):
        """Best-of-reps wall time (s) of one full batch solve, including the
        network and the dual completion for warm modes, and its iterations."""
        torch = self.torch
        best = 1e30
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            self.solve(x0, mode, tol=tol)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        it = self.iters.cpu().numpy().copy()
        return best, it


class Family:
    """Several trained systems solved as one batch: every system's
    instances in one persistent launch (a batch finishes with its slowest
    instance, so one launch over all systems overlaps their tails).  Each
    system's network writes its block of the initial trajectories; the
    dual completion and the solve run once for the whole batch."""

    def __init__(self, starts, device: int = 0):
        import torch
        self.torch = torch
        self.starts = list(starts)
        insts = []
        for ws in self.starts:
            insts += [_Inst(ws.sys)] * ws.batch
        self.solver = MPCm.MPCBatch(insts, rho=1.0, device=device)
        dev = torch.device("cuda", device)
        self.z = torch.zeros(self.solver.z_total, dtype=torch.float32, device=dev)
        self.z0 = torch.zeros(self.solver.z_total, dtype=torch.float32, device=dev)
        self.iters = torch.zeros(self.solver.n_inst, dtype=torch.int32, device=dev)
        self.blocks = []
        off = 0
        for ws in self.starts:
            n = ws.batch * ws.sys.z_dim
            self.blocks.append((off, n))
            off += n

    def solve(self, x0s, x0_all, mode: str, tol: float = 1e-4, max_iter: int = 20000):
        """x0s: per system device [batch, n]; x0_all: their concatenation
        (flat).  Modes as WarmStart.solve."""
        if mode == "cold":
            self.solver.solve(x0_all, self.z, self.iters, tol=tol, max_iter=max_iter)
        else:
            for ws, x0, (off, n) in zip(self.starts, x0s, self.blocks):
                ws.net.forward(x0, self.z0[off:off + n].view(ws.batch, -1))
            self.solver.solve(x0_all, self.z, self.iters, z_init=self.z0,
                              dual=(mode == "warm"), tol=tol, max_iter=max_iter)
        return self.z, self.iters

    def timed(self, x0s, x0_all, mode: str, reps: int = 3, tol: float = 1e-4):
        torch = self.torch
        best = 1e30
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            self.solve(x0s, x0_all, mode, tol=tol)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best, self.iters.cpu().numpy().copy()

