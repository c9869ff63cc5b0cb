"""Oracle of the MPC warm start (test infrastructure only, FP64 numpy).

Dual completion: given a predicted trajectory z (per step (u_t, x_{t+1})),
choose the initial duals u^0 of every edge so that (z, u^0) would be a fixed
point of Algorithm 2 if z were optimal.  At a fixed point x = z for every
factor, so -rho u_a is a subgradient of f_a at z, and the duals around each
variable sum to zero (the z- and u-updates keep that sum at zero from
u^0 = 0).  For the MPC graph this fixes every dual by one backward pass over
the dynamics multipliers mu_t:
    mu_{T-1} = Q x_T,   mu_{t-1} = A^T mu_t + Q x_t
    rho u[dyn_t]  = (-A^T mu_t, -B^T mu_t, mu_t)  on (x_t, u_t, x_{t+1})
                    (t = 0: (-B^T mu_0, mu_0) on (u_0, x_1))
    rho u[quad x_t] = -Q x_t,   rho u[quad u_t] = -R u_t
    rho u[box u_t]  = B^T mu_t + R u_t
The returned vector follows the edge order of ``workloads.mpc_graph``.

Receding-horizon shift (``receding_shift``): one controller cycle's update of
the initial state and of the previous cycle's ADMM state.

Also a plain FP64 MLP (forward, mean-squared-error backward, Adam step) that
the GPU training kernels are checked against.
"""
from __future__ import annotations

import numpy as np


def dual_completion(inst, z, rho: float = 1.0) -> np.ndarray:
    T, n, m = inst.T, inst.n, inst.m
    blk = np.asarray(z, dtype=np.float64).reshape(T, n + m)
    U = blk[:, :m]                  # u_0..u_{T-1}
    X = blk[:, m:]                  # x_1..x_T
    Q, R = np.diag(inst.q), np.diag(inst.r)
    A, B = inst.A, inst.B
    mu = np.zeros((T, n))
    mu[T - 1] = Q @ X[T - 1]
    for t in range(T - 1, 0, -1):
        mu[t - 1] = A.T @ mu[t] + Q @ X[t - 1]
    out = []
    # dyn_0 on (u_0, x_1)
    out.append(-(B.T @ mu[0]) / rho)
    out.append(mu[0] / rho)
    # dyn_t on (x_t, u_t, x_{t+1}), t = 1..T-1
    for t in range(1, T):
        out.append(-(A.T @ mu[t]) / rho)
        out.append(-(B.T @ mu[t]) / rho)
        out.append(mu[t] / rho)
    # quadratic on x_1..x_T, then on u_0..u_{T-1}
    for t in range(T):
        out.append(-(Q @ X[t]) / rho)
    for t in range(T):
        out.append(-(R @ U[t]) / rho)
    if inst.u_box > 0:
        for t in range(T):
            out.append((B.T @ mu[t] + R @ U[t]) / rho)
    return np.concatenate(out)


def _edge_blocks(inst):
    """(start, length) of every dual block of ``workloads.mpc_graph``'s edge
    order, by name: dyn0 = (u_0, x_1); dyn[t] = (x_t, u_t, x_{t+1}) for
    t = 1..T-1; qx[t] on x_{t+1}; qu[t] and box[t] on u_t."""
    T, n, m = inst.T, inst.n, inst.m
    off = 0
    blocks = {"dyn0": (off, m + n)}
    off += m + n
    for t in range(1, T):
        blocks[("dyn", t)] = (off, 2 * n + m)
        off += 2 * n + m
    for t in range(T):
        blocks[("qx", t)] = (off, n)
        off += n
    for t in range(T):
        blocks[("qu", t)] = (off, m)
        off += m
    if inst.u_box > 0:
        for t in range(T):
            blocks[("box", t)] = (off, m)
            off += m
    return blocks, off


def receding_shift(inst, x0, z, u=None, w=None):
    """One controller cycle of receding-horizon MPC (Sec. V-B: the state is
    updated and the ADMM continues from the previous cycle's solution).

    The plant applies the first planned input, x0' = A x0 + B u_0 (+ w).
    The trajectory moves one step forward: step t of the new z is step t+1
    of the old one, and the new last step is u = 0, x = A x_T (the old
    horizon's end propagated with no input).  Every edge's dual moves with
    its step; the step-1 dynamics factor's dual on x_1 has no counterpart
    (the step-0 factor has x_0 as a parameter) and is dropped, and the new
    last step's duals are zero.  ``u`` follows ``workloads.mpc_graph``'s edge
    order.  Returns (x0', z', u') in FP64 (u' is None when u is)."""
    T, n, m = inst.T, inst.n, inst.m
    A, B = np.asarray(inst.A, np.float64), np.asarray(inst.B, np.float64)
    blk = np.asarray(z, dtype=np.float64).reshape(T, n + m)
    x0n = A @ np.asarray(x0, np.float64) + B @ blk[0, :m]
    if w is not None:
        x0n = x0n + np.asarray(w, np.float64)
    zn = np.zeros_like(blk)
    zn[:T - 1] = blk[1:]
    zn[T - 1, m:] = A @ blk[T - 1, m:]
    if u is None:
        return x0n, zn.ravel(), None
    u = np.asarray(u, dtype=np.float64)
    blocks, total = _edge_blocks(inst)
    assert u.shape == (total,)
    un = np.zeros(total)

    def get(key):
        s, ln = blocks[key]
        return u[s:s + ln]

    def put(key, v):
        s, ln = blocks[key]
        un[s:s + ln] = v

    if T > 1:
        put("dyn0", get(("dyn", 1))[n:])        # (u_1, x_2) parts become (u_0, x_1)
    for t in range(1, T - 1):
        put(("dyn", t), get(("dyn", t + 1)))
    for name in ("qx", "qu") + (("box",) if inst.u_box > 0 else ()):
        for t in range(T - 1):
            put((name, t), get((name, t + 1)))
    return x0n, zn.ravel(), un


# ---------------------------------------------------------------------------
# Plain MLP: y = W3 relu(W2 relu(W1 x + b1) + b2) + b3, loss = mean((y - t)^2)
# With bf16=True every matrix product takes its two operands rounded to
# bf16 (round to nearest even from float32), as the GPU's matrix cores do;
# the products themselves are exact FP64 sums.
# ---------------------------------------------------------------------------

def bf16_round(a):
    """Round to bf16 (nearest even), via float32, returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    return out.astype(np.float64)


def _mm(a, b, bf16):
    if bf16:
        return bf16_round(a) @ bf16_round(b)
    return a @ b


def mlp_forward(params, x, bf16=False, mean=None, sd=None):
    """Raw output yhat; with mean/sd given, also the denormalised
    y = mean + sd * yhat (returned as the first value)."""
    W1, b1, W2, b2, W3, b3 = params
    h1p = _mm(x, W1.T, bf16) + b1
    h1 = np.maximum(h1p, 0.0)
    h2p = _mm(h1, W2.T, bf16) + b2
    h2 = np.maximum(h2p, 0.0)
    y = _mm(h2, W3.T, bf16) + b3
    if mean is not None:
        y = mean + sd * y
    return y, (x, h1p, h1, h2p, h2)


def mlp_loss_grad(params, x, target, bf16=False, mean=None, sd=None):
    """Mean over all batch*outputs entries of (yhat - (target - mean)/sd)^2
    (mean 0, sd 1 when not given) and its gradient."""
    W1, b1, W2, b2, W3, b3 = params
    y, (x, h1p, h1, h2p, h2) = mlp_forward(params, x, bf16)
    if mean is not None:
        target = (target - mean) / sd
    N = y.size
    diff = y - target
    loss = float(np.sum(diff * diff) / N)
    gy = 2.0 * diff / N
    gW3 = _mm(gy.T, h2, bf16)
    gb3 = gy.sum(0)
    gh2 = _mm(gy, W3, bf16) * (h2 > 0)
    gW2 = _mm(gh2.T, h1, bf16)
    gb2 = gh2.sum(0)
    gh1 = _mm(gh2, W2, bf16) * (h1 > 0)
    gW1 = _mm(gh1.T, x, bf16)
    gb1 = gh1.sum(0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) in place; step counts from 1."""
    for p, g, mm, vv in zip(params, grads, m, v):
        mm *= beta1
        mm += (1 - beta1) * g
        vv *= beta2
        vv += (1 - beta2) * g * g
        mhat = mm / (1 - beta1 ** step)
        vhat = vv / (1 - beta2 ** step)
        p -= lr * mhat / (np.sqrt(vhat) + eps)


def mlp_shapes(n_in, hidden, n_out):
    return [(hidden, n_in), (hidden,), (hidden, hidden), (hidden,), (n_out, hidden), (n_out,)]


def unflatten(flat, n_in, hidden, n_out):
    out, o = [], 0
    for s in mlp_shapes(n_in, hidden, n_out):
        k = int(np.prod(s))
        out.append(np.asarray(flat[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def flatten(params):
    return np.concatenate([np.asarray(p).ravel() for p in params])
