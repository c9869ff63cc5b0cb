"""Independent closed forms and brute-force solvers that pin the oracle.

None of these reuse the oracle's formulas: each solves the defining
optimisation problem another way (Riccati recursion, an active-set KKT
system, scipy's SLSQP, dense least squares).
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import minimize


def riccati_lqr(inst):
    """Unconstrained finite-horizon LQR for x_{t+1} = A x_t + B u_t with cost
    1/2 sum_{t=1..T} x^T Q x + 1/2 sum_{t=0..T-1} u^T R u.  Returns z laid
    out per step as (u_t, x_{t+1})."""
    A, B, T = inst.A, inst.B, inst.T
    Q, R = np.diag(inst.q), np.diag(inst.r)
    P = Q.copy()
    K = [None] * T
    for t in range(T - 1, -1, -1):
        K[t] = np.linalg.solve(R + B.T @ P @ B, B.T @ P @ A)
        P = Q + A.T @ P @ A - A.T @ P @ B @ K[t]
    x = inst.x0.copy()
    out = []
    for t in range(T):
        u = -K[t] @ x
        x = A @ x + B @ u
        out.append(np.concatenate([u, x]))
    return np.concatenate(out)


def mpc_qp_matrices(inst):
    """Dense QP  min 1/2 y^T H y  s.t.  E y = f  for y = (u_0, x_1, ..., u_{T-1}, x_T)."""
    T, n, m = inst.T, inst.n, inst.m
    k = n + m
    N = T * k
    H = np.zeros((N, N))
    E = np.zeros((T * n, N))
    f = np.zeros(T * n)
    for t in range(T):
        o = t * k
        H[o:o + m, o:o + m] = np.diag(inst.r)
        H[o + m:o + k, o + m:o + k] = np.diag(inst.q)
        # x_{t+1} - B u_t - A x_t = 0
        E[t * n:(t + 1) * n, o + m:o + k] = np.eye(n)
        E[t * n:(t + 1) * n, o:o + m] = -inst.B
        if t == 0:
            f[0:n] = inst.A @ inst.x0
        else:
            E[t * n:(t + 1) * n, o - n:o] = -inst.A
    return H, E, f


def mpc_active_set_kkt(inst, z, tol=1e-6):
    """Given a candidate optimum z of the box-constrained MPC QP, fix the
    inputs that sit on the box, solve the equality-constrained KKT system
    exactly and return (y, max multiplier sign violation, inactive
    interior margin)."""
    T, n, m = inst.T, inst.n, inst.m
    k = n + m
    H, E, f = mpc_qp_matrices(inst)
    N = H.shape[0]
    u_idx = np.concatenate([np.arange(t * k, t * k + m) for t in range(T)])
    act = [i for i in u_idx if abs(abs(z[i]) - inst.u_box) < tol]
    J = np.zeros((len(act), N))
    bnd = np.zeros(len(act))
    for r, i in enumerate(act):
        J[r, i] = 1.0
        bnd[r] = np.sign(z[i]) * inst.u_box
    C = np.vstack([E, J])
    rhs_c = np.concatenate([f, bnd])
    K = np.block([[H, C.T], [C, np.zeros((C.shape[0], C.shape[0]))]])
    sol = np.linalg.solve(K, np.concatenate([np.zeros(N), rhs_c]))
    y = sol[:N]
    mu = sol[N + E.shape[0]:]
    # stationarity H y + E^T lam + J^T mu = 0; an upper bound needs mu >= 0,
    # a lower bound mu <= 0.
    sign_bad = 0.0
    for r, i in enumerate(act):
        sign_bad = max(sign_bad, -mu[r] * np.sign(bnd[r]))
    inactive = [i for i in u_idx if i not in act]
    margin = min([inst.u_box - abs(y[i]) for i in inactive], default=1.0)
    return y, sign_bad, margin


def svm_primal_slsqp(a, y, C, l2_weight=1.0):
    """min lambda/2 |w|^2 + C sum xi  s.t.  y_i (w.a_i + b) >= 1 - xi_i, xi >= 0."""
    Npt, d = a.shape

    def obj(v):
        w, xi = v[:d], v[d + 1:]
        return 0.5 * l2_weight * w @ w + C * xi.sum()

    def jac(v):
        g = np.zeros_like(v)
        g[:d] = l2_weight * v[:d]
        g[d + 1:] = C
        return g

    cons = [dict(type="ineq",
                 fun=lambda v: y * (a @ v[:d] + v[d]) - 1.0 + v[d + 1:],
                 jac=lambda v: np.hstack([y[:, None] * a, y[:, None],
                                          np.eye(Npt)]))]
    bounds = [(None, None)] * (d + 1) + [(0.0, None)] * Npt
    v0 = np.zeros(d + 1 + Npt)
    v0[d + 1:] = 1.0
    res = minimize(obj, v0, jac=jac, constraints=cons, bounds=bounds,
                   method="SLSQP", options=dict(ftol=1e-15, maxiter=2000))
    return res.x[:d], res.x[d], res.fun


def slsqp(obj, x0, cons=(), bounds=None):
    res = minimize(obj, x0, constraints=list(cons), bounds=bounds,
                   method="SLSQP", options=dict(ftol=1e-15, maxiter=1000))
    return res.x, res.fun
