"""Seeded synthetic problem generators for factor-graph ADMM.

This module describes *problems*: the variables, the factors that couple
them and the data those factors carry.  It performs none of the ADMM
arithmetic (no proximal operator, no averaging, no dual update), so the
CPU oracle under ``oracle/`` and the HIP library can both be fed from it
without sharing any of the method's code.

The problem families follow the paper's numerical section:

* circle packing (Sec. V-A): N disks with centre ``c_i`` (2-D variable)
  and radius ``r_i`` (1-D variable); one non-overlap factor per pair, one
  wall factor per disk and half-plane, one radius-maximisation factor per
  disk.  The paper's count is ``2N^2 - N + 2NS`` edges,
  ``0.5N(N-1) + N + NS`` factors and ``2N`` variable nodes.
* linear MPC (Sec. V-B): state nodes ``x_t`` and input nodes ``u_t`` with a
  linear-dynamics equality factor per step, a quadratic stage-cost factor
  per node and an input box factor per input node.
* soft-margin linear SVM (Sec. V-C): scalar nodes ``w_1..w_d, b``, one hinge
  factor per data point and one squared-norm factor on ``w``.

Every generator is a pure function of its arguments and seed
(``numpy.random.default_rng``), so both sides of a parity test see
bit-identical inputs.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np

KINDS = ("nonoverlap", "wall", "radius", "quad", "box", "hinge", "l2",
         "lindyn", "lindyn0", "minerr", "equal", "margin")


@dataclasses.dataclass
class FactorGroup:
    """``n`` factors of one kind with the same edge signature.

    var_ids: int32 [n, arity]; params: float64 [n, param_len] or, when
    ``shared`` is true, [param_len] used by every factor of the group.
    rho, alpha: the edge weights of this group's edges (None: the
    problem's values).
    """
    kind: str
    var_ids: np.ndarray
    params: np.ndarray
    shared: bool = False
    rho: Optional[float] = None
    alpha: Optional[float] = None

    @property
    def n(self) -> int:
        return int(self.var_ids.shape[0])

    @property
    def arity(self) -> int:
        return int(self.var_ids.shape[1])

    @property
    def param_len(self) -> int:
        return int(self.params.shape[-1]) if self.params.size else 0


@dataclasses.dataclass
class Problem:
    """A factor graph plus its ADMM parameters and initial z."""
    name: str
    var_dims: np.ndarray            # int32 [n_vars]
    groups: List[FactorGroup]
    z0: np.ndarray                  # float64 [sum(var_dims)], variable order
    rho: float = 1.0
    alpha: float = 1.0
    meta: Dict = dataclasses.field(default_factory=dict)

    @property
    def n_vars(self) -> int:
        return int(self.var_dims.shape[0])

    @property
    def n_scalars(self) -> int:
        return int(self.var_dims.sum())

    @property
    def n_factors(self) -> int:
        return sum(g.n for g in self.groups)

    @property
    def n_edges(self) -> int:
        return sum(g.n * g.arity for g in self.groups)

    @property
    def n_slots(self) -> int:
        return sum(int(self.var_dims[g.var_ids].sum()) for g in self.groups)

    def var_offsets(self) -> np.ndarray:
        off = np.zeros(self.n_vars + 1, dtype=np.int64)
        np.cumsum(self.var_dims, out=off[1:])
        return off


# ----------------------------------------------------------------------------
# Circle packing
# ----------------------------------------------------------------------------

SQRT3 = float(np.sqrt(3.0))

# Unit-side equilateral triangle, vertices (0,0), (1,0), (1/2, sqrt(3)/2).
# Each wall is the half-plane Q^T (c - V) >= r with an inward unit normal Q.
TRIANGLE_WALLS = (
    ((0.0, 1.0), (0.0, 0.0)),
    ((SQRT3 / 2.0, -0.5), (0.0, 0.0)),
    ((-SQRT3 / 2.0, -0.5), (1.0, 0.0)),
)
# Unit square [0,1]^2.
SQUARE_WALLS = (
    ((1.0, 0.0), (0.0, 0.0)),
    ((-1.0, 0.0), (1.0, 0.0)),
    ((0.0, 1.0), (0.0, 0.0)),
    ((0.0, -1.0), (0.0, 1.0)),
)


def _sample_triangle(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform points in the unit triangle by parallelogram reflection."""
    u = rng.random(n)
    v = rng.random(n)
    flip = (u + v) > 1.0
    u = np.where(flip, 1.0 - u, u)
    v = np.where(flip, 1.0 - v, v)
    b = np.array([1.0, 0.0])
    c = np.array([0.5, SQRT3 / 2.0])
    return u[:, None] * b[None, :] + v[:, None] * c[None, :]


def packing(n_circles: int, shape: str = "triangle", r_max: float = 0.1,
            seed: int = 1000, gamma: float = 0.5, rho: float = 1.0,
            alpha: float = 1.0, with_walls: bool = True,
            with_radius: bool = True) -> Problem:
    """Disks in a polygon (Sec. V-A).

    Variable ids: ``c_i = 2i`` (dim 2), ``r_i = 2i + 1`` (dim 1).
    Factor order: all pairs ``i < j`` in lexicographic order, then the wall
    factors (disk-major, wall-minor), then one radius factor per disk with
    weight ``gamma`` on ``-1/2 r^2``.
    """
    rng = np.random.default_rng(seed)
    N = int(n_circles)
    if shape == "triangle":
        walls = TRIANGLE_WALLS
        centres = _sample_triangle(rng, N)
    elif shape == "square":
        walls = SQUARE_WALLS
        centres = rng.random((N, 2))
    else:
        raise ValueError(f"unknown shape {shape!r}")
    radii = rng.random(N) * r_max

    dims = np.tile(np.array([2, 1], dtype=np.int32), N)
    z0 = np.empty(3 * N, dtype=np.float64)
    z0[0::3] = centres[:, 0]
    z0[1::3] = centres[:, 1]
    z0[2::3] = radii

    groups: List[FactorGroup] = []
    if N >= 2:
        ii, jj = np.triu_indices(N, k=1)
        vid = np.stack([2 * ii, 2 * ii + 1, 2 * jj, 2 * jj + 1], axis=1)
        groups.append(FactorGroup("nonoverlap", vid.astype(np.int32),
                                  np.zeros((0,), np.float64), shared=True))
    if with_walls:
        S = len(walls)
        disk = np.repeat(np.arange(N), S)
        wall = np.tile(np.arange(S), N)
        vid = np.stack([2 * disk, 2 * disk + 1], axis=1).astype(np.int32)
        wp = np.array([[q[0], q[1], v[0], v[1]] for q, v in walls])
        groups.append(FactorGroup("wall", vid, wp[wall].copy()))
    if with_radius:
        vid = (2 * np.arange(N) + 1).astype(np.int32)[:, None]
        groups.append(FactorGroup("radius", vid,
                                  np.array([gamma], np.float64), shared=True))
    return Problem(name=f"packing_{shape}_{N}", var_dims=dims, groups=groups,
                   z0=z0, rho=rho, alpha=alpha,
                   meta=dict(n_circles=N, shape=shape, walls=walls,
                             gamma=gamma, r_max=r_max, seed=seed))


def packing_counts(N: int, S: int) -> Dict[str, int]:
    """The paper's graph-size formulas for N disks and S half-planes."""
    return dict(edges=2 * N * N - N + 2 * N * S,
                factors=N * (N - 1) // 2 + N + N * S,
                var_nodes=2 * N)


# ----------------------------------------------------------------------------
# Soft-margin linear SVM
# ----------------------------------------------------------------------------

def svm_data(n_points: int, d: int, seed: int, sep: float = 0.5):
    """Two Gaussian classes, labels +-1 with probability 1/2, class means
    ``+-sep * 1_d`` and unit covariance."""
    rng = np.random.default_rng(seed)
    y = np.where(rng.random(n_points) < 0.5, -1.0, 1.0)
    a = rng.standard_normal((n_points, d)) + sep * y[:, None]
    return a, y


def svm(n_points: int, d: int = 20, seed: int = 1002, C: float = 1.0,
        rho: float = 1.0, alpha: float = 1.0, sep: float = 0.5,
        l2_weight: float = 1.0) -> Problem:
    """Hinge-factor SVM graph: scalar nodes ``w_1..w_d`` (ids 0..d-1) and
    ``b`` (id d).  Factors: one hinge per point over (w_1..w_d, b) with
    data (a_i, y_i, C), then one squared-norm factor over w_1..w_d."""
    a, y = svm_data(n_points, d, seed, sep)
    dims = np.ones(d + 1, dtype=np.int32)
    vid = np.broadcast_to(np.arange(d + 1, dtype=np.int32),
                          (n_points, d + 1)).copy()
    hp = np.concatenate([a, y[:, None], np.full((n_points, 1), C)], axis=1)
    groups = [
        FactorGroup("hinge", vid, hp),
        FactorGroup("l2", np.arange(d, dtype=np.int32)[None, :],
                    np.array([l2_weight], np.float64), shared=True),
    ]
    return Problem(name=f"svm_{n_points}x{d}", var_dims=dims, groups=groups,
                   z0=np.zeros(d + 1), rho=rho, alpha=alpha,
                   meta=dict(a=a, y=y, C=C, d=d, seed=seed,
                             l2_weight=l2_weight))


def svm_copies(n_points: int, d: int = 20, seed: int = 1002, lam: float = 1.0,
               rho: float = 1.0, alpha: float = 1.0, sep: float = 0.5) -> Problem:
    """The paper's own SVM graph (Sec. V-C): one copy ``w_i`` (dim d) of the
    weight vector per point, the bias ``b`` and one slack ``xi_i`` per point.

    Variable ids: ``w_i = i`` (dim d), ``b = N`` (dim 1), ``xi_i = N + 1 + i``
    (dim 1).  Factors, in this order: one margin factor per point on
    (w_i, b, xi_i) with data (a_i, y_i); one minimal-error factor per slack
    (weight ``lam``); one squared-norm factor per copy with weight 1/N (the
    1/2 |w|^2 term split into N equal parts); equality factors joining
    consecutive copies (w_i, w_{i+1}), a chain (the paper's figure is not
    available; a chain keeps every copy's degree at most four).  At
    consensus the objective is 1/2 |w|^2 + lam sum xi_i subject to the
    margins, the problem ``svm`` states with hinge factors and C = lam."""
    a, y = svm_data(n_points, d, seed, sep)
    N = int(n_points)
    dims = np.concatenate([np.full(N, d, np.int32), np.ones(1 + N, np.int32)])
    i = np.arange(N, dtype=np.int32)
    groups = [
        FactorGroup("margin", np.stack([i, np.full(N, N, np.int32), N + 1 + i], axis=1),
                    np.concatenate([a, y[:, None]], axis=1)),
        FactorGroup("minerr", (N + 1 + i)[:, None], np.array([lam], np.float64), shared=True),
        FactorGroup("l2", i[:, None], np.array([1.0 / N], np.float64), shared=True),
    ]
    if N > 1:
        groups.append(FactorGroup("equal", np.stack([i[:-1], i[1:]], axis=1),
                                  np.zeros((0,), np.float64), shared=True))
    return Problem(name=f"svm_copies_{N}x{d}", var_dims=dims, groups=groups,
                   z0=np.zeros(int(dims.sum())), rho=rho, alpha=alpha,
                   meta=dict(a=a, y=y, C=lam, d=d, seed=seed))


# ----------------------------------------------------------------------------
# Linear MPC
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class MPCInstance:
    """x_{t+1} = A x_t + B u_t, t = 0..T-1, x_0 given.  Stage cost
    1/2 (x_t^T diag(q) x_t + u_t^T diag(r) u_t) on x_1..x_T and u_0..u_{T-1};
    |u_t|_inf <= u_box (u_box <= 0 means no box)."""
    T: int
    n: int
    m: int
    A: np.ndarray
    B: np.ndarray
    x0: np.ndarray
    q: np.ndarray
    r: np.ndarray
    u_box: float = 1.0


def mpc_system(rng: np.random.Generator, n: int, m: int, rho_spec=0.95):
    G = rng.standard_normal((n, n))
    A = rho_spec * G / np.max(np.abs(np.linalg.eigvals(G)))
    B = rng.standard_normal((n, m)) / np.sqrt(n)
    return A, B


def mpc_batch(n_inst: int, seed: int = 1003, T_range=(20, 200),
              n_range=(4, 12), m_range=(2, 4), q=1.0, r=0.1,
              u_box=1.0) -> List[MPCInstance]:
    """Uneven batch: T, n, m uniform integers (inclusive ranges); A with
    spectral radius 0.95, B Gaussian / sqrt(n), Q = qI, R = rI, x0 ~ N(0, I)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_inst):
        T = int(rng.integers(T_range[0], T_range[1] + 1))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        A, B = mpc_system(rng, n, m)
        x0 = rng.standard_normal(n)
        out.append(MPCInstance(T, n, m, A, B, x0, np.full(n, q),
                               np.full(m, r), u_box))
    return out


def mpc_family(n_systems: int = 8, n: int = 8, m: int = 3, T: int = 100,
               system_seed0: int = 2000):
    """Fixed systems of the warm-start family: system s uses seed
    ``system_seed0 + s`` and the batch generation rule for A and B."""
    systems = []
    for s in range(n_systems):
        rng = np.random.default_rng(system_seed0 + s)
        A, B = mpc_system(rng, n, m)
        systems.append((A, B))
    return systems


def mpc_x0(n: int, count: int, seed: int) -> np.ndarray:
    """Initial states x0 ~ N(0, I), shape [count, n]."""
    return np.random.default_rng(seed).standard_normal((count, n))


def mpc_disturbance(total: int, cycles: int, seed: int, sd: float = 0.1) -> np.ndarray:
    """Plant disturbances of a closed loop, w ~ N(0, sd^2 I) per state entry
    and cycle, shape [cycles, total] (float32)."""
    return (sd * np.random.default_rng(seed).standard_normal((cycles, total))).astype(np.float32)


def mpc_graph(inst: MPCInstance, box: bool = True) -> Problem:
    """Factor graph of one MPC instance.

    Variable ids: ``u_t = 2t`` (dim m) and ``x_{t+1} = 2t + 1`` (dim n) for
    t = 0..T-1, so z is laid out per step as (u_t, x_{t+1}).
    Factors (in this order): the t = 0 dynamics factor on (u_0, x_1) carrying
    (A, B, x0); the dynamics factors on (x_t, u_t, x_{t+1}) for t = 1..T-1
    carrying (A, B); a quadratic factor on every x_t and on every u_t; a box
    factor on every u_t.
    """
    T, n, m = inst.T, inst.n, inst.m
    dims = np.empty(2 * T, dtype=np.int32)
    dims[0::2] = m
    dims[1::2] = n
    AB = np.concatenate([inst.A.ravel(), inst.B.ravel()])
    groups = [FactorGroup("lindyn0", np.array([[0, 1]], np.int32),
                          np.concatenate([AB, inst.x0])[None, :])]
    if T > 1:
        t = np.arange(1, T)
        vid = np.stack([2 * t - 1, 2 * t, 2 * t + 1], axis=1).astype(np.int32)
        groups.append(FactorGroup("lindyn", vid, AB.copy(), shared=True))
    groups.append(FactorGroup("quad", (2 * np.arange(T) + 1).astype(np.int32)[:, None],
                              inst.q.astype(np.float64).copy(), shared=True))
    groups.append(FactorGroup("quad", (2 * np.arange(T)).astype(np.int32)[:, None],
                              inst.r.astype(np.float64).copy(), shared=True))
    if box and inst.u_box > 0:
        groups.append(FactorGroup("box", (2 * np.arange(T)).astype(np.int32)[:, None],
                                  np.array([-inst.u_box, inst.u_box]), shared=True))
    return Problem(name=f"mpc_T{T}_n{n}_m{m}", var_dims=dims, groups=groups,
                   z0=np.zeros(int(dims.sum())), rho=1.0, alpha=1.0,
                   meta=dict(T=T, n=n, m=m))


# ----------------------------------------------------------------------------
# The paper's Fig. 1 example topology
# ----------------------------------------------------------------------------

def fig1_topology():
    """f = f1(w1,w2,w3) + f2(w1,w4,w5) + f3(w2,w5) + f4(w5), 0-based ids.
    Returns the factor list; the edge order the paper states is the order
    of these lists concatenated."""
    return [[0, 1, 2], [0, 3, 4], [1, 4], [4]]


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def workload(name: str) -> Problem:
    """The named synthetic workloads of the benchmark configurations."""
    if name == "packing_tri10":
        return packing(10, "triangle", 0.1, seed=1000)
    if name == "packing_sq2000":
        return packing(2000, "square", 0.02, seed=1001)
    if name == "packing_sq5000":
        return packing(5000, "square", 0.008, seed=1005)
    if name == "svm_100k_d20":
        return svm(100_000, 20, seed=1002)
    raise KeyError(name)
