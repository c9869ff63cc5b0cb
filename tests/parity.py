"""Parity measures shared by the GPU tests (no ADMM arithmetic here).

Every comparison of (z, u, x) is made twice: as a relative norm over the
whole vector and element by element, so that a few wrong slots cannot
hide inside a norm over millions of correct ones.

Scales: z relative to |z|; u and x relative to |o_e| + |z_b(e)| (u = m - z
cancels, so its rounding error follows the operands it is formed from,
not |u| itself); element-wise denominators also carry a floor of
FLOOR * (largest scale) so that entries that are zero in exact arithmetic
do not demand an error of zero.

Element-wise bound with the oracle's own sensitivity: some entries are
ill-conditioned in exact arithmetic (two nearly coincident disk centres
make the non-overlap direction d/|d| amplify any rounding of the centres
by |c|/|d|; disks passing through each other flip it).  `sensitivity`
reruns the oracle from the same start with rounding-size noise injected
into z and u every iteration and records, per entry, how far the oracle
itself moves.  The element bound is then |g_e - o_e| <= tol * scale_e +
K * sens_e: an entry may deviate by K times what rounding alone moves it
in the oracle, plus the tolerance.  A wrong entry in a well-conditioned
place still fails; an entry that rounding alone moves by 1e-3 is judged
against that.
"""
import numpy as np

FLOOR = 1e-2
K_SENS = 20.0


def _norm_rel(a, b, scale):
    d = np.linalg.norm(np.asarray(a, np.float64) - b)
    s = np.linalg.norm(scale)
    return float(d / s) if s > 0 else float(d)


def _elem_rel(a, b, scale, sens=None):
    scale = np.asarray(scale, np.float64)
    if scale.size == 0:
        return 0.0
    f = FLOOR * float(np.max(scale)) + 1e-300
    d = np.abs(np.asarray(a, np.float64) - b)
    if sens is not None:
        d = np.maximum(0.0, d - K_SENS * sens)
    return float(np.max(d / (scale + f)))


def errors(gz, gu, gx, oz, ou, ox, sz, sens=None):
    """Norm and element-wise relative errors of (z, u, x) against (oz, ou,
    ox); sz maps every edge slot to its z index; gx/ox may be None; sens:
    optional per-entry sensitivities {'z', 'u', 'x'} (see module doc)."""
    sens = sens or {}
    oz = np.asarray(oz, np.float64)
    zs = np.abs(oz[sz])
    out = {"z": _norm_rel(gz, oz, np.abs(oz)),
           "z_elem": _elem_rel(gz, oz, np.abs(oz), sens.get("z"))}
    ou = np.asarray(ou, np.float64)
    out["u"] = _norm_rel(gu, ou, np.abs(ou) + zs)
    out["u_elem"] = _elem_rel(gu, ou, np.abs(ou) + zs, sens.get("u"))
    if gx is not None and ox is not None:
        ox = np.asarray(ox, np.float64)
        out["x"] = _norm_rel(gx, ox, np.abs(ox) + zs)
        out["x_elem"] = _elem_rel(gx, ox, np.abs(ox) + zs, sens.get("x"))
    return out


def norm_part(errs):
    return max(v for k, v in errs.items() if not k.endswith("_elem"))


def sensitivity(problem, iters, eps, alpha=None, z0=None, u0=None, runs=2):
    """The oracle's own response to rounding-size relative noise eps (1e-16
    for FP64, 6e-8 for FP32) injected into z and u after every iteration,
    as the GPU's own rounding perturbs them, from the start (z0, u0)
    (default: the problem's z0, u = 0).  Returns (norm errors of the
    perturbed runs against the clean one, worst over runs, in the measures
    of `errors`; per-entry sensitivities {'z', 'u', 'x'}: the largest
    |perturbed - clean| over the runs)."""
    import oracle as O
    from tests.helpers import slot_z
    sz = slot_z(problem)
    z0 = problem.z0 if z0 is None else z0
    a = O.OracleGraph(problem, alpha=alpha)
    a.set_state(z0, u0)
    a.run(iters)
    worst = {}
    sens = {"z": np.zeros_like(a.z), "u": np.zeros_like(a.u), "x": np.zeros_like(a.x)}
    for r in range(runs):
        b = O.OracleGraph(problem, alpha=alpha)
        rng = np.random.default_rng(100 + r)
        z = np.asarray(z0, np.float64)
        u = np.zeros(problem.n_slots) if u0 is None else np.asarray(u0, np.float64)
        for k in range(iters):
            zn = z * (1 + eps * rng.standard_normal(z.shape))
            un = u + eps * (np.abs(u) + np.abs(z[sz])) * rng.standard_normal(u.shape)
            b.set_state(zn, un)
            b.run(1)
            z, u = b.z, b.u
        e = errors(b.z, b.u, b.x, a.z, a.u, a.x, sz)
        for k, v in e.items():
            worst[k] = max(worst.get(k, 0.0), v)
        sens["z"] = np.maximum(sens["z"], np.abs(b.z - a.z))
        sens["u"] = np.maximum(sens["u"], np.abs(b.u - a.u))
        sens["x"] = np.maximum(sens["x"], np.abs(b.x - a.x))
    return worst, sens
