"""Parity measures shared by the GPU tests (no ADMM arithmetic here).

Every comparison of (z, u, x) is made twice: as a relative norm over the
whole vector and element by element, so that a few wrong slots cannot
hide inside a norm over millions of correct ones.

Scales: z relative to |z|; u and x relative to |o_e| + |z_b(e)| (u = m - z
cancels, so its rounding error follows the operands it is formed from,
not |u| itself); element-wise denominators also carry a floor of
FLOOR * (largest scale) so that entries that are zero in exact arithmetic
do not demand an error of zero.

Element-wise bound and the oracle's own sensitivity: some entries are
ill-conditioned in exact arithmetic (two nearly coincident disk centres
make the non-overlap direction d/|d| amplify any rounding of the centres
by |c|/|d|; disks passing through each other flip it).  `sensitivity`
reruns the oracle from the same start with rounding-size noise injected
into z and u every iteration and records, per entry, the largest distance
the oracle itself moves over four runs.  The element bound is then
|g_e - o_e| <= tol * den_e + K_SENS * sens_e: an entry may deviate by
K_SENS times what rounding alone moves it in the oracle, plus the
tolerance.  A wrong entry in a well-conditioned place still fails; an
entry that rounding alone moves by 1e-3 is judged against that.  Single
runs are a poor estimate of an ill-conditioned entry's response (at 5000
random disks, three steps from a common state, one entry moved by 3e-6,
8e-4, 2.6e-3 and 3e-3 in four runs), hence the maximum over four runs and
a factor of 20.  The number of entries whose allowance exceeds the
tolerance is reported (`*_allowed`).
"""
import numpy as np

FLOOR = 1e-2
K_SENS = 20.0


def _norm_rel(a, b, scale):
    d = np.linalg.norm(np.asarray(a, np.float64) - b)
    s = np.linalg.norm(scale)
    return float(d / s) if s > 0 else float(d)


def _elem_rel(a, b, scale, sens=None, tol=None):
    """Largest element-wise relative error beyond the allowance for the
    oracle's own sensitivity, and the number of entries whose allowance
    exceeds the tolerance."""
    scale = np.asarray(scale, np.float64)
    if scale.size == 0:
        return 0.0, 0
    den = scale + FLOOR * float(np.max(scale)) + 1e-300
    d = np.abs(np.asarray(a, np.float64) - b)
    if sens is None:
        return float(np.max(d / den)), 0
    allowed = int(np.count_nonzero(K_SENS * sens > (tol or 0.0) * den))
    return float(np.max(np.maximum(0.0, d - K_SENS * sens) / den)), allowed


def errors(gz, gu, gx, oz, ou, ox, sz, sens=None, tol=None):
    """Norm and element-wise relative errors of (z, u, x) against (oz, ou,
    ox); sz maps every edge slot to its z index; gx/ox may be None; sens:
    optional per-entry sensitivities {'z', 'u', 'x'} with the tolerance
    they are judged against (see module doc)."""
    sens = sens or {}
    out = {}

    def put(key, g, o, scale):
        out[key] = _norm_rel(g, o, scale)
        out[key + "_elem"], al = _elem_rel(g, o, scale, sens.get(key), tol)
        if key in sens:
            out[key + "_allowed"] = al
    oz = np.asarray(oz, np.float64)
    zs = np.abs(oz[sz])
    put("z", gz, oz, np.abs(oz))
    ou = np.asarray(ou, np.float64)
    put("u", gu, ou, np.abs(ou) + zs)
    if gx is not None and ox is not None:
        ox = np.asarray(ox, np.float64)
        put("x", gx, ox, np.abs(ox) + zs)
    return out


def norm_part(errs):
    return max(v for k, v in errs.items() if not k.endswith(("_elem", "_allowed")))


def check(errs, tol):
    """Assert every norm and element-wise measure below tol."""
    bad = {k: v for k, v in errs.items() if not k.endswith("_allowed") and not v < tol}
    assert not bad, (bad, errs)


def sensitivity(problem, iters, eps, alpha=None, z0=None, u0=None, runs=4, twa=False):
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
    a = O.OracleGraph(problem, alpha=alpha, twa=twa)
    a.set_state(z0, u0)
    a.run(iters)
    worst = {}
    sens = {"z": np.zeros_like(a.z), "u": np.zeros_like(a.u), "x": np.zeros_like(a.x)}
    for r in range(runs):
        b = O.OracleGraph(problem, alpha=alpha, twa=twa)
        rng = np.random.default_rng(100 + r)
        z = np.asarray(z0, np.float64)
        u = np.zeros(problem.n_slots) if u0 is None else np.asarray(u0, np.float64)
        for k in range(iters):
            zn = z * (1 + eps * rng.standard_normal(z.shape))
            un = u + eps * (np.abs(u) + np.abs(z[sz])) * rng.standard_normal(u.shape)
            if twa:
                # keep the variant's weights; a dual it reset to 0 stays 0
                if k == 0:
                    b.set_state(zn, np.where(u == 0.0, 0.0, un))
                else:
                    b.replace_zu(zn, np.where(u == 0.0, 0.0, un))
            else:
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
