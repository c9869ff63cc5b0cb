// ADMM-on-a-factor-graph oracle: plain, serial, double precision.
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
// reference that the HIP library is checked against.  Only the tests, the
// smoke check and the CPU-baseline leg of the benchmark may load it; the
// product path never does.  It shares no code, header, table or helper
// with the GPU library.
//
// What it computes (paper Sec. II, Algorithm 2, and eq. (3) for the
// proximal operator):
//   repeat
//     x-update: for every factor a, x_(a,.) = Prox_{f_a,rho}(n_(a,.))
//     m-update: m_e = x_e + u_e                      for every edge e
//     z-update: z_b = sum_{a in db} rho m_(a,b) / sum_{a in db} rho
//     u-update: u_e = u_e + alpha (x_e - z_b)
//     n-update: n_e = z_b - u_e
// Each update is its own loop over factors, edges or variables, in the
// paper's order; the z-update sums each variable's incoming rho m in
// edge-creation order.  Every edge carries its own rho_(a,b) and
// alpha_(a,b) (Algorithm 2); here they are set per group of factors (all
// edges of one factor share them, as the appendix's closed forms assume),
// and default to one graph-wide value.
//
// The same source builds serially (the default) or with OpenMP for a
// multi-core timing: each of the loops is then a parallel loop over its own
// index (the paper's first CPU scheme, one parallel loop per update).
// Every element is still computed by the same arithmetic in the same order,
// so both builds give bit-identical results.
//
// Proximal operators (paper appendix, with the readings listed in the
// design notes):
//   nonoverlap  (App. A, first PO)  projection onto |c1-c2| >= r1+r2; the
//               radii move by -D/4 (the printed +1 radius direction leaves
//               the pair overlapping); n_hat = (1,0) when the centres meet.
//   wall        (App. A, second PO) projection onto Q^T(c-V) >= r, general
//               |Q|.
//   radius      (App. A, third PO)  argmin -gamma/2 r^2 + rho/2 (r-n)^2 over
//               r >= 0, which needs rho > gamma.
//   quad        (App. B, cost PO)   f = 1/2 sum_k q_k x_k^2.
//   lindyn(0)   (App. B, dynamics PO) projection onto x' = A x + B u
//               (x fixed to the parameter x0 for the first step), solved
//               from its normal equations with Gaussian elimination.
//   box         clip to [lo, hi] per component.
//   hinge       f = C max(0, 1 - y(w.a + b)), the minimal-error and margin
//               POs of App. C merged into one factor per point.
//   l2          f = lambda/2 |w|^2 (App. C, norm-two PO).
//   minerr      f = lambda sum xi_k with xi_k >= 0 (App. C, minimal-error
//               PO): xi = (n - lambda/rho)^+.
//   equal       w1 = w2 (App. C, equality PO): both take the mean.
//   margin      projection onto y(w.x + b) >= 1 - xi (App. C, one-point
//               margin PO).  The printed closed form has a garbled product
//               and signs that leave the output infeasible; the projection
//               is rederived from its Lagrange conditions.
//
// Stopping measures (the paper leaves them open): after the u-update,
//   r = max_e |x_e - z_b|        s = rho * max_b |z_b - z_b(previous)|.
//
// Three-weight variant (Sec. II names improved update schemes for the
// per-edge weights, citing the three-weight message-passing algorithm of
// Derbinsky et al.; the reading used here is listed in the design notes).
// Every message carries a weight in {0, rho_(a,b), infinity}; no operator
// here is ever certain of a value, so only 0 and rho occur:
//   x-update: each factor's prox uses the weights of the messages it
//     receives (left weights) and sets the weight of each message it
//     sends (right weights): a non-overlap or wall factor whose constraint
//     is inactive (the prox leaves n unchanged) sends weight 0 on all its
//     edges, every other factor sends rho.  A zero left weight marks a
//     variable no factor had an opinion on: among the factor's edges, the
//     zero-weight ones then absorb the whole correction, in equal shares.
//   z-update: z_b = sum w m / sum w over b's edges; when every weight is 0
//     z_b keeps its value.  Every edge of b then receives left weight rho
//     (its own) if some weight was positive, else 0.
//   u-update: u_e += alpha (x_e - z_b) for edges sent with weight rho; u_e
//     is reset to 0 for edges sent with weight 0 (an inactive constraint
//     carries no multiplier).
// With every weight equal to rho the iteration is Algorithm 2 exactly.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

enum Kind {
  K_NONOVERLAP = 1,
  K_WALL = 2,
  K_RADIUS = 3,
  K_QUAD = 4,
  K_BOX = 5,
  K_HINGE = 6,
  K_L2 = 7,
  K_LINDYN = 8,
  K_LINDYN0 = 9,
  K_MINERR = 10,
  K_EQUAL = 11,
  K_MARGIN = 12,
};

struct Factor {
  int kind;
  std::vector<int> vars;     // variable id of each edge, in edge order
  std::vector<long> slot;    // first slot of each edge in the edge arrays
  int nslots;                // total scalar slots of this factor
  std::vector<double> p;     // parameters
  double rho = 0.0, alpha = 0.0;  // this factor's edge weights (0: the graph's)
};

struct Graph {
  std::vector<int> dim;      // per variable
  std::vector<long> zoff;    // per variable, offset into z
  long nz = 0;
  std::vector<Factor> F;
  long nslot = 0;            // total edge slots
  std::vector<long> slot_z;  // z index of each edge slot
  std::vector<double> z, zprev, x, m, u, n;
  std::vector<long> zbeg, zedges;  // edges of each variable, in creation order
  std::vector<double> erho, ealpha, vrho;  // per edge slot rho, alpha; per z the largest rho
  long lists_for = -1;             // nslot the tables were built for
  double rho = 1.0, alpha = 1.0;
  double r_primal = 0.0, r_dual = 0.0;
  bool twa = false;                 // three-weight variant
  std::vector<double> wr, wl;       // per edge slot: sent and received weights
};

// ---------------------------------------------------------------------------
// Small dense linear solve: Gaussian elimination with partial pivoting.
// a is k x k row-major (destroyed), b is k (overwritten with the solution).
// ---------------------------------------------------------------------------
bool solve_dense(std::vector<double>& a, std::vector<double>& b, int k) {
  for (int c = 0; c < k; ++c) {
    int piv = c;
    for (int r = c + 1; r < k; ++r)
      if (std::fabs(a[r * k + c]) > std::fabs(a[piv * k + c])) piv = r;
    if (a[piv * k + c] == 0.0) return false;
    if (piv != c) {
      for (int j = 0; j < k; ++j) std::swap(a[c * k + j], a[piv * k + j]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < k; ++r) {
      double f = a[r * k + c] / a[c * k + c];
      if (f == 0.0) continue;
      for (int j = c; j < k; ++j) a[r * k + j] -= f * a[c * k + j];
      b[r] -= f * b[c];
    }
  }
  for (int r = k - 1; r >= 0; --r) {
    double s = b[r];
    for (int j = r + 1; j < k; ++j) s -= a[r * k + j] * b[j];
    b[r] = s / a[r * k + r];
  }
  return true;
}

// ---------------------------------------------------------------------------
// Proximal operators.  nv: the factor's n vector (its edges' slots
// concatenated), out: x for the same slots.  dims: dimension of each edge.
// ---------------------------------------------------------------------------

// |c1 - c2| >= r1 + r2 on edges (c1, r1, c2, r2).
void prox_nonoverlap(const double* nv, double rho, double* out) {
  (void)rho;  // equal weights on all four edges: the step does not depend on rho
  const double c1x = nv[0], c1y = nv[1], r1 = nv[2];
  const double c2x = nv[3], c2y = nv[4], r2 = nv[5];
  const double dx = c2x - c1x, dy = c2y - c1y;
  const double L = std::sqrt(dx * dx + dy * dy);
  double hx = 1.0, hy = 0.0;
  if (L > 0.0) { hx = dx / L; hy = dy / L; }
  const double D = std::max(0.0, r1 + r2 - L);
  // lambda = D / (1/rho + 1/rho + 1/rho + 1/rho); each edge moves lambda/rho.
  const double lam = D / (4.0 / rho);
  const double step = lam / rho;
  out[0] = c1x - step * hx;
  out[1] = c1y - step * hy;
  out[2] = r1 - step;
  out[3] = c2x + step * hx;
  out[4] = c2y + step * hy;
  out[5] = r2 - step;
}

// Q^T (c - V) >= r on edges (c, r); p = (Qx, Qy, Vx, Vy).
void prox_wall(const double* nv, const double* p, double rho, double* out) {
  const double Qx = p[0], Qy = p[1], Vx = p[2], Vy = p[3];
  const double g = Qx * (nv[0] - Vx) + Qy * (nv[1] - Vy) - nv[2];
  out[0] = nv[0]; out[1] = nv[1]; out[2] = nv[2];
  if (g >= 0.0) return;
  const double lam = -g / ((Qx * Qx + Qy * Qy) / rho + 1.0 / rho);
  out[0] = nv[0] + (lam / rho) * Qx;
  out[1] = nv[1] + (lam / rho) * Qy;
  out[2] = nv[2] - lam / rho;
}

// argmin_{r >= 0} -gamma/2 r^2 + rho/2 (r - n)^2.
void prox_radius(const double* nv, double gamma, double rho, double* out) {
  out[0] = std::max(0.0, rho * nv[0] / (rho - gamma));
}

// f = 1/2 sum q_k x_k^2.
void prox_quad(const double* nv, int k, const double* q, double rho, double* out) {
  for (int i = 0; i < k; ++i) out[i] = rho * nv[i] / (rho + q[i]);
}

void prox_box(const double* nv, int k, double lo, double hi, double* out) {
  for (int i = 0; i < k; ++i) out[i] = std::min(hi, std::max(lo, nv[i]));
}

// f = C max(0, 1 - y (w.a + b)) on scalar edges (w_1..w_d, b);
// p = (a_1..a_d, y, C).
void prox_hinge(const double* nv, int d, const double* p, double rho, double* out) {
  const double y = p[d], C = p[d + 1];
  double s = nv[d];
  double aa = 0.0;
  for (int k = 0; k < d; ++k) { s += nv[k] * p[k]; aa += p[k] * p[k]; }
  s *= y;
  const double D = aa / rho + 1.0 / rho;
  const double tau = std::min(C, std::max(0.0, (1.0 - s) / D));
  for (int k = 0; k < d; ++k) out[k] = nv[k] + tau * y * p[k] / rho;
  out[d] = nv[d] + tau * y / rho;
}

// f = lam/2 |w|^2.
void prox_l2(const double* nv, int k, double lam, double rho, double* out) {
  for (int i = 0; i < k; ++i) out[i] = rho * nv[i] / (rho + lam);
}

// lambda sum xi_k over xi_k >= 0: a shifted clamp at zero.
void prox_minerr(const double* nv, int k, double lam, double rho, double* out) {
  for (int i = 0; i < k; ++i) out[i] = std::max(0.0, nv[i] - lam / rho);
}

// w1 = w2 with equal weights on both edges: the nearest point of the
// diagonal is the mean of the two inputs.
void prox_equal(const double* nv, int d, double* out) {
  for (int i = 0; i < d; ++i) {
    const double v = 0.5 * (nv[i] + nv[d + i]);
    out[i] = v;
    out[d + i] = v;
  }
}

// Edges (w (d), b, xi), p = (x_1..x_d, y).  minimise rho/2 |(w,b,xi) - n|^2
// subject to y(w.x + b) + xi >= 1.  If n satisfies the constraint it is its
// own projection.  Otherwise the constraint is active with multiplier
// mu >= 0: w = n_w + mu y x / rho, b = n_b + mu y / rho, xi = n_xi + mu / rho,
// and substituting into the active constraint (y^2 = 1) gives
// mu = (1 - g0) / ((|x|^2 + 2) / rho) with g0 = y(n_w.x + n_b) + n_xi.
void prox_margin(const double* nv, int d, const double* p, double rho, double* out) {
  const double y = p[d];
  double wx = 0.0, xx = 0.0;
  for (int k = 0; k < d; ++k) { wx += nv[k] * p[k]; xx += p[k] * p[k]; }
  const double g0 = y * (wx + nv[d]) + nv[d + 1];
  for (int k = 0; k < d + 2; ++k) out[k] = nv[k];
  if (g0 >= 1.0) return;
  const double mu = (1.0 - g0) / ((xx + 2.0) / rho);
  for (int k = 0; k < d; ++k) out[k] = nv[k] + mu * y * p[k] / rho;
  out[d] = nv[d] + mu * y / rho;
  out[d + 1] = nv[d + 1] + mu / rho;
}

// Projection onto x' = A x + B u on edges (x, u, x') with A n x n, B n x m
// (row-major).  Minimise |a - a_n|^2 + |M a - b|^2 with a = (x, u),
// M = [A B], b = n_x': normal equations (I + M^T M) a = a_n + M^T b.
void prox_lindyn(const double* nv, int n, int m, const double* A,
                 const double* B, double* out) {
  const int k = n + m;
  std::vector<double> M(static_cast<size_t>(n) * k);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) M[i * k + j] = A[i * n + j];
    for (int j = 0; j < m; ++j) M[i * k + n + j] = B[i * m + j];
  }
  const double* an = nv;
  const double* b = nv + k;
  std::vector<double> H(static_cast<size_t>(k) * k, 0.0), rhs(k);
  for (int i = 0; i < k; ++i) {
    H[i * k + i] = 1.0;
    double s = an[i];
    for (int r = 0; r < n; ++r) s += M[r * k + i] * b[r];
    rhs[i] = s;
    for (int j = 0; j < k; ++j) {
      double h = 0.0;
      for (int r = 0; r < n; ++r) h += M[r * k + i] * M[r * k + j];
      H[i * k + j] += h;
    }
  }
  solve_dense(H, rhs, k);
  for (int i = 0; i < k; ++i) out[i] = rhs[i];
  for (int r = 0; r < n; ++r) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += M[r * k + j] * rhs[j];
    out[k + r] = s;
  }
}

// First step: x1 = A x0 + B u0 with x0 a parameter; edges (u0, x1).
void prox_lindyn0(const double* nv, int n, int m, const double* A,
                  const double* B, const double* x0, double* out) {
  std::vector<double> c(n);
  for (int r = 0; r < n; ++r) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += A[r * n + j] * x0[j];
    c[r] = s;
  }
  const double* nu = nv;
  const double* b = nv + m;
  // minimise |u - n_u|^2 + |B u + c - b|^2:  (I + B^T B) u = n_u + B^T (b - c)
  std::vector<double> H(static_cast<size_t>(m) * m, 0.0), rhs(m);
  for (int i = 0; i < m; ++i) {
    H[i * m + i] = 1.0;
    double s = nu[i];
    for (int r = 0; r < n; ++r) s += B[r * m + i] * (b[r] - c[r]);
    rhs[i] = s;
    for (int j = 0; j < m; ++j) {
      double h = 0.0;
      for (int r = 0; r < n; ++r) h += B[r * m + i] * B[r * m + j];
      H[i * m + j] += h;
    }
  }
  solve_dense(H, rhs, m);
  for (int i = 0; i < m; ++i) out[i] = rhs[i];
  for (int r = 0; r < n; ++r) {
    double s = c[r];
    for (int j = 0; j < m; ++j) s += B[r * m + j] * rhs[j];
    out[m + r] = s;
  }
}

// Dispatch one factor.  dims: the dimension of each of its edges.
int prox_apply(int kind, int arity, const int* dims, const double* p, int plen,
               double rho, const double* nv, double* out) {
  switch (kind) {
    case K_NONOVERLAP:
      if (arity != 4 || dims[0] != 2 || dims[1] != 1 || dims[2] != 2 || dims[3] != 1) return -1;
      prox_nonoverlap(nv, rho, out);
      return 0;
    case K_WALL:
      if (arity != 2 || dims[0] != 2 || dims[1] != 1 || plen != 4) return -1;
      prox_wall(nv, p, rho, out);
      return 0;
    case K_RADIUS:
      if (arity != 1 || dims[0] != 1 || plen != 1) return -1;
      if (!(rho > p[0])) return -2;
      prox_radius(nv, p[0], rho, out);
      return 0;
    case K_QUAD: {
      int k = 0;
      for (int e = 0; e < arity; ++e) k += dims[e];
      if (plen != k) return -1;
      prox_quad(nv, k, p, rho, out);
      return 0;
    }
    case K_BOX: {
      int k = 0;
      for (int e = 0; e < arity; ++e) k += dims[e];
      if (plen != 2) return -1;
      prox_box(nv, k, p[0], p[1], out);
      return 0;
    }
    case K_HINGE: {
      const int d = arity - 1;
      for (int e = 0; e < arity; ++e) if (dims[e] != 1) return -1;
      if (d < 1 || plen != d + 2) return -1;
      prox_hinge(nv, d, p, rho, out);
      return 0;
    }
    case K_L2: {
      int k = 0;
      for (int e = 0; e < arity; ++e) k += dims[e];
      if (plen != 1) return -1;
      prox_l2(nv, k, p[0], rho, out);
      return 0;
    }
    case K_MINERR: {
      int k = 0;
      for (int e = 0; e < arity; ++e) k += dims[e];
      if (plen != 1 || !(p[0] >= 0.0)) return -1;
      prox_minerr(nv, k, p[0], rho, out);
      return 0;
    }
    case K_EQUAL:
      if (arity != 2 || dims[0] != dims[1] || plen != 0) return -1;
      prox_equal(nv, dims[0], out);
      return 0;
    case K_MARGIN: {
      if (arity != 3 || dims[1] != 1 || dims[2] != 1) return -1;
      const int d = dims[0];
      if (plen != d + 1 || (p[d] != 1.0 && p[d] != -1.0)) return -1;
      prox_margin(nv, d, p, rho, out);
      return 0;
    }
    case K_LINDYN: {
      if (arity != 3 || dims[0] != dims[2]) return -1;
      const int n = dims[0], m = dims[1];
      if (plen != n * n + n * m) return -1;
      prox_lindyn(nv, n, m, p, p + n * n, out);
      return 0;
    }
    case K_LINDYN0: {
      if (arity != 2) return -1;
      const int m = dims[0], n = dims[1];
      if (plen != n * n + n * m + n) return -1;
      prox_lindyn0(nv, n, m, p, p + n * n, p + n * n + n * m, out);
      return 0;
    }
    default:
      return -1;
  }
}

// The edges of every variable in creation order (the order in which the
// z-update adds them), and every edge slot's rho and alpha.
void build_lists(Graph& g) {
  g.erho.assign(g.nslot, g.rho);
  g.ealpha.assign(g.nslot, g.alpha);
  for (const Factor& f : g.F)
    for (long e = f.slot[0]; e < f.slot[0] + f.nslots; ++e) {
      if (f.rho > 0.0) g.erho[e] = f.rho;
      if (f.alpha > 0.0) g.ealpha[e] = f.alpha;
    }
  g.vrho.assign(g.nz, 0.0);
  for (long e = 0; e < g.nslot; ++e) g.vrho[g.slot_z[e]] = std::max(g.vrho[g.slot_z[e]], g.erho[e]);
  g.zbeg.assign(g.nz + 1, 0);
  for (long e = 0; e < g.nslot; ++e) g.zbeg[g.slot_z[e] + 1]++;
  for (long b = 0; b < g.nz; ++b) g.zbeg[b + 1] += g.zbeg[b];
  g.zedges.resize(g.nslot);
  std::vector<long> next(g.zbeg.begin(), g.zbeg.end() - 1);
  for (long e = 0; e < g.nslot; ++e) g.zedges[next[g.slot_z[e]]++] = e;
  g.lists_for = g.nslot;
}

// One iteration of Algorithm 2, each update its own loop.
void iterate(Graph& g) {
  const long S = g.nslot;
  const long NF = static_cast<long>(g.F.size());
  if (g.lists_for != S) build_lists(g);
  // n-update of the previous iteration (n = z - u), kept explicit.
#pragma omp parallel for schedule(static)
  for (long e = 0; e < S; ++e) g.n[e] = g.z[g.slot_z[e]] - g.u[e];
  // x-update.
#pragma omp parallel
  {
    std::vector<int> dims;
#pragma omp for schedule(dynamic, 256)
    for (long i = 0; i < NF; ++i) {
      const Factor& f = g.F[i];
      dims.resize(f.vars.size());
      for (size_t k = 0; k < f.vars.size(); ++k) dims[k] = g.dim[f.vars[k]];
      const long s0 = f.slot[0];
      prox_apply(f.kind, static_cast<int>(f.vars.size()), dims.data(),
                 f.p.data(), static_cast<int>(f.p.size()), f.rho > 0.0 ? f.rho : g.rho,
                 &g.n[s0], &g.x[s0]);
    }
  }
  // m-update.
#pragma omp parallel for schedule(static)
  for (long e = 0; e < S; ++e) g.m[e] = g.x[e] + g.u[e];
  // z-update: each variable's incoming m summed in edge-creation order; a
  // variable with no edge keeps z.
  g.zprev = g.z;
#pragma omp parallel for schedule(static)
  for (long b = 0; b < g.nz; ++b) {
    double num = 0.0, den = 0.0;
    for (long q = g.zbeg[b]; q < g.zbeg[b + 1]; ++q) {
      const long e = g.zedges[q];
      num += g.erho[e] * g.m[e];
      den += g.erho[e];
    }
    if (den > 0.0) g.z[b] = num / den;
  }
  // u-update.
#pragma omp parallel for schedule(static)
  for (long e = 0; e < S; ++e) g.u[e] += g.ealpha[e] * (g.x[e] - g.z[g.slot_z[e]]);
  // Stopping measures (maxima: the same in any order); the dual residual
  // weighs each variable's change by the largest rho of its edges.
  double r = 0.0, s = 0.0;
#pragma omp parallel for schedule(static) reduction(max : r)
  for (long e = 0; e < S; ++e) r = std::max(r, std::fabs(g.x[e] - g.z[g.slot_z[e]]));
#pragma omp parallel for schedule(static) reduction(max : s)
  for (long b = 0; b < g.nz; ++b) s = std::max(s, g.vrho[b] * std::fabs(g.z[b] - g.zprev[b]));
  g.r_primal = r;
  g.r_dual = s;
}

// Three-weight prox of the two constraint factors of circle packing with
// received weights wl (per slot; the slots of one edge share their weight)
// that include a zero.  The zero-weight edges take the correction in equal
// shares (the limit of the weighted projection as their weights go to 0
// together) and every other edge keeps its input.
void prox_nonoverlap_free(const double* nv, const double* wl, double* out) {
  const double c1x = nv[0], c1y = nv[1], r1 = nv[2];
  const double c2x = nv[3], c2y = nv[4], r2 = nv[5];
  const double dx = c2x - c1x, dy = c2y - c1y;
  const double L = std::sqrt(dx * dx + dy * dy);
  double hx = 1.0, hy = 0.0;
  if (L > 0.0) { hx = dx / L; hy = dy / L; }
  const double D = std::max(0.0, r1 + r2 - L);
  // edges c1, r1, c2, r2 start at slots 0, 2, 3, 5
  const bool z0 = wl[0] == 0.0, z1 = wl[2] == 0.0, z2 = wl[3] == 0.0, z3 = wl[5] == 0.0;
  const double nzero = (z0 ? 1.0 : 0.0) + (z1 ? 1.0 : 0.0) + (z2 ? 1.0 : 0.0) + (z3 ? 1.0 : 0.0);
  const double share = D / nzero;
  out[0] = c1x - (z0 ? share : 0.0) * hx;
  out[1] = c1y - (z0 ? share : 0.0) * hy;
  out[2] = r1 - (z1 ? share : 0.0);
  out[3] = c2x + (z2 ? share : 0.0) * hx;
  out[4] = c2y + (z2 ? share : 0.0) * hy;
  out[5] = r2 - (z3 ? share : 0.0);
}

void prox_wall_free(const double* nv, const double* p, const double* wl, double* out) {
  const double Qx = p[0], Qy = p[1], Vx = p[2], Vy = p[3];
  const double g = Qx * (nv[0] - Vx) + Qy * (nv[1] - Vy) - nv[2];
  out[0] = nv[0]; out[1] = nv[1]; out[2] = nv[2];
  if (g >= 0.0) return;
  // edges c (slots 0, 1) and r (slot 2); equal weights on the free ones
  const bool zc = wl[0] == 0.0, zr = wl[2] == 0.0;
  const double den = (zc ? Qx * Qx + Qy * Qy : 0.0) + (zr ? 1.0 : 0.0);
  const double lam = -g / den;
  if (zc) { out[0] = nv[0] + lam * Qx; out[1] = nv[1] + lam * Qy; }
  if (zr) out[2] = nv[2] - lam;
}

// One iteration of the three-weight variant, each update its own loop.
void iterate_twa(Graph& g) {
  const long S = g.nslot;
  const long NF = static_cast<long>(g.F.size());
  if (g.lists_for != S) build_lists(g);
  if (static_cast<long>(g.wl.size()) != S) g.wl = g.erho;   // start: every weight rho
  g.wr.resize(S);
  for (long e = 0; e < S; ++e) g.n[e] = g.z[g.slot_z[e]] - g.u[e];
  // x-update with received weights; sent weights
  std::vector<int> dims;
  for (long i = 0; i < NF; ++i) {
    const Factor& f = g.F[i];
    dims.resize(f.vars.size());
    for (size_t k = 0; k < f.vars.size(); ++k) dims[k] = g.dim[f.vars[k]];
    const long s0 = f.slot[0];
    const double rho = f.rho > 0.0 ? f.rho : g.rho;
    bool free_edge = false;
    for (int q = 0; q < f.nslots; ++q) free_edge = free_edge || g.wl[s0 + q] == 0.0;
    const bool constraint = f.kind == K_NONOVERLAP || f.kind == K_WALL;
    if (constraint && free_edge) {
      if (f.kind == K_NONOVERLAP) prox_nonoverlap_free(&g.n[s0], &g.wl[s0], &g.x[s0]);
      else prox_wall_free(&g.n[s0], f.p.data(), &g.wl[s0], &g.x[s0]);
    } else {
      prox_apply(f.kind, static_cast<int>(f.vars.size()), dims.data(), f.p.data(),
                 static_cast<int>(f.p.size()), rho, &g.n[s0], &g.x[s0]);
    }
    bool moved = !constraint;
    for (int q = 0; q < f.nslots && !moved; ++q) moved = g.x[s0 + q] != g.n[s0 + q];
    for (int q = 0; q < f.nslots; ++q) g.wr[s0 + q] = moved ? g.erho[s0 + q] : 0.0;
  }
  for (long e = 0; e < S; ++e) g.m[e] = g.x[e] + g.u[e];
  // z-update with the sent weights; received weights for the next x-update
  g.zprev = g.z;
  for (long b = 0; b < g.nz; ++b) {
    double num = 0.0, den = 0.0;
    for (long q = g.zbeg[b]; q < g.zbeg[b + 1]; ++q) {
      const long e = g.zedges[q];
      num += g.wr[e] * g.m[e];
      den += g.wr[e];
    }
    if (den > 0.0) g.z[b] = num / den;
    for (long q = g.zbeg[b]; q < g.zbeg[b + 1]; ++q) {
      const long e = g.zedges[q];
      g.wl[e] = den > 0.0 ? g.erho[e] : 0.0;
    }
  }
  // u-update: edges sent with weight 0 carry no multiplier
  for (long e = 0; e < S; ++e)
    g.u[e] = g.wr[e] > 0.0 ? g.u[e] + g.ealpha[e] * (g.x[e] - g.z[g.slot_z[e]]) : 0.0;
  double r = 0.0, s = 0.0;
  for (long e = 0; e < S; ++e) r = std::max(r, std::fabs(g.x[e] - g.z[g.slot_z[e]]));
  for (long b = 0; b < g.nz; ++b) s = std::max(s, g.vrho[b] * std::fabs(g.z[b] - g.zprev[b]));
  g.r_primal = r;
  g.r_dual = s;
}

// The whole run as one parallel region (the paper's second CPU scheme,
// Sec. III-A): the threads live for every iteration, each update type is a
// work-shared loop over its own index, and the barrier at the end of each
// loop separates one update type from the next.  Every element gets the
// same arithmetic in the same order as in iterate(), so the results equal
// the serial ones bit for bit; the stopping test reads the two maxima after
// the barrier that ends their loops, so every thread leaves at the same
// iteration.  Returns the iterations done.
int run_region(Graph& g, int max_iter, double tol) {
  const long S = g.nslot;
  const long NF = static_cast<long>(g.F.size());
  if (g.lists_for != S) build_lists(g);
  int done = max_iter;
  double r = 0.0, s = 0.0;
#pragma omp parallel
  {
    std::vector<int> dims;
    for (int k = 1; k <= max_iter; ++k) {
#pragma omp for schedule(static)
      for (long e = 0; e < S; ++e) g.n[e] = g.z[g.slot_z[e]] - g.u[e];
#pragma omp for schedule(dynamic, 256)
      for (long i = 0; i < NF; ++i) {
        const Factor& f = g.F[i];
        dims.resize(f.vars.size());
        for (size_t q = 0; q < f.vars.size(); ++q) dims[q] = g.dim[f.vars[q]];
        const long s0 = f.slot[0];
        prox_apply(f.kind, static_cast<int>(f.vars.size()), dims.data(),
                   f.p.data(), static_cast<int>(f.p.size()), f.rho > 0.0 ? f.rho : g.rho,
                   &g.n[s0], &g.x[s0]);
      }
#pragma omp for schedule(static)
      for (long e = 0; e < S; ++e) g.m[e] = g.x[e] + g.u[e];
#pragma omp single
      {
        g.zprev = g.z;
        r = 0.0;
        s = 0.0;
      }
#pragma omp for schedule(static)
      for (long b = 0; b < g.nz; ++b) {
        double num = 0.0, den = 0.0;
        for (long q = g.zbeg[b]; q < g.zbeg[b + 1]; ++q) {
          const long e = g.zedges[q];
          num += g.erho[e] * g.m[e];
          den += g.erho[e];
        }
        if (den > 0.0) g.z[b] = num / den;
      }
#pragma omp for schedule(static)
      for (long e = 0; e < S; ++e) g.u[e] += g.ealpha[e] * (g.x[e] - g.z[g.slot_z[e]]);
#pragma omp for schedule(static) reduction(max : r)
      for (long e = 0; e < S; ++e) r = std::max(r, std::fabs(g.x[e] - g.z[g.slot_z[e]]));
#pragma omp for schedule(static) reduction(max : s)
      for (long b = 0; b < g.nz; ++b) s = std::max(s, g.vrho[b] * std::fabs(g.z[b] - g.zprev[b]));
      if (tol > 0.0 && r <= tol && s <= tol) {
#pragma omp single nowait
        done = k;
        break;
      }
    }
  }
  g.r_primal = r;
  g.r_dual = s;
  return done;
}

}  // namespace

extern "C" {

// Threads the loops run on (1 in the serial build).
int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void* orc_graph_create(int n_vars, const int* dims) {
  Graph* g = new Graph();
  g->dim.assign(dims, dims + n_vars);
  g->zoff.resize(n_vars);
  long off = 0;
  for (int i = 0; i < n_vars; ++i) { g->zoff[i] = off; off += dims[i]; }
  g->nz = off;
  g->z.assign(off, 0.0);
  g->zprev.assign(off, 0.0);
  return g;
}

void orc_graph_destroy(void* h) { delete static_cast<Graph*>(h); }

// Append one factor; returns 0 or -1 on a bad variable id.
int orc_add_factor(void* h, int kind, int arity, const int* vars,
                   const double* params, int plen) {
  Graph* g = static_cast<Graph*>(h);
  Factor f;
  f.kind = kind;
  f.nslots = 0;
  for (int k = 0; k < arity; ++k) {
    if (vars[k] < 0 || vars[k] >= static_cast<int>(g->dim.size())) return -1;
    f.vars.push_back(vars[k]);
    f.slot.push_back(g->nslot + f.nslots);
    for (int c = 0; c < g->dim[vars[k]]; ++c)
      g->slot_z.push_back(g->zoff[vars[k]] + c);
    f.nslots += g->dim[vars[k]];
  }
  f.p.assign(params, params + plen);
  g->nslot += f.nslots;
  g->F.push_back(std::move(f));
  return 0;
}

// Add n factors of one kind; vars [n*arity]; params [n*plen] or, when
// shared != 0, [plen] for all.
int orc_add_factors(void* h, int kind, int n, int arity, const int* vars,
                    const double* params, int plen, int shared) {
  for (int i = 0; i < n; ++i) {
    const double* p = shared ? params : params + static_cast<long>(i) * plen;
    int rc = orc_add_factor(h, kind, arity, vars + static_cast<long>(i) * arity, p, plen);
    if (rc) return rc;
  }
  return 0;
}

// rho and alpha of factors [first, first + count) (> 0; 0 restores the
// graph's value).
int orc_set_factor_weights(void* h, long first, long count, double rho, double alpha) {
  Graph* g = static_cast<Graph*>(h);
  if (first < 0 || count < 0 || first + count > static_cast<long>(g->F.size())) return -1;
  for (long i = first; i < first + count; ++i) {
    g->F[i].rho = rho;
    g->F[i].alpha = alpha;
  }
  g->lists_for = -1;
  return 0;
}

void orc_set_params(void* h, double rho, double alpha) {
  Graph* g = static_cast<Graph*>(h);
  g->rho = rho;
  g->alpha = alpha;
  g->lists_for = -1;
}

long orc_num_slots(void* h) { return static_cast<Graph*>(h)->nslot; }
long orc_num_z(void* h) { return static_cast<Graph*>(h)->nz; }

// Initial state: z given, u = 0 (or given per edge slot when u != null).
void orc_set_state(void* h, const double* z, const double* u) {
  Graph* g = static_cast<Graph*>(h);
  std::memcpy(g->z.data(), z, sizeof(double) * g->nz);
  g->u.assign(g->nslot, 0.0);
  if (u) std::memcpy(g->u.data(), u, sizeof(double) * g->nslot);
  g->x.assign(g->nslot, 0.0);
  g->m.assign(g->nslot, 0.0);
  g->n.assign(g->nslot, 0.0);
  g->wl.clear();
  g->wr.clear();
}

// Run up to max_iter iterations; when tol > 0 stop at the first iteration
// whose r and s are both <= tol.  Returns the iterations done.
int orc_run(void* h, int max_iter, double tol) {
  Graph* g = static_cast<Graph*>(h);
  if (static_cast<long>(g->u.size()) != g->nslot) orc_set_state(h, g->z.data(), nullptr);
  for (int k = 1; k <= max_iter; ++k) {
    if (g->twa) iterate_twa(*g);
    else iterate(*g);
    if (tol > 0.0 && g->r_primal <= tol && g->r_dual <= tol) return k;
  }
  return max_iter;
}

// Replace z and u in place, keeping every other part of the iteration
// state (the three-weight variant's received weights), for tests that
// perturb a running iteration.
void orc_set_zu(void* h, const double* z, const double* u) {
  Graph* g = static_cast<Graph*>(h);
  std::memcpy(g->z.data(), z, sizeof(double) * g->nz);
  std::memcpy(g->u.data(), u, sizeof(double) * g->nslot);
}

// Run iterations with relative noise of size eps added to z and u before
// each one (z_b *= 1 + eps g, u_e += eps (|u_e| + |z_b(e)|) g with g
// uniform in [-sqrt(3), sqrt(3)], unit variance, from SplitMix64 on
// (seed, iteration, index)): a test-only model of a lower working
// precision's rounding, for measuring how far rounding alone moves a
// trajectory.  Plain Algorithm 2 only (the serial or OpenMP loops).
namespace {
inline double noise_unit(uint64_t key) {
  uint64_t x = key + 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  x ^= x >> 31;
  const double u01 = static_cast<double>(x >> 11) * (1.0 / 9007199254740992.0);
  return (2.0 * u01 - 1.0) * 1.7320508075688772;
}
}  // namespace

int orc_run_noisy(void* h, int iters, double eps, unsigned long long seed) {
  Graph* g = static_cast<Graph*>(h);
  if (g->twa) return -1;
  if (static_cast<long>(g->u.size()) != g->nslot) orc_set_state(h, g->z.data(), nullptr);
  const uint64_t base = static_cast<uint64_t>(seed) << 40;
  for (int k = 0; k < iters; ++k) {
    const uint64_t kb = base + (static_cast<uint64_t>(k) << 20) * 0x100000001ULL;
    std::vector<double> zc = g->z;
#pragma omp parallel for schedule(static)
    for (long b = 0; b < g->nz; ++b) g->z[b] = zc[b] * (1.0 + eps * noise_unit(kb ^ (2 * b)));
#pragma omp parallel for schedule(static)
    for (long e = 0; e < g->nslot; ++e)
      g->u[e] += eps * (std::fabs(g->u[e]) + std::fabs(zc[g->slot_z[e]])) *
                 noise_unit(kb ^ (2 * e + 1) ^ 0x5555555555ULL);
    iterate(*g);
  }
  return iters;
}

// Three-weight variant on (1) or off (0).  Switching resets every received
// weight to rho.
void orc_set_twa(void* h, int on) {
  Graph* g = static_cast<Graph*>(h);
  g->twa = on != 0;
  g->wl.clear();
  g->wr.clear();
}

// Weights sent by the factors in the last three-weight x-update, per slot.
void orc_get_wr(void* h, double* w) {
  Graph* g = static_cast<Graph*>(h);
  for (long e = 0; e < g->nslot; ++e) w[e] = e < static_cast<long>(g->wr.size()) ? g->wr[e] : 0.0;
}

// orc_run with the one-region scheme (run_region); the same results.
int orc_run_region(void* h, int max_iter, double tol) {
  Graph* g = static_cast<Graph*>(h);
  if (g->twa) return -1;   // the region scheme runs Algorithm 2 only
  if (static_cast<long>(g->u.size()) != g->nslot) orc_set_state(h, g->z.data(), nullptr);
  if (max_iter < 1) return 0;
  return run_region(*g, max_iter, tol);
}

void orc_get_z(void* h, double* z) {
  Graph* g = static_cast<Graph*>(h);
  std::memcpy(z, g->z.data(), sizeof(double) * g->nz);
}
void orc_get_u(void* h, double* u) {
  Graph* g = static_cast<Graph*>(h);
  std::memcpy(u, g->u.data(), sizeof(double) * g->nslot);
}
void orc_get_x(void* h, double* x) {
  Graph* g = static_cast<Graph*>(h);
  std::memcpy(x, g->x.data(), sizeof(double) * g->nslot);
}
void orc_get_m(void* h, double* m) {
  Graph* g = static_cast<Graph*>(h);
  std::memcpy(m, g->m.data(), sizeof(double) * g->nslot);
}
void orc_get_slot_z(void* h, long* idx) {
  Graph* g = static_cast<Graph*>(h);
  std::memcpy(idx, g->slot_z.data(), sizeof(long) * g->nslot);
}
void orc_residuals(void* h, double* r, double* s) {
  Graph* g = static_cast<Graph*>(h);
  *r = g->r_primal;
  *s = g->r_dual;
}

// The three-weight constraint prox with received weights wl (per slot; at
// least one zero), for the tests that pin it.
int orc_prox_free(int kind, const double* params, const double* wl, const double* nv,
                  double* out) {
  if (kind == K_NONOVERLAP) prox_nonoverlap_free(nv, wl, out);
  else if (kind == K_WALL) prox_wall_free(nv, params, wl, out);
  else return -1;
  return 0;
}

// A single proximal operator, for the tests that pin each one.
int orc_prox(int kind, int arity, const int* dims, const double* params,
             int plen, double rho, const double* nv, double* out) {
  return prox_apply(kind, arity, dims, params, plen, rho, nv, out);
}

}  // extern "C"
