// Factor-graph ADMM engine: host-side graph compiler and the C ABI of
// include/admm.h for graphs.
//
// The compiler turns the user's factor lists (paper Sec. III: nodes added
// one call at a time, edges stored in creation order) into a device layout
// built for gfx950 instead of the paper's one-array-per-variable-kind
// layout:
//  - factors are bucketed by proximal-operator kind, so every workgroup of
//    the fused x-pass runs a single operator;
//  - per-edge state is structure-of-arrays, [slot][factor], so a wavefront
//    streams each slot with unit stride;
//  - complete pairwise non-overlap buckets (every unordered pair of disks
//    once, as in circle packing) are stored as dense 64x64 pair tiles with
//    implicit indices, and each tile emits row/column partial sums;
//  - hinge buckets whose factors share one variable list (the SVM) emit one
//    partial per variable per workgroup;
//  - everything else keeps explicit per-edge variable offsets, and the
//    z-update sums its m slots directly.
// Each scalar of z gets a list of contributions (partials or m slots) in a
// fixed order, which the z-pass sums deterministically.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <vector>

#include "graph_plan.h"

using namespace admmg;

namespace admmg {

int64_t zpass_blocks(const Plan& P) {
  return ((int64_t)P.var_t.size() + P.t_lpb - 1) / P.t_lpb + (int64_t)P.var_b.size() +
         ((int64_t)P.var_w.size() + ZPB - 1) / ZPB + ((int64_t)P.var_l.size() + NT - 1) / NT;
}

// Bytes of the resident driver's LDS image: every region rounded up to 16 B,
// in the order resident_layout assigns them.
int64_t resident_image_bytes(const Plan& P, int64_t nz, int64_t es) {
  auto r16 = [](int64_t b) { return (b + 15) / 16 * 16; };
  int64_t b = r16((P.zc_span + 2 * P.n_m) * es) + 2 * r16(nz * es) + r16((int64_t)P.par.size() * es) +
              r16((int64_t)P.idx.size() * 4);
  b += r16((int64_t)P.var_b.size() * 4) + r16((int64_t)P.rng_b.size() * 8) + r16((int64_t)P.deg_b.size() * es);
  b += r16((int64_t)P.var_w.size() * 4) + r16((int64_t)P.rng_w.size() * 8) + r16((int64_t)P.deg_w.size() * es);
  b += r16((int64_t)P.var_l.size() * 4) + r16((int64_t)P.deg_l.size() * es);
  b += r16((int64_t)P.bt.size() * (int64_t)sizeof(BucketDesc));
  return b;
}

}  // namespace admmg

namespace {

struct Group {
  int32_t kind, n, arity, plen;
  bool shared;
  double rho = 0.0;            // rho of this group's edges (0: the graph's)
  double alpha = 0.0;          // alpha of this group's edges (0: the graph's)
  std::vector<int32_t> vids;   // [n * arity]
  std::vector<double> params;  // [n * plen] or [plen]
  const double* prm(int64_t f) const {
    return plen == 0 ? nullptr : params.data() + (shared ? 0 : f * (int64_t)plen);
  }
};

}  // namespace

struct admm_graph {
  int32_t precision = ADMM_FP32;
  std::vector<int32_t> dim;
  std::vector<int64_t> zoff;
  int64_t nz = 0;
  std::vector<Group> groups;
  double rho = 1.0, alpha = 1.0;
  int32_t pair_rows = 0;  // rows per dense pair tile (0: chosen at finalize)
  int32_t driver = ADMM_DRIVER_AUTO;
  int32_t graph_block = 32;  // iterations per recorded block of the graph driver
  int32_t twa = 0;           // three-weight variant
  int32_t zlist = 0;         // contribution layout of pair-tile entities (ADMM_OPT_ZLIST)
  int32_t pair_state = ADMM_PAIR_STATE_AUTO;
  int64_t n_factors = 0, n_edges = 0, n_slots = 0;
  int state = 0;  // 0 building, 1 validated (no device), 2 ready
  int device = -1;
  Plan plan;
  admm_graph_info info{};
  std::unique_ptr<EngineBase> eng;
};

namespace {

inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

int32_t kind_dim_ok(const admm_graph& g, const Group& gr, std::string& why, int32_t& nn,
                    int32_t& mm) {
  const int A = gr.arity;
  auto D = [&](int64_t f, int e) { return g.dim[gr.vids[f * A + e]]; };
  nn = mm = 0;
  switch (gr.kind) {
    case KD_NONOVERLAP:
      if (A != 4 || gr.plen != 0) { why = "NONOVERLAP needs arity 4 and no params"; return 0; }
      for (int64_t f = 0; f < gr.n; ++f)
        if (D(f, 0) != 2 || D(f, 1) != 1 || D(f, 2) != 2 || D(f, 3) != 1) {
          why = "NONOVERLAP edges must have dims (2,1,2,1)"; return 0;
        }
      return 1;
    case KD_WALL:
      if (A != 2 || gr.plen != 4) { why = "WALL needs arity 2 and 4 params"; return 0; }
      for (int64_t f = 0; f < gr.n; ++f)
        if (D(f, 0) != 2 || D(f, 1) != 1) { why = "WALL edges must have dims (2,1)"; return 0; }
      return 1;
    case KD_RADIUS:
      if (A != 1 || gr.plen != 1) { why = "RADIUS needs arity 1 and 1 param"; return 0; }
      for (int64_t f = 0; f < gr.n; ++f)
        if (D(f, 0) != 1) { why = "RADIUS edge must have dim 1"; return 0; }
      return 1;
    case KD_QUAD:
      for (int64_t f = 0; f < gr.n; ++f) {
        int k = 0;
        for (int e = 0; e < A; ++e) k += D(f, e);
        if (k != gr.plen) { why = "QUAD needs one weight per scalar slot"; return 0; }
      }
      return 1;
    case KD_BOX:
      if (gr.plen != 2) { why = "BOX needs 2 params (lo, hi)"; return 0; }
      for (int64_t f = 0; f < gr.n; ++f)
        if (gr.prm(f)[0] > gr.prm(f)[1]) { why = "BOX needs lo <= hi"; return 0; }
      return 1;
    case KD_HINGE:
      if (A < 2 || gr.plen != A + 1) { why = "HINGE needs arity d+1 >= 2 and d+2 params"; return 0; }
      for (int64_t f = 0; f < gr.n; ++f) {
        for (int e = 0; e < A; ++e)
          if (D(f, e) != 1) { why = "HINGE edges must be scalar"; return 0; }
        if (gr.prm(f)[A] < 0) { why = "HINGE needs C >= 0"; return 0; }
      }
      return 1;
    case KD_L2:
      if (gr.plen != 1) { why = "L2 needs 1 param"; return 0; }
      return 1;
    case KD_MINERR:
      if (gr.plen != 1) { why = "MINERR needs 1 param"; return 0; }
      for (int64_t f = 0; f < gr.n; ++f)
        if (!(gr.prm(f)[0] >= 0.0)) { why = "MINERR needs lambda >= 0"; return 0; }
      return 1;
    case KD_EQUAL:
      if (A != 2 || gr.plen != 0) { why = "EQUAL needs arity 2 and no params"; return 0; }
      for (int64_t f = 0; f < gr.n; ++f)
        if (D(f, 0) != D(f, 1)) { why = "EQUAL edges must have equal dims"; return 0; }
      return 1;
    case KD_MARGIN: {
      if (A != 3) { why = "MARGIN needs arity 3 (w, b, xi)"; return 0; }
      const int d = gr.n > 0 ? D(0, 0) : 0;
      if (gr.plen != d + 1) { why = "MARGIN needs d+1 params (x_1..x_d, y)"; return 0; }
      for (int64_t f = 0; f < gr.n; ++f) {
        if (D(f, 0) != d || D(f, 1) != 1 || D(f, 2) != 1) {
          why = "MARGIN edges must have dims (d,1,1), d the same within one call"; return 0;
        }
        const double y = gr.prm(f)[d];
        if (y != 1.0 && y != -1.0) { why = "MARGIN needs y = +1 or -1"; return 0; }
      }
      return 1;
    }
    case KD_LINDYN:
    case KD_LINDYN0: {
      const bool first = gr.kind == KD_LINDYN0;
      if (A != (first ? 2 : 3)) { why = "LINDYN needs arity 3, LINDYN0 arity 2"; return 0; }
      for (int64_t f = 0; f < gr.n; ++f) {
        int n = first ? D(f, 1) : D(f, 0), m = first ? D(f, 0) : D(f, 1);
        if (!first && D(f, 2) != n) { why = "LINDYN edges must have dims (n,m,n)"; return 0; }
        if (f == 0) { nn = n; mm = m; }
        if (n != nn || m != mm) { why = "LINDYN dims must agree within one call"; return 0; }
      }
      if (gr.plen != nn * nn + nn * mm + (first ? nn : 0)) { why = "LINDYN param_len mismatch"; return 0; }
      return 1;
    }
    default:
      why = "unknown factor kind";
      return 0;
  }
}

// Inverse of a small symmetric positive definite matrix (Gauss-Jordan).
std::vector<double> spd_inverse(std::vector<double> a, int n) {
  std::vector<double> inv(n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[r * n + c]) > std::fabs(a[piv * n + c])) piv = r;
    for (int j = 0; j < n; ++j) {
      std::swap(a[c * n + j], a[piv * n + j]);
      std::swap(inv[c * n + j], inv[piv * n + j]);
    }
    const double d = a[c * n + c];
    for (int j = 0; j < n; ++j) { a[c * n + j] /= d; inv[c * n + j] /= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) { a[r * n + j] -= f * a[c * n + j]; inv[r * n + j] -= f * inv[c * n + j]; }
    }
  }
  return inv;
}

// True when a NONOVERLAP bucket lists every unordered pair of "entities"
// (a centre variable and its radius variable) exactly once, each factor
// naming the entity with the smaller centre id first.  Fills the entities'
// z offsets and the entity pair of every factor.
bool detect_complete_pairs(const admm_graph& g, const Group& gr, std::vector<int32_t>& ent_zc,
                           std::vector<int32_t>& ent_zr, std::vector<int32_t>& fe1,
                           std::vector<int32_t>& fe2) {
  const int32_t nv = (int32_t)g.dim.size();
  std::vector<int32_t> c2r(nv, -1), r2c(nv, -1);
  for (int64_t f = 0; f < gr.n; ++f)
    for (int h = 0; h < 2; ++h) {
      const int32_t c = gr.vids[f * 4 + 2 * h], r = gr.vids[f * 4 + 2 * h + 1];
      if (c2r[c] < 0) c2r[c] = r; else if (c2r[c] != r) return false;
      if (r2c[r] < 0) r2c[r] = c; else if (r2c[r] != c) return false;
    }
  // entities in increasing order of their centre variable id
  std::vector<int32_t> eid(nv, -1);
  ent_zc.clear();
  ent_zr.clear();
  for (int32_t c = 0; c < nv; ++c) {
    if (c2r[c] < 0) continue;
    eid[c] = (int32_t)ent_zc.size();
    ent_zc.push_back((int32_t)g.zoff[c]);
    ent_zr.push_back((int32_t)g.zoff[c2r[c]]);
  }
  const int64_t E = (int64_t)ent_zc.size();
  if (E < 2 || gr.n != E * (E - 1) / 2) return false;
  fe1.resize(gr.n);
  fe2.resize(gr.n);
  std::vector<uint8_t> seen((size_t)E * E, 0);
  for (int64_t f = 0; f < gr.n; ++f) {
    const int32_t a = eid[gr.vids[f * 4]], b = eid[gr.vids[f * 4 + 2]];
    if (a >= b) return false;
    if (seen[(size_t)a * E + b]) return false;
    seen[(size_t)a * E + b] = 1;
    fe1[f] = a;
    fe2[f] = b;
  }
  return true;
}

// Hinge and margin factors take up to NT - 1 weight components: one
// register per component up to 64 (dmax 32 or 64), two sweeps over memory
// above that (dmax 0).
constexpr int HINGE_DMAX = NT - 1;
int hinge_dmax(int d) { return d <= 32 ? 32 : d <= 64 ? 64 : 0; }

constexpr int32_t DEFAULT_T_LPB = 32;   // transposed lists per z-pass block (measured best of 16, 32, 64)

bool hinge_uniform(const Group& gr) {
  for (int64_t f = 1; f < gr.n; ++f)
    for (int e = 0; e < gr.arity; ++e)
      if (gr.vids[f * gr.arity + e] != gr.vids[e]) return false;
  return gr.n >= 1;
}

// Build the device layout.  Validation errors return non-OK.
// True when every edge's alpha is 1 (the graph's or its group's).
bool all_alpha_one(const admm_graph& g) {
  for (const Group& gr : g.groups)
    if ((gr.alpha > 0.0 ? gr.alpha : g.alpha) != 1.0) return false;
  return g.groups.empty() ? g.alpha == 1.0 : true;
}

admm_status build_plan(admm_graph& g, Plan& P, bool no_tiles) {
  P = Plan();
  P.alpha_one = all_alpha_one(g);
  bool alpha_mixed = false;
  for (const Group& gr : g.groups)
    if (gr.alpha > 0.0 && gr.alpha != g.alpha) alpha_mixed = true;
  if (alpha_mixed) P.ualpha.assign(g.n_slots, g.alpha);
  P.no_tiles = no_tiles;
  // Every contribution to a z scalar, in emission order: z index and the
  // index-buffer slot that will receive its position in the z-major buffer.
  struct Emit { int64_t z; int64_t key; };
  std::vector<Emit> em;
  // Pair-tile partials in the transposed layout (64-row tiles, one pair
  // bucket): scalar z, slot j of its transposed list, index-buffer key,
  // relative rho.  Entity e's slots: the column partial of tile (I', B) at
  // j = I' (I' <= B), the row partial of tile (B, J) at j = J + 1 (J >= B),
  // B = e / 64; its other contributions follow at j >= NBC + 1.
  struct TEmit { int64_t z; int32_t j; int64_t key; double rw; };
  std::vector<TEmit> tem;
  std::vector<int64_t> tz;     // scalars of the transposed lists, list order
  int32_t t_tiles = 0;         // tile slots per transposed list (NBC + 1)
  int n_pair_buckets = 0;
  std::vector<double> deg(g.nz, 0.0);   // sum of relative rho over each scalar's edges
  std::vector<double> rmz(g.nz, 0.0);
  struct EmRange { size_t end; double rho; };
  std::vector<EmRange> em_rho;
  P.upos.assign(g.n_slots, 0);
  P.uz.assign(g.n_slots, 0);
  int64_t us = 0;      // running user slot
  int64_t blocks = 0;
  for (const Group& gr : g.groups) {
    const double rg = gr.rho > 0.0 ? gr.rho : g.rho;
    // z-sum weight relative to the graph's rho: exactly 1 for every edge of a
    // graph without group weights, so such graphs keep their unweighted sums
    const double rw = rg / g.rho;
    if (rg != g.rho) P.weighted = true;
    const double ag = gr.alpha > 0.0 ? gr.alpha : g.alpha;
    const int64_t us0 = us;
    std::string why;
    int32_t nn = 0, mm = 0;
    if (!kind_dim_ok(g, gr, why, nn, mm)) return admmi::set_err(ADMM_E_ARG, "%s", why.c_str());
    if (gr.kind == KD_RADIUS)
      for (int64_t f = 0; f < gr.n; ++f)
        if (!(rg > gr.prm(f)[0]))
          return admmi::set_err(ADMM_E_NUMERIC, "RADIUS factor needs rho > gamma (rho=%g, gamma=%g)",
                                rg, gr.prm(f)[0]);
    if (gr.n == 0) continue;
    BucketDesc b{};
    b.kind = gr.kind;
    b.arity = gr.arity;
    b.idx_off = (int64_t)P.idx.size();
    b.par_off = (int64_t)P.par.size();
    P.n_m = round_up(P.n_m, 64);  // every bucket's state starts 256-byte aligned
    b.m_off = P.n_m;
    // slots per factor (constant within a group for every kind but QUAD/BOX/L2)
    auto fslots = [&](int64_t f) {
      int k = 0;
      for (int e = 0; e < gr.arity; ++e) k += g.dim[gr.vids[f * gr.arity + e]];
      return k;
    };
    // user-slot walk helper: for factor f, edge e, comp c -> z index
    auto zof = [&](int64_t f, int e) { return g.zoff[gr.vids[f * gr.arity + e]]; };

    std::vector<int32_t> ezc, ezr, fe1, fe2;
    const bool separable = gr.kind == KD_RADIUS || gr.kind == KD_QUAD || gr.kind == KD_BOX ||
                           gr.kind == KD_L2 || gr.kind == KD_MINERR;
    // the three-weight variant runs on pair tiles only with their sparse state
    const bool tiles_ok = !P.no_tiles &&
                          (!g.twa || (g.precision == ADMM_FP32 && P.alpha_one &&
                                      g.pair_state != ADMM_PAIR_STATE_DENSE));
    if (gr.kind == KD_NONOVERLAP && tiles_ok &&
        detect_complete_pairs(g, gr, ezc, ezr, fe1, fe2)) {
      // ---------------- dense pair tiles ----------------
      b.mode = BM_PAIR;
      b.E = (int32_t)ezc.size();
      int RB = g.pair_rows;
      if (RB == 0) RB = 64;  // measured fastest at 2000 disks (64: 19.4 us, 32: 21.6, 16: 23.5)
      const int CB = PB;
      b.rb = RB;
      const int NBR = (b.E + RB - 1) / RB, NBC = (b.E + CB - 1) / CB;
      b.NB = NBC;
      b.nslot = 6;
      std::vector<int32_t> tI, tJ;
      std::vector<int64_t> tid((size_t)NBR * NBC, -1);
      for (int I = 0; I < NBR; ++I)
        for (int J = 0; J < NBC; ++J) {
          const int maxej = std::min(b.E, (J + 1) * CB) - 1;
          if (maxej <= I * RB) continue;  // no pair e_i < e_j in this tile
          tid[(size_t)I * NBC + J] = (int64_t)tI.size();
          tI.push_back(I);
          tJ.push_back(J);
        }
      b.n = (int64_t)tI.size();
      b.nfp = b.n;
      P.n_pair_tiles += b.n;
      {
        bool aff = b.E > 0;
        for (int e = 0; e < b.E && aff; ++e)
          aff = ezc[e] == ezc[0] + 3 * e && ezr[e] == ezc[e] + 2;
        b.ent_aff = aff ? 1 : 0;
        b.ent_base = aff ? ezc[0] : 0;
      }
      {
        // the kernels compute (I, J) when the tiles are the whole upper
        // triangle in row-major order
        bool tri = RB == CB && b.n == (int64_t)NBC * (NBC + 1) / 2;
        for (int64_t t = 0, I = 0, J = 0; tri && t < b.n; ++t) {
          tri = tI[t] == I && tJ[t] == J;
          if (++J == NBC) J = ++I;
        }
        b.tri = tri ? 1 : 0;
      }
      b.sparse = (g.precision == ADMM_FP32 && P.alpha_one &&
                  g.pair_state != ADMM_PAIR_STATE_DENSE) ? 1 : 0;
      b.flag0 = P.n_flags;
      if (b.sparse) P.n_flags += b.n * NT;
      for (int64_t t = 0; t < b.n; ++t) { P.idx.push_back(tI[t]); P.idx.push_back(tJ[t]); }
      for (int e = 0; e < b.E; ++e) { P.idx.push_back(ezc[e]); P.idx.push_back(ezr[e]); }
      const int64_t TS = 6LL * RB * CB;
      const int64_t PS = 3LL * (RB + CB);
      P.n_m += b.n * TS;
      b.dst_off = (int64_t)P.idx.size();
      P.idx.resize(P.idx.size() + b.n * PS, -1);
      b.blk0 = (int32_t)blocks;
      blocks += b.n;
      b.blk1 = (int32_t)blocks;
      // 64-row tiles of the only pair bucket write their partials into
      // transposed lists: each tile's 192 row and 192 column partials land
      // at consecutive positions
      const bool tlay = RB == CB && ++n_pair_buckets == 1 && g.zlist != ADMM_ZLIST_ZMAJOR;
      if (tlay) {
        t_tiles = NBC + 1;
        for (int e = 0; e < b.E; ++e) {
          tz.push_back(ezc[e]);
          tz.push_back(ezc[e] + 1);
          tz.push_back(ezr[e]);
        }
      }
      // contributions: per tile, rows then columns with at least one pair
      for (int64_t t = 0; t < b.n; ++t) {
        const int I = tI[t], J = tJ[t];
        const int maxej = std::min(b.E, (J + 1) * CB) - 1;
        const int64_t pb = b.dst_off + t * PS;
        for (int li = 0; li < RB; ++li) {
          const int ei = I * RB + li;
          if (ei >= b.E || ei >= maxej) break;
          if (tlay) {
            for (int c = 0; c < 3; ++c)
              tem.push_back({c < 2 ? ezc[ei] + c : ezr[ei], J + 1, pb + li * 3 + c, rw});
          } else {
            em.push_back({ezc[ei], pb + li * 3});
            em.push_back({ezc[ei] + 1, pb + li * 3 + 1});
            em.push_back({ezr[ei], pb + li * 3 + 2});
          }
        }
        for (int lj = 0; lj < CB; ++lj) {
          const int ej = J * CB + lj;
          if (ej >= b.E) break;
          if (ej <= I * RB) continue;
          if (tlay) {
            for (int c = 0; c < 3; ++c)
              tem.push_back({c < 2 ? ezc[ej] + c : ezr[ej], I, pb + 3 * RB + lj * 3 + c, rw});
          } else {
            em.push_back({ezc[ej], pb + 3 * RB + lj * 3});
            em.push_back({ezc[ej] + 1, pb + 3 * RB + lj * 3 + 1});
            em.push_back({ezr[ej], pb + 3 * RB + lj * 3 + 2});
          }
        }
      }
      for (int64_t f = 0; f < gr.n; ++f) {
        const int e1 = fe1[f], e2 = fe2[f];
        const int I = e1 / RB, li = e1 % RB, J = e2 / CB, lj = e2 % CB;
        const int64_t t = tid[(size_t)I * NBC + J];
        const int64_t base = b.m_off + t * TS + (int64_t)li * CB + lj;
        const int64_t zs[6] = {ezc[e1], ezc[e1] + 1, ezr[e1], ezc[e2], ezc[e2] + 1, ezr[e2]};
        for (int s = 0; s < 6; ++s) {
          P.upos[us] = base + (int64_t)s * RB * CB;
          P.uz[us] = (int32_t)zs[s];
          deg[zs[s]] += rw; rmz[zs[s]] = std::max(rmz[zs[s]], rg);
          ++us;
        }
      }
      P.algo_elems += 2 * (int64_t)gr.n * 6;

    } else if (gr.kind == KD_HINGE && gr.arity - 1 <= HINGE_DMAX && hinge_uniform(gr)) {
      // ---------------- hinge, shared variable list ----------------
      b.mode = BM_UNIF_HINGE;
      b.d = gr.arity - 1;
      b.dmax = hinge_dmax(b.d);
      b.n = gr.n;
      // d < 32: four lanes per four factors in FP32 with alpha = 1 (NT
      // factors per workgroup, rows padded to whole workgroups so that every
      // 16-byte access stays in its row), else two lanes per factor (NT / 2)
      // (not in a plan built for the resident driver, whose LDS image keeps
      // the rows at their 64-factor padding)
      b.quad = (b.dmax == 32 && b.d < 32 && g.precision == ADMM_FP32 && P.alpha_one &&
                !P.no_tiles) ? 1 : 0;
      b.nfp = round_up(gr.n, b.quad ? NT : 64);
      b.nslot = gr.arity;
      for (int e = 0; e < gr.arity; ++e) P.idx.push_back((int32_t)zof(0, e));
      const int d = b.d;
      if (b.quad) {
        // 16-byte aligned parameter rows
        P.par.resize((size_t)round_up((int64_t)P.par.size(), 4), 0.0);
        b.par_off = (int64_t)P.par.size();
      }
      P.par.resize(P.par.size() + (size_t)(d + 3) * b.nfp, 0.0);
      double* par = P.par.data() + b.par_off;
      for (int64_t f = 0; f < gr.n; ++f) {
        const double* p = gr.prm(f);
        const double y = p[d], C = p[d + 1];
        double aa = 0.0;
        for (int k = 0; k < d; ++k) { par[k * b.nfp + f] = y * p[k]; aa += p[k] * p[k]; }
        par[d * b.nfp + f] = y;
        par[(d + 1) * b.nfp + f] = C;
        par[(d + 2) * b.nfp + f] = rg / (aa + 1.0);
      }
      P.n_m += (int64_t)gr.arity * b.nfp;
      const int64_t fpb = b.quad ? NT : (b.dmax == 32 ? NT / 2 : NT);
      const int64_t tiles = (gr.n + fpb - 1) / fpb;
      b.dst_off = (int64_t)P.idx.size();
      P.idx.resize(P.idx.size() + tiles * gr.arity, -1);
      b.blk0 = (int32_t)blocks;
      blocks += tiles;
      b.blk1 = (int32_t)blocks;
      for (int64_t t = 0; t < tiles; ++t)
        for (int e = 0; e < gr.arity; ++e) em.push_back({zof(0, e), b.dst_off + t * gr.arity + e});
      for (int64_t f = 0; f < gr.n; ++f)
        for (int e = 0; e < gr.arity; ++e) {
          P.upos[us] = b.m_off + (int64_t)e * b.nfp + f;
          P.uz[us] = (int32_t)zof(f, e);
          deg[zof(f, e)] += rw; rmz[zof(f, e)] = std::max(rmz[zof(f, e)], rg);
          ++us;
        }
      P.algo_elems += (int64_t)gr.n * (2 * gr.arity + d + 3);
    } else if (gr.kind == KD_EQUAL) {
      // ---------------- equality: one thread per component pair ----------------
      b.mode = BM_GEN_FACTOR;
      b.arity = 2;
      b.nslot = 2;
      int64_t np = 0;
      for (int64_t f = 0; f < gr.n; ++f) np += g.dim[gr.vids[f * 2]];
      b.n = np;
      b.nfp = round_up(np, 64);
      const int64_t i0 = (int64_t)P.idx.size();
      P.idx.resize(i0 + 2 * b.nfp, 0);
      P.n_m += 2 * b.nfp;
      b.dst_off = (int64_t)P.idx.size();
      P.idx.resize(P.idx.size() + 2 * b.nfp, -1);
      int64_t j = 0;
      for (int64_t f = 0; f < gr.n; ++f) {
        const int dm = g.dim[gr.vids[f * 2]];
        for (int e = 0; e < 2; ++e)
          for (int c = 0; c < dm; ++c) {
            const int64_t zi = zof(f, e) + c;
            P.idx[i0 + e * b.nfp + j + c] = (int32_t)zi;
            P.upos[us] = b.m_off + (int64_t)e * b.nfp + j + c;
            P.uz[us] = (int32_t)zi;
            deg[zi] += rw; rmz[zi] = std::max(rmz[zi], rg);
            ++us;
            em.push_back({zi, b.dst_off + (int64_t)e * b.nfp + j + c});
          }
        j += dm;
      }
      b.blk0 = (int32_t)blocks;
      blocks += (np + NT - 1) / NT;
      b.blk1 = (int32_t)blocks;
      P.algo_elems += 4 * np;
      P.layout_idx_bytes += 2 * np * 4;
    } else if (gr.kind == KD_MARGIN) {
      // ---------------- margin: the general hinge path with a slack slot ----------------
      b.mode = BM_GEN_FACTOR;
      b.n = gr.n;
      b.nfp = round_up(gr.n, 64);
      const int d = g.dim[gr.vids[0]];
      b.d = d;
      if (d > HINGE_DMAX)
        return admmi::set_err(ADMM_E_UNSUPPORTED, "MARGIN with d > %d is not supported", HINGE_DMAX);
      b.dmax = hinge_dmax(d);
      b.nslot = d + 2;
      const int64_t i0 = (int64_t)P.idx.size();
      P.idx.resize(i0 + (int64_t)(d + 2) * b.nfp, 0);
      P.par.resize(P.par.size() + (size_t)(d + 3) * b.nfp, 0.0);
      double* par = P.par.data() + b.par_off;
      for (int64_t f = 0; f < gr.n; ++f) {
        for (int k = 0; k < d; ++k) P.idx[i0 + k * b.nfp + f] = (int32_t)(zof(f, 0) + k);
        P.idx[i0 + d * b.nfp + f] = (int32_t)zof(f, 1);
        P.idx[i0 + (d + 1) * b.nfp + f] = (int32_t)zof(f, 2);
        const double* p = gr.prm(f);
        const double y = p[d];
        double xx = 0.0;
        for (int k = 0; k < d; ++k) { par[k * b.nfp + f] = y * p[k]; xx += p[k] * p[k]; }
        par[d * b.nfp + f] = y;
        par[(d + 1) * b.nfp + f] = INFINITY;
        par[(d + 2) * b.nfp + f] = rg / (xx + 2.0);
      }
      P.n_m += (int64_t)b.nslot * b.nfp;
      b.dst_off = (int64_t)P.idx.size();
      P.idx.resize(P.idx.size() + (int64_t)b.nslot * b.nfp, -1);
      // one bias for every factor (the usual graph): one partial per workgroup
      b.ub = 1;
      for (int64_t f = 1; f < gr.n && b.ub; ++f) b.ub = zof(f, 1) == zof(0, 1);
      const int64_t tiles = (gr.n + NT - 1) / NT;
      for (int64_t f = 0; f < gr.n; ++f)
        for (int s = 0; s < d + 2; ++s) {
          const int64_t zi = P.idx[i0 + s * b.nfp + f];
          P.upos[us] = b.m_off + (int64_t)s * b.nfp + f;
          P.uz[us] = (int32_t)zi;
          deg[zi] += rw; rmz[zi] = std::max(rmz[zi], rg);
          ++us;
          if (!(b.ub && s == d)) em.push_back({zi, b.dst_off + (int64_t)s * b.nfp + f});
        }
      if (b.ub)
        for (int64_t t = 0; t < tiles; ++t) em.push_back({zof(0, 1), b.dst_off + (int64_t)d * b.nfp + t});
      b.blk0 = (int32_t)blocks;
      blocks += tiles;
      b.blk1 = (int32_t)blocks;
      P.algo_elems += (int64_t)gr.n * (2 * b.nslot + d + 3);
      P.layout_idx_bytes += (int64_t)gr.n * b.nslot * 4;
    } else if (separable) {
      // ---------------- separable operators: one thread per slot ----------------
      b.mode = BM_GEN_SLOT;
      int64_t ns = 0;
      for (int64_t f = 0; f < gr.n; ++f) ns += fslots(f);
      b.n = ns;
      b.nfp = round_up(ns, 64);
      b.nslot = 1;
      const int64_t i0 = (int64_t)P.idx.size();
      P.idx.resize(i0 + b.nfp, 0);
      b.dst_off = (int64_t)P.idx.size();
      P.idx.resize(P.idx.size() + b.nfp, -1);
      P.par.resize(P.par.size() + 2 * (size_t)b.nfp, 0.0);
      double* par = P.par.data() + b.par_off;
      int64_t s = 0;
      for (int64_t f = 0; f < gr.n; ++f) {
        const double* p = gr.prm(f);
        int comp = 0;
        for (int e = 0; e < gr.arity; ++e) {
          const int dm = g.dim[gr.vids[f * gr.arity + e]];
          for (int c = 0; c < dm; ++c, ++comp, ++s) {
            const int64_t zi = zof(f, e) + c;
            P.idx[i0 + s] = (int32_t)zi;
            double p0 = 0.0, p1 = 0.0;
            switch (gr.kind) {
              case KD_RADIUS: p0 = rg / (rg - p[0]); break;
              case KD_QUAD: p0 = rg / (rg + p[comp]); break;
              case KD_L2: p0 = rg / (rg + p[0]); break;
              case KD_BOX: p0 = p[0]; p1 = p[1]; break;
              case KD_MINERR: p0 = p[0] / rg; break;
            }
            par[s] = p0;
            par[b.nfp + s] = p1;
            P.upos[us] = b.m_off + s;
            P.uz[us] = (int32_t)zi;
            deg[zi] += rw; rmz[zi] = std::max(rmz[zi], rg);
            ++us;
            em.push_back({zi, b.dst_off + s});
          }
        }
      }
      P.n_m += b.nfp;
      b.blk0 = (int32_t)blocks;
      blocks += (ns + NT - 1) / NT;
      b.blk1 = (int32_t)blocks;
      P.algo_elems += ns * (2 + (gr.kind == KD_BOX ? 2 : 1));
      P.layout_idx_bytes += ns * 4;
    } else {
      // ---------------- general: one thread per factor ----------------
      b.mode = BM_GEN_FACTOR;
      b.n = gr.n;
      b.nfp = round_up(gr.n, 64);
      b.nslot = fslots(0);
      if (gr.kind == KD_HINGE) {
        b.d = gr.arity - 1;
        if (b.d > HINGE_DMAX)
          return admmi::set_err(ADMM_E_UNSUPPORTED, "HINGE with d > %d is not supported", HINGE_DMAX);
        b.dmax = hinge_dmax(b.d);
      }
      if (gr.kind == KD_LINDYN || gr.kind == KD_LINDYN0) {
        b.nn = nn;
        b.mm = mm;
        if (nn > MAXN || mm > MAXM)
          return admmi::set_err(ADMM_E_UNSUPPORTED, "LINDYN supports n <= %d, m <= %d", MAXN, MAXM);
      }
      const int64_t i0 = (int64_t)P.idx.size();
      const bool lind = gr.kind == KD_LINDYN || gr.kind == KD_LINDYN0;
      P.idx.resize(i0 + (int64_t)(gr.arity + (lind ? 1 : 0)) * b.nfp, 0);
      for (int64_t f = 0; f < gr.n; ++f)
        for (int e = 0; e < gr.arity; ++e) P.idx[i0 + e * b.nfp + f] = (int32_t)zof(f, e);
      if (gr.kind == KD_WALL) {
        P.par.resize(P.par.size() + 4 * (size_t)b.nfp, 0.0);
        double* par = P.par.data() + b.par_off;
        for (int64_t f = 0; f < gr.n; ++f) {
          const double* p = gr.prm(f);
          par[f] = p[0];
          par[b.nfp + f] = p[1];
          par[2 * b.nfp + f] = p[0] * p[2] + p[1] * p[3];
          par[3 * b.nfp + f] = 1.0 / (p[0] * p[0] + p[1] * p[1] + 1.0);
        }
        P.algo_elems += gr.n * 4;
      } else if (gr.kind == KD_HINGE) {
        const int d = b.d;
        P.par.resize(P.par.size() + (size_t)(d + 3) * b.nfp, 0.0);
        double* par = P.par.data() + b.par_off;
        for (int64_t f = 0; f < gr.n; ++f) {
          const double* p = gr.prm(f);
          double aa = 0.0;
          for (int k = 0; k < d; ++k) { par[k * b.nfp + f] = p[d] * p[k]; aa += p[k] * p[k]; }
          par[d * b.nfp + f] = p[d];
          par[(d + 1) * b.nfp + f] = p[d + 1];
          par[(d + 2) * b.nfp + f] = rg / (aa + 1.0);
        }
        P.algo_elems += gr.n * (d + 3);
      } else if (lind) {
        // parameter blocks: one per factor, or one for the group when shared
        const int n = nn, m = mm;
        const bool first = gr.kind == KD_LINDYN0;
        const int k = first ? m : n + m;
        const int64_t nblk = gr.shared ? 1 : gr.n;
        const int64_t bl = (int64_t)n * k + (int64_t)n * n + (first ? n : 0);
        for (int64_t q = 0; q < nblk; ++q) {
          const double* p = gr.prm(q);
          const double* A = p;
          const double* B = p + n * n;
          std::vector<double> Mx((size_t)n * k);
          for (int r = 0; r < n; ++r) {
            if (first) {
              for (int j = 0; j < m; ++j) Mx[r * k + j] = B[r * m + j];
            } else {
              for (int j = 0; j < n; ++j) Mx[r * k + j] = A[r * n + j];
              for (int j = 0; j < m; ++j) Mx[r * k + n + j] = B[r * m + j];
            }
          }
          std::vector<double> G((size_t)n * n, 0.0);
          for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) {
              double s = (r == c) ? 1.0 : 0.0;
              for (int j = 0; j < k; ++j) s += Mx[r * k + j] * Mx[c * k + j];
              G[r * n + c] = s;
            }
          std::vector<double> S = spd_inverse(G, n);
          const int64_t off = (int64_t)P.par.size() - b.par_off;
          P.par.insert(P.par.end(), Mx.begin(), Mx.end());
          P.par.insert(P.par.end(), S.begin(), S.end());
          if (first) {
            const double* x0 = p + n * n + n * m;
            for (int r = 0; r < n; ++r) {
              double s = 0.0;
              for (int j = 0; j < n; ++j) s += A[r * n + j] * x0[j];
              P.par.push_back(s);
            }
          }
          if (gr.shared) {
            for (int64_t f = 0; f < gr.n; ++f) P.idx[i0 + gr.arity * b.nfp + f] = (int32_t)off;
          } else {
            P.idx[i0 + gr.arity * b.nfp + q] = (int32_t)off;
          }
          (void)bl;
        }
      }
      P.n_m += (int64_t)b.nslot * b.nfp;
      b.dst_off = (int64_t)P.idx.size();
      P.idx.resize(P.idx.size() + (int64_t)b.nslot * b.nfp, -1);
      for (int64_t f = 0; f < gr.n; ++f) {
        int s = 0;
        for (int e = 0; e < gr.arity; ++e) {
          const int dm = g.dim[gr.vids[f * gr.arity + e]];
          for (int c = 0; c < dm; ++c, ++s) {
            const int64_t zi = zof(f, e) + c;
            const int64_t pos = b.m_off + (int64_t)s * b.nfp + f;
            P.upos[us] = pos;
            P.uz[us] = (int32_t)zi;
            deg[zi] += rw; rmz[zi] = std::max(rmz[zi], rg);
            ++us;
            em.push_back({zi, b.dst_off + (int64_t)s * b.nfp + f});
          }
        }
      }
      b.blk0 = (int32_t)blocks;
      blocks += (gr.n + NT - 1) / NT;
      b.blk1 = (int32_t)blocks;
      P.algo_elems += 2 * (int64_t)gr.n * b.nslot;
      P.layout_idx_bytes += (int64_t)gr.n * gr.arity * 4;
    }
    b.irho = 1.0 / rg;
    b.alpha = ag;
    if (!P.ualpha.empty())
      for (int64_t q = us0; q < us; ++q) P.ualpha[q] = ag;
    P.bt.push_back(b);
    em_rho.push_back({em.size(), rw});
  }
  if (us != g.n_slots) return admmi::set_err(ADMM_E_ARG, "internal: slot count mismatch");
  if (blocks > 0x7fffffff) return admmi::set_err(ADMM_E_UNSUPPORTED, "graph too large for one launch");
  P.xblocks = blocks;
  // Contribution positions.  Each scalar's contributions are contiguous, in
  // emission order.  Long lists (more than ZB_MIN) are packed one after the
  // other and found through explicit ranges.  Medium lists get one fixed
  // stride, the longest of them rounded up to the lanes that sum one list,
  // when that at most doubles their space (else explicit ranges), and short
  // lists a stride of LANE_MAX: the z-pass then reads them without first
  // reading a range.  Padding is never written and stays zero.
  // Transposed lists first: tile slots, then the scalar's other
  // contributions in emission order; every list padded to the longest.
  P.n_zc = (int64_t)em.size() + (int64_t)tem.size();
  std::vector<int64_t> tk(g.nz, -1);   // scalar -> transposed list
  for (size_t k = 0; k < tz.size(); ++k) tk[tz[k]] = (int64_t)k;
  std::vector<int64_t> len(g.nz, 0);
  for (auto& e : em) len[e.z]++;
  const int64_t n_t = (int64_t)tz.size();
  int64_t t_rest = 0;
  for (int64_t k = 0; k < n_t; ++k) t_rest = std::max(t_rest, len[tz[k]]);
  P.t_len = n_t ? (int32_t)(t_tiles + t_rest) : 0;
  P.t_lpb = g.zlist >= 16 ? g.zlist : DEFAULT_T_LPB;
  P.t_base = 0;
  const int64_t t_span = round_up(n_t * P.t_len, 16);
  for (int64_t k = 0; k < n_t; ++k) {
    P.var_t.push_back((int32_t)tz[k]);
    P.deg_t.push_back(deg[tz[k]]);
  }
  int64_t sum_w = 0, max_w = 0, n_wl = 0, n_ll = 0, sum_b = 0;
  for (int64_t zi = 0; zi < g.nz; ++zi) {
    if (tk[zi] >= 0) continue;
    if (len[zi] > ZB_MIN) sum_b += len[zi];
    else if (len[zi] > LANE_MAX) { sum_w += len[zi]; max_w = std::max(max_w, len[zi]); ++n_wl; }
    else ++n_ll;
  }
  const int64_t S_w = round_up(std::max<int64_t>(max_w, 1), ZSEG);
  const bool pad_w = n_wl > 0 && S_w * n_wl <= 2 * sum_w + 4096;
  P.w_stride = pad_w ? S_w : 0;
  P.w_base = round_up(t_span + sum_b, 16);
  P.l_base = round_up(P.w_base + (pad_w ? S_w * n_wl : sum_w), 16);
  const int64_t zc_total = P.l_base + LANE_MAX * n_ll;
  std::vector<int64_t> base(g.nz, 0);
  {
    int64_t pb = t_span, pw = P.w_base, kw = 0, kl = 0;
    for (int64_t zi = 0; zi < g.nz; ++zi) {
      const int64_t L = len[zi];
      if (tk[zi] >= 0) {
        base[zi] = t_tiles;   // next free slot of the transposed list
      } else if (L > ZB_MIN) {
        base[zi] = pb;
        P.var_b.push_back((int32_t)zi);
        P.rng_b.push_back(pb);
        P.rng_b.push_back(pb + L);
        P.deg_b.push_back(deg[zi]);
        pb += L;
      } else if (L > LANE_MAX) {
        base[zi] = pad_w ? P.w_base + kw * S_w : pw;
        P.var_w.push_back((int32_t)zi);
        if (!pad_w) {
          P.rng_w.push_back(pw);
          P.rng_w.push_back(pw + L);
          pw += L;
        }
        P.deg_w.push_back(deg[zi]);
        ++kw;
      } else {
        base[zi] = P.l_base + kl * LANE_MAX;
        P.var_l.push_back((int32_t)zi);
        P.deg_l.push_back(deg[zi]);
        ++kl;
      }
    }
    if (P.weighted) {
      P.wz.assign(zc_total, 0.0);
      P.rmz = rmz;
    }
    size_t gi = 0;
    for (size_t q = 0; q < em.size(); ++q) {
      const Emit& e = em[q];
      const int64_t pos = tk[e.z] >= 0 ? P.t_base + (base[e.z]++) * n_t + tk[e.z] : base[e.z]++;
      P.idx[e.key] = (int32_t)pos;
      if (P.weighted) {
        while (q >= em_rho[gi].end) ++gi;
        P.wz[pos] = em_rho[gi].rho;
      }
    }
    for (const TEmit& e : tem) {
      const int64_t pos = P.t_base + (int64_t)e.j * n_t + tk[e.z];
      P.idx[e.key] = (int32_t)pos;
      if (P.weighted) P.wz[pos] = e.rw;
    }
  }
  // pool = [contributions | m regions | x regions], each region aligned
  P.n_m = round_up(P.n_m, 64);
  P.zc_span = round_up(zc_total, 64);
  for (BucketDesc& b : P.bt) {
    b.m_off += P.zc_span;
    b.x_off = b.m_off + P.n_m;
  }
  for (auto& v : P.upos) v += P.zc_span;
  if (P.zc_span + 2 * P.n_m > 0x7fffffffLL)
    return admmi::set_err(ADMM_E_UNSUPPORTED, "more than 2^31 pool elements");
  // each contribution is written once and read once; its destination index read once
  P.layout_elems += 2 * P.n_zc;
  P.layout_idx_bytes += P.n_zc * 4;
  return ADMM_OK;
}

constexpr int64_t RES_LDS_BYTES = 96 * 1024;   // image limit of the resident driver
constexpr int32_t DEFAULT_GRAPH_BLOCK = 32;     // iterations per block of the graph driver
constexpr int64_t RES_AUTO_MAX_BLOCKS = 64;    // auto: resident up to this many pass blocks

admm_status check_graph(admm_graph* g) {
  if (!g) return admmi::set_err(ADMM_E_ARG, "graph handle is NULL");
  return ADMM_OK;
}

admm_status check_ready(admm_graph* g) {
  if (!g) return admmi::set_err(ADMM_E_ARG, "graph handle is NULL");
  if (g->state != 2) return admmi::set_err(ADMM_E_STATE, "graph is not finalized on a device");
  return ADMM_OK;
}

}  // namespace

extern "C" {

admm_status admm_graph_create(int32_t n_vars, const int32_t* var_dim, int32_t precision,
                              admm_graph** out) {
  admmi::clear_err();
  if (!out) return admmi::set_err(ADMM_E_ARG, "out is NULL");
  *out = nullptr;
  if (n_vars < 0 || (n_vars > 0 && !var_dim)) return admmi::set_err(ADMM_E_ARG, "bad variable list");
  if (precision != ADMM_FP32 && precision != ADMM_FP64)
    return admmi::set_err(ADMM_E_ARG, "precision must be ADMM_FP32 or ADMM_FP64");
  std::unique_ptr<admm_graph> g(new admm_graph());
  g->precision = precision;
  g->dim.assign(var_dim, var_dim + n_vars);
  g->zoff.resize(n_vars);
  int64_t off = 0;
  for (int32_t i = 0; i < n_vars; ++i) {
    if (var_dim[i] < 1) return admmi::set_err(ADMM_E_ARG, "variable %d has dimension %d < 1", i, var_dim[i]);
    g->zoff[i] = off;
    off += var_dim[i];
  }
  if (off > 0x7fffffffLL) return admmi::set_err(ADMM_E_UNSUPPORTED, "more than 2^31 scalars in z");
  g->nz = off;
  *out = g.release();
  return ADMM_OK;
}

admm_status admm_graph_add_factors(admm_graph* g, int32_t kind, int32_t n_factors, int32_t arity,
                                   const int32_t* var_ids, const double* params, int32_t param_len,
                                   int32_t shared_params) {
  admmi::clear_err();
  if (admm_status s = check_graph(g)) return s;
  if (g->state != 0) return admmi::set_err(ADMM_E_STATE, "graph already finalized");
  if (kind < KD_NONOVERLAP || kind > KD_MARGIN) return admmi::set_err(ADMM_E_ARG, "unknown factor kind %d", kind);
  if (n_factors < 0 || arity < 1 || param_len < 0) return admmi::set_err(ADMM_E_ARG, "bad sizes");
  if (n_factors > 0 && !var_ids) return admmi::set_err(ADMM_E_ARG, "var_ids is NULL");
  if (param_len > 0 && !params) return admmi::set_err(ADMM_E_ARG, "params is NULL");
  Group gr;
  gr.kind = kind;
  gr.n = n_factors;
  gr.arity = arity;
  gr.plen = param_len;
  gr.shared = shared_params != 0;
  gr.vids.assign(var_ids, var_ids + (int64_t)n_factors * arity);
  int64_t slots = 0;
  for (int64_t i = 0; i < (int64_t)gr.vids.size(); ++i) {
    const int32_t v = gr.vids[i];
    if (v < 0 || v >= (int32_t)g->dim.size())
      return admmi::set_err(ADMM_E_ARG, "variable id %d out of range [0,%d)", v, (int)g->dim.size());
    slots += g->dim[v];
  }
  for (int64_t f = 0; f < n_factors; ++f)
    for (int e = 0; e < arity; ++e)
      for (int e2 = e + 1; e2 < arity; ++e2)
        if (gr.vids[f * arity + e] == gr.vids[f * arity + e2])
          return admmi::set_err(ADMM_E_ARG, "factor %lld lists variable %d twice", (long long)f,
                                gr.vids[f * arity + e]);
  const int64_t np = gr.shared ? param_len : (int64_t)n_factors * param_len;
  if (np) gr.params.assign(params, params + np);
  {
    std::string why;
    int32_t nn = 0, mm = 0;
    if (!kind_dim_ok(*g, gr, why, nn, mm)) return admmi::set_err(ADMM_E_ARG, "%s", why.c_str());
  }
  g->n_factors += n_factors;
  g->n_edges += (int64_t)n_factors * arity;
  g->n_slots += slots;
  g->groups.push_back(std::move(gr));
  return ADMM_OK;
}

admm_status admm_graph_set_rho(admm_graph* g, double rho) {
  admmi::clear_err();
  if (admm_status s = check_graph(g)) return s;
  if (g->state != 0) return admmi::set_err(ADMM_E_STATE, "graph already finalized");
  if (!(rho > 0.0) || !std::isfinite(rho)) return admmi::set_err(ADMM_E_ARG, "rho must be > 0");
  g->rho = rho;
  return ADMM_OK;
}

admm_status admm_graph_set_group_rho(admm_graph* g, int32_t group, double rho) {
  admmi::clear_err();
  if (admm_status s = check_graph(g)) return s;
  if (g->state != 0) return admmi::set_err(ADMM_E_STATE, "graph already finalized");
  if (group < 0 || group >= (int32_t)g->groups.size())
    return admmi::set_err(ADMM_E_ARG, "group %d out of range (%d groups)", group, (int)g->groups.size());
  if (!(rho > 0.0) || !std::isfinite(rho)) return admmi::set_err(ADMM_E_ARG, "rho must be > 0");
  g->groups[group].rho = rho;
  return ADMM_OK;
}

admm_status admm_graph_set_group_alpha(admm_graph* g, int32_t group, double alpha) {
  admmi::clear_err();
  if (admm_status s = check_graph(g)) return s;
  if (g->state != 0) return admmi::set_err(ADMM_E_STATE, "graph already finalized");
  if (group < 0 || group >= (int32_t)g->groups.size())
    return admmi::set_err(ADMM_E_ARG, "group %d out of range (%d groups)", group, (int)g->groups.size());
  if (!(alpha > 0.0) || !std::isfinite(alpha)) return admmi::set_err(ADMM_E_ARG, "alpha must be > 0");
  g->groups[group].alpha = alpha;
  return ADMM_OK;
}

admm_status admm_graph_set_alpha(admm_graph* g, double alpha) {
  admmi::clear_err();
  if (admm_status s = check_graph(g)) return s;
  if (g->state != 0) return admmi::set_err(ADMM_E_STATE, "graph already finalized");
  if (!(alpha > 0.0) || !std::isfinite(alpha)) return admmi::set_err(ADMM_E_ARG, "alpha must be > 0");
  g->alpha = alpha;
  return ADMM_OK;
}

admm_status admm_graph_set_option(admm_graph* g, int32_t option, int64_t value) {
  admmi::clear_err();
  if (admm_status s = check_graph(g)) return s;
  if (g->state != 0) return admmi::set_err(ADMM_E_STATE, "graph already finalized");
  switch (option) {
    case ADMM_OPT_PAIR_ROWS:
      if (value != 0 && value != 16 && value != 32 && value != 64)
        return admmi::set_err(ADMM_E_ARG, "pair tile rows must be 0, 16, 32 or 64");
      g->pair_rows = (int32_t)value;
      return ADMM_OK;
    case ADMM_OPT_PAIR_STATE:
      if (value != ADMM_PAIR_STATE_AUTO && value != ADMM_PAIR_STATE_DENSE)
        return admmi::set_err(ADMM_E_ARG, "pair state must be 0 (auto) or 1 (dense)");
      g->pair_state = (int32_t)value;
      return ADMM_OK;
    case ADMM_OPT_DRIVER:
      if (value != ADMM_DRIVER_AUTO && value != ADMM_DRIVER_LAUNCHES &&
          value != ADMM_DRIVER_RESIDENT && value != ADMM_DRIVER_GRAPH)
        return admmi::set_err(ADMM_E_ARG,
                              "driver must be 0 (auto), 1 (launches), 2 (resident) or 3 (graph)");
      g->driver = (int32_t)value;
      return ADMM_OK;
    case ADMM_OPT_ZLIST:
      if (value != 0 && value != ADMM_ZLIST_ZMAJOR && value != 16 && value != 32 && value != 64)
        return admmi::set_err(ADMM_E_ARG, "z-list layout must be 0, 1, 16, 32 or 64");
      g->zlist = (int32_t)value;
      return ADMM_OK;
    case ADMM_OPT_THREE_WEIGHT:
      if (value != 0 && value != 1) return admmi::set_err(ADMM_E_ARG, "three-weight must be 0 or 1");
      g->twa = (int32_t)value;
      return ADMM_OK;
    case ADMM_OPT_GRAPH_BLOCK:
      if (value != 0 && (value < 2 || value > 4096 || (value & 1)))
        return admmi::set_err(ADMM_E_ARG, "graph block must be 0 (default) or even in [2, 4096]");
      g->graph_block = value ? (int32_t)value : DEFAULT_GRAPH_BLOCK;
      return ADMM_OK;
    default:
      return admmi::set_err(ADMM_E_ARG, "unknown option %d", option);
  }
}

admm_status admm_graph_finalize(admm_graph* g, int32_t device) {
  admmi::clear_err();
  if (admm_status s = check_graph(g)) return s;
  if (g->state == 2) return admmi::set_err(ADMM_E_STATE, "graph already finalized");
  const int64_t es_ = g->precision == ADMM_FP64 ? 8 : 4;
  // Resident candidates: the m and x regions alone must fit the LDS image.
  if (g->twa && g->driver == ADMM_DRIVER_RESIDENT)
    return admmi::set_err(ADMM_E_UNSUPPORTED, "the three-weight variant runs with launches or graph blocks");
  bool want_res = (g->driver == ADMM_DRIVER_AUTO || g->driver == ADMM_DRIVER_RESIDENT) &&
                  !g->twa && g->n_slots * 2 * es_ <= RES_LDS_BYTES;
  if (g->driver == ADMM_DRIVER_RESIDENT && !want_res)
    return admmi::set_err(ADMM_E_UNSUPPORTED, "resident driver: %lld slots do not fit in LDS",
                          (long long)g->n_slots);
  if (admm_status s = build_plan(*g, g->plan, want_res)) return s;
  if (want_res) {
    const int64_t bytes = resident_image_bytes(g->plan, g->nz, es_);
    const int64_t blocks = g->plan.xblocks + zpass_blocks(g->plan);
    bool ok = bytes <= RES_LDS_BYTES;
    if (g->driver == ADMM_DRIVER_RESIDENT && !ok)
      return admmi::set_err(ADMM_E_UNSUPPORTED, "resident driver: LDS image of %lld B exceeds %lld B",
                            (long long)bytes, (long long)RES_LDS_BYTES);
    if (g->driver == ADMM_DRIVER_AUTO && blocks > RES_AUTO_MAX_BLOCKS) ok = false;
    if (!ok) {
      if (admm_status s = build_plan(*g, g->plan, false)) return s;
    }
    g->plan.resident = ok;
  }
  const Plan& P = g->plan;
  const int64_t es = g->precision == ADMM_FP64 ? 8 : 4;
  if (g->twa) {
    // the three-weight variant is built for packing graphs: non-overlap
    // (pair tiles with their sparse state, or general), wall and separable
    // factors, one rho and alpha = 1
    if (!P.alpha_one || P.weighted)
      return admmi::set_err(ADMM_E_UNSUPPORTED, "the three-weight variant needs alpha = 1 and one rho");
    for (const BucketDesc& b : P.bt) {
      const bool ok = (b.mode == BM_PAIR && b.sparse) || b.mode == BM_GEN_SLOT ||
                      (b.mode == BM_GEN_FACTOR && (b.kind == KD_NONOVERLAP || b.kind == KD_WALL));
      if (!ok)
        return admmi::set_err(ADMM_E_UNSUPPORTED,
                              "the three-weight variant supports non-overlap, wall and separable "
                              "factors (kind %d is not one)", (int)b.kind);
    }
  }
  admm_graph_info& I = g->info;
  I.n_vars = (int64_t)g->dim.size();
  I.n_scalars = g->nz;
  I.n_factors = g->n_factors;
  I.n_edges = g->n_edges;
  I.n_slots = g->n_slots;
  I.n_buckets = (int64_t)P.bt.size();
  I.n_pair_tiles = P.n_pair_tiles;
  I.n_contributions = P.n_zc;
  I.precision = g->precision;
  I.alpha_is_one = P.alpha_one;
  I.state_bytes = (P.zc_span + 2 * P.n_m) * es;
  // algorithmic: state read + write per slot (m; plus x when alpha != 1) and
  // per-factor prox data; layout: indices, partial sums and their reads.
  I.algo_bytes_per_iter = P.algo_elems * es * (P.alpha_one ? 1 : 2);
  I.layout_bytes_per_iter = P.layout_elems * es + P.layout_idx_bytes;
  // without the resident driver: launches when asked for, else recorded
  // iteration blocks (the same kernels in the same order)
  const int32_t eager = g->driver == ADMM_DRIVER_LAUNCHES ? ADMM_DRIVER_LAUNCHES : ADMM_DRIVER_GRAPH;
  I.driver = P.resident ? ADMM_DRIVER_RESIDENT : eager;
  I.sparse_pair_state = P.n_flags > 0 ? 1 : 0;
  I.three_weight = g->twa;
  I.resident_lds_bytes = P.resident ? (int32_t)resident_image_bytes(P, g->nz, es) : 0;
  if (admm_status s = admmi::probe_device(device)) {
    g->state = 1;
    return s;
  }
  ADMM_HIP(hipSetDevice(device));
  std::unique_ptr<EngineBase> eng(g->precision == ADMM_FP64 ? make_engine_f64(device)
                                                              : make_engine_f32(device));
  if (g->plan.resident) {
    if (admm_status s = eng->resident_check(P, g->nz, P.alpha_one)) {
      if (g->driver == ADMM_DRIVER_RESIDENT) return s;
      admmi::clear_err();
      g->plan.resident = false;  // auto: the same plan runs with launches
      I.driver = eager;
      I.resident_lds_bytes = 0;
    }
  }
  eng->graph_block = I.driver == ADMM_DRIVER_GRAPH ? g->graph_block : 0;
  eng->twa = g->twa != 0;
  std::vector<double> z0(g->nz, 0.0);
  if (admm_status s = eng->upload(P, z0, g->rho, g->alpha)) return s;
  g->eng = std::move(eng);
  g->device = device;
  g->state = 2;
  // host copies only needed for the layout; keep user slot map on device only
  g->plan.idx.clear(); g->plan.idx.shrink_to_fit();
  g->plan.par.clear(); g->plan.par.shrink_to_fit();
  g->plan.upos.clear(); g->plan.upos.shrink_to_fit();
  g->plan.uz.clear(); g->plan.uz.shrink_to_fit();
  return ADMM_OK;
}

admm_status admm_graph_info_get(const admm_graph* g, admm_graph_info* info) {
  admmi::clear_err();
  if (!g || !info) return admmi::set_err(ADMM_E_ARG, "NULL argument");
  if (g->state == 0) return admmi::set_err(ADMM_E_STATE, "graph not finalized");
  *info = g->info;
  return ADMM_OK;
}

admm_status admm_set_state(admm_graph* g, const double* z, const double* u, void* stream) {
  admmi::clear_err();
  if (admm_status s = check_ready(g)) return s;
  if (!z) return admmi::set_err(ADMM_E_ARG, "z is NULL");
  return g->eng->set_state(z, u, (hipStream_t)stream);
}

admm_status admm_run(admm_graph* g, int32_t iters, void* stream) {
  admmi::clear_err();
  if (admm_status s = check_ready(g)) return s;
  if (iters < 0) return admmi::set_err(ADMM_E_ARG, "iters < 0");
  return g->eng->run(iters, (hipStream_t)stream);
}

admm_status admm_run_profiled(admm_graph* g, int32_t iters, void* stream, double* xpass_ms,
                              double* zpass_ms) {
  admmi::clear_err();
  if (admm_status s = check_ready(g)) return s;
  if (iters < 0 || !xpass_ms || !zpass_ms) return admmi::set_err(ADMM_E_ARG, "bad arguments");
  return g->eng->run_profiled(iters, (hipStream_t)stream, xpass_ms, zpass_ms);
}

admm_status admm_get_z(admm_graph* g, double* z, void* stream) {
  admmi::clear_err();
  if (admm_status s = check_ready(g)) return s;
  if (!z) return admmi::set_err(ADMM_E_ARG, "z is NULL");
  return g->eng->get_z(z, (hipStream_t)stream);
}

admm_status admm_get_u(admm_graph* g, double* u, void* stream) {
  admmi::clear_err();
  if (admm_status s = check_ready(g)) return s;
  if (!u) return admmi::set_err(ADMM_E_ARG, "u is NULL");
  return g->eng->get_slots(u, 0, (hipStream_t)stream);
}

admm_status admm_get_x(admm_graph* g, double* x, void* stream) {
  admmi::clear_err();
  if (admm_status s = check_ready(g)) return s;
  if (!x) return admmi::set_err(ADMM_E_ARG, "x is NULL");
  return g->eng->get_slots(x, 1, (hipStream_t)stream);
}

admm_status admm_get_residuals(admm_graph* g, double* r, double* s, void* stream) {
  admmi::clear_err();
  if (admm_status st = check_ready(g)) return st;
  if (!r || !s) return admmi::set_err(ADMM_E_ARG, "NULL output");
  return g->eng->residuals(r, s, (hipStream_t)stream);
}

admm_status admm_z_device_ptr(admm_graph* g, void** z_dev) {
  admmi::clear_err();
  if (admm_status s = check_ready(g)) return s;
  if (!z_dev) return admmi::set_err(ADMM_E_ARG, "NULL output");
  *z_dev = g->eng->z_ptr();
  return ADMM_OK;
}

admm_status admm_graph_destroy(admm_graph* g) {
  admmi::clear_err();
  delete g;
  return ADMM_OK;
}

}  // extern "C"
