// Device side of the factor-graph ADMM engine (gfx950, wave64).
//
// One iteration of Algorithm 2 (paper Sec. II) is two launches:
//   x-pass  one fused launch over every factor bucket.  Per edge slot it
//           reads the persistent state, forms u and n = z - u, applies the
//           bucket's proximal operator (eq. (3), appendix closed forms),
//           forms m = x + u and writes the new state.  Structured buckets
//           also emit per-tile partial sums of m for the z-update.
//   z-pass  z_b = (sum of b's contributions) / deg(b), summed in a fixed
//           order (one lane per short list, a wavefront tree per long list):
//           deterministic, no atomics.
// Contributions (per-tile partial sums, or m itself for unstructured
// buckets) are written by the x-pass straight into a z-major buffer at the
// start of the pool, through destination tables built at finalize, so each
// variable's contributions are contiguous for the z-pass.
// State per slot: with alpha == 1 only m is kept (u = m - z, n = 2z - m);
// otherwise m and x are kept and u = (m - x) + alpha (x - z).
#pragma once

#include "internal.h"

namespace admmg {

constexpr int NT = 256;              // threads per workgroup, every pass
constexpr int PB = 64;               // entity block of dense pair tiles
constexpr int PR = PB * PB / NT;     // pair rows per thread
constexpr int MAXN = 16;             // lindyn state dim limit (general path)
constexpr int MAXM = 8;              // lindyn input dim limit (general path)
constexpr int LANE_MAX = 4;          // z-lists up to this length: one lane
constexpr int ZB_MIN = 128;          // z-lists longer than this: one workgroup

enum BucketMode : int32_t {
  BM_PAIR = 1,        // complete pairwise non-overlap, dense 64x64 tiles
  BM_UNIF_HINGE = 2,  // hinge factors that all share one variable list
  BM_GEN_FACTOR = 3,  // one thread per factor, per-edge z offsets
  BM_GEN_SLOT = 4,    // separable prox: one thread per scalar slot
};

enum PassMode : int { PM_NORMAL = 0, PM_SAVE = 1, PM_RESID = 2 };

enum Kind : int32_t {
  KD_NONOVERLAP = 1, KD_WALL = 2, KD_RADIUS = 3, KD_QUAD = 4, KD_BOX = 5,
  KD_HINGE = 6, KD_L2 = 7, KD_LINDYN = 8, KD_LINDYN0 = 9,
  KD_MINERR = 10, KD_EQUAL = 11, KD_MARGIN = 12,
};

// Descriptor of one bucket, read by the x-pass from device memory.
struct BucketDesc {
  int32_t mode, kind;
  int32_t blk0, blk1;   // x-pass workgroups [blk0, blk1)
  int64_t n;            // factors (factor modes), slots (GEN_SLOT), tiles (PAIR)
  int64_t nfp;          // SoA row stride
  int32_t arity, nslot; // edges / scalar slots per factor
  int32_t d, nn, mm, dmax;  // hinge d (and its register bound); lindyn n, m
  int32_t E, NB;        // pair layout: entities, column blocks
  int32_t rb;           // pair layout: entities per row block (16, 32 or 64)
  int32_t sparse;       // pair layout: state of unmoved pairs kept implicit (FP32, alpha = 1)
  int64_t flag0;        // pair layout: first flag word of this bucket (per tile NT words)
  int32_t ent_aff;      // pair layout: entity e's z offsets are ent_base + 3e (centre), + 2 (radius)
  int32_t ent_base;
  int32_t ub;           // hinge/margin: the b edge is one variable for every factor
                        // of the bucket, which takes one partial sum per workgroup
  int32_t tri;          // pair layout: 64-row tiles in row-major order of the whole
                        // upper triangle (J >= I), so (I, J) follows from the tile index
  int32_t quad;         // shared-variable hinge: four factors per lane (FP32, alpha = 1)
  int32_t quad_pad;
  int64_t m_off, x_off;  // element offsets of the state regions in the pool
  int64_t twb_off;      // three-weight variant: first byte of this bucket's active flags
  int64_t dst_off;      // index-buffer offset of the contribution destinations
  int64_t idx_off;      // offset in the int32 index buffer
  int64_t par_off;      // element offset in the parameter buffer
  double irho;          // 1 / rho of this bucket's edges
  double alpha;         // alpha of this bucket's edges
};

template <typename T>
struct XArgs {
  T* pool;
  const int32_t* idx;
  const T* par;
  const T* z;
  const T* zprev;       // z of the previous iteration (sparse pair state)
  uint16_t* flags;      // sparse pair state: bit set = m stored explicitly
  T* blockmax;
  const BucketDesc* bt;
  int32_t nb;
  T alpha, inv_rho;
  // three-weight variant (null otherwise): per contribution position the
  // weight written with it, per z scalar "no edge weighted" from the last
  // z-update, per constraint factor "sent weight rho" in the last x-update
  T* wc;
  const uint8_t* zfree;
  uint8_t* twb;
};

template <typename T>
struct ZArgs {
  const T* pool;
  const int32_t* var_t;   // transposed lists (pair-tile entities): 64 per block
  const T* deg_t;
  int64_t n_t, t_base;
  int32_t nb_t, t_len, t_lpb;  // blocks, padded length, lists per block (16, 32 or 64)
  const int32_t* var_b;   // lists of more than ZB_MIN contributions: one block each
  const int64_t* rng_b;
  const T* deg_b;
  int32_t n_b;
  const int32_t* var_w;   // lists of LANE_MAX+1 .. ZB_MIN: one 16-lane row each
  const int64_t* rng_w;   // explicit ranges when w_stride == 0
  const T* deg_w;
  int64_t n_w;
  int32_t nb_w;
  const int32_t* var_l;   // lists of at most LANE_MAX: one lane each, stride LANE_MAX
  const T* deg_l;         // 0: no edge, z keeps its value
  int64_t n_l;
  int64_t w_stride, w_base, l_base;  // padded list layout (pool positions)
  const T* zin;
  T* zout;
  T* blockmax;
  const T* wz;            // per contribution position: its edge's rho (null: all equal)
  const T* rmz;           // per z scalar: the largest rho of its edges (with wz)
  int32_t check;
  // three-weight variant (null otherwise): z = sum(contributions) /
  // sum(weights written with them), z kept and zfree set when every weight is 0
  const T* wc;
  uint8_t* zfree;
};

template <typename T>
__device__ __forceinline__ T tabs(T v) { return v < T(0) ? -v : v; }
template <typename T>
__device__ __forceinline__ T tmax(T a, T b) { return a > b ? a : b; }
template <typename T>
__device__ __forceinline__ T tmin(T a, T b) { return a < b ? a : b; }

// Block-wide max of non-negative values, stored by thread 0 at *out (the
// caller points out at its block's slot).  A NaN enters as +infinity, so a
// non-finite iterate anywhere in the block always reaches the result (a
// plain max can drop a NaN operand).
template <typename T>
__device__ __forceinline__ void block_max_store(T v, T* out) {
  __shared__ T red[NT / 64];
  if (!(v == v)) v = T(INFINITY);
  v = admmi::wave_max(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    T mx = red[0];
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) mx = tmax(mx, red[i]);
    out[0] = mx;
  }
}

// u and n of one slot from the stored state.
template <typename T, bool A1>
__device__ __forceinline__ void state_un(T m, T xo, T zv, T alpha, T& u, T& n) {
  if constexpr (A1) {
    u = m - zv;
  } else {
    u = (m - xo) + alpha * (xo - zv);
  }
  n = zv - u;
}

// ---------------------------------------------------------------------------
// Proximal operators in working precision (appendix closed forms).
// ---------------------------------------------------------------------------

// Square root and reciprocal: FP32 uses the hardware instructions (within
// 1 ulp), FP64 the correctly rounded library forms.
__device__ __forceinline__ float tsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double tsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float trcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double trcp(double x) { return 1.0 / x; }

// Non-overlap |c1 - c2| >= r1 + r2 with equal weights: move both centres
// apart along n_hat and shrink both radii by D/4, D = max(0, r1+r2-|c2-c1|);
// n_hat = (1,0) when the centres coincide.
template <typename T>
__device__ __forceinline__ bool prox_nonoverlap(T* v) {
  const T dx = v[3] - v[0], dy = v[4] - v[1];
  const T L = tsqrt(dx * dx + dy * dy);
  const T D = v[2] + v[5] - L;
  const bool moved = D > T(0);
  if (moved) {
    T hx = T(1), hy = T(0);
    if (L > T(0)) {
      const T il = trcp(L);
      hx = dx * il;
      hy = dy * il;
    }
    const T st = D * T(0.25);
    v[0] -= st * hx;
    v[1] -= st * hy;
    v[2] -= st;
    v[3] += st * hx;
    v[4] += st * hy;
    v[5] -= st;
  }
  return moved;
}

// Wall Q^T(c - V) >= r; p = (Qx, Qy, Q.V, 1/(|Q|^2+1)).  Returns whether
// the constraint was active (the prox moved its input).
template <typename T>
__device__ __forceinline__ bool prox_wall(T* v, T qx, T qy, T qv, T ik) {
  const T g = qx * v[0] + qy * v[1] - qv - v[2];
  if (g < T(0)) {
    const T st = -g * ik;
    v[0] += st * qx;
    v[1] += st * qy;
    v[2] -= st;
  }
  return g < T(0);
}

// Three-weight variant (Sec. II's per-edge weights; every message weight is
// 0 or rho).  An edge received with weight 0 belongs to a variable no
// factor weighted in the last z-update; the zero-weight edges of a
// constraint factor absorb its whole correction in equal shares and the
// other edges keep their input.  Non-overlap: bits of fr = c1, r1, c2, r2
// received with weight 0 (at least one set).
template <typename T>
__device__ __forceinline__ bool prox_nonoverlap_free(T* v, unsigned fr) {
  const T dx = v[3] - v[0], dy = v[4] - v[1];
  const T L = tsqrt(dx * dx + dy * dy);
  const T D = v[2] + v[5] - L;
  const bool moved = D > T(0);
  if (moved) {
    T hx = T(1), hy = T(0);
    if (L > T(0)) {
      const T il = trcp(L);
      hx = dx * il;
      hy = dy * il;
    }
    const T st = D / T(__popc(fr));
    if (fr & 1u) { v[0] -= st * hx; v[1] -= st * hy; }
    if (fr & 2u) v[2] -= st;
    if (fr & 4u) { v[3] += st * hx; v[4] += st * hy; }
    if (fr & 8u) v[5] -= st;
  }
  return moved;
}

// Wall with bits of fr = c, r received with weight 0 (at least one set).
template <typename T>
__device__ __forceinline__ bool prox_wall_free(T* v, T qx, T qy, T qv, unsigned fr) {
  const T g = qx * v[0] + qy * v[1] - qv - v[2];
  if (!(g < T(0))) return false;
  const T den = ((fr & 1u) ? qx * qx + qy * qy : T(0)) + ((fr & 2u) ? T(1) : T(0));
  const T lam = -g / den;
  if (fr & 1u) { v[0] += lam * qx; v[1] += lam * qy; }
  if (fr & 2u) v[2] -= lam;
  return true;
}

// Row and column block of pair tile `tile`: computed when the tiles are the
// whole upper triangle in row-major order (row I holds NB - I tiles and
// starts at tile I NB - I (I - 1) / 2; a root estimate, then exact integer
// steps), else read from the tile list.  Uniform across the workgroup.
__device__ __forceinline__ void pair_tile(const BucketDesc& b, const int32_t* tiles, int tile,
                                          int& I, int& J) {
  if (b.tri) {
    const int nb = b.NB;
    const float q = (float)(2 * nb + 1);
    int i = (int)(0.5f * (q - sqrtf(q * q - 8.f * (float)tile)));
    i = i < 0 ? 0 : (i > nb - 1 ? nb - 1 : i);
    auto first = [nb](int r) { return r * nb - r * (r - 1) / 2; };
    while (i + 1 < nb && first(i + 1) <= tile) ++i;
    while (i > 0 && first(i) > tile) --i;
    I = i;
    J = i + (tile - first(i));
  } else {
    I = tiles[2 * tile];
    J = tiles[2 * tile + 1];
  }
}

// ---------------------------------------------------------------------------
// Dense pairwise non-overlap tiles.  Tile (I, J) holds the pairs
// (e_i, e_j) = (I*RB + li, J*64 + lj), li < RB, lj < 64, of which those with
// e_i < e_j < E are real factors; storage [slot 0..5][li*64 + lj] with slots
// (c_i.x, c_i.y, r_i, c_j.x, c_j.y, r_j).  Thread t owns column lj = t % 64
// and rows (t/64)*RB/4 .. +RB/4-1; rows are summed across the wavefront,
// columns in registers and then across the four wavefronts.
// Partials per tile: [row li][3] (RB rows) then [col lj][3] (64 columns).
// ---------------------------------------------------------------------------
constexpr int PAIR_UNROLL_F64 = 4;   // FP64 pair rows per unrolled step
template <typename T, bool A1, int MODE, int RB>
__device__ __forceinline__ void xpass_pair(const XArgs<T>& a, const BucketDesc& b, int tile) {
  constexpr int CB = PB;              // columns per tile
  constexpr int PRR = RB * CB / NT;   // rows per thread
  constexpr int TSZ = RB * CB;        // pairs per tile
  __shared__ T zrow[RB * 3];
  __shared__ T zcol[CB * 3];
  __shared__ T cacc[NT / 64][CB * 3];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int32_t* tiles = a.idx + b.idx_off;
  const int32_t* ent = tiles + 2 * b.n;
  int I, J;
  pair_tile(b, tiles, tile, I, J);
  if (t < RB + CB) {
    const bool isrow = t < RB;
    const int l = isrow ? t : t - RB;
    const int e = isrow ? I * RB + l : J * CB + l;
    T cx = T(0), cy = T(0), r = T(0);
    if (e < b.E) {
      const int zc = ent[2 * e], zr = ent[2 * e + 1];
      cx = a.z[zc];
      cy = a.z[zc + 1];
      r = a.z[zr];
    }
    T* dst = isrow ? zrow : zcol;
    dst[l * 3 + 0] = cx;
    dst[l * 3 + 1] = cy;
    dst[l * 3 + 2] = r;
  }
  __syncthreads();
  const int lj = lane;
  const int ej = J * CB + lj;
  const T zj0 = zcol[lj * 3 + 0], zj1 = zcol[lj * 3 + 1], zj2 = zcol[lj * 3 + 2];
  constexpr int64_t TS = 6 * (int64_t)TSZ;
  T* mt = a.pool + b.m_off + (int64_t)tile * TS;
  T* xt = a.pool + b.x_off + (int64_t)tile * TS;
  T ca0 = T(0), ca1 = T(0), ca2 = T(0);
  T rv0 = T(0), rv1 = T(0), rv2 = T(0);
  T rmax = T(0);
  // FP64: rows four at a time, so that the loads in flight stay within the
  // registers of four wavefronts per SIMD
  constexpr int UNR = sizeof(T) == 8 ? PAIR_UNROLL_F64 : PRR;
#pragma unroll UNR
  for (int k = 0; k < PRR; ++k) {
    const int li = w * PRR + k;
    const int ei = I * RB + li;
    const bool valid = (ei < ej) && (ej < b.E);
    const int p = li * CB + lj;
    const T zz[6] = {zrow[li * 3 + 0], zrow[li * 3 + 1], zrow[li * 3 + 2], zj0, zj1, zj2};
    T mv[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) mv[s] = mt[s * TSZ + p];
    if constexpr (MODE == PM_RESID) {
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        const T xv = xt[s * TSZ + p];
        if (valid) rmax = tmax(rmax, tabs(xv - zz[s]));
      }
    } else {
      T u[6], v[6];
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        T xo = T(0);
        if constexpr (!A1) xo = xt[s * TSZ + p];
        state_un<T, A1>(mv[s], xo, zz[s], (T)b.alpha, u[s], v[s]);
      }
      prox_nonoverlap(v);
      T mn[6];
#pragma unroll
      for (int s = 0; s < 6; ++s) mn[s] = v[s] + u[s];
      if (valid) {
#pragma unroll
        for (int s = 0; s < 6; ++s) {
          mt[s * TSZ + p] = mn[s];
          if constexpr (!A1 || MODE == PM_SAVE) xt[s * TSZ + p] = v[s];
        }
      }
      ca0 += valid ? mn[3] : T(0);
      ca1 += valid ? mn[4] : T(0);
      ca2 += valid ? mn[5] : T(0);
      const T r0 = admmi::wave_sum(valid ? mn[0] : T(0));
      const T r1 = admmi::wave_sum(valid ? mn[1] : T(0));
      const T r2 = admmi::wave_sum(valid ? mn[2] : T(0));
      if (lane == k) {
        rv0 = r0;
        rv1 = r1;
        rv2 = r2;
      }
    }
  }
  if constexpr (MODE == PM_RESID) {
    block_max_store(rmax, a.blockmax);
  } else {
    const int32_t* dst = a.idx + b.dst_off + (int64_t)tile * (3 * (RB + CB));
    if (lane < PRR) {
      const int li = w * PRR + lane;
      const int d0 = dst[li * 3];
      if (d0 >= 0) {
        a.pool[d0] = rv0;
        a.pool[dst[li * 3 + 1]] = rv1;
        a.pool[dst[li * 3 + 2]] = rv2;
      }
    }
    cacc[w][lj * 3 + 0] = ca0;
    cacc[w][lj * 3 + 1] = ca1;
    cacc[w][lj * 3 + 2] = ca2;
    __syncthreads();
    if (t < CB * 3) {
      T s = cacc[0][t];
#pragma unroll
      for (int q = 1; q < NT / 64; ++q) s += cacc[q][t];
      const int d = dst[3 * RB + t];
      if (d >= 0) a.pool[d] = s;
    }
  }
}

// FP32 with alpha = 1: the same tile computation with 16-byte accesses.
// Thread (w, rg = lane / 16, cq = lane % 16) owns columns 4cq .. 4cq+3 and
// rows li = w*RB/4 + 4k + rg, k < RB/16, so that one load instruction of a
// wavefront covers four whole rows (1 KB).  Every load of a thread is issued
// before its first prox.  Row sums: over the thread's four columns, then a
// 16-lane DPP tree (one DPP row holds exactly the lanes of one tile row).
// Column sums: over the thread's rows, across the four DPP rows (xor 16,
// 32), then across the four wavefronts in LDS in wavefront order.  State of
// pairs that are not factors (lower triangle of diagonal tiles, padding) is
// updated too but never summed or returned, so that stores cover whole rows.
typedef float f4v __attribute__((ext_vector_type(4)));

template <int RB>
struct PairMap {
  static constexpr int CB = PB;
  static constexpr int PRT = RB / 16;   // rows per thread
  static constexpr int TSZ = RB * CB;   // pairs per tile
  static __device__ __forceinline__ int row(int w, int k, int rg) { return w * (RB / 4) + 4 * k + rg; }
};

// z offsets of pair-tile entity e (centre x, radius).
__device__ __forceinline__ void pair_entity(const BucketDesc& b, const int32_t* ent, int e,
                                            int& zc, int& zr) {
  if (b.ent_aff) {
    zc = b.ent_base + 3 * e;
    zr = zc + 2;
  } else {
    zc = ent[2 * e];
    zr = ent[2 * e + 1];
  }
}

// Column sums of a thread's four columns (three scalars each) across the
// four DPP rows of its wavefront and then the four wavefronts, in a fixed
// order; thread t < 192 returns the total for column t / 3, scalar t % 3.
__device__ __forceinline__ float pair_colsum(float (&cs)[4][3], float (*cacc)[PB * 3], int w,
                                            int rg, int cq, int t) {
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      float v = cs[c][s];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      cs[c][s] = v;
    }
  if (rg == 0) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int s = 0; s < 3; ++s) cacc[w][(4 * cq + c) * 3 + s] = cs[c][s];
  }
  __syncthreads();
  float sum = 0.f;
  if (t < PB * 3) {
    sum = cacc[0][t];
#pragma unroll
    for (int q = 1; q < NT / 64; ++q) sum += cacc[q][t];
  }
  return sum;
}

template <int MODE, int RB, bool TW = false>
__device__ __forceinline__ void xpass_pair_v4(const XArgs<float>& a, const BucketDesc& b,
                                              int tile) {
  using PM = PairMap<RB>;
  constexpr int CB = PM::CB, PRT = PM::PRT, TSZ = PM::TSZ;
  __shared__ float zrow4[RB * 3];
  __shared__ float zcol4[CB * 3];
  __shared__ float cacc4[NT / 64][CB * 3];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int rg = lane >> 4, cq = lane & 15;
  const int32_t* tiles = a.idx + b.idx_off;
  const int32_t* ent = tiles + 2 * b.n;
  int I, J;
  pair_tile(b, tiles, tile, I, J);
  constexpr int64_t TS = 6 * (int64_t)TSZ;
  const float* src = a.pool + (MODE == PM_RESID ? b.x_off : b.m_off) + (int64_t)tile * TS;
  f4v mv[PRT][6];
#pragma unroll
  for (int k = 0; k < PRT; ++k) {
    const int li = PM::row(w, k, rg);
#pragma unroll
    for (int s = 0; s < 6; ++s)
      mv[k][s] = *(const f4v*)(src + s * TSZ + li * CB + 4 * cq);
  }
  if (t < RB + CB) {
    const bool isrow = t < RB;
    const int l = isrow ? t : t - RB;
    const int e = isrow ? I * RB + l : J * CB + l;
    float cx = 0.f, cy = 0.f, r = 0.f;
    if (e < b.E) {
      int zc, zr;
      pair_entity(b, ent, e, zc, zr);
      cx = a.z[zc];
      cy = a.z[zc + 1];
      r = a.z[zr];
    }
    float* dst = isrow ? zrow4 : zcol4;
    dst[l * 3 + 0] = cx;
    dst[l * 3 + 1] = cy;
    dst[l * 3 + 2] = r;
  }
  __syncthreads();
  float zcl[4][3];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int s = 0; s < 3; ++s) zcl[c][s] = zcol4[(4 * cq + c) * 3 + s];
  const int ej0 = J * CB + 4 * cq;
  if constexpr (MODE == PM_RESID) {
    float rmax = 0.f;
#pragma unroll
    for (int k = 0; k < PRT; ++k) {
      const int li = PM::row(w, k, rg);
      const int ei = I * RB + li;
      float zr[3];
#pragma unroll
      for (int s = 0; s < 3; ++s) zr[s] = zrow4[li * 3 + s];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int ej = ej0 + c;
        if (ei < ej && ej < b.E) {
#pragma unroll
          for (int s = 0; s < 6; ++s)
            rmax = tmax(rmax, tabs(mv[k][s][c] - (s < 3 ? zr[s] : zcl[c][s - 3])));
        }
      }
    }
    block_max_store(rmax, a.blockmax);
    if constexpr (TW) {
      // three-weight variant: pairs the last iteration did not move sent
      // weight 0, so their dual is 0 and their m is the final z; then every
      // pair's m is explicit again
      uint16_t* flagp = a.flags + b.flag0 + (int64_t)tile * NT + t;
      const uint32_t fl = *flagp;
      float* mt = a.pool + b.m_off + (int64_t)tile * TS;
#pragma unroll
      for (int k = 0; k < PRT; ++k) {
        const int li = PM::row(w, k, rg);
        if (((fl >> (4 * k)) & 0xFu) == 0xFu) continue;
        f4v m4[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) m4[s] = *(const f4v*)(mt + s * TSZ + li * CB + 4 * cq);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if ((fl >> (4 * k + c)) & 1u) continue;
#pragma unroll
          for (int s = 0; s < 6; ++s) m4[s][c] = s < 3 ? zrow4[li * 3 + s] : zcl[c][s - 3];
        }
#pragma unroll
        for (int s = 0; s < 6; ++s) *(f4v*)(mt + s * TSZ + li * CB + 4 * cq) = m4[s];
      }
      *flagp = 0xFFFFu;
    }
  } else {
    float* mt = a.pool + b.m_off + (int64_t)tile * TS;
    float* xt = a.pool + b.x_off + (int64_t)tile * TS;
    const int32_t* dst = a.idx + b.dst_off + (int64_t)tile * (3 * (RB + CB));
    float cs[4][3];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int s = 0; s < 3; ++s) cs[c][s] = 0.f;
#pragma unroll
    for (int k = 0; k < PRT; ++k) {
      const int li = PM::row(w, k, rg);
      const int ei = I * RB + li;
      float zr[3];
#pragma unroll
      for (int s = 0; s < 3; ++s) zr[s] = zrow4[li * 3 + s];
      float rs[3] = {0.f, 0.f, 0.f};
      f4v xv[6];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int ej = ej0 + c;
        const bool valid = (ei < ej) && (ej < b.E);
        float u[6], v[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) {
          const float zv = s < 3 ? zr[s] : zcl[c][s - 3];
          u[s] = mv[k][s][c] - zv;
          v[s] = zv - u[s];
        }
        prox_nonoverlap(v);
#pragma unroll
        for (int s = 0; s < 6; ++s) {
          const float mn = v[s] + u[s];
          mv[k][s][c] = mn;
          xv[s][c] = v[s];
          if (s < 3) rs[s] += valid ? mn : 0.f;
          else cs[c][s - 3] += valid ? mn : 0.f;
        }
      }
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        *(f4v*)(mt + s * TSZ + li * CB + 4 * cq) = mv[k][s];
        if constexpr (MODE == PM_SAVE) *(f4v*)(xt + s * TSZ + li * CB + 4 * cq) = xv[s];
      }
#pragma unroll
      for (int s = 0; s < 3; ++s) rs[s] = admmi::row16_sum(rs[s]);
      if (cq < 3) {
        const int d = dst[li * 3 + cq];
        if (d >= 0) a.pool[d] = cq == 0 ? rs[0] : (cq == 1 ? rs[1] : rs[2]);
      }
    }
    const float sum = pair_colsum(cs, cacc4, w, rg, cq, t);
    if (t < CB * 3) {
      const int d = dst[3 * RB + t];
      if (d >= 0) a.pool[d] = sum;
    }
  }
}

// Sparse pair state (b.sparse; FP32, alpha = 1, x-pass modes NORMAL and
// SAVE).  A pair whose prox leaves n where it is (no overlap) ends the
// iteration with m = n + u = z exactly, the z the iteration started from.
// Such a pair stores nothing: its bit in the thread's 16-bit flag word is
// cleared, and the next iteration takes its m from the previous z.  Only
// pairs the prox moves store m (whole float4 rows of the thread, read back
// only where the flag is set).  Every pair's prox is evaluated every
// iteration: for a pair with implicit m, n and u depend on the two entities
// only and are formed once per entity (u = z_prev - z, n = z - u, the same
// formulas as for stored m); the overlap test D = r_i + r_j - |c_j - c_i| > 0
// is first taken without the square root, with a relative margin of 2^-18
// on |c_j - c_i|^2 (far above the rounding of the squares and of the root),
// and only pairs inside the margin or with stored m go through the full
// operator, so every decision equals the operator's own.  An unmoved pair
// contributes z to both partial sums: a row's partial is the sum of its
// moved pairs' m plus (valid pairs - moved pairs) * z, the valid count
// being known from the tile position; the DPP and cross-wavefront sums of
// the moved pairs are skipped when no pair of the wavefront (workgroup)
// moved.  All independent loads (flags, destinations, z of both
// iterations) are issued together at the start.  The last iteration of a
// run stores m and x of every pair and sets every flag, so that the dense
// arrays are complete between runs.
// TW (three-weight variant): an unmoved pair is an inactive constraint and
// sends weight 0, so its dual is 0 (n = z; no storage) and it adds nothing
// to the partial sums; the tile writes, with each partial, the number of
// moved pairs in it (the weight of that contribution).  A pair with an
// entity that no factor weighted takes the three-weight operator.  The
// last iteration keeps the flags of the moved pairs for the residual pass,
// which stores z as the m of every other pair (their dual is 0).
template <int MODE, int RB, bool TW = false>
__device__ __forceinline__ void xpass_pair_sparse(const XArgs<float>& a, const BucketDesc& b,
                                                  int tile) {
  using PM = PairMap<RB>;
  constexpr int CB = PM::CB, PRT = PM::PRT, TSZ = PM::TSZ;
  constexpr bool SAVE = MODE == PM_SAVE;
  __shared__ float erow[3][RB * 3];   // z, n, u of the row entities
  __shared__ float ecol[3][CB * 3];   // z, n, u of the column entities
  __shared__ float cacc5[NT / 64][CB * 3];
  __shared__ float cnt5[NT / 64][CB];
  __shared__ int any5;
  __shared__ uint8_t efr[TW ? RB + CB : 1];   // TW: bit 0 centre, bit 1 radius unweighted
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int rg = lane >> 4, cq = lane & 15;
  const int32_t* tiles = a.idx + b.idx_off;
  const int32_t* ent = tiles + 2 * b.n;
  int I, J;
  pair_tile(b, tiles, tile, I, J);
  constexpr int64_t TS = 6 * (int64_t)TSZ;
  uint16_t* flagp = a.flags + b.flag0 + (int64_t)tile * NT + t;
  const uint32_t fl = *flagp;       // set: m of the pair is stored
  const int32_t* dst = a.idx + b.dst_off + (int64_t)tile * (3 * (RB + CB));
  int drow[PRT];
#pragma unroll
  for (int k = 0; k < PRT; ++k) drow[k] = cq < 3 ? dst[PM::row(w, k, rg) * 3 + cq] : -1;
  const int dcol = t < CB * 3 ? dst[3 * RB + t] : -1;
  if (t < RB + CB) {
    const bool isrow = t < RB;
    const int l = isrow ? t : t - RB;
    const int e = isrow ? I * RB + l : J * CB + l;
    float zv[3] = {0.f, 0.f, 0.f}, zp[3] = {0.f, 0.f, 0.f};
    uint8_t fr = 0;
    if (e < b.E) {
      int zc, zr;
      pair_entity(b, ent, e, zc, zr);
      zv[0] = a.z[zc];
      zv[1] = a.z[zc + 1];
      zv[2] = a.z[zr];
      if constexpr (TW) {
        fr = (uint8_t)((a.zfree[zc] ? 1 : 0) | (a.zfree[zr] ? 2 : 0));
      } else {
        zp[0] = a.zprev[zc];
        zp[1] = a.zprev[zc + 1];
        zp[2] = a.zprev[zr];
      }
    }
    if constexpr (TW) efr[t] = fr;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const float u = TW ? 0.f : zp[s] - zv[s];
      const float n = TW ? zv[s] : zv[s] - u;
      if (isrow) {
        erow[0][l * 3 + s] = zv[s];
        erow[1][l * 3 + s] = n;
        erow[2][l * 3 + s] = u;
      } else {
        ecol[0][l * 3 + s] = zv[s];
        ecol[1][l * 3 + s] = n;
        ecol[2][l * 3 + s] = u;
      }
    }
  }
  if (t == 0) any5 = 0;
  __syncthreads();
  float cz[4][3], cn[4][3];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      cz[c][s] = ecol[0][(4 * cq + c) * 3 + s];
      cn[c][s] = ecol[1][(4 * cq + c) * 3 + s];
    }
  const int ej0 = J * CB + 4 * cq;
  // pairs that need the full operator: factors (e_i < e_j < E) with stored
  // m or whose overlap the test does not exclude; the last iteration of a
  // run takes every factor through it.  Other tile slots (the lower
  // triangle and the diagonal of diagonal tiles, padding) are never
  // evaluated: their state is not part of the method.
  uint32_t valid = 0;
#pragma unroll
  for (int k = 0; k < PRT; ++k) {
    const int ei = I * RB + PM::row(w, k, rg);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int ej = ej0 + c;
      valid |= ((ei < ej && ej < b.E) ? 1u : 0u) << (4 * k + c);
    }
  }
  uint32_t work = SAVE ? valid : (fl & valid);
  if constexpr (!SAVE) {
#pragma unroll
    for (int k = 0; k < PRT; ++k) {
      const int li = PM::row(w, k, rg);
      const float r0 = erow[1][li * 3 + 0], r1 = erow[1][li * 3 + 1], r2 = erow[1][li * 3 + 2];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float dx = cn[c][0] - r0, dy = cn[c][1] - r1;
        const float S = r2 + cn[c][2];
        const float L2 = dx * dx + dy * dy;
        const bool maybe = S > 0.f && S * S >= L2 * (1.f - 0x1p-18f);
        work |= (maybe ? 1u : 0u) << (4 * k + c);
      }
    }
    work &= valid;
  }
  float* mt = a.pool + b.m_off + (int64_t)tile * TS;
  float* xt = a.pool + b.x_off + (int64_t)tile * TS;
  // One row of the thread at a time, its partial emitted before the next
  // row starts, so that only the column sums live across rows (register
  // pressure sets how many workgroups share a CU).
  float cs[4][3], cmc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    cmc[c] = 0.f;
#pragma unroll
    for (int s = 0; s < 3; ++s) cs[c][s] = 0.f;
  }
  uint32_t movedall = 0;
  bool wave_moved = false;
#pragma unroll
  for (int k = 0; k < PRT; ++k) {
    const int li = PM::row(w, k, rg);
    const uint32_t rowwork = (work >> (4 * k)) & 0xFu;
    float rs[3] = {0.f, 0.f, 0.f}, rmc = 0.f;
    uint32_t moved_bits = 0;
    if (rowwork) {
      const uint32_t rowbits = (fl >> (4 * k)) & 0xFu;
      // mo: the row's m, read where stored and overwritten column by column
      f4v mo[6];
      if (rowbits) {
#pragma unroll
        for (int s = 0; s < 6; ++s)
          mo[s] = *(const f4v*)(mt + s * TSZ + li * CB + 4 * cq);
      }
      float rz[3], rn[3], ru[3];
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        rz[s] = erow[0][li * 3 + s];
        rn[s] = erow[1][li * 3 + s];
        ru[s] = erow[2][li * 3 + s];
      }
      f4v xo[6];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        float zv[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) zv[s] = s < 3 ? rz[s] : cz[c][s - 3];
        if (!((rowwork >> c) & 1u)) {
          // not a factor of this iteration's work: m = z, x = n
#pragma unroll
          for (int s = 0; s < 6; ++s) {
            mo[s][c] = zv[s];
            if constexpr (SAVE) xo[s][c] = s < 3 ? rn[s] : cn[c][s - 3];
          }
          continue;
        }
        const bool expl = (rowbits >> c) & 1u;
        float u[6], v[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) {
          if (expl) {
            u[s] = mo[s][c] - zv[s];
            v[s] = zv[s] - u[s];
          } else {
            u[s] = s < 3 ? ru[s] : ecol[2][(4 * cq + c) * 3 + s - 3];
            v[s] = s < 3 ? rn[s] : cn[c][s - 3];
          }
        }
        bool moved;
        if constexpr (TW) {
          const unsigned fr = (unsigned)efr[li] | ((unsigned)efr[RB + 4 * cq + c] << 2);
          moved = fr ? prox_nonoverlap_free(v, fr) : prox_nonoverlap(v);
        } else {
          moved = prox_nonoverlap(v);
        }
        if constexpr (SAVE) {
#pragma unroll
          for (int s = 0; s < 6; ++s) xo[s][c] = v[s];
        }
        if (moved) {
          moved_bits |= 1u << c;
#pragma unroll
          for (int s = 0; s < 6; ++s) mo[s][c] = v[s] + u[s];
#pragma unroll
          for (int s = 0; s < 3; ++s) {
            rs[s] += mo[s][c];
            cs[c][s] += mo[s + 3][c];
          }
          rmc += 1.f;
          cmc[c] += 1.f;
        } else {
#pragma unroll
          for (int s = 0; s < 6; ++s) mo[s][c] = zv[s];
        }
      }
      if (SAVE || moved_bits) {
#pragma unroll
        for (int s = 0; s < 6; ++s) {
          *(f4v*)(mt + s * TSZ + li * CB + 4 * cq) = mo[s];
          if constexpr (SAVE) *(f4v*)(xt + s * TSZ + li * CB + 4 * cq) = xo[s];
        }
      }
    }
    movedall |= moved_bits << (4 * k);
    // row partial: moved pairs' m plus (valid - moved) * z (TW: moved
    // pairs' m, with their number as the weight); the DPP sums are skipped
    // when no pair of the row's wavefront moved (they would add zeros)
    const bool row_moved = __ballot(moved_bits != 0) != 0;
    wave_moved |= row_moved;
    const int ei = I * RB + li;
    const int lo = ei + 1 > J * CB ? ei + 1 : J * CB;
    const int hi = b.E < J * CB + CB ? b.E : J * CB + CB;
    float cnt = (float)(hi > lo ? hi - lo : 0);
    float ms[3] = {0.f, 0.f, 0.f};
    if (row_moved) {
#pragma unroll
      for (int s = 0; s < 3; ++s) ms[s] = admmi::row16_sum(rs[s]);
      cnt -= admmi::row16_sum(rmc);
    }
    if (drow[k] >= 0) {
      const float m = cq == 0 ? ms[0] : (cq == 1 ? ms[1] : ms[2]);
      if constexpr (TW) {
        const float vc = (float)(hi > lo ? hi - lo : 0);
        a.pool[drow[k]] = m;
        a.wc[drow[k]] = vc - cnt;
      } else {
        a.pool[drow[k]] = fmaf(cnt, erow[0][li * 3 + (cq < 3 ? cq : 0)], m);
      }
    }
  }
  *flagp = (uint16_t)((SAVE && !TW) ? 0xFFFFu : movedall);
  // column partials
  if (wave_moved && lane == 0) any5 = 1;
  __syncthreads();
  float ms = 0.f, mcnt = 0.f;
  if (any5) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      float v = cmc[c];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      cmc[c] = v;
    }
    if (rg == 0) {
#pragma unroll
      for (int c = 0; c < 4; ++c) cnt5[w][4 * cq + c] = cmc[c];
    }
    ms = pair_colsum(cs, cacc5, w, rg, cq, t);
    if (t < CB * 3) {
      const int col = t / 3;
      mcnt = cnt5[0][col];
#pragma unroll
      for (int q = 1; q < NT / 64; ++q) mcnt += cnt5[q][col];
    }
  }
  if (dcol >= 0) {
    const int ej = J * CB + t / 3;
    const int rows = ej < b.E ? (ej - I * RB < RB ? ej - I * RB : RB) : 0;
    const float cnt = (float)(rows > 0 ? rows : 0) - mcnt;
    if constexpr (TW) {
      a.pool[dcol] = ms;
      a.wc[dcol] = mcnt;
    } else {
      a.pool[dcol] = fmaf(cnt, ecol[0][t], ms);
    }
  }
}

// ---------------------------------------------------------------------------
// Hinge factor C max(0, 1 - y(w.a + b)) over scalar edges (w_1..w_d, b).
// Parameters SoA [d+3][nfp]: y*a_1..y*a_d, y, C, rho/(|a|^2+1).
// UNIF: every factor shares the variable list (z offsets [d+1]); each
// workgroup of 256 factors emits column partials [tile][d+1].
// Otherwise z offsets are per edge [d+1][nfp] and m itself is summed.
// MARGIN (App. C, one-point margin, sign-corrected): the same projection
// onto y(w.x + b) + xi >= 1 with the slack xi as slot d+1, no upper bound
// (C = +inf) and rho/(|x|^2+2) as the last parameter.
// ---------------------------------------------------------------------------
template <typename T, bool A1, int MODE, bool UNIF, int DM>
__device__ __forceinline__ void xpass_hinge(const XArgs<T>& a, const BucketDesc& b, int blk) {
  __shared__ T wsum[NT / 64][DM + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int d = b.d;
  const int64_t f = (int64_t)blk * NT + t;
  const bool valid = f < b.n;
  const int64_t ff = valid ? f : 0;
  const int64_t nfp = b.nfp;
  const int32_t* zo = a.idx + b.idx_off;
  const T* P = a.par + b.par_off;
  T* M = a.pool + b.m_off;
  T* X = a.pool + b.x_off;
  T nv[DM], uv[DM], ya[DM];
  T dot = T(0);
  T rmax = T(0);
#pragma unroll
  for (int k = 0; k < DM; ++k) {
    if (k < d) {
      const T zk = UNIF ? a.z[zo[k]] : a.z[zo[k * nfp + ff]];
      const T mk = M[k * nfp + ff];
      T xo = T(0);
      if constexpr (!A1 || MODE == PM_RESID) xo = X[k * nfp + ff];
      if constexpr (MODE == PM_RESID) {
        if (valid) rmax = tmax(rmax, tabs(xo - zk));
      } else {
        state_un<T, A1>(mk, xo, zk, (T)b.alpha, uv[k], nv[k]);
        ya[k] = P[k * nfp + ff];
        dot += nv[k] * ya[k];
      }
    }
  }
  const T zb = UNIF ? a.z[zo[d]] : a.z[zo[d * nfp + ff]];
  const T mb = M[d * nfp + ff];
  T xob = T(0);
  if constexpr (!A1 || MODE == PM_RESID) xob = X[d * nfp + ff];
  const bool margin = !UNIF && b.kind == KD_MARGIN;
  T zs = T(0), ms = T(0), xos = T(0);
  if (margin) {
    zs = a.z[zo[(d + 1) * nfp + ff]];
    ms = M[(d + 1) * nfp + ff];
    if constexpr (!A1 || MODE == PM_RESID) xos = X[(d + 1) * nfp + ff];
  }
  if constexpr (MODE == PM_RESID) {
    if (valid) rmax = tmax(rmax, tabs(xob - zb));
    if (valid && margin) rmax = tmax(rmax, tabs(xos - zs));
    block_max_store(rmax, a.blockmax);
    return;
  } else {
    T ub, nb;
    state_un<T, A1>(mb, xob, zb, (T)b.alpha, ub, nb);
    const T y = P[d * nfp + ff], C = P[(d + 1) * nfp + ff], iD = P[(d + 2) * nfp + ff];
    dot += y * nb;
    T us = T(0), ns = T(0);
    if (margin) {
      state_un<T, A1>(ms, xos, zs, (T)b.alpha, us, ns);
      dot += ns;
    }
    const T tau = tmin(C, tmax(T(0), (T(1) - dot) * iD));
    const T st = tau * (T)b.irho;
    const T xb = nb + st * y;
    const T mnb = xb + ub;
    const bool shared_b = !UNIF && b.ub;
    if (valid) {
      M[d * nfp + ff] = mnb;
      if constexpr (!A1 || MODE == PM_SAVE) X[d * nfp + ff] = xb;
      if constexpr (!UNIF) {
        if (!shared_b) a.pool[a.idx[b.dst_off + d * nfp + ff]] = mnb;
      }
      if (margin) {
        const T xs = ns + st;
        M[(d + 1) * nfp + ff] = xs + us;
        if constexpr (!A1 || MODE == PM_SAVE) X[(d + 1) * nfp + ff] = xs;
        a.pool[a.idx[b.dst_off + (d + 1) * nfp + ff]] = xs + us;
      }
    }
#pragma unroll
    for (int k = 0; k < DM; ++k) {
      if (k < d) {
        const T xk = nv[k] + st * ya[k];
        const T mk = xk + uv[k];
        if (valid) {
          M[k * nfp + ff] = mk;
          if constexpr (!A1 || MODE == PM_SAVE) X[k * nfp + ff] = xk;
          if constexpr (!UNIF) a.pool[a.idx[b.dst_off + k * nfp + ff]] = mk;
        }
        if constexpr (UNIF) {
          const T s = admmi::wave_sum(valid ? mk : T(0));
          if (lane == 0) wsum[w][k] = s;
        }
      }
    }
    if (shared_b) {
      // the shared b edge: this workgroup's sum of m in a fixed order
      const T sb = admmi::wave_sum(valid ? mnb : T(0));
      if (lane == 0) wsum[w][0] = sb;
      __syncthreads();
      if (t == 0) {
        T acc = wsum[0][0];
#pragma unroll
        for (int q = 1; q < NT / 64; ++q) acc += wsum[q][0];
        a.pool[a.idx[b.dst_off + d * nfp + blk]] = acc;
      }
    }
    if constexpr (UNIF) {
      const T s = admmi::wave_sum(valid ? mnb : T(0));
      if (lane == 0) wsum[w][d] = s;
      __syncthreads();
      if (t <= d) {
        T acc = wsum[0][t];
#pragma unroll
        for (int q = 1; q < NT / 64; ++q) acc += wsum[q][t];
        a.pool[a.idx[b.dst_off + (int64_t)blk * (d + 1) + t]] = acc;
      }
    }
  }
}

// Hinge factors sharing one variable list with d <= 32 (the SVM): two lanes
// per factor, NT / 2 factors per workgroup, so twice as many wavefronts
// keep loads in flight.  Lane h of a pair takes components [h dh, (h+1) dh)
// (dh = ceil(d / 2)) and lane 1 also the b edge; both lanes form the same
// dot product (partial sums exchanged, added in the same order) and step.
// Every component's m is summed over the workgroup's factors: over the
// lanes of one parity of a wavefront (xor butterfly over lane bits 1..5),
// then over the four wavefronts in order.
template <typename T>
__device__ __forceinline__ T sum_parity_row(T v);

// Sum over the lanes of one parity within each 16-lane row (lane bits 1..3),
// DPP only; every lane returns its row's sum for its parity.
template <>
__device__ __forceinline__ float sum_parity_row<float>(float v) {
  v += ADMM_DPP(v, 0x4E, 0xF);    // quad_perm [2,3,0,1]: lanes i, i ^ 2
  v += ADMM_DPP(v, 0x124, 0xF);   // row_ror:4
  v += ADMM_DPP(v, 0x128, 0xF);   // row_ror:8
  return v;
}

template <>
__device__ __forceinline__ double sum_parity_row<double>(double v) {
#pragma unroll
  for (int o = 2; o < 16; o <<= 1) v += __shfl_xor(v, o, 16);
  return v;
}

// LDS of the shared-variable hinge paths, one allocation per precision
// whatever the register width they are instantiated for.
template <typename T>
struct HingeSmem {
  T wsum[NT / 16][33];   // per 16-lane row (or per wavefront), per component
  T zsh[33];             // z of the bucket's d + 1 variables
};
template <typename T>
__device__ __forceinline__ HingeSmem<T>& hinge_smem() {
  __shared__ HingeSmem<T> sm;
  return sm;
}

template <typename T, bool A1, int MODE, int DH>
__device__ __forceinline__ void xpass_hinge2(const XArgs<T>& a, const BucketDesc& b, int blk) {
  constexpr int FPB = NT / 2;
  auto& wsum2 = hinge_smem<T>().wsum;
  auto& zsh = hinge_smem<T>().zsh;
  const int t = threadIdx.x, lane = t & 63, h = t & 1, row = t >> 4;
  const int d = b.d, dh = (d + 1) / 2;
  const int64_t f = (int64_t)blk * FPB + (t >> 1);
  const bool valid = f < b.n;
  const int64_t ff = valid ? f : 0;
  const int64_t nfp = b.nfp;
  const int32_t* zo = a.idx + b.idx_off;
  const T* P = a.par + b.par_off;
  T* M = a.pool + b.m_off;
  T* X = a.pool + b.x_off;
  const T alpha = (T)b.alpha;
  const int k0 = h ? dh : 0, k1 = h ? d : dh;
  if (t <= d) zsh[t] = a.z[zo[t]];
  // every load of the factor first (a valid component index everywhere,
  // k0 <= d, so no load sits behind a branch), then the arithmetic
  T mv[DH], pv[DH], xv[DH];
#pragma unroll
  for (int i = 0; i < DH; ++i) {
    const int kc = k0 + i < k1 ? k0 + i : k0;
    mv[i] = M[kc * nfp + ff];
    pv[i] = MODE == PM_RESID ? T(0) : P[kc * nfp + ff];
    xv[i] = (!A1 || MODE == PM_RESID) ? X[kc * nfp + ff] : T(0);
  }
  const T mb = M[d * nfp + ff];
  const T xob = (!A1 || MODE == PM_RESID) ? X[d * nfp + ff] : T(0);
  T y = T(0), C = T(0), iD = T(0);
  if constexpr (MODE != PM_RESID) {
    y = P[d * nfp + ff];
    C = P[(d + 1) * nfp + ff];
    iD = P[(d + 2) * nfp + ff];
  }
  __syncthreads();
  const T zb = zsh[d];
  if constexpr (MODE == PM_RESID) {
    T rmax = T(0);
#pragma unroll
    for (int i = 0; i < DH; ++i) {
      const int k = k0 + i;
      if (valid && k < k1) rmax = tmax(rmax, tabs(xv[i] - zsh[k]));
    }
    if (valid && h) rmax = tmax(rmax, tabs(xob - zb));
    block_max_store(rmax, a.blockmax);
    return;
  } else {
    T uv[DH], nv[DH];
    T dot = T(0);
#pragma unroll
    for (int i = 0; i < DH; ++i) {
      const int k = k0 + i;
      const bool on = k < k1;
      state_un<T, A1>(mv[i], xv[i], zsh[on ? k : k0], alpha, uv[i], nv[i]);
      if (on) dot += nv[i] * pv[i];
    }
    T ub = T(0), nb = T(0);
    state_un<T, A1>(mb, xob, zb, alpha, ub, nb);
    if (!h) ub = nb = T(0);
    // both lanes: (even partial + odd partial) + y nb, the same bits in each
    const T other = __shfl_xor(dot, 1, 64);
    const T nbb = __shfl_xor(nb, 1, 64);
    const T full = (h ? other + dot : dot + other) + y * (h ? nb : nbb);
    const T tau = tmin(C, tmax(T(0), (T(1) - full) * iD));
    const T st = tau * (T)b.irho;
    T mnb = T(0);
    if (h) {
      const T xb = nb + st * y;
      mnb = xb + ub;
      if (valid) {
        M[d * nfp + ff] = mnb;
        if constexpr (!A1 || MODE == PM_SAVE) X[d * nfp + ff] = xb;
      }
    }
#pragma unroll
    for (int i = 0; i < DH; ++i) {   // i < dh is uniform: every lane takes part
      if (i >= dh) break;
      const int k = k0 + i;
      const bool on = k < k1;
      const T xk = nv[i] + st * pv[i];
      const T mn = xk + uv[i];
      if (valid && on) {
        M[k * nfp + ff] = mn;
        if constexpr (!A1 || MODE == PM_SAVE) X[k * nfp + ff] = xk;
      }
      const T s = sum_parity_row<T>((valid && on) ? mn : T(0));
      if ((lane & 15) < 2 && on) wsum2[row][k] = s;
    }
    {
      const T s = sum_parity_row<T>((valid && h) ? mnb : T(0));
      if ((lane & 15) == 1) wsum2[row][d] = s;
    }
    __syncthreads();
    if (t <= d) {
      T acc = wsum2[0][t];
#pragma unroll
      for (int q = 1; q < NT / 16; ++q) acc += wsum2[q][t];
      a.pool[a.idx[b.dst_off + (int64_t)blk * (d + 1) + t]] = acc;
    }
  }
}

// Shared-variable hinge with d < 32, FP32 and alpha = 1: each group of
// four lanes takes four consecutive factors, so that every load and store
// of a lane is 16 bytes (four factors' values of one edge).  Lane q of a
// group takes the edges [q DQ, (q + 1) DQ) of the d + 1 (the b edge last,
// its parameter y); its partial dot products of the four factors are added
// over the group in a fixed order, so all four lanes hold the same bits.
// The edges' m are summed over the workgroup's factors: over a lane's four
// factors, over the lanes of the same q in each 16-lane row (DPP), across
// the rows, then across the wavefronts in order.  NT factors per workgroup.
__device__ __forceinline__ float quad_sum4(float v) {
  // (v0 + v1) + (v2 + v3) of the group's four lanes, the same in each
  const float v0 = ADMM_DPP(v, 0x00, 0xF), v1 = ADMM_DPP(v, 0x55, 0xF);
  const float v2 = ADMM_DPP(v, 0xAA, 0xF), v3 = ADMM_DPP(v, 0xFF, 0xF);
  return (v0 + v1) + (v2 + v3);
}

template <bool A1, int MODE, int DQ>
__device__ __forceinline__ void xpass_hinge4(const XArgs<float>& a, const BucketDesc& b, int blk) {
  auto& wsum4 = hinge_smem<float>().wsum;   // rows 0 .. NT / 64 - 1 used
  auto& zsh4 = hinge_smem<float>().zsh;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, q = t & 3;
  const int d = b.d;
  const int64_t f0 = (int64_t)blk * NT + 4 * (t >> 2);   // the group's first factor
  const int64_t nfp = b.nfp;
  const int32_t* zo = a.idx + b.idx_off;
  const float* P = a.par + b.par_off;
  float* M = a.pool + b.m_off;
  float* X = a.pool + b.x_off;
  const int k0 = q * DQ;
  if (t <= d) zsh4[t] = a.z[zo[t]];
  // loads first: the lane's edges (an edge index past d reads edge d) and
  // the four factors' y, C and rho / (|a|^2 + 1)
  f4v mv[DQ], pv[DQ];
#pragma unroll
  for (int i = 0; i < DQ; ++i) {
    const int k = k0 + i <= d ? k0 + i : d;
    if constexpr (MODE == PM_RESID) {
      mv[i] = *(const f4v*)(X + k * nfp + f0);
    } else {
      mv[i] = *(const f4v*)(M + k * nfp + f0);
      pv[i] = *(const f4v*)(P + k * nfp + f0);
    }
  }
  f4v C4 = {0.f, 0.f, 0.f, 0.f}, iD4 = C4;
  if constexpr (MODE != PM_RESID) {
    C4 = *(const f4v*)(P + (d + 1) * nfp + f0);
    iD4 = *(const f4v*)(P + (d + 2) * nfp + f0);
  }
  __syncthreads();
  bool valid[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) valid[j] = f0 + j < b.n;
  if constexpr (MODE == PM_RESID) {
    float rmax = 0.f;
#pragma unroll
    for (int i = 0; i < DQ; ++i) {
      const int k = k0 + i;
      if (k <= d) {
        const float zk = zsh4[k];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (valid[j]) rmax = tmax(rmax, tabs(mv[i][j] - zk));
      }
    }
    block_max_store(rmax, a.blockmax);
    return;
  } else {
    // u = m - z, n = z - u; partial dot products of the lane's edges
    f4v dot = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < DQ; ++i) {
      const int k = k0 + i;
      const float zk = zsh4[k <= d ? k : d];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float u = mv[i][j] - zk;
        const float n = zk - u;
        mv[i][j] = u;          // mv holds u from here on
        pv[i][j] = k <= d ? pv[i][j] : 0.f;
        dot[j] += n * pv[i][j];
      }
    }
    f4v st;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float full = quad_sum4(dot[j]);
      const float tau = tmin(C4[j], tmax(0.f, (1.f - full) * iD4[j]));
      st[j] = tau * (float)b.irho;
    }
    // x = n + st p, m = x + u; the edges' sums over the workgroup's factors
#pragma unroll
    for (int i = 0; i < DQ; ++i) {
      const int k = k0 + i;
      const float zk = zsh4[k <= d ? k : d];
      f4v mn, xk;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float u = mv[i][j];
        xk[j] = (zk - u) + st[j] * pv[i][j];
        mn[j] = xk[j] + u;
      }
      if (k <= d) {
        *(f4v*)(M + k * nfp + f0) = mn;
        if constexpr (MODE == PM_SAVE) *(f4v*)(X + k * nfp + f0) = xk;
      }
      float sv = ((valid[0] ? mn[0] : 0.f) + (valid[1] ? mn[1] : 0.f)) +
                 ((valid[2] ? mn[2] : 0.f) + (valid[3] ? mn[3] : 0.f));
      sv += ADMM_DPP(sv, 0x124, 0xF);   // row_ror:4
      sv += ADMM_DPP(sv, 0x128, 0xF);   // row_ror:8
      sv += __shfl_xor(sv, 16, 64);
      sv += __shfl_xor(sv, 32, 64);
      if (lane < 4 && k <= d) wsum4[w][k] = sv;
    }
    __syncthreads();
    if (t <= d) {
      float acc = wsum4[0][t];
#pragma unroll
      for (int r = 1; r < NT / 64; ++r) acc += wsum4[r][t];
      a.pool[a.idx[b.dst_off + (int64_t)blk * (d + 1) + t]] = acc;
    }
  }
}

// Hinge and margin factors with d > 64 weight components (up to NT - 1):
// the same operator as xpass_hinge without register arrays.  A first sweep
// over the components forms the dot product s = y(n_w.a + n_b) (+ n_xi);
// once tau is known a second sweep reads each component's m, z and y a
// again and writes its outputs, in the same order as xpass_hinge.
template <typename T, bool A1, int MODE, bool UNIF>
__device__ __forceinline__ void xpass_hinge_wide(const XArgs<T>& a, const BucketDesc& b,
                                                 int blk) {
  __shared__ T wsw[NT / 64][NT];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int d = b.d;
  const int64_t f = (int64_t)blk * NT + t;
  const bool valid = f < b.n;
  const int64_t ff = valid ? f : 0;
  const int64_t nfp = b.nfp;
  const int32_t* zo = a.idx + b.idx_off;
  const T* P = a.par + b.par_off;
  T* M = a.pool + b.m_off;
  T* X = a.pool + b.x_off;
  const T alpha = (T)b.alpha;
  T dot = T(0), rmax = T(0);
  for (int k = 0; k < d; ++k) {
    const T zk = UNIF ? a.z[zo[k]] : a.z[zo[k * nfp + ff]];
    const T mk = M[k * nfp + ff];
    T xo = T(0);
    if constexpr (!A1 || MODE == PM_RESID) xo = X[k * nfp + ff];
    if constexpr (MODE == PM_RESID) {
      if (valid) rmax = tmax(rmax, tabs(xo - zk));
    } else {
      T uk, nk;
      state_un<T, A1>(mk, xo, zk, alpha, uk, nk);
      dot += nk * P[k * nfp + ff];
    }
  }
  const T zb = UNIF ? a.z[zo[d]] : a.z[zo[d * nfp + ff]];
  const T mb = M[d * nfp + ff];
  T xob = T(0);
  if constexpr (!A1 || MODE == PM_RESID) xob = X[d * nfp + ff];
  const bool margin = !UNIF && b.kind == KD_MARGIN;
  T zs = T(0), ms = T(0), xos = T(0);
  if (margin) {
    zs = a.z[zo[(d + 1) * nfp + ff]];
    ms = M[(d + 1) * nfp + ff];
    if constexpr (!A1 || MODE == PM_RESID) xos = X[(d + 1) * nfp + ff];
  }
  if constexpr (MODE == PM_RESID) {
    if (valid) rmax = tmax(rmax, tabs(xob - zb));
    if (valid && margin) rmax = tmax(rmax, tabs(xos - zs));
    block_max_store(rmax, a.blockmax);
    return;
  } else {
    T ub, nb;
    state_un<T, A1>(mb, xob, zb, alpha, ub, nb);
    const T y = P[d * nfp + ff], C = P[(d + 1) * nfp + ff], iD = P[(d + 2) * nfp + ff];
    dot += y * nb;
    T us = T(0), ns = T(0);
    if (margin) {
      state_un<T, A1>(ms, xos, zs, alpha, us, ns);
      dot += ns;
    }
    const T tau = tmin(C, tmax(T(0), (T(1) - dot) * iD));
    const T st = tau * (T)b.irho;
    const T xb = nb + st * y;
    const T mnb = xb + ub;
    const bool shared_b = !UNIF && b.ub;
    if (valid) {
      M[d * nfp + ff] = mnb;
      if constexpr (!A1 || MODE == PM_SAVE) X[d * nfp + ff] = xb;
      if constexpr (!UNIF) {
        if (!shared_b) a.pool[a.idx[b.dst_off + d * nfp + ff]] = mnb;
      }
      if (margin) {
        const T xs = ns + st;
        M[(d + 1) * nfp + ff] = xs + us;
        if constexpr (!A1 || MODE == PM_SAVE) X[(d + 1) * nfp + ff] = xs;
        a.pool[a.idx[b.dst_off + (d + 1) * nfp + ff]] = xs + us;
      }
    }
    for (int k = 0; k < d; ++k) {
      const T zk = UNIF ? a.z[zo[k]] : a.z[zo[k * nfp + ff]];
      const T mk = M[k * nfp + ff];
      T xo = T(0);
      if constexpr (!A1) xo = X[k * nfp + ff];
      T uk, nk;
      state_un<T, A1>(mk, xo, zk, alpha, uk, nk);
      const T xk = nk + st * P[k * nfp + ff];
      const T mn = xk + uk;
      if (valid) {
        M[k * nfp + ff] = mn;
        if constexpr (!A1 || MODE == PM_SAVE) X[k * nfp + ff] = xk;
        if constexpr (!UNIF) a.pool[a.idx[b.dst_off + k * nfp + ff]] = mn;
      }
      if constexpr (UNIF) {
        const T s = admmi::wave_sum(valid ? mn : T(0));
        if (lane == 0) wsw[w][k] = s;
      }
    }
    if (shared_b) {
      const T sb = admmi::wave_sum(valid ? mnb : T(0));
      if (lane == 0) wsw[w][0] = sb;
      __syncthreads();
      if (t == 0) {
        T acc = wsw[0][0];
#pragma unroll
        for (int q = 1; q < NT / 64; ++q) acc += wsw[q][0];
        a.pool[a.idx[b.dst_off + d * nfp + blk]] = acc;
      }
    }
    if constexpr (UNIF) {
      const T s = admmi::wave_sum(valid ? mnb : T(0));
      if (lane == 0) wsw[w][d] = s;
      __syncthreads();
      if (t <= d) {
        T acc = wsw[0][t];
#pragma unroll
        for (int q = 1; q < NT / 64; ++q) acc += wsw[q][t];
        a.pool[a.idx[b.dst_off + (int64_t)blk * (d + 1) + t]] = acc;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Separable operators, one thread per scalar slot.  Params [2][nfp]:
//   RADIUS  x = max(0, p0 n), p0 = rho/(rho - gamma)
//   QUAD    x = p0 n,         p0 = rho/(rho + q_k)
//   L2      x = p0 n,         p0 = rho/(rho + lambda)
//   BOX     x = min(p1, max(p0, n)), (p0, p1) = (lo, hi)
//   MINERR  x = max(0, n - p0),  p0 = lambda/rho  (App. C, minimal error)
// ---------------------------------------------------------------------------
template <typename T, bool A1, int MODE>
__device__ __forceinline__ void xpass_slot(const XArgs<T>& a, const BucketDesc& b, int blk) {
  const int64_t s = (int64_t)blk * NT + threadIdx.x;
  T rmax = T(0);
  if (s < b.n) {
    const int32_t* zi = a.idx + b.idx_off;
    const T* P = a.par + b.par_off;
    T* M = a.pool + b.m_off;
    T* X = a.pool + b.x_off;
    const T zv = a.z[zi[s]];
    if constexpr (MODE == PM_RESID) {
      rmax = tabs(X[s] - zv);
    } else {
      T xo = T(0);
      if constexpr (!A1) xo = X[s];
      T u, n;
      state_un<T, A1>(M[s], xo, zv, (T)b.alpha, u, n);
      const T p0 = P[s];
      T x;
      if (b.kind == KD_BOX) {
        x = tmin(P[b.nfp + s], tmax(p0, n));
      } else if (b.kind == KD_RADIUS) {
        x = tmax(T(0), p0 * n);
      } else if (b.kind == KD_MINERR) {
        x = tmax(T(0), n - p0);
      } else {
        x = p0 * n;
      }
      M[s] = x + u;
      if constexpr (!A1 || MODE == PM_SAVE) X[s] = x;
      a.pool[a.idx[b.dst_off + s]] = x + u;
    }
  }
  if constexpr (MODE == PM_RESID) block_max_store(rmax, a.blockmax);
}

// ---------------------------------------------------------------------------
// General factor buckets, one thread per factor, explicit per-edge z offsets
// [edge][nfp].  Register arrays have compile-time sizes so nothing spills.
// ---------------------------------------------------------------------------

// Gather u and n for a factor whose edge e has dimension dims[e].
template <typename T, bool A1, int MODE, int NSL>
__device__ __forceinline__ void gen_gather(const XArgs<T>& a, const BucketDesc& b, int64_t f,
                                           const int (&dims)[4], int arity, T (&u)[NSL],
                                           T (&v)[NSL], T& rmax) {
  const int64_t nfp = b.nfp;
  const int32_t* zo = a.idx + b.idx_off;
  const T* M = a.pool + b.m_off;
  const T* X = a.pool + b.x_off;
  int s = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (e < arity) {
      const int z0 = zo[e * nfp + f];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        if (c < dims[e]) {
          const T zv = a.z[z0 + c];
          const T mv = M[s * nfp + f];
          T xo = T(0);
          if constexpr (!A1 || MODE == PM_RESID) xo = X[s * nfp + f];
          if constexpr (MODE == PM_RESID) {
            rmax = tmax(rmax, tabs(xo - zv));
          } else {
            state_un<T, A1>(mv, xo, zv, (T)b.alpha, u[s], v[s]);
          }
          ++s;
        }
      }
    }
  }
}

template <typename T, bool A1, int MODE, int NSL>
__device__ __forceinline__ void gen_store(const XArgs<T>& a, const BucketDesc& b, int64_t f,
                                          const T (&u)[NSL], const T (&v)[NSL]) {
  T* M = a.pool + b.m_off;
  T* X = a.pool + b.x_off;
  const int32_t* dst = a.idx + b.dst_off;
#pragma unroll
  for (int s = 0; s < NSL; ++s) {
    const T mn = v[s] + u[s];
    M[s * b.nfp + f] = mn;
    if constexpr (!A1 || MODE == PM_SAVE) X[s * b.nfp + f] = v[s];
    a.pool[dst[s * b.nfp + f]] = mn;
  }
}

// Three-weight variant of a non-overlap (NS = 6) or wall (NS = 3) factor
// on arbitrary variables, alpha = 1.  The factor's dual is m - z when it
// sent weight rho in the last iteration and 0 when it sent weight 0 (its
// constraint was inactive); edges of variables no factor weighted are
// received with weight 0.  Each contribution goes out with its weight (m
// and 1 when the constraint is active, 0 and 0 when not).  The residual
// pass stores z as the m of inactive factors (dual 0) and marks them
// active again, so the stored state is explicit between runs.
template <typename T, int MODE, int NS>
__device__ __forceinline__ void geom_tw(const XArgs<T>& a, const BucketDesc& b, int64_t f,
                                        const int (&dims)[4], int arity, T& rmax) {
  const int64_t nfp = b.nfp;
  const int32_t* zo = a.idx + b.idx_off;
  T* M = a.pool + b.m_off;
  T* X = a.pool + b.x_off;
  const int32_t* dst = a.idx + b.dst_off;
  uint8_t* act = a.twb + b.twb_off + f;
  const bool was = *act != 0;
  T z[NS], u[NS], v[NS];
  unsigned fr = 0;
  int s = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (e < arity) {
      const int z0 = zo[e * nfp + f];
      if (a.zfree[z0]) fr |= 1u << e;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        if (c < dims[e]) {
          z[s] = a.z[z0 + c];
          ++s;
        }
      }
    }
  }
  if constexpr (MODE == PM_RESID) {
#pragma unroll
    for (int q = 0; q < NS; ++q) rmax = tmax(rmax, tabs(X[q * nfp + f] - z[q]));
    if (!was) {
#pragma unroll
      for (int q = 0; q < NS; ++q) M[q * nfp + f] = z[q];
      *act = 1;
    }
    return;
  } else {
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      u[q] = was ? M[q * nfp + f] - z[q] : T(0);
      v[q] = z[q] - u[q];
    }
    bool moved;
    if constexpr (NS == 6) {
      moved = fr ? prox_nonoverlap_free(v, fr) : prox_nonoverlap(v);
    } else {
      const T* P = a.par + b.par_off;
      // fr bit 0: the centre edge, bit 1: the radius edge
      if (fr)
        moved = prox_wall_free(v, P[f], P[nfp + f], P[2 * nfp + f], fr);
      else
        moved = prox_wall(v, P[f], P[nfp + f], P[2 * nfp + f], P[3 * nfp + f]);
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const T mn = v[q] + u[q];
      M[q * nfp + f] = mn;
      if constexpr (MODE == PM_SAVE) X[q * nfp + f] = v[q];
      a.pool[dst[q * nfp + f]] = moved ? mn : T(0);
      a.wc[dst[q * nfp + f]] = moved ? T(1) : T(0);
    }
    *act = moved ? 1 : 0;
  }
}

// Non-overlap and wall factors on arbitrary variables, and equality
// factors split into scalar component pairs (App. C: with equal weights
// both copies take the mean of the pair).
template <typename T, bool A1, int MODE, bool TW = false>
__device__ __forceinline__ void xpass_geom(const XArgs<T>& a, const BucketDesc& b, int blk) {
  const int64_t f = (int64_t)blk * NT + threadIdx.x;
  T rmax = T(0);
  if (TW && f < b.n && b.kind != KD_EQUAL) {
    if (b.kind == KD_NONOVERLAP) {
      const int dims[4] = {2, 1, 2, 1};
      geom_tw<T, MODE, 6>(a, b, f, dims, 4, rmax);
    } else {
      const int dims[4] = {2, 1, 0, 0};
      geom_tw<T, MODE, 3>(a, b, f, dims, 2, rmax);
    }
  } else if (f < b.n) {
    if (b.kind == KD_EQUAL) {
      const int dims[4] = {1, 1, 0, 0};
      T u[2], v[2];
      gen_gather<T, A1, MODE, 2>(a, b, f, dims, 2, u, v, rmax);
      if constexpr (MODE != PM_RESID) {
        const T mean = (v[0] + v[1]) * T(0.5);
        v[0] = mean;
        v[1] = mean;
        gen_store<T, A1, MODE, 2>(a, b, f, u, v);
      }
    } else if (b.kind == KD_NONOVERLAP) {
      const int dims[4] = {2, 1, 2, 1};
      T u[6], v[6];
      gen_gather<T, A1, MODE, 6>(a, b, f, dims, 4, u, v, rmax);
      if constexpr (MODE != PM_RESID) {
        prox_nonoverlap(v);
        gen_store<T, A1, MODE, 6>(a, b, f, u, v);
      }
    } else {
      const int dims[4] = {2, 1, 0, 0};
      T u[3], v[3];
      gen_gather<T, A1, MODE, 3>(a, b, f, dims, 2, u, v, rmax);
      if constexpr (MODE != PM_RESID) {
        const T* P = a.par + b.par_off;
        const int64_t nfp = b.nfp;
        prox_wall(v, P[f], P[nfp + f], P[2 * nfp + f], P[3 * nfp + f]);
        gen_store<T, A1, MODE, 3>(a, b, f, u, v);
      }
    }
  }
  if constexpr (MODE == PM_RESID) block_max_store(rmax, a.blockmax);
}

// Linear-dynamics projections, one thread per factor.
//   LINDYN  edges (x, u, x'), params [M = [A B] (n x (n+m)), S = (I+MM^T)^-1]:
//           v = S (M a - x'), a <- a - M^T v, x' <- x' + v, a = (x, u).
//   LINDYN0 edges (u, x'), params [B (n x m), S0 = (I+BB^T)^-1, c = A x0]:
//           v = S0 (B u + c - x'), u <- u - B^T v, x' <- x' + v.
// Slot s of the factor is stored at [s][nfp]; a occupies slots [0, k), x'
// slots [k, k+n).
template <typename T, bool A1, int MODE>
__device__ __forceinline__ void xpass_lindyn(const XArgs<T>& a, const BucketDesc& b, int blk) {
  constexpr int MK = MAXN + MAXM;
  const int64_t f = (int64_t)blk * NT + threadIdx.x;
  T rmax = T(0);
  if (f < b.n) {
    const int64_t nfp = b.nfp;
    const int32_t* zo = a.idx + b.idx_off;
    T* M = a.pool + b.m_off;
    T* X = a.pool + b.x_off;
    const bool first = (b.kind == KD_LINDYN0);
    const int n = b.nn, m = b.mm;
    const int k = first ? m : n + m;
    // z offset of slot s: edges (x, u, x') or (u, x')
    const int zx = first ? 0 : zo[f];
    const int zu = first ? zo[f] : zo[nfp + f];
    const int zx1 = first ? zo[nfp + f] : zo[2 * nfp + f];
    T ua[MK], va[MK], ub[MAXN], vb[MAXN];
#pragma unroll
    for (int j = 0; j < MK; ++j) {
      if (j < k) {
        const int zi = first ? (zu + j) : (j < n ? zx + j : zu + (j - n));
        const T zv = a.z[zi];
        T xo = T(0);
        if constexpr (!A1 || MODE == PM_RESID) xo = X[j * nfp + f];
        if constexpr (MODE == PM_RESID) {
          rmax = tmax(rmax, tabs(xo - zv));
        } else {
          state_un<T, A1>(M[j * nfp + f], xo, zv, (T)b.alpha, ua[j], va[j]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < MAXN; ++r) {
      if (r < n) {
        const T zv = a.z[zx1 + r];
        T xo = T(0);
        if constexpr (!A1 || MODE == PM_RESID) xo = X[(k + r) * nfp + f];
        if constexpr (MODE == PM_RESID) {
          rmax = tmax(rmax, tabs(xo - zv));
        } else {
          state_un<T, A1>(M[(k + r) * nfp + f], xo, zv, (T)b.alpha, ub[r], vb[r]);
        }
      }
    }
    if constexpr (MODE != PM_RESID) {
      const T* P = a.par + b.par_off + zo[b.arity * nfp + f];
      const T* Mx = P;
      const T* S = P + n * k;
      const T* cc = S + n * n;
      T wv[MAXN], vv[MAXN];
#pragma unroll
      for (int r = 0; r < MAXN; ++r) {
        if (r < n) {
          T s = first ? (cc[r] - vb[r]) : -vb[r];
#pragma unroll
          for (int j = 0; j < MK; ++j)
            if (j < k) s += Mx[r * k + j] * va[j];
          wv[r] = s;
        }
      }
#pragma unroll
      for (int r = 0; r < MAXN; ++r) {
        if (r < n) {
          T s = T(0);
#pragma unroll
          for (int j = 0; j < MAXN; ++j)
            if (j < n) s += S[r * n + j] * wv[j];
          vv[r] = s;
        }
      }
#pragma unroll
      for (int j = 0; j < MK; ++j) {
        if (j < k) {
          T s = T(0);
#pragma unroll
          for (int r = 0; r < MAXN; ++r)
            if (r < n) s += Mx[r * k + j] * vv[r];
          va[j] -= s;
          M[j * nfp + f] = va[j] + ua[j];
          if constexpr (!A1 || MODE == PM_SAVE) X[j * nfp + f] = va[j];
          a.pool[a.idx[b.dst_off + j * nfp + f]] = va[j] + ua[j];
        }
      }
#pragma unroll
      for (int r = 0; r < MAXN; ++r) {
        if (r < n) {
          vb[r] += vv[r];
          M[(k + r) * nfp + f] = vb[r] + ub[r];
          if constexpr (!A1 || MODE == PM_SAVE) X[(k + r) * nfp + f] = vb[r];
          a.pool[a.idx[b.dst_off + (k + r) * nfp + f]] = vb[r] + ub[r];
        }
      }
    }
  }
  if constexpr (MODE == PM_RESID) block_max_store(rmax, a.blockmax);
}

// Feature sets compiled into one x-pass kernel; the host picks the
// smallest set that covers a graph's buckets, so the register budget of a
// launch is that of the paths it can take.
enum Features : int {
  FT_PAIR = 1,     // dense pair tiles
  FT_UHINGE = 2,   // shared-variable hinge, d <= 32
  FT_GEN = 4,      // non-overlap/wall on arbitrary variables, separable slots
  FT_WIDE = 8,     // general hinge and margin with d <= 32
  FT_PAIRSP = 16,  // dense pair tiles with sparse pair state
  FT_XWIDE = 32,   // hinge and margin with 64 < d < NT (two sweeps, no register arrays)
  FT_TWA = 64,     // three-weight variant (packing graphs: pair tiles, constraints, slots)
  FT_W64 = 128,    // hinge (shared-variable or general) with 32 < d <= 64
  FT_LINDYN = 256, // linear-dynamics projections
};
constexpr int FS_PAIR = FT_PAIR | FT_GEN;
constexpr int FS_PAIRSP = FT_PAIRSP | FT_GEN;
constexpr int FS_HINGE = FT_UHINGE | FT_GEN;
constexpr int FS_WIDE = FT_GEN | FT_WIDE;
constexpr int FS_DYN = FT_GEN | FT_LINDYN;
constexpr int FS_ALL = FT_PAIR | FT_UHINGE | FT_GEN | FT_WIDE | FT_PAIRSP | FT_W64 | FT_LINDYN;
constexpr int FS_XW = FT_XWIDE | FT_GEN;
constexpr int FS_PAIRSP_TW = FT_PAIRSP | FT_GEN | FT_TWA;
constexpr int FS_GEN_TW = FT_GEN | FT_TWA;
constexpr int FS_ALLX = FS_ALL | FT_XWIDE;

// The bucket of x-pass block blk, from the table in memory.
template <typename T>
__device__ __forceinline__ BucketDesc find_bucket(const XArgs<T>& a, int blk) {
  int bi = 0;
  while (bi + 1 < a.nb && blk >= a.bt[bi].blk1) ++bi;
  return a.bt[bi];
}

// Bucket table passed in the kernel arguments when a graph has at most
// XB_INLINE buckets: a workgroup then finds its bucket in the argument
// segment, read together with the other arguments, instead of through two
// dependent loads from memory before its first data load.
constexpr int XB_INLINE = 8;
struct BTab {
  BucketDesc d[XB_INLINE];
};

// One x-pass workgroup's work; blk indexes the x-pass blocks of all
// buckets, b is the bucket that holds it.
template <typename T, bool A1, int MODE, int FS>
__device__ __forceinline__ void xpass_block(XArgs<T> a, int blk, const BucketDesc& b) {
  constexpr bool TW = (FS & FT_TWA) != 0;
  a.blockmax += blk;
  const int local = blk - b.blk0;
  if ((FS & (FT_PAIR | FT_PAIRSP)) && b.mode == BM_PAIR) {
    if constexpr (sizeof(T) == 4 && A1) {
      if constexpr ((FS & FT_PAIRSP) && MODE != PM_RESID) {
        if (b.sparse) {
          if (b.rb == 16)
            xpass_pair_sparse<MODE, 16, TW>(a, b, local);
          else if (b.rb == 32)
            xpass_pair_sparse<MODE, 32, TW>(a, b, local);
          else
            xpass_pair_sparse<MODE, 64, TW>(a, b, local);
          return;
        }
      }
      if constexpr ((FS & FT_PAIR) || MODE == PM_RESID) {
        if (b.rb == 16)
          xpass_pair_v4<MODE, 16, TW>(a, b, local);
        else if (b.rb == 32)
          xpass_pair_v4<MODE, 32, TW>(a, b, local);
        else
          xpass_pair_v4<MODE, 64, TW>(a, b, local);
      }
    } else {
      if (b.rb == 16)
        xpass_pair<T, A1, MODE, 16>(a, b, local);
      else if (b.rb == 32)
        xpass_pair<T, A1, MODE, 32>(a, b, local);
      else
        xpass_pair<T, A1, MODE, 64>(a, b, local);
    }
  } else if ((FS & (FT_UHINGE | FT_W64 | FT_XWIDE)) && b.mode == BM_UNIF_HINGE) {
    if ((FS & FT_UHINGE) && b.dmax == 32 && b.quad) {
      if constexpr (sizeof(T) == 4 && A1) {
        // four lanes per four factors, ceil((d + 1) / 4) <= 8 edges per lane
        const int dq = (b.d + 4) / 4;
        if (dq <= 2)
          xpass_hinge4<A1, MODE, 2>(a, b, local);
        else if (dq <= 4)
          xpass_hinge4<A1, MODE, 4>(a, b, local);
        else if (dq <= 6)
          xpass_hinge4<A1, MODE, 6>(a, b, local);
        else
          xpass_hinge4<A1, MODE, 8>(a, b, local);
      }
    } else if ((FS & FT_UHINGE) && b.dmax == 32) {
      // per lane ceil(d / 2) components, register arrays sized to the next
      // multiple of 4 (no loads of unused components)
      const int dh = (b.d + 1) / 2;
      if (dh <= 4)
        xpass_hinge2<T, A1, MODE, 4>(a, b, local);
      else if (dh <= 8)
        xpass_hinge2<T, A1, MODE, 8>(a, b, local);
      else if (dh <= 12)
        xpass_hinge2<T, A1, MODE, 12>(a, b, local);
      else
        xpass_hinge2<T, A1, MODE, 16>(a, b, local);
    }
    else if ((FS & FT_W64) && b.dmax == 64)
      xpass_hinge<T, A1, MODE, true, 64>(a, b, local);
    else if ((FS & FT_XWIDE) && b.dmax == 0)
      xpass_hinge_wide<T, A1, MODE, true>(a, b, local);
  } else if ((FS & FT_GEN) && b.mode == BM_GEN_SLOT) {
    xpass_slot<T, A1, MODE>(a, b, local);
  } else if ((FS & FT_GEN) && (b.kind == KD_NONOVERLAP || b.kind == KD_WALL || b.kind == KD_EQUAL)) {
    xpass_geom<T, A1, MODE, TW>(a, b, local);
  } else if ((FS & FT_XWIDE) && (b.kind == KD_HINGE || b.kind == KD_MARGIN) && b.dmax == 0) {
    xpass_hinge_wide<T, A1, MODE, false>(a, b, local);
  } else if ((FS & FT_W64) && (b.kind == KD_HINGE || b.kind == KD_MARGIN) && b.dmax == 64) {
    xpass_hinge<T, A1, MODE, false, 64>(a, b, local);
  } else if ((FS & FT_WIDE) && (b.kind == KD_HINGE || b.kind == KD_MARGIN)) {
    xpass_hinge<T, A1, MODE, false, 32>(a, b, local);
  } else if (FS & FT_LINDYN) {
    xpass_lindyn<T, A1, MODE>(a, b, local);
  }
}

template <typename T, bool A1, int MODE, int FS>
__global__ __launch_bounds__(NT) void xpass_kernel(XArgs<T> a, BTab tab) {
  const int blk = blockIdx.x;
  BucketDesc b;
  if (a.nb <= XB_INLINE) {
    int bi = 0;
    while (bi + 1 < a.nb && blk >= tab.d[bi].blk1) ++bi;
    b = tab.d[bi];
  } else {
    b = find_bucket(a, blk);
  }
  xpass_block<T, A1, MODE, FS>(a, blk, b);
}

// z_b = sum(contributions) / deg(b), contributions read from one contiguous
// range per scalar.  Blocks [0, n_b): one long list each (lanes stride the
// list, then wavefront DPP trees and the four wavefront sums in order);
// the next nb_w blocks: sixteen lists each, one 16-lane row per list;
// remaining blocks: one short list per lane, summed in order.
constexpr int ZSEG = 16;                  // lanes per medium list
constexpr int ZPB = NT / ZSEG;            // medium lists per block
constexpr int ZUN = 8;                    // loads per lane issued at once (medium lists)
constexpr int ZTU = 16;                   // loads per thread issued at once (transposed)

// Transposed lists (the scalars of pair-tile entities): contribution j of
// list k at t_base + j * n_t + k.  A block takes L = t_lpb consecutive
// lists and NT / L threads per list: thread q of a list sums slots
// j = q, q + NT/L, ... (loads coalesced across the L lists, the first ZTU
// issued together), and the per-thread sums are added in order of q.  TW:
// the weights written with the contributions are summed the same way
// (three-weight variant).
template <typename T, bool TW>
__device__ __forceinline__ void zpass_tlist(const ZArgs<T>& a, int blk, T& dmax) {
  __shared__ T zt[2][NT];
  const int L = a.t_lpb, nq = NT / L;
  const int kk = threadIdx.x & (L - 1), q = threadIdx.x / L;
  const int64_t k = (int64_t)blk * L + kk;
  const bool ok = k < a.n_t;
  // the list's z index and degree, read with the contributions (not after
  // the reduction's barrier)
  int zi = 0;
  T dg = T(1);
  if (ok && q == 0) {
    zi = a.var_t[k];
    if (!TW) dg = a.deg_t[k];
  }
  T num = T(0), den = T(0);
  if (ok) {
    const T* p = a.pool + a.t_base + k;
    const T* w = TW ? a.wc + a.t_base + k : (a.wz ? a.wz + a.t_base + k : nullptr);
    T v[ZTU], c[ZTU];
#pragma unroll
    for (int i = 0; i < ZTU; ++i) {
      const int j = q + nq * i;
      v[i] = T(0);
      c[i] = T(0);
      if (j < a.t_len) {
        v[i] = p[(int64_t)j * a.n_t];
        if (TW || w) c[i] = w[(int64_t)j * a.n_t];
      }
    }
#pragma unroll
    for (int i = 0; i < ZTU; ++i) {
      if (TW) {
        num += v[i];
        den += c[i];
      } else {
        num += w ? c[i] * v[i] : v[i];
      }
    }
    for (int j = q + nq * ZTU; j < a.t_len; j += nq) {
      const T vj = p[(int64_t)j * a.n_t];
      if (TW) {
        num += vj;
        den += w[(int64_t)j * a.n_t];
      } else {
        num += w ? w[(int64_t)j * a.n_t] * vj : vj;
      }
    }
  }
  zt[0][threadIdx.x] = num;
  zt[1][threadIdx.x] = den;
  __syncthreads();
  if (ok && q == 0) {
    T tn = zt[0][kk], td = zt[1][kk];
    for (int i = 1; i < nq; ++i) {
      tn += zt[0][i * L + kk];
      td += zt[1][i * L + kk];
    }
    T zn = a.zin[zi];
    if (TW) {
      if (td > T(0)) zn = tn / td;
      a.zfree[zi] = td > T(0) ? 0 : 1;
    } else {
      zn = tn / dg;
    }
    a.zout[zi] = zn;
    if (a.check) dmax = tabs(zn - a.zin[zi]) * ((!TW && a.rmz) ? a.rmz[zi] : T(1));
  }
}
// Three-weight variant: z_b = (sum of the contributions) / (sum of the
// weights written with them), over the same lists in the same order; when
// the weights sum to 0 no factor weighted b, z_b keeps its value and zfree
// marks b for the next x-update.
template <typename T>
__device__ __forceinline__ void zpass_block_tw(ZArgs<T> a, int blk) {
  __shared__ T zr2[2][NT / 64];
  T dmax = T(0);
  if (blk < a.nb_t) {
    zpass_tlist<T, true>(a, blk, dmax);
    if (a.check) block_max_store(dmax, a.blockmax + blk);
    return;
  }
  a.blockmax += a.nb_t;
  blk -= a.nb_t;
  auto finish = [&](int zi, T num, T den) {
    T zn = a.zin[zi];
    if (den > T(0)) zn = num / den;
    a.zout[zi] = zn;
    a.zfree[zi] = den > T(0) ? 0 : 1;
    if (a.check) dmax = tabs(zn - a.zin[zi]);
  };
  if (blk < a.n_b) {
    const int64_t o1 = a.rng_b[2 * blk + 1];
    T num = T(0), den = T(0);
    for (int64_t j = a.rng_b[2 * blk] + threadIdx.x; j < o1; j += NT) {
      num += a.pool[j];
      den += a.wc[j];
    }
    num = admmi::wave_sum(num);
    den = admmi::wave_sum(den);
    if ((threadIdx.x & 63) == 0) {
      zr2[0][threadIdx.x >> 6] = num;
      zr2[1][threadIdx.x >> 6] = den;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      T tn = zr2[0][0], td = zr2[1][0];
#pragma unroll
      for (int q = 1; q < NT / 64; ++q) {
        tn += zr2[0][q];
        td += zr2[1][q];
      }
      finish(a.var_b[blk], tn, td);
    }
  } else if (blk < a.n_b + a.nb_w) {
    const int sl = threadIdx.x & (ZSEG - 1);
    const int64_t k = (int64_t)(blk - a.n_b) * ZPB + (threadIdx.x / ZSEG);
    const bool ok = k < a.n_w;
    T num = T(0), den = T(0);
    if (ok) {
      int64_t j0, j1;
      if (a.w_stride) {
        j0 = a.w_base + k * a.w_stride;
        j1 = j0 + a.w_stride;
      } else {
        j0 = a.rng_w[2 * k];
        j1 = a.rng_w[2 * k + 1];
      }
      for (int64_t j = j0 + sl; j < j1; j += ZSEG) {
        num += a.pool[j];
        den += a.wc[j];
      }
    }
    num = admmi::row16_sum(num);
    den = admmi::row16_sum(den);
    if (ok && sl == 0) finish(a.var_w[k], num, den);
  } else {
    const int64_t k = (int64_t)(blk - a.n_b - a.nb_w) * NT + threadIdx.x;
    if (k < a.n_l) {
      const int64_t o = a.l_base + k * LANE_MAX;
      T num = a.pool[o], den = a.wc[o];
#pragma unroll
      for (int j = 1; j < LANE_MAX; ++j) {
        num += a.pool[o + j];
        den += a.wc[o + j];
      }
      finish(a.var_l[k], num, den);
    }
  }
  if (a.check) block_max_store(dmax, a.blockmax + blk);
}

template <typename T>
__device__ __forceinline__ void zpass_block(ZArgs<T> a, int blk) {
  if (a.wc) {
    zpass_block_tw(a, blk);
    return;
  }
  if (blk < a.nb_t) {
    T dt = T(0);
    zpass_tlist<T, false>(a, blk, dt);
    if (a.check) block_max_store(dt, a.blockmax + blk);
    return;
  }
  a.blockmax += a.nb_t;
  blk -= a.nb_t;
  __shared__ T zred[NT / 64];
  a.blockmax += blk;
  T dmax = T(0);
  if (blk < a.n_b) {
    const int64_t o1 = a.rng_b[2 * blk + 1];
    const int zi = a.var_b[blk];       // read before the reduction
    const T dg = a.deg_b[blk];
    T s = T(0);
    if (a.wz) {
      for (int64_t j = a.rng_b[2 * blk] + threadIdx.x; j < o1; j += NT) s += a.wz[j] * a.pool[j];
    } else {
      for (int64_t j = a.rng_b[2 * blk] + threadIdx.x; j < o1; j += NT) s += a.pool[j];
    }
    s = admmi::wave_sum(s);
    if ((threadIdx.x & 63) == 0) zred[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      T t = zred[0];
#pragma unroll
      for (int q = 1; q < NT / 64; ++q) t += zred[q];
      const T zn = t / dg;
      a.zout[zi] = zn;
      if (a.check) dmax = tabs(zn - a.zin[zi]) * (a.rmz ? a.rmz[zi] : T(1));
    }
  } else if (blk < a.n_b + a.nb_w) {
    const int sl = threadIdx.x & (ZSEG - 1);
    const int64_t k = (int64_t)(blk - a.n_b) * ZPB + (threadIdx.x / ZSEG);
    const bool ok = k < a.n_w;
    const int zi = ok ? a.var_w[k] : 0;   // read with the contributions
    const T dg = ok ? a.deg_w[k] : T(1);
    T s = T(0);
    if (ok) {
      if (a.w_stride) {
        // The first ZUN loads of each lane are issued together before any
        // sum (the list is a few strides long: one memory round trip instead
        // of one per stride); the sum order is the same as a sequential loop.
        const int64_t o = a.w_base + k * a.w_stride;
        const T* p = a.pool + o;
        T v[ZUN];
#pragma unroll
        for (int q = 0; q < ZUN; ++q) {
          const int64_t j = sl + q * ZSEG;
          v[q] = T(0);
          if (j < a.w_stride) v[q] = a.wz ? a.wz[o + j] * p[j] : p[j];
        }
#pragma unroll
        for (int q = 0; q < ZUN; ++q) s += v[q];
        for (int64_t j = sl + ZUN * ZSEG; j < a.w_stride; j += ZSEG)
          s += a.wz ? a.wz[o + j] * p[j] : p[j];
      } else {
        const int64_t o1 = a.rng_w[2 * k + 1];
        if (a.wz) {
          for (int64_t j = a.rng_w[2 * k] + sl; j < o1; j += ZSEG) s += a.wz[j] * a.pool[j];
        } else {
          for (int64_t j = a.rng_w[2 * k] + sl; j < o1; j += ZSEG) s += a.pool[j];
        }
      }
    }
    s = admmi::row16_sum(s);
    if (ok && sl == 0) {
      const T zn = s / dg;
      a.zout[zi] = zn;
      if (a.check) dmax = tabs(zn - a.zin[zi]) * (a.rmz ? a.rmz[zi] : T(1));
    }
  } else {
    const int64_t k = (int64_t)(blk - a.n_b - a.nb_w) * NT + threadIdx.x;
    if (k < a.n_l) {
      const int zi = a.var_l[k];
      const T d = a.deg_l[k];
      const int64_t o = a.l_base + k * LANE_MAX;
      const T* p = a.pool + o;
      T s;
      if (a.wz) {
        s = a.wz[o] * p[0];
#pragma unroll
        for (int j = 1; j < LANE_MAX; ++j) s += a.wz[o + j] * p[j];
      } else {
        s = p[0];
#pragma unroll
        for (int j = 1; j < LANE_MAX; ++j) s += p[j];
      }
      T zn;
      if (d > T(0))
        zn = s / d;
      else
        zn = a.zin[zi];   // no edge: z keeps its value
      a.zout[zi] = zn;
      if (a.check) dmax = tabs(zn - a.zin[zi]) * (a.rmz ? a.rmz[zi] : T(1));
    }
  }
  if (a.check) block_max_store(dmax, a.blockmax);
}

template <typename T>
__global__ __launch_bounds__(NT) void zpass_kernel(ZArgs<T> a) {
  zpass_block<T>(a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Resident driver for graphs whose whole state fits in one workgroup's LDS:
// every iteration of a run in one launch of one workgroup.  The regions the
// passes touch (pool, z ping-pong, parameters, indices, contribution lists)
// are copied into LDS at the start, the x-pass and z-pass blocks run one
// after another with workgroup barriers in between (the order that separate
// launches would impose), and the pool and the final z are copied back.
// The bucket table is staged in LDS too.  Pair tiles are not used here.
// ---------------------------------------------------------------------------
constexpr int RES_MAX_REG = 16;
constexpr int FS_RES = FT_UHINGE | FT_GEN | FT_WIDE | FT_XWIDE | FT_W64 | FT_LINDYN;

struct ResRegion {
  const void* src;  // global source
  void* back;       // global destination of the copy-back (NULL: none)
  int32_t off;      // byte offset in LDS (multiple of 16)
  int32_t words;    // 4-byte words
};

template <typename T>
struct ResArgs {
  ResRegion reg[RES_MAX_REG];
  int32_t nreg;
  int32_t o_pool, o_par, o_idx, o_z0, o_z1;
  int32_t o_var_b, o_rng_b, o_deg_b, o_var_w, o_rng_w, o_deg_w, o_var_l, o_deg_l;
  int32_t o_bt;     // the bucket table
  int32_t zc, iters, xblocks, zblocks, z_words;
  T* z_back[2];     // global z buffers (the final z is copied to z_back[final index])
};

template <typename T, bool A1>
__global__ __launch_bounds__(NT) void resident_kernel(XArgs<T> xa, ZArgs<T> za, ResArgs<T> r) {
  extern __shared__ __align__(16) unsigned char lds_img[];
  for (int q = 0; q < r.nreg; ++q) {
    const uint32_t* src = (const uint32_t*)r.reg[q].src;
    uint32_t* dst = (uint32_t*)(lds_img + r.reg[q].off);
    for (int i = threadIdx.x; i < r.reg[q].words; i += NT) dst[i] = src[i];
  }
  __syncthreads();
  xa.pool = (T*)(lds_img + r.o_pool);
  xa.par = (const T*)(lds_img + r.o_par);
  xa.idx = (const int32_t*)(lds_img + r.o_idx);
  xa.bt = (const BucketDesc*)(lds_img + r.o_bt);
  za.pool = xa.pool;
  za.var_b = (const int32_t*)(lds_img + r.o_var_b);
  za.rng_b = (const int64_t*)(lds_img + r.o_rng_b);
  za.deg_b = (const T*)(lds_img + r.o_deg_b);
  za.var_w = (const int32_t*)(lds_img + r.o_var_w);
  za.rng_w = (const int64_t*)(lds_img + r.o_rng_w);
  za.deg_w = (const T*)(lds_img + r.o_deg_w);
  za.var_l = (const int32_t*)(lds_img + r.o_var_l);
  za.deg_l = (const T*)(lds_img + r.o_deg_l);
  // z buffers are addressed as lds_img + offset each iteration (not through a
  // pointer carried across iterations) so that every z access stays an LDS
  // access.
  int zc = r.zc;
  const int32_t zoff[2] = {r.o_z0, r.o_z1};
  for (int k = 0; k < r.iters; ++k) {
    const bool last = (k == r.iters - 1);
    xa.z = (const T*)(lds_img + zoff[zc]);
    for (int b = 0; b < r.xblocks; ++b) {
      if (A1 && last)
        xpass_block<T, A1, PM_SAVE, FS_RES>(xa, b, find_bucket(xa, b));
      else
        xpass_block<T, A1, PM_NORMAL, FS_RES>(xa, b, find_bucket(xa, b));
      __syncthreads();
    }
    za.zin = (const T*)(lds_img + zoff[zc]);
    za.zout = (T*)(lds_img + zoff[zc ^ 1]);
    za.check = last ? 1 : 0;
    for (int b = 0; b < r.zblocks; ++b) {
      zpass_block<T>(za, b);
      __syncthreads();
    }
    zc ^= 1;
  }
  xa.z = (const T*)(lds_img + zoff[zc]);
  for (int b = 0; b < r.xblocks; ++b) {
    xpass_block<T, A1, PM_RESID, FS_RES>(xa, b, find_bucket(xa, b));
    __syncthreads();
  }
  for (int q = 0; q < r.nreg; ++q) {
    if (!r.reg[q].back) continue;
    const uint32_t* src = (const uint32_t*)(lds_img + r.reg[q].off);
    uint32_t* dst = (uint32_t*)r.reg[q].back;
    for (int i = threadIdx.x; i < r.reg[q].words; i += NT) dst[i] = src[i];
  }
  const uint32_t* zs = (const uint32_t*)(lds_img + zoff[zc]);
  uint32_t* zd = (uint32_t*)r.z_back[zc];
  for (int i = threadIdx.x; i < r.z_words; i += NT) zd[i] = zs[i];
}

// State import: m = u + z_b (x = z_b) for every user slot.
template <typename T>
__global__ void set_state_kernel(int64_t ns, const int64_t* upos, const int32_t* uz,
                                 const double* u, const T* z, T* pool, int64_t xdelta,
                                 int write_x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const T zv = z[uz[i]];
  const T uv = u ? (T)u[i] : T(0);
  pool[upos[i]] = uv + zv;
  if (write_x) pool[upos[i] + xdelta] = zv;
}

// Export of u (which = 0), x (which = 1) in user slot order.
template <typename T, bool A1>
__global__ void get_slots_kernel(int64_t ns, const int64_t* upos, const int32_t* uz,
                                 const T* pool, const T* z, int64_t xdelta, T alpha,
                                 const T* ualpha, int which, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const int64_t p = upos[i];
  const T zv = z[uz[i]];
  if (which == 1) {
    out[i] = (double)pool[p + xdelta];
    return;
  }
  T u;
  if constexpr (A1) {
    u = pool[p] - zv;
  } else {
    const T xo = pool[p + xdelta];
    u = (pool[p] - xo) + (ualpha ? ualpha[i] : alpha) * (xo - zv);
  }
  out[i] = (double)u;
}

template <typename W>
__global__ void fill_kernel(int64_t n, W v, W* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v;
}

template <typename T>
__global__ void convert_kernel(int64_t n, const double* in, T* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (T)in[i];
}

template <typename T>
__global__ void widen_kernel(int64_t n, const T* in, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}

}  // namespace admmg
