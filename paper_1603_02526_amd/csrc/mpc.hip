// Batched linear MPC: thousands of uneven instances solved by the ADMM of
// Algorithm 2 (paper Sec. II) in one persistent launch.
//
// Each instance is the MPC factor graph of the paper's Sec. V-B with split
// variable nodes: u_t (dim m, t = 0..T-1) and x_{t+1} (dim n).  Factors per
// step t: the linear-dynamics projection on (x_t, u_t, x_{t+1}) (x_0 is a
// parameter at t = 0), a quadratic cost on u_t and on x_{t+1}, and a box on
// u_t.  Every variable has degree <= 3, so the z-update is a 2- or 3-term
// average.  alpha = 1, so the per-edge state is m alone (u = m - z).
//
// Mapping to gfx950: one lane per time step.  Instances with T <= 64 run one
// per wavefront, up to four independent wavefronts per workgroup; longer
// instances use ceil(T/64) wavefronts of one workgroup in lockstep.  All of
// an instance's per-edge state and z stay in registers for the whole solve;
// neighbouring time steps exchange z and m through LDS; the matrices of the
// projection are read from a per-instance parameter block with wavefront-
// uniform addresses.  Workgroups take work items from a queue until it is
// empty.  Each instance stops at the first iteration with
//   r = max_e |x_e - z_b| <= tol  and  s = rho max_b |z_b - z_b(prev)| <= tol.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <numeric>
#include <vector>

#include "internal.h"

namespace {

constexpr int WGT = 256;   // threads per workgroup (batches with an instance of T > 128)
constexpr int WGS = 128;   // threads per workgroup when every instance has T <= 128
constexpr int MN = 12;     // largest state dimension
constexpr int MM = 4;      // largest input dimension
constexpr int MK = MN + MM;
constexpr int TMAX = 256;  // longest horizon (four wavefronts)

struct MpcInst {
  int32_t T, n, m, box;
  int32_t par_off, x0_off, pad0, pad1;
  int64_t z_off, u_off;
};

// Parameter block (floats).  The state dimension is padded to N =
// max(n, 4) (the solver is compiled for each N) and the input dimension to
// 4, with zero rows and columns, so every matrix row has a fixed length:
//   M [N][N+4] = [A B], S [N][N] = (I + M M^T)^-1, B [N][4],
//   S0 [N][N] = (I + B B^T)^-1, A [N][N], cq [N] = rho/(rho+q), cr [4] =
//   rho/(rho+r), q [N], r [4], lo, hi
// Padded components of z and m stay exactly zero through every update.
struct ParOff {
  int N4, K4;  // N rounded up to 4; row width of M
  int M, MT, S, S0, B, A, cq, cr, q, r, lo, size;
};
__host__ __device__ constexpr ParOff par_offsets(int N) {
  ParOff o{};
  o.N4 = (N + 3) / 4 * 4;
  o.K4 = o.N4 + MM;
  o.M = 0;                         // [N][K4]: A row | 0 .. | B row
  o.MT = o.M + N * o.K4;           // [K4][N4]: column j of [A 0 B], zero padded
  o.S = o.MT + o.K4 * o.N4;        // [N][N4]
  o.S0 = o.S + N * o.N4;           // [N][N4]
  o.B = o.S0 + N * o.N4;           // [N][MM]
  o.A = o.B + N * MM;              // [N][N]
  o.cq = o.A + N * N;
  o.cr = o.cq + N;
  o.q = o.cr + MM;
  o.r = o.q + N;
  o.lo = o.r + MM;
  o.size = (o.lo + 2 + 3) / 4 * 4;
  return o;
}
__host__ __device__ constexpr int pad_n(int n) { return n < 4 ? 4 : n; }
constexpr int PBLK = par_offsets(MN).size + MN;  // parameter block + c = A x0 (floats)
static_assert(PBLK % 4 == 0, "parameter slots must stay 16-byte aligned");

struct SolveArgs {
  const MpcInst* inst;
  const float* par;
  const float* x0;
  const float* zinit;   // nullable: z0 = 0
  const float* uinit;   // nullable: u0 = 0
  float* zout;
  float* uout;          // nullable: final per-edge duals
  int32_t* iters;
  const int32_t* items; // [n_items][5]: G, id0..id3 (-1 = none)
  int32_t n_items;
  int32_t* counter;
  float tol;
  int32_t max_iter;
  float rho;
};

template <bool LOCK>
__device__ __forceinline__ void isync() {
  if constexpr (LOCK) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  }
}


typedef float f4v __attribute__((ext_vector_type(4)));

// Whole-wavefront shifts by one lane (DPP wave_shr:1 / wave_shl:1): lane t
// receives lane t-1's (resp. t+1's) value; lane 0 (resp. 63) receives 0.
// Every lane of the wavefront must be active.
__device__ __forceinline__ float lane_prev(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_next(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, false));
}

// out[i] += sum_c P[i*C + c] x[c] for i < R, P in LDS with 16-byte aligned
// rows of C floats (C % 4 == 0), terms added in c order.  Row i+1 is read
// while row i is summed; the scheduling barrier per row keeps the compiler
// from reading every row ahead (the whole block would not fit in registers).
template <int R, int C>
__device__ __forceinline__ void mv_rows(const float* P, const float (&x)[C], float (&out)[R]) {
  f4v cur[C / 4], nxt[C / 4];
#pragma unroll
  for (int q = 0; q < C / 4; ++q) cur[q] = ((const f4v*)P)[q];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    if (i + 1 < R) {
#pragma unroll
      for (int q = 0; q < C / 4; ++q) nxt[q] = ((const f4v*)(P + (i + 1) * C))[q];
    }
    float s = out[i];
#pragma unroll
    for (int q = 0; q < C / 4; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) s = fmaf(cur[q][e], x[4 * q + e], s);
    out[i] = s;
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < C / 4; ++q) cur[q] = nxt[q];
  }
}

// One instance.  LOCK: all four wavefronts of the workgroup work on it in
// lockstep (t = threadIdx.x); otherwise this wavefront alone (t = lane).
// xb: first exchange slot of this instance.  red: per-wavefront residuals.
// N: padded state dimension; inputs are padded to MM = 4.
template <bool LOCK, int N>
__device__ __forceinline__ void solve_one(const SolveArgs a, int id, int t, int xb, float* xz,
                                          float* xm, float* red, float* ps) {
  constexpr ParOff o = par_offsets(N);
  const MpcInst I = a.inst[id];
  const int T = __builtin_amdgcn_readfirstlane(I.T);
  const int n = __builtin_amdgcn_readfirstlane(I.n);
  const int m = __builtin_amdgcn_readfirstlane(I.m);
  const int k = n + m;  // unpadded step width of z and of the u layout / 3
  const bool box = __builtin_amdgcn_readfirstlane(I.box) != 0;
  const bool act = t < T;
  // Stage the parameter block in this instance's LDS slot.
  {
    const float* __restrict__ Pg = a.par + __builtin_amdgcn_readfirstlane(I.par_off);
    const int nthr = LOCK ? (int)blockDim.x : 64;
    const int tid = LOCK ? (int)threadIdx.x : (int)(threadIdx.x & 63);
    for (int q = tid; q < o.size; q += nthr) ps[q] = Pg[q];
  }
  isync<LOCK>();
  const float* Pb = ps;
  const float lo = Pb[o.lo], hi = Pb[o.lo + 1];

  float zu[MM], zx1[N];
  float mdx[N], mdu[MM], mdx1[N], mqu[MM], mbx[MM], mqx[N];
  float cvec[N];  // c = A x0, used by time step 0 only
#pragma unroll
  for (int i = 0; i < N; ++i) cvec[i] = 0.f;
#pragma unroll
  for (int i = 0; i < N; ++i) { zx1[i] = 0.f; mdx[i] = 0.f; mdx1[i] = 0.f; mqx[i] = 0.f; }
#pragma unroll
  for (int j = 0; j < MM; ++j) { zu[j] = 0.f; mdu[j] = 0.f; mqu[j] = 0.f; mbx[j] = 0.f; }

  if (act && a.zinit) {
    const float* zi = a.zinit + I.z_off + (int64_t)t * k;
#pragma unroll
    for (int j = 0; j < MM; ++j) if (j < m) zu[j] = zi[j];
#pragma unroll
    for (int i = 0; i < N; ++i) if (i < n) zx1[i] = zi[m + i];
  }
  // z of x_t, the previous step's x_{t+1} (0 at t = 0).  One wavefront per
  // instance exchanges neighbours by lane shifts; lockstep wavefronts
  // through LDS.  The same value is carried across iterations in zxpc.
  float zxpc[N];
  if constexpr (LOCK) {
    if (act) {
#pragma unroll
      for (int i = 0; i < N; ++i) xz[(xb + t) * MN + i] = zx1[i];
    }
    isync<LOCK>();
#pragma unroll
    for (int i = 0; i < N; ++i) zxpc[i] = (act && t >= 1) ? xz[(xb + t - 1) * MN + i] : 0.f;
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) zxpc[i] = lane_prev(zx1[i]);
  }
  if (act) {
    float zxp[N];
#pragma unroll
    for (int i = 0; i < N; ++i) zxp[i] = zxpc[i];
    // m = u + z per edge; u per step laid out [dx n | du m | dx1 n | qu m | bx m | qx n]
    if (a.uinit) {
      const float* ui = a.uinit + I.u_off + (int64_t)t * 3 * k;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        if (i < n) {
          mdx[i] = ui[i];
          mdx1[i] = ui[n + m + i];
          mqx[i] = ui[2 * n + 3 * m + i];
        }
      }
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        if (j < m) {
          mdu[j] = ui[n + j];
          mqu[j] = ui[2 * n + m + j];
          mbx[j] = ui[2 * n + 2 * m + j];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      mdx[i] += zxp[i];
      mdx1[i] += zx1[i];
      mqx[i] += zx1[i];
    }
  }
  if (act) {
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      mdu[j] += zu[j];
      mqu[j] += zu[j];
      mbx[j] += zu[j];
    }
    if (t == 0) {
      const float* x0 = a.x0 + I.x0_off;
      float xv[N];
#pragma unroll
      for (int j = 0; j < N; ++j) xv[j] = (j < n) ? x0[j] : 0.f;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        float s = 0.f;
#pragma unroll
        for (int j = 0; j < N; ++j) s += Pb[o.A + i * N + j] * xv[j];
        cvec[i] = s;
      }
    }
  }

  int done_it = -1;
  const int nw = LOCK ? (T + 63) / 64 : 1;
  const int w = threadIdx.x >> 6;
  for (int it = 1; it <= a.max_iter; ++it) {
    float ax[N], au[MM], bv[N], xqu[MM], xbx[MM], xqx[N];
    float rloc = 0.f, sloc = 0.f;
    // The parameter block is re-read from LDS every iteration: an opaque
    // zero offset keeps the compiler from hoisting several hundred
    // loop-invariant matrix entries into registers.
    int zoff;
    asm volatile("s_mov_b32 %0, 0" : "=s"(zoff));
    const float* P = Pb + zoff;
    float zxp[N];
#pragma unroll
    for (int i = 0; i < N; ++i) zxp[i] = zxpc[i];
    if (act) {
      // ---- x-update.  n = z - u = 2z - m on every edge.
#pragma unroll
      for (int i = 0; i < N; ++i) ax[i] = (t >= 1) ? (2.f * zxp[i] - mdx[i]) : 0.f;
#pragma unroll
      for (int j = 0; j < MM; ++j) au[j] = 2.f * zu[j] - mdu[j];
#pragma unroll
      for (int i = 0; i < N; ++i) bv[i] = 2.f * zx1[i] - mdx1[i];
      // dynamics: w = M a + c - b; v = S w (S0 at t = 0); a -= M^T v; b += v
      constexpr int N4 = o.N4, K4 = o.K4;
      float xa[K4], wv[N], wp[N4], vv[N], vp[N4], sx[N], su[MM];
#pragma unroll
      for (int c = 0; c < K4; ++c) xa[c] = c < N ? ax[c < N ? c : 0] : (c >= N4 ? au[c >= N4 ? c - N4 : 0] : 0.f);
#pragma unroll
      for (int i = 0; i < N; ++i) wv[i] = cvec[i] - bv[i];
      mv_rows<N, K4>(P + o.M, xa, wv);
#pragma unroll
      for (int c = 0; c < N4; ++c) wp[c] = c < N ? wv[c < N ? c : 0] : 0.f;
#pragma unroll
      for (int i = 0; i < N; ++i) vv[i] = 0.f;
      mv_rows<N, N4>(P + ((t >= 1) ? o.S : o.S0), wp, vv);
#pragma unroll
      for (int c = 0; c < N4; ++c) vp[c] = c < N ? vv[c < N ? c : 0] : 0.f;
#pragma unroll
      for (int i = 0; i < N; ++i) sx[i] = 0.f;
#pragma unroll
      for (int j = 0; j < MM; ++j) su[j] = 0.f;
      mv_rows<N, N4>(P + o.MT, vp, sx);
      mv_rows<MM, N4>(P + o.MT + N4 * N4, vp, su);
#pragma unroll
      for (int j = 0; j < N; ++j) ax[j] -= sx[j];
#pragma unroll
      for (int j = 0; j < MM; ++j) au[j] -= su[j];
#pragma unroll
      for (int i = 0; i < N; ++i) bv[i] += vv[i];
      // separable costs and the box
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        xqu[j] = P[o.cr + j] * (2.f * zu[j] - mqu[j]);
        const float nb = 2.f * zu[j] - mbx[j];
        xbx[j] = nb < lo ? lo : (nb > hi ? hi : nb);
      }
#pragma unroll
      for (int i = 0; i < N; ++i) xqx[i] = P[o.cq + i] * (2.f * zx1[i] - mqx[i]);
      // ---- m-update: m = x + u, u = m_old - z_old
#pragma unroll
      for (int i = 0; i < N; ++i) {
        mdx[i] = ax[i] + (mdx[i] - zxp[i]);
        mdx1[i] = bv[i] + (mdx1[i] - zx1[i]);
        mqx[i] = xqx[i] + (mqx[i] - zx1[i]);
      }
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        mdu[j] = au[j] + (mdu[j] - zu[j]);
        mqu[j] = xqu[j] + (mqu[j] - zu[j]);
        mbx[j] = xbx[j] + (mbx[j] - zu[j]);
      }
    }
    // From step t+1 (lane t+1): the m and the x of its dynamics edge on
    // x_{t+1}.  Lane shifts inside a wavefront; in lockstep mode lane 63
    // takes them from the next wavefront's lane 0 through LDS.
    float xmn[N], axn[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      xmn[i] = lane_next(mdx[i]);
      axn[i] = lane_next(ax[i]);
    }
    if constexpr (LOCK) {
      if ((t & 63) == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
          xm[w * 2 * MN + i] = mdx[i];
          xm[w * 2 * MN + MN + i] = ax[i];
        }
      }
      __syncthreads();
      if ((t & 63) == 63 && w + 1 < nw) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
          xmn[i] = xm[(w + 1) * 2 * MN + i];
          axn[i] = xm[(w + 1) * 2 * MN + MN + i];
        }
      }
    }
    float zx1n[N];
#pragma unroll
    for (int i = 0; i < N; ++i) zx1n[i] = 0.f;
    // residual maxima use v_max (which drops NaN): a NaN in this step's new
    // z makes chk NaN, and the step then reports an infinite residual
    float chk = 0.f;
    if (act) {
      // ---- z-update: 3-term averages (x_T and box-free inputs: 2 terms).
      // The residual of step t+1's dynamics edge on x_{t+1} is taken here,
      // where the new z of x_{t+1} is.
      const bool nxt = (t + 1 < T);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        float s = mdx1[i] + mqx[i];
        if (nxt) s += xmn[i];
        const float zn = s * (nxt ? (1.f / 3.f) : 0.5f);
        sloc = fmaxf(sloc, fabsf(zn - zx1[i]));
        rloc = fmaxf(rloc, fmaxf(fabsf(bv[i] - zn), fabsf(xqx[i] - zn)));
        if (nxt) rloc = fmaxf(rloc, fabsf(axn[i] - zn));
        zx1n[i] = zn;
        chk += zn;
      }
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        const float s = box ? (mdu[j] + mqu[j] + mbx[j]) : (mdu[j] + mqu[j]);
        const float zn = s * (box ? (1.f / 3.f) : 0.5f);
        sloc = fmaxf(sloc, fabsf(zn - zu[j]));
        float r = fmaxf(fabsf(au[j] - zn), fabsf(xqu[j] - zn));
        if (box) r = fmaxf(r, fabsf(xbx[j] - zn));
        rloc = fmaxf(rloc, r);
        chk += zn;
        zu[j] = zn;
      }
#pragma unroll
      for (int i = 0; i < N; ++i) zx1[i] = zx1n[i];
    }
    // next iteration's z of x_t: the new z of step t-1 (lane t-1); in
    // lockstep mode lane 0 takes it from the previous wavefront's lane 63
    // through LDS, across the barrier of the stopping-rule reduction
#pragma unroll
    for (int i = 0; i < N; ++i) zxpc[i] = lane_prev(zx1n[i]);
    if constexpr (LOCK) {
      if ((t & 63) == 63) {
#pragma unroll
        for (int i = 0; i < N; ++i) xz[w * MN + i] = zx1n[i];
      }
    }
    if (!(chk == chk)) rloc = __builtin_inff();
    // ---- stopping rule, reduced over the instance
    float r = admmi::wave_max_nonneg(rloc), s = admmi::wave_max_nonneg(sloc);
    if constexpr (LOCK) {
      if ((threadIdx.x & 63) == 0) { red[2 * w] = r; red[2 * w + 1] = s; }
      __syncthreads();
      r = red[0];
      s = red[1];
      for (int q = 1; q < nw; ++q) { r = fmaxf(r, red[2 * q]); s = fmaxf(s, red[2 * q + 1]); }
      if ((t & 63) == 0 && w >= 1) {
#pragma unroll
        for (int i = 0; i < N; ++i) zxpc[i] = xz[(w - 1) * MN + i];
      }
    }
    s *= a.rho;
    if (r <= a.tol && s <= a.tol) {
      done_it = it;
      break;
    }
  }
  if (act) {
    float* zo = a.zout + I.z_off + (int64_t)t * k;
#pragma unroll
    for (int j = 0; j < MM; ++j) if (j < m) zo[j] = zu[j];
#pragma unroll
    for (int i = 0; i < N; ++i) if (i < n) zo[m + i] = zx1[i];
    if (a.uout) {
      // u = m - z with the final z (the state the next solve continues from);
      // zxpc already holds the final z of x_t
      float* uo = a.uout + I.u_off + (int64_t)t * 3 * k;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        if (i < n) {
          uo[i] = t >= 1 ? mdx[i] - zxpc[i] : 0.f;
          uo[n + m + i] = mdx1[i] - zx1[i];
          uo[2 * n + 3 * m + i] = mqx[i] - zx1[i];
        }
      }
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        if (j < m) {
          uo[n + j] = mdu[j] - zu[j];
          uo[2 * n + m + j] = mqu[j] - zu[j];
          uo[2 * n + 2 * m + j] = mbx[j] - zu[j];
        }
      }
    }
  }
  if (t == 0) a.iters[id] = done_it > 0 ? done_it : -a.max_iter;
}

template <bool LOCK>
__device__ __forceinline__ void solve_dispatch(const SolveArgs a, int id, int t, int xb, float* xz,
                                               float* xm, float* red, float* ps) {
  const int N = pad_n(__builtin_amdgcn_readfirstlane(a.inst[id].n));
  switch (N) {
    case 4: solve_one<LOCK, 4>(a, id, t, xb, xz, xm, red, ps); break;
    case 5: solve_one<LOCK, 5>(a, id, t, xb, xz, xm, red, ps); break;
    case 6: solve_one<LOCK, 6>(a, id, t, xb, xz, xm, red, ps); break;
    case 7: solve_one<LOCK, 7>(a, id, t, xb, xz, xm, red, ps); break;
    case 8: solve_one<LOCK, 8>(a, id, t, xb, xz, xm, red, ps); break;
    case 9: solve_one<LOCK, 9>(a, id, t, xb, xz, xm, red, ps); break;
    case 10: solve_one<LOCK, 10>(a, id, t, xb, xz, xm, red, ps); break;
    case 11: solve_one<LOCK, 11>(a, id, t, xb, xz, xm, red, ps); break;
    default: solve_one<LOCK, 12>(a, id, t, xb, xz, xm, red, ps); break;
  }
}

// WG threads per workgroup: WG/64 one-wavefront instances, or one instance
// of up to WG/64 lockstep wavefronts, per work item.  The register budget
// is held at two waves per SIMD for both sizes.
template <int WG>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(2, 2))) void mpc_solve_kernel(
    const MpcInst* __restrict__ inst, const float* __restrict__ par, const float* __restrict__ x0,
    const float* __restrict__ zinit, const float* __restrict__ uinit, float* __restrict__ zout,
    float* __restrict__ uout, int32_t* __restrict__ iters, const int32_t* __restrict__ items,
    int32_t n_items, int32_t* __restrict__ counter, float tol, int32_t max_iter, float rho) {
  SolveArgs a;
  a.inst = inst;
  a.par = par;
  a.x0 = x0;
  a.zinit = zinit;
  a.uinit = uinit;
  a.zout = zout;
  a.uout = uout;
  a.iters = iters;
  a.items = items;
  a.n_items = n_items;
  a.counter = counter;
  a.tol = tol;
  a.max_iter = max_iter;
  a.rho = rho;
  __shared__ float xz[WG * MN];
  __shared__ float xm[WG * MN];
  __shared__ float red[8];
  __shared__ __align__(16) float ps[(WG / 64) * PBLK];   // rows read as 16-byte vectors
  __shared__ int s_item;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (item >= a.n_items) break;
    const int G = __builtin_amdgcn_readfirstlane(a.items[5 * item]);
    if (G == 1) {
      const int id = __builtin_amdgcn_readfirstlane(a.items[5 * item + 1 + w]);
      if (id >= 0) solve_dispatch<false>(a, id, lane, w * 64, xz, xm, red, ps + w * PBLK);
    } else {
      const int id = __builtin_amdgcn_readfirstlane(a.items[5 * item + 1]);
      solve_dispatch<true>(a, id, threadIdx.x, 0, xz, xm, red, ps);
    }
    __syncthreads();
  }
}

__global__ void reset_counter_kernel(int32_t* c) {
  if (threadIdx.x == 0) c[0] = 0;
}

// Dual completion from z: mu_{T-1} = Q x_T, mu_{t-1} = A^T mu_t + Q x_t, then
//   rho u[dyn_t]  = (-A^T mu_t, -B^T mu_t, mu_t)  (no x part at t = 0)
//   rho u[quad u] = -R u_t, rho u[box] = B^T mu_t + R u_t, rho u[quad x] = -Q x_{t+1}
// One 64-lane workgroup per instance: lanes r < n run the backward pass,
// then every lane writes the duals of its time steps.
// Dual completion, four instances per wavefront (one 16-lane DPP row
// each; lane i of a row is state component i).  Backward over t, with
// X[t] = x_{t+1} and U[t] = u_t from z:
//   mu_{T-1} = Q X[T-1],  mu_{t-1} = A^T mu_t + Q X[t-1],
// and at step t (u layout [dx n | du m | dx1 n | qu m | bx m | qx n]):
//   dx = -A^T mu_t (0 at t = 0), du = -B^T mu_t, dx1 = mu_t,
//   qu = -R U[t], bx = B^T mu_t + R U[t], qx = -Q X[t], all divided by rho.
// Lane i holds column i of A and of B; mu_t[j] reaches every lane of the
// row by DPP row broadcast (row_newbcast:j), so a step is 2n FMAs.  The
// instance's z is staged in LDS first.  Rows run max(T) steps; a row
// whose instance is shorter or absent computes on zeros and stores
// nothing.
template <int J>
__device__ __forceinline__ float row_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + J, 0xF, 0xF, false));
}

__global__ __launch_bounds__(64) void mpc_dual_kernel(const MpcInst* inst, int32_t n_inst,
                                                      const float* par, const float* z, float* u,
                                                      float inv_rho) {
  __shared__ float zs[4][TMAX * 16];
  const int lane = threadIdx.x, row = lane >> 4, li = lane & 15;
  const int id = blockIdx.x * 4 + row;
  const bool have = id < n_inst;
  const MpcInst I = inst[have ? id : 0];
  const int T = have ? I.T : 0, n = I.n, m = I.m, k = n + m;
  const int N = pad_n(n);
  const ParOff o = par_offsets(N);
  const float* P = par + I.par_off;
  const float* zz = z + I.z_off;
  // eight loads in flight per lane before the first store waits
#pragma unroll 8
  for (int e = li; e < T * k; e += 16) zs[row][e] = zz[e];
  float acol[MN], bcol[MN];
#pragma unroll
  for (int j = 0; j < MN; ++j) {
    acol[j] = (li < n && j < n) ? P[o.A + j * N + li] : 0.f;
    bcol[j] = (li < m && j < n) ? P[o.B + j * MM + li] : 0.f;
  }
  const float ql = li < n ? P[o.q + li] : 0.f;
  const float rl = li < m ? P[o.r + li] : 0.f;
  __syncthreads();
  int Tmax = T;
  Tmax = max(Tmax, __shfl_xor(Tmax, 16, 64));
  Tmax = max(Tmax, __shfl_xor(Tmax, 32, 64));
  const float* zr = zs[row];
  float mu = (T > 0 && li < n) ? ql * zr[(T - 1) * k + m + li] : 0.f;
  for (int s = 0; s < Tmax; ++s) {
    const int t = T - 1 - s;            // this row's step (< 0: nothing to do)
    // this step's x_{t+1} and u_t and the previous step's x_t, read together
    // (indices clamped into the instance; unused values are never stored)
    const int tc = t > 0 ? t : 0, tp = t > 1 ? t - 1 : 0;
    const int ix = m + (li < n ? li : 0), iu = li < m ? li : 0;
    const float xt = zr[tc * k + ix];
    const float uu = zr[tc * k + iu];
    const float xp = zr[tp * k + ix];
    float a = 0.f, b = 0.f;
    static_assert(MN == 12, "the broadcast sequence below covers 12 components");
#define ADMM_DUAL_TERM(J)                   \
  {                                         \
    const float mj = row_bcast<J>(mu);      \
    a = fmaf(acol[J], mj, a);               \
    b = fmaf(bcol[J], mj, b);               \
  }
    ADMM_DUAL_TERM(0) ADMM_DUAL_TERM(1) ADMM_DUAL_TERM(2) ADMM_DUAL_TERM(3)
    ADMM_DUAL_TERM(4) ADMM_DUAL_TERM(5) ADMM_DUAL_TERM(6) ADMM_DUAL_TERM(7)
    ADMM_DUAL_TERM(8) ADMM_DUAL_TERM(9) ADMM_DUAL_TERM(10) ADMM_DUAL_TERM(11)
#undef ADMM_DUAL_TERM
    if (t >= 0) {
      float* ut = u + I.u_off + (int64_t)t * 3 * k;
      if (li < n) {
        ut[li] = t >= 1 ? -a * inv_rho : 0.f;             // dynamics, x_t edge
        ut[n + m + li] = mu * inv_rho;                     // dynamics, x_{t+1} edge
        ut[2 * n + 3 * m + li] = -ql * xt * inv_rho;       // quadratic on x_{t+1}
      }
      if (li < m) {
        ut[n + li] = -b * inv_rho;                         // dynamics, u_t edge
        ut[2 * n + m + li] = -rl * uu * inv_rho;           // quadratic on u_t
        ut[2 * n + 2 * m + li] = (b + rl * uu) * inv_rho;  // box on u_t
      }
    }
    mu = (t >= 1 && li < n) ? a + ql * xp : 0.f;
  }
}

// One receding-horizon step of every instance (the paper's Sec. V-B: each
// controller cycle updates the current state and continues the ADMM from the
// previous cycle's solution).  The plant applies the first planned input:
//   x0' = A x0 + B u_0 (+ w),  u_0 = z of u_0.
// With zn: the trajectory moves one step forward, z'(t) = z(t+1) for
// t < T-1, and the new last step holds u = 0 and x = A x_T.  With un: every
// edge's dual moves with its step (the dynamics factor of step 0 has no x_t
// edge, so that part of step 1 is dropped) and the new last step's duals are
// zero; the duals around every variable keep their sum.
// One workgroup per instance, one thread per step (T <= 256).
__global__ __launch_bounds__(WGT) void mpc_shift_kernel(
    const MpcInst* __restrict__ inst, const float* __restrict__ par, const float* __restrict__ x0,
    const float* __restrict__ z, const float* __restrict__ u, const float* __restrict__ w,
    float* __restrict__ x0n, float* __restrict__ zn, float* __restrict__ un) {
  const MpcInst I = inst[blockIdx.x];
  const int t = threadIdx.x;
  const int T = I.T, n = I.n, m = I.m, k = n + m;
  const int Np = pad_n(n);
  const ParOff o = par_offsets(Np);
  const float* P = par + I.par_off;
  const float* zi = z + I.z_off;
  if (t == 0) {
    const float* xi = x0 + I.x0_off;
    for (int r = 0; r < n; ++r) {
      float s = 0.f;
      for (int j = 0; j < n; ++j) s = fmaf(P[o.A + r * Np + j], xi[j], s);
      for (int j = 0; j < m; ++j) s = fmaf(P[o.B + r * MM + j], zi[j], s);
      if (w) s += w[I.x0_off + r];
      x0n[I.x0_off + r] = s;
    }
  }
  if (t >= T) return;
  if (zn) {
    float* zo = zn + I.z_off + (int64_t)t * k;
    if (t + 1 < T) {
      const float* src = zi + (int64_t)(t + 1) * k;
      for (int q = 0; q < k; ++q) zo[q] = src[q];
    } else {
      const float* xT = zi + (int64_t)t * k + m;
      for (int j = 0; j < m; ++j) zo[j] = 0.f;
      for (int r = 0; r < n; ++r) {
        float s = 0.f;
        for (int j = 0; j < n; ++j) s = fmaf(P[o.A + r * Np + j], xT[j], s);
        zo[m + r] = s;
      }
    }
  }
  if (un) {
    float* uo = un + I.u_off + (int64_t)t * 3 * k;
    if (t + 1 < T) {
      const float* src = u + I.u_off + (int64_t)(t + 1) * 3 * k;
      for (int q = 0; q < 3 * k; ++q) uo[q] = (t == 0 && q < n) ? 0.f : src[q];
    } else {
      for (int q = 0; q < 3 * k; ++q) uo[q] = 0.f;
    }
  }
}

std::vector<double> inv_spd(std::vector<double> a, int n) {
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

struct Plan {
  int pack1 = 4;  // instances per workgroup when T <= 64
  int order = 1;  // 0 as given, 1 longest first, 2 by (n, m) then longest first,
                  // 3 longest measured solve first (iterations of the last tuning solve)
  int grid = 0;   // persistent workgroups; 0: resident capacity
};

}  // namespace

struct admm_mpc_batch {
  int device = 0;
  int32_t n_inst = 0;
  double rho = 1.0;
  std::vector<MpcInst> h_inst;
  int64_t z_total = 0, u_total = 0, x0_total = 0;
  MpcInst* d_inst = nullptr;
  float* d_par = nullptr;
  float* d_u = nullptr;       // dual-completion output
  int32_t* d_items = nullptr;
  int32_t n_items = 0;
  int32_t* d_counter = nullptr;
  Plan plan;
  int resident = 0;          // workgroups resident per device at full occupancy
  int wg = WGT;              // threads per workgroup of the persistent launch
  std::vector<int32_t> measured;  // iterations per instance from the last tuning solve
  std::vector<void*> allocs;
  ~admm_mpc_batch() {
    if (!allocs.empty()) {
      hipSetDevice(device);
      for (void* p : allocs) hipFree(p);
    }
  }
};

namespace {

admm_status mpc_alloc(admm_mpc_batch* b, void** p, size_t bytes) {
  ADMM_HIP(hipMalloc(p, std::max<size_t>(bytes, 4)));
  b->allocs.push_back(*p);
  return ADMM_OK;
}

// Work items for a plan: instances of more than 64 steps get a workgroup of
// their own; shorter ones are packed pack1 to a workgroup (one wavefront
// each).  Items are ordered by the plan's order key.
admm_status build_items(admm_mpc_batch* b, const Plan& pl) {
  std::vector<int32_t> ids(b->n_inst);
  std::iota(ids.begin(), ids.end(), 0);
  auto cost = [&](int i) {
    const MpcInst& I = b->h_inst[i];
    return (double)I.T * (2.0 * I.n * (I.n + I.m) + I.n * I.n + 8.0 * (I.n + I.m));
  };
  // expected duration of a solve: measured iterations x the latency of one
  // iteration, which grows with the padded state size and with the number
  // of lockstep wavefronts (fitted to single-instance timings)
  auto duration = [&](int i) {
    const MpcInst& I = b->h_inst[i];
    const double Np = I.n < 4 ? 4.0 : (double)I.n;
    const int G = (I.T + 63) / 64;
    const double it = std::max<int32_t>(1, std::abs(b->measured[i]));
    return it * (0.6 + 0.016 * Np * Np + 0.3 * (G - 1));
  };
  if (pl.order == 3 && (int)b->measured.size() == b->n_inst) {
    std::stable_sort(ids.begin(), ids.end(),
                     [&](int x, int y) { return duration(x) > duration(y); });
  } else if (pl.order == 1 || pl.order == 3) {
    std::stable_sort(ids.begin(), ids.end(), [&](int x, int y) { return cost(x) > cost(y); });
  } else if (pl.order == 2) {
    std::stable_sort(ids.begin(), ids.end(), [&](int x, int y) {
      const MpcInst &X = b->h_inst[x], &Y = b->h_inst[y];
      if (X.n != Y.n) return X.n > Y.n;
      if (X.m != Y.m) return X.m > Y.m;
      return X.T > Y.T;
    });
  }
  std::vector<int32_t> items;
  std::vector<int32_t> pend;
  auto flush = [&]() {
    if (pend.empty()) return;
    items.push_back(1);
    for (int q = 0; q < 4; ++q) items.push_back(q < (int)pend.size() ? pend[q] : -1);
    pend.clear();
  };
  // a workgroup holds at most wg/64 one-wavefront instances
  const int pack = std::min(pl.pack1, b->wg / 64);
  for (int32_t i : ids) {
    const int G = (b->h_inst[i].T + 63) / 64;
    if (G == 1) {
      pend.push_back(i);
      if ((int)pend.size() == pack) flush();
    } else {
      items.push_back(G);
      items.push_back(i);
      items.push_back(-1);
      items.push_back(-1);
      items.push_back(-1);
    }
  }
  flush();
  b->n_items = (int32_t)(items.size() / 5);
  ADMM_HIP(hipMemcpy(b->d_items, items.data(), items.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  b->plan = pl;
  return ADMM_OK;
}

admm_status launch_solve(admm_mpc_batch* b, const float* x0, const float* zinit, const float* uinit,
                         float tol, int32_t max_iter, float* zout, float* uout, int32_t* iters,
                         hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  reset_counter_kernel<<<1, 64, 0, st>>>(b->d_counter);
  SolveArgs a;
  a.inst = b->d_inst;
  a.par = b->d_par;
  a.x0 = x0;
  a.zinit = zinit;
  a.uinit = uinit;
  a.zout = zout;
  a.uout = uout;
  a.iters = iters;
  a.items = b->d_items;
  a.n_items = b->n_items;
  a.counter = b->d_counter;
  a.tol = tol;
  a.max_iter = max_iter;
  a.rho = (float)b->rho;
  int grid = b->plan.grid > 0 ? b->plan.grid : b->resident;
  grid = std::max(1, std::min(grid, b->n_items));
  hipExtLaunchKernelGGL(b->wg == WGS ? mpc_solve_kernel<WGS> : mpc_solve_kernel<WGT>, dim3(grid),
                        dim3(b->wg), 0, st, e0, e1, 0,
                        (const MpcInst*)a.inst, a.par, a.x0, a.zinit, a.uinit, a.zout, a.uout,
                        a.iters, a.items, a.n_items, a.counter, a.tol, a.max_iter, a.rho);
  ADMM_HIP(hipGetLastError());
  return ADMM_OK;
}

}  // namespace

extern "C" {

admm_status admm_mpc_batch_create(int32_t n_inst, const int32_t* T, const int32_t* n,
                                  const int32_t* m, const double* A, const double* B,
                                  const double* q, const double* r, const double* u_box,
                                  double rho, int32_t device, admm_mpc_batch** out) {
  admmi::clear_err();
  if (!out) return admmi::set_err(ADMM_E_ARG, "out is NULL");
  *out = nullptr;
  if (n_inst < 1 || !T || !n || !m || !A || !B || !q || !r || !u_box)
    return admmi::set_err(ADMM_E_ARG, "NULL array or n_inst < 1");
  if (!(rho > 0.0)) return admmi::set_err(ADMM_E_ARG, "rho must be > 0");
  for (int32_t i = 0; i < n_inst; ++i) {
    if (T[i] < 1 || n[i] < 1 || m[i] < 1) return admmi::set_err(ADMM_E_ARG, "instance %d: T, n, m must be >= 1", i);
    if (T[i] > TMAX || n[i] > MN || m[i] > MM)
      return admmi::set_err(ADMM_E_UNSUPPORTED, "instance %d: needs T <= %d, n <= %d, m <= %d", i, TMAX, MN, MM);
  }
  std::unique_ptr<admm_mpc_batch> b(new admm_mpc_batch());
  b->device = device;
  b->n_inst = n_inst;
  b->rho = rho;
  std::vector<float> par;
  int64_t aoff = 0, boff = 0, qoff = 0, roff = 0;
  for (int32_t i = 0; i < n_inst; ++i) {
    const int ni = n[i], mi = m[i], ki = ni + mi;
    MpcInst I{};
    I.T = T[i];
    I.n = ni;
    I.m = mi;
    I.box = u_box[i] > 0.0 ? 1 : 0;
    I.par_off = (int32_t)par.size();
    I.x0_off = (int32_t)b->x0_total;
    I.z_off = b->z_total;
    I.u_off = b->u_total;
    b->x0_total += ni;
    b->z_total += (int64_t)T[i] * ki;
    b->u_total += (int64_t)T[i] * 3 * ki;
    const double* Ai = A + aoff;
    const double* Bi = B + boff;
    const double* qi = q + qoff;
    const double* ri = r + roff;
    aoff += ni * ni;
    boff += ni * mi;
    qoff += ni;
    roff += mi;
    const int Np = pad_n(ni);
    const ParOff o = par_offsets(Np);
    std::vector<double> blk(o.size, 0.0);
    for (int rr = 0; rr < ni; ++rr) {
      for (int j = 0; j < ni; ++j) {
        blk[o.M + rr * o.K4 + j] = Ai[rr * ni + j];
        blk[o.MT + j * o.N4 + rr] = Ai[rr * ni + j];
      }
      for (int j = 0; j < mi; ++j) {
        blk[o.M + rr * o.K4 + o.N4 + j] = Bi[rr * mi + j];
        blk[o.MT + (o.N4 + j) * o.N4 + rr] = Bi[rr * mi + j];
      }
    }
    std::vector<double> G(ni * ni, 0.0), G0(ni * ni, 0.0);
    for (int a1 = 0; a1 < ni; ++a1)
      for (int a2 = 0; a2 < ni; ++a2) {
        double s = (a1 == a2) ? 1.0 : 0.0, s0 = s;
        for (int j = 0; j < ni; ++j) s += Ai[a1 * ni + j] * Ai[a2 * ni + j];
        for (int j = 0; j < mi; ++j) {
          s += Bi[a1 * mi + j] * Bi[a2 * mi + j];
          s0 += Bi[a1 * mi + j] * Bi[a2 * mi + j];
        }
        G[a1 * ni + a2] = s;
        G0[a1 * ni + a2] = s0;
      }
    std::vector<double> S = inv_spd(G, ni), S0 = inv_spd(G0, ni);
    for (int a1 = 0; a1 < ni; ++a1)
      for (int a2 = 0; a2 < ni; ++a2) {
        blk[o.S + a1 * o.N4 + a2] = S[a1 * ni + a2];
        blk[o.S0 + a1 * o.N4 + a2] = S0[a1 * ni + a2];
        blk[o.A + a1 * Np + a2] = Ai[a1 * ni + a2];
      }
    for (int a1 = 0; a1 < ni; ++a1)
      for (int j = 0; j < mi; ++j) blk[o.B + a1 * MM + j] = Bi[a1 * mi + j];
    for (int j = 0; j < ni; ++j) {
      if (qi[j] < 0.0) return admmi::set_err(ADMM_E_ARG, "instance %d: q must be >= 0", i);
      blk[o.cq + j] = rho / (rho + qi[j]);
      blk[o.q + j] = qi[j];
    }
    for (int j = 0; j < mi; ++j) {
      if (ri[j] < 0.0) return admmi::set_err(ADMM_E_ARG, "instance %d: r must be >= 0", i);
      blk[o.cr + j] = rho / (rho + ri[j]);
      blk[o.r + j] = ri[j];
    }
    blk[o.lo] = u_box[i] > 0.0 ? -u_box[i] : -INFINITY;
    blk[o.lo + 1] = u_box[i] > 0.0 ? u_box[i] : INFINITY;
    for (double v : blk) par.push_back((float)v);
    b->h_inst.push_back(I);
  }
  if (par.size() > 0x7fffffffULL) return admmi::set_err(ADMM_E_UNSUPPORTED, "batch parameters too large");
  if (admm_status s = admmi::probe_device(device)) return s;
  ADMM_HIP(hipSetDevice(device));
  admm_status s;
  if ((s = mpc_alloc(b.get(), (void**)&b->d_inst, sizeof(MpcInst) * n_inst))) return s;
  if ((s = mpc_alloc(b.get(), (void**)&b->d_par, sizeof(float) * par.size()))) return s;
  if ((s = mpc_alloc(b.get(), (void**)&b->d_u, sizeof(float) * b->u_total))) return s;
  if ((s = mpc_alloc(b.get(), (void**)&b->d_items, sizeof(int32_t) * 5 * (size_t)n_inst))) return s;
  if ((s = mpc_alloc(b.get(), (void**)&b->d_counter, sizeof(int32_t)))) return s;
  ADMM_HIP(hipMemcpy(b->d_inst, b->h_inst.data(), sizeof(MpcInst) * n_inst, hipMemcpyHostToDevice));
  ADMM_HIP(hipMemcpy(b->d_par, par.data(), sizeof(float) * par.size(), hipMemcpyHostToDevice));
  int per_cu = 0, cus = 0;
  int maxT = 0;
  for (int32_t i = 0; i < n_inst; ++i) maxT = std::max(maxT, (int)T[i]);
  b->wg = maxT <= WGS ? WGS : WGT;
  if (b->wg == WGS)
    ADMM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mpc_solve_kernel<WGS>, WGS, 0));
  else
    ADMM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mpc_solve_kernel<WGT>, WGT, 0));
  ADMM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  b->resident = std::max(1, per_cu) * std::max(1, cus);
  if ((s = build_items(b.get(), Plan()))) return s;
  *out = b.release();
  return ADMM_OK;
}

admm_status admm_mpc_batch_sizes(const admm_mpc_batch* b, int64_t* z_total, int64_t* u_total,
                                 int64_t* x0_total) {
  admmi::clear_err();
  if (!b) return admmi::set_err(ADMM_E_ARG, "batch is NULL");
  if (z_total) *z_total = b->z_total;
  if (u_total) *u_total = b->u_total;
  if (x0_total) *x0_total = b->x0_total;
  return ADMM_OK;
}

admm_status admm_mpc_batch_dual_complete(admm_mpc_batch* b, const float* z, float* u, void* stream) {
  admmi::clear_err();
  if (!b || !z || !u) return admmi::set_err(ADMM_E_ARG, "NULL argument");
  ADMM_HIP(hipSetDevice(b->device));
  mpc_dual_kernel<<<(b->n_inst + 3) / 4, 64, 0, (hipStream_t)stream>>>(b->d_inst, b->n_inst, b->d_par, z, u,
                                                              (float)(1.0 / b->rho));
  ADMM_HIP(hipGetLastError());
  return ADMM_OK;
}

admm_status admm_mpc_batch_solve(admm_mpc_batch* b, const float* x0, const float* z_init,
                                 int32_t dual_mode, float tol, int32_t max_iter, float* z_out,
                                 int32_t* iters_out, void* stream) {
  admmi::clear_err();
  if (!b || !x0 || !z_out || !iters_out) return admmi::set_err(ADMM_E_ARG, "NULL argument");
  if (max_iter < 1 || !(tol > 0.f)) return admmi::set_err(ADMM_E_ARG, "need max_iter >= 1 and tol > 0");
  if (dual_mode != 0 && dual_mode != 1) return admmi::set_err(ADMM_E_ARG, "dual_mode must be 0 or 1");
  if (dual_mode == 1 && !z_init) return admmi::set_err(ADMM_E_ARG, "dual completion needs z_init");
  ADMM_HIP(hipSetDevice(b->device));
  hipStream_t st = (hipStream_t)stream;
  const float* uinit = nullptr;
  if (dual_mode == 1) {
    mpc_dual_kernel<<<(b->n_inst + 3) / 4, 64, 0, st>>>(b->d_inst, b->n_inst, b->d_par, z_init, b->d_u,
                                                          (float)(1.0 / b->rho));
    ADMM_HIP(hipGetLastError());
    uinit = b->d_u;
  }
  return launch_solve(b, x0, z_init, uinit, tol, max_iter, z_out, nullptr, iters_out, st, nullptr,
                      nullptr);
}

admm_status admm_mpc_batch_solve_state(admm_mpc_batch* b, const float* x0, const float* z_init,
                                       const float* u_init, float tol, int32_t max_iter,
                                       float* z_out, float* u_out, int32_t* iters_out,
                                       void* stream) {
  admmi::clear_err();
  if (!b || !x0 || !z_out || !iters_out) return admmi::set_err(ADMM_E_ARG, "NULL argument");
  if (max_iter < 1 || !(tol > 0.f)) return admmi::set_err(ADMM_E_ARG, "need max_iter >= 1 and tol > 0");
  if (u_init && !z_init) return admmi::set_err(ADMM_E_ARG, "u_init needs z_init");
  if (u_out && (u_out == u_init)) return admmi::set_err(ADMM_E_ARG, "u_out must not be u_init");
  if (z_out == z_init) return admmi::set_err(ADMM_E_ARG, "z_out must not be z_init");
  ADMM_HIP(hipSetDevice(b->device));
  return launch_solve(b, x0, z_init, u_init, tol, max_iter, z_out, u_out, iters_out,
                      (hipStream_t)stream, nullptr, nullptr);
}

admm_status admm_mpc_batch_shift(admm_mpc_batch* b, const float* x0, const float* z, const float* u,
                                 const float* w, float* x0_next, float* z_next, float* u_next,
                                 void* stream) {
  admmi::clear_err();
  if (!b || !x0 || !z || !x0_next) return admmi::set_err(ADMM_E_ARG, "NULL argument");
  if ((u == nullptr) != (u_next == nullptr)) return admmi::set_err(ADMM_E_ARG, "u and u_next go together");
  if (x0_next == x0 || (z_next && z_next == z) || (u_next && u_next == u))
    return admmi::set_err(ADMM_E_ARG, "outputs must not overlap the inputs");
  ADMM_HIP(hipSetDevice(b->device));
  mpc_shift_kernel<<<b->n_inst, WGT, 0, (hipStream_t)stream>>>(b->d_inst, b->d_par, x0, z, u, w,
                                                              x0_next, z_next, u_next);
  ADMM_HIP(hipGetLastError());
  return ADMM_OK;
}

admm_status admm_mpc_batch_set_plan(admm_mpc_batch* b, int32_t pack1, int32_t order, int32_t grid) {
  admmi::clear_err();
  if (!b) return admmi::set_err(ADMM_E_ARG, "batch is NULL");
  if ((pack1 != 1 && pack1 != 2 && pack1 != 4) || order < 0 || order > 3 || grid < 0)
    return admmi::set_err(ADMM_E_ARG, "bad plan");
  ADMM_HIP(hipSetDevice(b->device));
  Plan p;
  p.pack1 = pack1;
  p.order = order;
  p.grid = grid;
  return build_items(b, p);
}

admm_status admm_mpc_batch_get_plan(const admm_mpc_batch* b, int32_t* pack1, int32_t* order,
                                    int32_t* grid, int32_t* resident) {
  admmi::clear_err();
  if (!b) return admmi::set_err(ADMM_E_ARG, "batch is NULL");
  if (pack1) *pack1 = b->plan.pack1;
  if (order) *order = b->plan.order;
  if (grid) *grid = b->plan.grid;
  if (resident) *resident = b->resident;
  return ADMM_OK;
}

admm_status admm_mpc_batch_tune(admm_mpc_batch* b, const float* x0, float tol, int32_t max_iter,
                                float* z_scratch, int32_t* iters_scratch, int32_t reps,
                                float* times_ms, int32_t max_candidates, int32_t* n_candidates,
                                void* stream) {
  admmi::clear_err();
  if (!b || !x0 || !z_scratch || !iters_scratch) return admmi::set_err(ADMM_E_ARG, "NULL argument");
  ADMM_HIP(hipSetDevice(b->device));
  hipStream_t st = (hipStream_t)stream;
  // one cold solve first: its iteration counts drive the measured order
  {
    admm_status s = build_items(b, Plan());
    if (s) return s;
    s = launch_solve(b, x0, nullptr, nullptr, tol, max_iter, z_scratch, nullptr, iters_scratch, st,
                     nullptr, nullptr);
    if (s) return s;
    b->measured.assign(b->n_inst, 0);
    ADMM_HIP(hipMemcpyAsync(b->measured.data(), iters_scratch, sizeof(int32_t) * b->n_inst,
                            hipMemcpyDeviceToHost, st));
    ADMM_HIP(hipStreamSynchronize(st));
  }
  std::vector<Plan> cands;
  for (int pack : {4, 2, 1})
    for (int order : {1, 2, 3})
      for (int gmul : {0, 1}) {
        Plan p;
        p.pack1 = pack;
        p.order = order;
        p.grid = gmul == 0 ? 0 : b->n_inst;  // resident set, or one workgroup per item
        cands.push_back(p);
      }
  hipEvent_t e0, e1;
  ADMM_HIP(hipEventCreate(&e0));
  ADMM_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  Plan bestp = b->plan;
  int nc = 0;
  for (const Plan& p : cands) {
    admm_status s = build_items(b, p);
    if (s) { hipEventDestroy(e0); hipEventDestroy(e1); return s; }
    float tmin = 1e30f;
    for (int rep = 0; rep < std::max(1, reps); ++rep) {
      s = launch_solve(b, x0, nullptr, nullptr, tol, max_iter, z_scratch, nullptr, iters_scratch, st,
                       e0, e1);
      if (s) { hipEventDestroy(e0); hipEventDestroy(e1); return s; }
      hipError_t he = hipEventSynchronize(e1);
      if (he != hipSuccess) { hipEventDestroy(e0); hipEventDestroy(e1); ADMM_HIP(he); }
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      tmin = std::min(tmin, ms);
    }
    if (times_ms && nc < max_candidates) times_ms[nc] = tmin;
    ++nc;
    if (tmin < best) { best = tmin; bestp = p; }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (n_candidates) *n_candidates = nc;
  return build_items(b, bestp);
}

admm_status admm_mpc_batch_destroy(admm_mpc_batch* b) {
  admmi::clear_err();
  delete b;
  return ADMM_OK;
}

}  // extern "C"
