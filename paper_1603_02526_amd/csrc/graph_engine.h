// Device engine of the factor-graph ADMM for one working precision: owns
// the device buffers of a finalized graph and enqueues the x-pass and
// z-pass kernels of graph_kernels.h (launches, recorded iteration blocks,
// or the resident driver).  Instantiated once per precision in
// engine_f32.hip and engine_f64.hip.
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

#include <hip/hip_ext.h>

#include "graph_plan.h"

namespace admmg {

// ---------------------------------------------------------------------------
// Device engine for one working precision.
// ---------------------------------------------------------------------------
template <typename T>
struct Engine : EngineBase {
  int device = 0;
  bool alpha1 = true;
  T alpha = T(1), inv_rho = T(1);
  int nb = 0;
  int fs = FS_ALL;  // x-pass feature set
  BTab btab{};      // the bucket table as a kernel argument (first XB_INLINE buckets)
  int64_t xblocks = 0, zblocks = 0, nb_w = 0, n_w = 0, n_l = 0, n_slots = 0, nz = 0, xdelta = 0;
  int64_t n_b = 0;
  int64_t w_stride = 0, w_base = 0, l_base = 0;
  int32_t *var_b = nullptr;
  int64_t* rng_b = nullptr;
  T* deg_b = nullptr;
  bool resident = false;
  uint16_t* flags = nullptr;
  int64_t n_flags = 0;
  ResArgs<T> ra{};
  size_t res_lds = 0;
  T* pool = nullptr;
  T* par = nullptr;
  int32_t* idx = nullptr;
  BucketDesc* bt = nullptr;
  T* z[2] = {nullptr, nullptr};
  int zc = 0;
  int32_t *var_w = nullptr, *var_l = nullptr;
  int64_t* rng_w = nullptr;
  T *deg_w = nullptr, *deg_l = nullptr;
  int64_t* upos = nullptr;
  int32_t* uz = nullptr;
  T *bmx = nullptr, *bmz = nullptr;
  bool weighted = false;           // groups with different rho
  T* ualpha = nullptr;             // groups with different alpha: alpha per user slot
  T *wz = nullptr, *rmz = nullptr;  // weighted: rho per contribution position, largest rho per z
  double* io = nullptr;
  int64_t io_n = 0;
  bool have_resid = false;
  int32_t* var_t = nullptr;     // transposed z lists (pair-tile entities)
  T* deg_t = nullptr;
  int64_t n_t = 0, t_base = 0;
  int32_t t_len = 0, t_lpb = 64;
  T* wc = nullptr;              // three-weight variant: weight per contribution position
  uint8_t* zfree = nullptr;     // three-weight variant: per z scalar, no edge weighted
  uint8_t* twb = nullptr;       // three-weight variant: per constraint factor, sent rho
  int64_t n_twb = 0;
  bool numeric_fail = false;  // sticky until the next state import
  std::vector<void*> allocs;

  ~Engine() override {
    hipSetDevice(device);
    for (hipGraphExec_t& e : gexec)
      if (e) hipGraphExecDestroy(e);
    if (cap) hipStreamDestroy(cap);
    for (void* p : allocs) hipFree(p);
  }

  template <typename U>
  admm_status alloc(U** p, int64_t n) {
    *p = nullptr;
    const size_t bytes = (size_t)std::max<int64_t>(n, 1) * sizeof(U);
    ADMM_HIP(hipMalloc((void**)p, bytes));
    allocs.push_back(*p);
    return ADMM_OK;
  }

  template <typename U>
  admm_status put(U** p, const std::vector<U>& v) {
    admm_status s = alloc(p, (int64_t)v.size());
    if (s) return s;
    if (!v.empty()) ADMM_HIP(hipMemcpy(*p, v.data(), v.size() * sizeof(U), hipMemcpyHostToDevice));
    return ADMM_OK;
  }

  admm_status put_conv(T** p, const std::vector<double>& v) {
    std::vector<T> t(v.begin(), v.end());
    return put(p, t);
  }

  template <bool A1>
  static const void* resident_fn() {
    return reinterpret_cast<const void*>(&resident_kernel<T, A1>);
  }

  admm_status resident_check(const Plan& P, int64_t nz_, bool a1) override {
    const int64_t bytes = resident_image_bytes(P, nz_, (int64_t)sizeof(T));
    hipFuncAttributes fa;
    ADMM_HIP(hipFuncGetAttributes(&fa, a1 ? resident_fn<true>() : resident_fn<false>()));
    int maxsh = 0;
    ADMM_HIP(hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    if ((int64_t)fa.sharedSizeBytes + bytes > (int64_t)maxsh)
      return admmi::set_err(ADMM_E_UNSUPPORTED,
                            "resident driver: LDS image %lld B + static %zu B exceeds %d B",
                            (long long)bytes, (size_t)fa.sharedSizeBytes, maxsh);
    if (bytes > 64 * 1024) {
      ADMM_HIP(hipFuncSetAttribute(a1 ? resident_fn<true>() : resident_fn<false>(),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    }
    return ADMM_OK;
  }

  // Region table and LDS offsets of the resident driver (same order and
  // rounding as resident_image_bytes).
  void resident_layout() {
    ResArgs<T>& r = ra;
    r = ResArgs<T>{};
    int32_t off = 0;
    auto add = [&](const void* src, void* back, int64_t bytes) {
      const int32_t o = off;
      if (bytes > 0) {
        ResRegion& q = r.reg[r.nreg++];
        q.src = src;
        q.back = back;
        q.off = o;
        q.words = (int32_t)(bytes / 4);
      }
      off += (int32_t)((bytes + 15) / 16 * 16);
      return o;
    };
    const int64_t es = (int64_t)sizeof(T);
    r.o_pool = add(pool, pool, pool_n * es);
    r.o_z0 = add(z[0], nullptr, nz * es);
    r.o_z1 = add(z[1], nullptr, nz * es);
    r.o_par = add(par, nullptr, par_n * es);
    r.o_idx = add(idx, nullptr, idx_n * 4);
    r.o_var_b = add(var_b, nullptr, n_b * 4);
    r.o_rng_b = add(rng_b, nullptr, n_b * 16);
    r.o_deg_b = add(deg_b, nullptr, n_b * es);
    r.o_var_w = add(var_w, nullptr, n_w * 4);
    r.o_rng_w = add(rng_w, nullptr, w_stride ? 0 : n_w * 16);
    r.o_deg_w = add(deg_w, nullptr, n_w * es);
    r.o_var_l = add(var_l, nullptr, n_l * 4);
    r.o_deg_l = add(deg_l, nullptr, n_l * es);
    r.o_bt = add(bt, nullptr, (int64_t)nb * (int64_t)sizeof(BucketDesc));
    r.xblocks = (int32_t)xblocks;
    r.zblocks = (int32_t)zblocks;
    r.z_words = (int32_t)(nz * es / 4);
    r.z_back[0] = z[0];
    r.z_back[1] = z[1];
    res_lds = (size_t)off;
  }

  int64_t pool_n = 0, par_n = 0, idx_n = 0;

  admm_status upload(const Plan& P, const std::vector<double>& z0, double rho,
                     double alpha_) override {
    alpha1 = P.alpha_one;
    (void)alpha_;
    alpha = (T)alpha_;
    inv_rho = (T)(1.0 / rho);
    nb = (int)P.bt.size();
    xblocks = P.xblocks;
    {
      int need = 0;
      for (const BucketDesc& b : P.bt) {
        if (b.mode == BM_PAIR) need |= b.sparse ? FT_PAIRSP : FT_PAIR;
        else if ((b.kind == KD_HINGE || b.kind == KD_MARGIN) && b.dmax == 0) need |= FT_XWIDE;
        else if (b.mode == BM_UNIF_HINGE && b.dmax == 32) need |= FT_UHINGE;
        else if ((b.mode == BM_UNIF_HINGE || b.kind == KD_HINGE || b.kind == KD_MARGIN) &&
                 b.dmax == 64)
          need |= FT_W64;
        else if (b.mode == BM_GEN_SLOT || b.kind == KD_NONOVERLAP || b.kind == KD_WALL ||
                 b.kind == KD_EQUAL)
          need |= FT_GEN;
        else if (b.kind == KD_HINGE || b.kind == KD_MARGIN) need |= FT_WIDE;
        else need |= FT_LINDYN;
      }
      if (twa) need |= FT_TWA;
      fs = (need & FT_TWA) ? ((need & FT_PAIRSP) ? FS_PAIRSP_TW : FS_GEN_TW)
           : ((need & ~FS_PAIR) == 0)   ? FS_PAIR
           : ((need & ~FS_PAIRSP) == 0) ? FS_PAIRSP
           : ((need & ~FS_HINGE) == 0)  ? FS_HINGE
           : ((need & ~FS_WIDE) == 0)   ? FS_WIDE
           : ((need & ~FS_DYN) == 0)    ? FS_DYN
           : ((need & ~FS_XW) == 0)     ? FS_XW
           : ((need & ~FS_ALL) == 0)    ? FS_ALL
                                        : FS_ALLX;
    }
    n_b = (int64_t)P.var_b.size();
    w_stride = P.w_stride;
    w_base = P.w_base;
    l_base = P.l_base;
    n_w = (int64_t)P.var_w.size();
    n_l = (int64_t)P.var_l.size();
    nb_w = (n_w + ZPB - 1) / ZPB;
    zblocks = zpass_blocks(P);
    resident = P.resident;
    n_slots = (int64_t)P.upos.size();
    nz = (int64_t)z0.size();
    xdelta = P.n_m;
    admm_status s;
    pool_n = P.zc_span + 2 * P.n_m;
    par_n = (int64_t)P.par.size();
    idx_n = (int64_t)P.idx.size();
    if ((s = alloc(&pool, pool_n))) return s;
    ADMM_HIP(hipMemset(pool, 0, (size_t)std::max<int64_t>(pool_n, 1) * sizeof(T)));
    if ((s = put_conv(&par, P.par))) return s;
    if ((s = put(&idx, P.idx))) return s;
    {
      // three-weight variant: each constraint factor of the general layout
      // keeps one byte (whether it sent weight rho in the last iteration)
      std::vector<BucketDesc> btc = P.bt;
      n_twb = 0;
      for (BucketDesc& b : btc) {
        b.twb_off = n_twb;
        if (twa && b.mode == BM_GEN_FACTOR && (b.kind == KD_NONOVERLAP || b.kind == KD_WALL))
          n_twb += b.n;
      }
      if ((s = put(&bt, btc))) return s;
      btab = BTab{};
      for (size_t i = 0; i < btc.size() && i < (size_t)XB_INLINE; ++i) btab.d[i] = btc[i];
    }
    if ((s = alloc(&z[0], nz))) return s;
    if ((s = alloc(&z[1], nz))) return s;
    n_t = (int64_t)P.var_t.size();
    t_base = P.t_base;
    t_len = P.t_len;
    t_lpb = P.t_lpb;
    if ((s = put(&var_t, P.var_t))) return s;
    if ((s = put_conv(&deg_t, P.deg_t))) return s;
    if ((s = put(&var_b, P.var_b))) return s;
    if ((s = put(&rng_b, P.rng_b))) return s;
    if ((s = put_conv(&deg_b, P.deg_b))) return s;
    if ((s = put(&var_w, P.var_w))) return s;
    if ((s = put(&var_l, P.var_l))) return s;
    if ((s = put(&rng_w, P.rng_w))) return s;
    if ((s = put_conv(&deg_w, P.deg_w))) return s;
    if ((s = put_conv(&deg_l, P.deg_l))) return s;
    if ((s = put(&upos, P.upos))) return s;
    if ((s = put(&uz, P.uz))) return s;
    if (!P.ualpha.empty())
      if ((s = put_conv(&ualpha, P.ualpha))) return s;
    weighted = P.weighted;
    if (weighted) {
      if ((s = put_conv(&wz, P.wz))) return s;
      if ((s = put_conv(&rmz, P.rmz))) return s;
    }
    if ((s = alloc(&bmx, xblocks))) return s;
    if ((s = alloc(&bmz, zblocks))) return s;
    io_n = std::max(n_slots, nz);
    if ((s = alloc(&io, io_n))) return s;
    n_flags = P.n_flags;
    if ((s = alloc(&flags, n_flags))) return s;
    if (twa) {
      // weights written with the contributions; those of separable factors
      // (always weight rho) once here, the others by every x-pass
      std::vector<T> w0((size_t)std::max<int64_t>(P.zc_span, 1), T(0));
      for (const BucketDesc& b : P.bt)
        if (b.mode == BM_GEN_SLOT)
          for (int64_t q = 0; q < b.n; ++q) w0[(size_t)P.idx[b.dst_off + q]] = T(1);
      if ((s = put(&wc, w0))) return s;
      if ((s = alloc(&zfree, nz))) return s;
      if ((s = alloc(&twb, n_twb))) return s;
    }
    if (resident) resident_layout();
    return set_state(z0.data(), nullptr, nullptr);
  }

  admm_status set_state(const double* zh, const double* uh, hipStream_t st) override {
    ADMM_HIP(hipSetDevice(device));
    ADMM_HIP(hipMemcpyAsync(io, zh, nz * sizeof(double), hipMemcpyHostToDevice, st));
    const int64_t gz = (nz + 255) / 256;
    if (gz) convert_kernel<T><<<gz, 256, 0, st>>>(nz, io, z[zc]);
    ADMM_HIP(hipGetLastError());
    if (uh) {
      ADMM_HIP(hipMemcpyAsync(io, uh, n_slots * sizeof(double), hipMemcpyHostToDevice, st));
    }
    const int64_t gs = (n_slots + 255) / 256;
    if (gs)
      set_state_kernel<T><<<gs, 256, 0, st>>>(n_slots, upos, uz, uh ? io : nullptr, z[zc], pool,
                                              xdelta, 1);
    // three-weight variant: a state import starts from weight rho everywhere
    if (zfree && nz)
      fill_kernel<uint8_t><<<(unsigned)((nz + 255) / 256), 256, 0, st>>>(nz, (uint8_t)0, zfree);
    if (twb && n_twb)
      fill_kernel<uint8_t><<<(unsigned)((n_twb + 255) / 256), 256, 0, st>>>(n_twb, (uint8_t)1, twb);
    // every pair's m is explicit in the dense arrays after a state import
    if (n_flags)
      fill_kernel<uint16_t><<<(unsigned)((n_flags + 255) / 256), 256, 0, st>>>(n_flags, (uint16_t)0xFFFF, flags);
    ADMM_HIP(hipGetLastError());
    ADMM_HIP(hipStreamSynchronize(st));
    have_resid = false;
    numeric_fail = false;
    return ADMM_OK;
  }

  XArgs<T> xargs() const {
    XArgs<T> a;
    a.pool = pool;
    a.idx = idx;
    a.par = par;
    a.z = z[zc];
    a.zprev = z[zc ^ 1];
    a.flags = flags;
    a.blockmax = bmx;
    a.wc = wc;
    a.zfree = zfree;
    a.twb = twb;
    a.bt = bt;
    a.nb = nb;
    a.alpha = alpha;
    a.inv_rho = inv_rho;
    return a;
  }

  // Launches take an optional start/stop event pair recorded at the
  // kernel's own begin and end (hipExtLaunchKernelGGL), used for timing.
  // Plain launches (also what stream capture records) unless an event pair
  // is asked for.
  template <typename K, typename... A>
  static void launch(K kern, dim3 g, hipStream_t st, hipEvent_t e0, hipEvent_t e1, const A&... a) {
    if (e0 || e1)
      hipExtLaunchKernelGGL(kern, g, dim3(NT), 0, st, e0, e1, 0, a...);
    else
      hipLaunchKernelGGL(kern, g, dim3(NT), 0, st, a...);
  }

  template <bool A1, int FS>
  void launch_x_fs(int mode, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    XArgs<T> a = xargs();
    const dim3 g((unsigned)xblocks);
    if (mode == PM_NORMAL)
      launch(xpass_kernel<T, A1, PM_NORMAL, FS>, g, st, e0, e1, a, btab);
    else if (mode == PM_SAVE)
      launch(xpass_kernel<T, A1, PM_SAVE, FS>, g, st, e0, e1, a, btab);
    else
      launch(xpass_kernel<T, A1, PM_RESID, FS>, g, st, e0, e1, a, btab);
  }

  template <bool A1>
  void launch_x(int mode, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    if (fs == FS_PAIR) launch_x_fs<A1, FS_PAIR>(mode, st, e0, e1);
    else if (fs == FS_PAIRSP) launch_x_fs<A1, FS_PAIRSP>(mode, st, e0, e1);
    else if (fs == FS_HINGE) launch_x_fs<A1, FS_HINGE>(mode, st, e0, e1);
    else if (fs == FS_WIDE) launch_x_fs<A1, FS_WIDE>(mode, st, e0, e1);
    else if (fs == FS_DYN) launch_x_fs<A1, FS_DYN>(mode, st, e0, e1);
    else if (fs == FS_XW) launch_x_fs<A1, FS_XW>(mode, st, e0, e1);
    else if (fs == FS_ALL) launch_x_fs<A1, FS_ALL>(mode, st, e0, e1);
    else if (fs == FS_ALLX) launch_x_fs<A1, FS_ALLX>(mode, st, e0, e1);
    else if constexpr (A1) {
      // the three-weight variant runs with alpha = 1 only
      if (fs == FS_PAIRSP_TW) launch_x_fs<A1, FS_PAIRSP_TW>(mode, st, e0, e1);
      else launch_x_fs<A1, FS_GEN_TW>(mode, st, e0, e1);
    }
  }

  ZArgs<T> zargs(int check) const {
    ZArgs<T> a;
    a.pool = pool;
    a.var_t = var_t;
    a.deg_t = deg_t;
    a.n_t = n_t;
    a.t_base = t_base;
    a.nb_t = (int32_t)((n_t + t_lpb - 1) / t_lpb);
    a.t_len = t_len;
    a.t_lpb = t_lpb;
    a.var_b = var_b;
    a.rng_b = rng_b;
    a.deg_b = deg_b;
    a.n_b = (int32_t)n_b;
    a.var_w = var_w;
    a.rng_w = rng_w;
    a.deg_w = deg_w;
    a.n_w = n_w;
    a.nb_w = (int32_t)nb_w;
    a.var_l = var_l;
    a.deg_l = deg_l;
    a.n_l = n_l;
    a.w_stride = w_stride;
    a.w_base = w_base;
    a.l_base = l_base;
    a.wz = wz;
    a.rmz = rmz;
    a.zin = z[zc];
    a.zout = z[zc ^ 1];
    a.blockmax = bmz;
    a.check = check;
    a.wc = wc;
    a.zfree = zfree;
    return a;
  }

  void launch_z(int check, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    ZArgs<T> a = zargs(check);
    if (zblocks) launch(zpass_kernel<T>, dim3((unsigned)zblocks), st, e0, e1, a);
    zc ^= 1;
  }

  // Graph driver: graph_block iterations (x-pass, z-pass per iteration,
  // nothing else) recorded once per starting z buffer into a hipGraph and
  // replayed with one graph launch per block.  graph_block is even, so a
  // block leaves z in the buffer it started from and the kernel arguments
  // recorded for that parity hold for every replay.
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};

  admm_status record_block(hipGraphExec_t* out) {
    if (!cap) ADMM_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    ADMM_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    const int zc0 = zc;
    for (int k = 0; k < graph_block; ++k) {
      if (xblocks) {
        if (alpha1) launch_x<true>(PM_NORMAL, cap);
        else launch_x<false>(PM_NORMAL, cap);
      }
      launch_z(0, cap);
    }
    zc = zc0;
    hipGraph_t gr = nullptr;
    const hipError_t le = hipGetLastError();
    const hipError_t ce = hipStreamEndCapture(cap, &gr);
    if (le != hipSuccess || ce != hipSuccess) {
      if (gr) hipGraphDestroy(gr);
      return admmi::set_err(ADMM_E_HIP, "recording the iteration block: %s",
                            hipGetErrorString(le != hipSuccess ? le : ce));
    }
    const hipError_t ie = hipGraphInstantiate(out, gr, nullptr, nullptr, 0);
    hipGraphDestroy(gr);
    if (ie != hipSuccess) {
      *out = nullptr;
      return admmi::set_err(ADMM_E_HIP, "instantiating the iteration block: %s",
                            hipGetErrorString(ie));
    }
    return ADMM_OK;
  }

  // The whole run in one launch of one workgroup (resident driver).
  void launch_resident(int32_t iters, hipStream_t st, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr) {
    ResArgs<T> r = ra;
    r.zc = zc;
    r.iters = iters;
    const XArgs<T> xa = xargs();
    const ZArgs<T> za = zargs(0);
    if (alpha1)
      hipExtLaunchKernelGGL((resident_kernel<T, true>), dim3(1), dim3(NT), res_lds, st, e0, e1, 0,
                            xa, za, r);
    else
      hipExtLaunchKernelGGL((resident_kernel<T, false>), dim3(1), dim3(NT), res_lds, st, e0, e1, 0,
                            xa, za, r);
    if (iters & 1) zc ^= 1;
  }

  admm_status run(int32_t iters, hipStream_t st) override {
    if (iters <= 0) return ADMM_OK;
    ADMM_HIP(hipSetDevice(device));
    if (resident) {
      launch_resident(iters, st);
      ADMM_HIP(hipGetLastError());
      have_resid = true;
      return ADMM_OK;
    }
    int32_t k = 0;
    if (graph_block > 0) {
      // every iteration but the last (which stores x and checks z) in
      // recorded blocks
      while (iters - 1 - k >= graph_block) {
        hipGraphExec_t& ex = gexec[zc];
        if (!ex)
          if (admm_status s = record_block(&ex)) return s;
        ADMM_HIP(hipGraphLaunch(ex, st));
        k += graph_block;
      }
    }
    for (; k < iters; ++k) {
      const bool last = (k == iters - 1);
      if (xblocks) {
        if (alpha1) launch_x<true>(last ? PM_SAVE : PM_NORMAL, st);
        else launch_x<false>(PM_NORMAL, st);
      }
      launch_z(last ? 1 : 0, st);
    }
    if (xblocks) {
      if (alpha1) launch_x<true>(PM_RESID, st);
      else launch_x<false>(PM_RESID, st);
    }
    ADMM_HIP(hipGetLastError());
    have_resid = true;
    return ADMM_OK;
  }

  // Same launches as run(), with an event pair around every kernel; returns
  // the summed x-pass and z-pass durations in milliseconds (synchronises).
  admm_status run_profiled(int32_t iters, hipStream_t st, double* x_ms, double* z_ms) override {
    *x_ms = 0.0;
    *z_ms = 0.0;
    if (iters <= 0) return ADMM_OK;
    ADMM_HIP(hipSetDevice(device));
    if (resident) {
      hipEvent_t e0, e1;
      ADMM_HIP(hipEventCreate(&e0));
      ADMM_HIP(hipEventCreate(&e1));
      launch_resident(iters, st, e0, e1);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      if (e != hipSuccess) return admmi::set_err(ADMM_E_HIP, "profiled run: %s", hipGetErrorString(e));
      *x_ms = ms;
      have_resid = true;
      return ADMM_OK;
    }
    std::vector<hipEvent_t> ev(4 * (size_t)iters);
    for (auto& e : ev) ADMM_HIP(hipEventCreate(&e));
    admm_status rc = ADMM_OK;
    for (int32_t k = 0; k < iters; ++k) {
      const bool last = (k == iters - 1);
      if (xblocks) {
        if (alpha1) launch_x<true>(last ? PM_SAVE : PM_NORMAL, st, ev[4 * k + 0], ev[4 * k + 1]);
        else launch_x<false>(PM_NORMAL, st, ev[4 * k + 0], ev[4 * k + 1]);
      } else {
        hipEventRecord(ev[4 * k + 0], st);
        hipEventRecord(ev[4 * k + 1], st);
      }
      if (zblocks) {
        launch_z(last ? 1 : 0, st, ev[4 * k + 2], ev[4 * k + 3]);
      } else {
        hipEventRecord(ev[4 * k + 2], st);
        launch_z(last ? 1 : 0, st);
        hipEventRecord(ev[4 * k + 3], st);
      }
    }
    if (xblocks) {
      if (alpha1) launch_x<true>(PM_RESID, st);
      else launch_x<false>(PM_RESID, st);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = admmi::set_err(ADMM_E_HIP, "profiled run: %s", hipGetErrorString(e));
    for (int32_t k = 0; rc == ADMM_OK && k < iters; ++k) {
      float a = 0.f, b = 0.f;
      hipEventElapsedTime(&a, ev[4 * k + 0], ev[4 * k + 1]);
      hipEventElapsedTime(&b, ev[4 * k + 2], ev[4 * k + 3]);
      *x_ms += a;
      *z_ms += b;
    }
    for (auto& ee : ev) hipEventDestroy(ee);
    have_resid = (rc == ADMM_OK);
    return rc;
  }

  admm_status get_z(double* out, hipStream_t st) override {
    ADMM_HIP(hipSetDevice(device));
    const int64_t g = (nz + 255) / 256;
    if (g) widen_kernel<T><<<g, 256, 0, st>>>(nz, z[zc], io);
    ADMM_HIP(hipGetLastError());
    ADMM_HIP(hipMemcpyAsync(out, io, nz * sizeof(double), hipMemcpyDeviceToHost, st));
    ADMM_HIP(hipStreamSynchronize(st));
    return ADMM_OK;
  }

  admm_status get_slots(double* out, int which, hipStream_t st) override {
    ADMM_HIP(hipSetDevice(device));
    const int64_t g = (n_slots + 255) / 256;
    if (g) {
      if (alpha1)
        get_slots_kernel<T, true><<<g, 256, 0, st>>>(n_slots, upos, uz, pool, z[zc], xdelta, alpha,
                                                      nullptr, which, io);
      else
        get_slots_kernel<T, false><<<g, 256, 0, st>>>(n_slots, upos, uz, pool, z[zc], xdelta,
                                                       alpha, ualpha, which, io);
    }
    ADMM_HIP(hipGetLastError());
    ADMM_HIP(hipMemcpyAsync(out, io, n_slots * sizeof(double), hipMemcpyDeviceToHost, st));
    ADMM_HIP(hipStreamSynchronize(st));
    return ADMM_OK;
  }

  admm_status residuals(double* r, double* s, hipStream_t st) override {
    if (!have_resid) return admmi::set_err(ADMM_E_STATE, "no iteration has been run since the last state change");
    if (numeric_fail)
      return admmi::set_err(ADMM_E_NUMERIC, "an iterate became NaN or infinite (set a new state)");
    ADMM_HIP(hipSetDevice(device));
    std::vector<T> hx(std::max<int64_t>(xblocks, 1), T(0)), hz(std::max<int64_t>(zblocks, 1), T(0));
    if (xblocks) ADMM_HIP(hipMemcpyAsync(hx.data(), bmx, xblocks * sizeof(T), hipMemcpyDeviceToHost, st));
    if (zblocks) ADMM_HIP(hipMemcpyAsync(hz.data(), bmz, zblocks * sizeof(T), hipMemcpyDeviceToHost, st));
    ADMM_HIP(hipStreamSynchronize(st));
    T a = T(0), b = T(0);
    for (T v : hx) a = std::max(a, v);
    for (T v : hz) b = std::max(b, v);
    *r = (double)a;
    // weighted graphs scale each variable's change by its largest rho in the kernel
    *s = weighted ? (double)b : (double)b / (double)inv_rho;
    // every block maximum turns a NaN into +infinity: a non-finite residual
    // means some x or z of the last iteration is not finite
    if (!std::isfinite(*r) || !std::isfinite(*s)) {
      numeric_fail = true;
      return admmi::set_err(ADMM_E_NUMERIC, "an iterate became NaN or infinite (r = %g, s = %g)",
                            *r, *s);
    }
    return ADMM_OK;
  }

  void* z_ptr() override { return z[zc]; }
};

}  // namespace admmg
