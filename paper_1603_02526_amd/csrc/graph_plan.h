// Host-side plan of a finalized graph and the interface of the per-precision
// device engines (graph.hip builds the plan; engine_f32.hip and
// engine_f64.hip instantiate the engine for one working precision each).
#pragma once

#include <cstdint>
#include <vector>

#include "graph_kernels.h"

namespace admmg {

// Host layout of a finalized graph (precision independent).
struct Plan {
  std::vector<BucketDesc> bt;
  std::vector<int32_t> idx;
  std::vector<double> par;
  int64_t n_zc = 0, n_m = 0;    // contribution buffer and m-region element counts
  int64_t zc_span = 0;          // contribution region incl. padding, rounded up to 64
  int64_t w_stride = 0;         // medium z lists: fixed stride (0: explicit ranges)
  int64_t w_base = 0, l_base = 0;  // medium / short z lists: first pool position
  std::vector<int32_t> var_b, var_w, var_l;   // z lists: long, medium, short
  std::vector<int64_t> rng_b, rng_w;
  std::vector<double> deg_b, deg_w, deg_l;  // per z list: sum of its edges' rho / graph rho
  // Transposed lists of the scalars of pair-tile entities (64-row tiles):
  // contribution j of list k at t_base + j * n_t + k, so that the 192
  // partials a tile writes for one entity block are contiguous.
  std::vector<int32_t> var_t;
  std::vector<double> deg_t;
  int64_t t_base = 0;
  int32_t t_len = 0;
  int32_t t_lpb = 32;           // transposed lists per z-pass block
  bool weighted = false;        // groups with different rho: weighted z-sums
  std::vector<double> wz;       // weighted: relative rho of every contribution position
  std::vector<double> rmz;      // weighted: per z scalar, the largest rho of its edges
  bool alpha_one = true;        // every edge has alpha = 1 (m-only state)
  std::vector<double> ualpha;   // groups with different alpha: alpha per user slot
  std::vector<int64_t> upos;    // user slot -> pool position of m
  std::vector<int32_t> uz;      // user slot -> z index
  int64_t xblocks = 0;
  int64_t algo_bytes = 0, layout_bytes = 0;  // per iteration, in T units x sizeof later
  int64_t algo_elems = 0, layout_idx_bytes = 0, layout_elems = 0;
  int64_t n_pair_tiles = 0;
  int64_t n_flags = 0;          // sparse pair-state flag words (NT per tile)
  bool no_tiles = false;        // input: build no dense pair tiles
  bool resident = false;        // output of finalize: resident driver chosen
};

struct EngineBase {
  int32_t graph_block = 0;  // graph driver: iterations per recorded block (0: launches)
  bool twa = false;         // three-weight variant (set before upload)
  virtual ~EngineBase() {}
  // Whether the resident driver can run this plan on the device (LDS image
  // plus the kernel's static LDS within the per-workgroup limit).
  virtual admm_status resident_check(const Plan& p, int64_t nz, bool alpha1) = 0;
  virtual admm_status upload(const Plan& p, const std::vector<double>& z0, double rho,
                             double alpha) = 0;
  virtual admm_status set_state(const double* z, const double* u, hipStream_t s) = 0;
  virtual admm_status run(int32_t iters, hipStream_t s) = 0;
  virtual admm_status run_profiled(int32_t iters, hipStream_t s, double* x_ms, double* z_ms) = 0;
  virtual admm_status get_z(double* z, hipStream_t s) = 0;
  virtual admm_status get_slots(double* out, int which, hipStream_t s) = 0;
  virtual admm_status residuals(double* r, double* s, hipStream_t st) = 0;
  virtual void* z_ptr() = 0;
};

// Pass blocks of the z-update and bytes of the resident driver's LDS image.
int64_t zpass_blocks(const Plan& P);
int64_t resident_image_bytes(const Plan& P, int64_t nz, int64_t es);

// Engines for one working precision on `device` (caller owns the result).
EngineBase* make_engine_f32(int device);
EngineBase* make_engine_f64(int device);

}  // namespace admmg
