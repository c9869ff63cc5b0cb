// Internal helpers shared by the library's translation units: error
// reporting across the C ABI and wavefront reductions for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "admm.h"

namespace admmi {

admm_status set_err(admm_status s, const char* fmt, ...);
void clear_err();

// Returns ADMM_OK when a GPU is usable, else ADMM_E_NO_DEVICE.
admm_status probe_device(int device);

#define ADMM_HIP(expr)                                                      \
  do {                                                                      \
    hipError_t e__ = (expr);                                                \
    if (e__ != hipSuccess)                                                  \
      return ::admmi::set_err(e__ == hipErrorOutOfMemory ? ADMM_E_OOM       \
                                                         : ADMM_E_HIP,      \
                              "%s: %s (%s:%d)", #expr,                      \
                              hipGetErrorString(e__), __FILE__, __LINE__);  \
  } while (0)

// ---------------------------------------------------------------------------
// Wavefront sums with a fixed combination order (bitwise reproducible).
// fp32: DPP butterfly inside each 16-lane row, then row broadcasts; the
// total is read from lane 63 and returned in every lane.
// fp64: xor-butterfly through ds_bpermute; a + b == b + a exactly, so every
// lane ends with the same bits.
// Every lane of the wavefront must be active at the call.
// ---------------------------------------------------------------------------
#define ADMM_DPP(v, ctrl, rowmask)                                              \
  __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), (ctrl),     \
                                             (rowmask), 0xF, false))

__device__ __forceinline__ float wave_sum(float v) {
  v += ADMM_DPP(v, 0xB1, 0xF);   // quad_perm [1,0,3,2]: pairs
  v += ADMM_DPP(v, 0x4E, 0xF);   // quad_perm [2,3,0,1]: quads
  v += ADMM_DPP(v, 0x141, 0xF);  // row_half_mirror: 8 lanes
  v += ADMM_DPP(v, 0x140, 0xF);  // row_mirror: 16 lanes (whole row)
  v += ADMM_DPP(v, 0x142, 0xA);  // row_bcast:15 into rows 1 and 3
  v += ADMM_DPP(v, 0x143, 0xC);  // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Max over the wavefront of non-negative values, DPP only (lanes a row
// mask leaves out read 0, which cannot exceed the max); every lane returns
// the result.  Every lane of the wavefront must be active at the call.
__device__ __forceinline__ float wave_max_nonneg(float v) {
  v = fmaxf(v, ADMM_DPP(v, 0xB1, 0xF));   // pairs
  v = fmaxf(v, ADMM_DPP(v, 0x4E, 0xF));   // quads
  v = fmaxf(v, ADMM_DPP(v, 0x141, 0xF));  // 8 lanes
  v = fmaxf(v, ADMM_DPP(v, 0x140, 0xF));  // 16 lanes
  v = fmaxf(v, ADMM_DPP(v, 0x142, 0xA));  // row_bcast:15 into rows 1 and 3
  v = fmaxf(v, ADMM_DPP(v, 0x143, 0xC));  // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Sum over each 16-lane row (DPP row), result in every lane of the row.
__device__ __forceinline__ float row16_sum(float v) {
  v += ADMM_DPP(v, 0xB1, 0xF);   // pairs
  v += ADMM_DPP(v, 0x4E, 0xF);   // quads
  v += ADMM_DPP(v, 0x141, 0xF);  // 8 lanes
  v += ADMM_DPP(v, 0x140, 0xF);  // 16 lanes
  return v;
}

__device__ __forceinline__ double row16_sum(double v) {
#pragma unroll
  for (int k = 8; k >= 1; k >>= 1) v += __shfl_xor(v, k, 16);
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) v += __shfl_xor(v, k, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) {
    T o = __shfl_xor(v, k, 64);
    v = o > v ? o : v;
  }
  return v;
}

}  // namespace admmi
