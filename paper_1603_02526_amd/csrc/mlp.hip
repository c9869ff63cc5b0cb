// Small MLP for the learned MPC warm start: y = W3 relu(W2 relu(W1 x + b1) +
// b2) + b3, mean-squared-error loss, Adam.  Every matrix product runs on the
// gfx950 matrix cores (v_mfma_f32_16x16x32_bf16): operands rounded to
// bf16 (round to nearest even) while staged through LDS, products
// accumulated in fp32.  Master weights, activations and gradients are fp32
// in device memory.  Bias, ReLU and the ReLU mask of the backward pass are
// fused into the product epilogues; reductions (loss, bias gradients) use a
// fixed order, so results are deterministic.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <mutex>
#include <vector>

#include "internal.h"

namespace {

typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int GT = 256;  // threads per GEMM workgroup (4 wavefronts)
constexpr int BM = 64, BN = 64, BK = 32;

__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}

enum Epi : int { EPI_PLAIN = 0, EPI_BIAS = 1, EPI_BIAS_RELU = 2, EPI_MASK = 3, EPI_BIAS_AFFINE = 4 };

// C[M x N] = sum_k A(m,k) B(k,n); A(m,k) = TA ? A[k*lda+m] : A[m*lda+k],
// B(k,n) = TB ? B[n*ldb+k] : B[k*ldb+n].  Epilogue per EPI.
// Workgroup tile 64 x 64, each wavefront a 32 x 32 quarter as 2 x 2 MFMA
// tiles of 16 x 16, K consumed 32 at a time through LDS: one gfx950
// v_mfma_f32_16x16x32_bf16 per tile and barrier (lane l holds row or
// column l % 16 and the eight k = 8 (l / 16) .. + 7 of the step).  Split K: workgroup z covers K range [z*kc, (z+1)*kc) and
// writes its partial product to C + z*M*N (plain epilogue only).
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(GT) void gemm_kernel(int M, int N, int K, int kc,
                                                 const float* __restrict__ A, int lda,
                                                 const float* __restrict__ B, int ldb,
                                                 float* __restrict__ C, int ldc,
                                                 const float* __restrict__ bias,
                                                 const float* __restrict__ mask, int ldm,
                                                 const float* __restrict__ mu,
                                                 const float* __restrict__ sd) {
  __shared__ unsigned short As[BM][BK + 4];
  __shared__ unsigned short Bs[BK][BN + 4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int kbeg = blockIdx.z * kc;
  const int kend = min(K, kbeg + kc);
  C += (int64_t)blockIdx.z * M * N;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  // The next K tile is read from global memory into registers while the
  // current one is multiplied from LDS.
  float ra[8], rb[8];
  auto load_tile = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + q * GT;
      int r, c;
      if (TA) { c = e / BM; r = e % BM; } else { r = e / BK; c = e % BK; }
      const int gm = m0 + r, gk = k0 + c;
      ra[q] = (gm < M && gk < kend) ? (TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk]) : 0.f;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + q * GT;
      int r, c;
      if (TB) { c = e / BK; r = e % BK; } else { r = e / BN; c = e % BN; }
      const int gk = k0 + r, gn = n0 + c;
      rb[q] = (gk < kend && gn < N) ? (TB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn]) : 0.f;
    }
  };
  if (kbeg < kend) load_tile(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    // A tile 64 x 32 and B tile 32 x 64: 2048 elements each, 8 per thread
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + q * GT;
      int r, c;
      if (TA) { c = e / BM; r = e % BM; } else { r = e / BK; c = e % BK; }
      As[r][c] = f2bf(ra[q]);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + q * GT;
      int r, c;
      if (TB) { c = e / BK; r = e % BK; } else { r = e / BN; c = e % BN; }
      Bs[r][c] = f2bf(rb[q]);
    }
    __syncthreads();
    if (k0 + BK < kend) load_tile(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      const int kq = kk + (lane >> 4) * 8;
      v8s af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int row = wm + i * 16 + (lane & 15);
#pragma unroll
        for (int j = 0; j < 8; ++j) af[i][j] = (short)As[row][kq + j];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int col = wn + i * 16 + (lane & 15);
#pragma unroll
        for (int j = 0; j < 8; ++j) bf[i][j] = (short)Bs[kq + j][col];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(v8bf, af[i]), __builtin_bit_cast(v8bf, bf[j]), acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn + j * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + wm + i * 16 + (lane >> 4) * 4 + q;
        if (row < M && col < N) {
          float v = acc[i][j][q];
          if (EPI == EPI_BIAS || EPI == EPI_BIAS_RELU || EPI == EPI_BIAS_AFFINE) v += bias[col];
          if (EPI == EPI_BIAS_AFFINE) v = mu[col] + sd[col] * v;
          if (EPI == EPI_BIAS_RELU) v = v > 0.f ? v : 0.f;
          if (EPI == EPI_MASK) v = mask[(int64_t)row * ldm + col] > 0.f ? v : 0.f;
          C[(int64_t)row * ldc + col] = v;
        }
      }
    }
}

// out[i] = sum_{z < nz} ws[z*n + i], z in order (split-K reduction).
__global__ void splitk_sum_kernel(int64_t n, int nz, const float* __restrict__ ws,
                                  float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int z = 0; z < nz; ++z) s += ws[(int64_t)z * n + i];
  out[i] = s;
}

// The same reduction of a [M][N] product followed by the ReLU-mask
// epilogue: out[r][c] = mask[r][c] > 0 ? sum : 0.
__global__ void splitk_sum_mask_kernel(int64_t n, int N, int nz, const float* __restrict__ ws,
                                       const float* __restrict__ mask, int ldm,
                                       float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int z = 0; z < nz; ++z) s += ws[(int64_t)z * n + i];
  const int64_t r = i / N, c = i % N;
  out[i] = mask[r * ldm + c] > 0.f ? s : 0.f;
}

// Loss on normalised outputs: with yh the network's raw output and
// th = (target - mu) / sd per column, dY = 2 (yh - th) / (rows * cols);
// per-block partial sums of (yh - th)^2.
__global__ __launch_bounds__(256) void mse_grad_kernel(int64_t n, int cols, const float* y,
                                                       const float* tg, const float* mu,
                                                       const float* sd, float scale, float* dy,
                                                       float* part) {
  __shared__ float red[256];
  float s = 0.f;
  // n < 2^31 (checked on the host): 32-bit index arithmetic
  const int nn = (int)n;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nn; i += gridDim.x * 256) {
    const int c = i % cols;
    const float d = y[i] - (tg[i] - mu[c]) / sd[c];
    dy[i] = 2.f * d * scale;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Sum of the per-block partials in a fixed order: 64 lanes sum strided
// subsets in order, then lane 0 adds the 64 results in lane order.
__global__ void finish_loss_kernel(int nb, const float* part, float scale, float* loss) {
  __shared__ float r64[64];
  float s = 0.f;
  for (int i = threadIdx.x; i < nb; i += 64) s += part[i];
  r64[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int i = 0; i < 64; ++i) t += r64[i];
    *loss = t * scale;
  }
}

// Per-column statistics of a [rows][cols] array in two deterministic
// stages.  colpart: part[k][c] = sum over the rows of chunk k, in order, of
// (a[r][c] - shift[c])^pw (pw = 1 or 2, shift = 0 when NULL), in FP64.
__global__ void colpart_kernel(int64_t rows, int cols, int64_t chunk, const float* __restrict__ a,
                               const double* __restrict__ shift, int pw,
                               double* __restrict__ part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  const int64_t r0 = (int64_t)blockIdx.y * chunk;
  const int64_t r1 = r0 + chunk < rows ? r0 + chunk : rows;
  const double sh = shift ? shift[c] : 0.0;
  double s = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const double d = (double)a[r * cols + c] - sh;
    s += pw == 1 ? d : d * d;
  }
  part[(int64_t)blockIdx.y * cols + c] = s;
}

// Sums the chunk partials in chunk order.  stage 0: mean (kept in FP64 as
// the shift of the second stage); stage 1: standard deviation, floored.
__global__ void colfinish_kernel(int cols, int nk, int64_t rows, const double* __restrict__ part,
                                 int stage, double* __restrict__ mean_d, float* __restrict__ mu,
                                 float* __restrict__ sd, float sd_min) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int k = 0; k < nk; ++k) s += part[(int64_t)k * cols + c];
  if (stage == 0) {
    const double m = s / (double)rows;
    mean_d[c] = m;
    mu[c] = (float)m;
  } else {
    const double v = sqrt(s / (double)rows);
    sd[c] = (float)(v > sd_min ? v : sd_min);
  }
}

__global__ void fill_kernel(int n, float v, float* a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// Bias gradients db[c] = sum_r dY[r][c] in two deterministic stages:
// colsum_part sums chunks of CS_ROWS rows in order into ws[k][c], and
// splitk_sum_kernel adds the chunks in order.
constexpr int CS_ROWS = 128;
__global__ void colsum_part_kernel(int rows, int cols, const float* __restrict__ dY,
                                   float* __restrict__ ws) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  const int r0 = blockIdx.y * CS_ROWS;
  const int r1 = r0 + CS_ROWS < rows ? r0 + CS_ROWS : rows;
  float s = 0.f;
#pragma unroll 8
  for (int r = r0; r < r1; ++r) s += dY[(int64_t)r * cols + c];
  ws[(int64_t)blockIdx.y * cols + c] = s;
}

// Adam (Kingma and Ba), bias-corrected, on the flat parameter vector.
__global__ void adam_kernel(int64_t n, float* p, const float* g, float* m, float* v, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

// Workspace of admm_mlp_fit_output_scaling_noalloc: a fixed array in device
// memory, one copy per device for the life of the process, shared by every
// call on that device.  Host code uses only its device address, looked up
// once per device with that device current; the symbol itself is a host
// stand-in and is never passed to a kernel or a copy.
constexpr int64_t SCRATCH_DOUBLES = int64_t(1) << 20;   // 8 MiB
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_dev[SCRATCH_MAX_DEVICES] = {};

// Device address of `scratch` on `device` (which must be current).
admm_status scratch_address(int device, double** out) {
  if (device < 0 || device >= SCRATCH_MAX_DEVICES)
    return admmi::set_err(ADMM_E_ARG, "device %d out of range", device);
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[device]) {
    void* p = nullptr;
    ADMM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return admmi::set_err(ADMM_E_HIP, "no device address for the workspace");
    scratch_dev[device] = static_cast<double*>(p);
  }
  *out = scratch_dev[device];
  return ADMM_OK;
}
}  // namespace

struct admm_mlp {
  int device = 0;
  int n_in = 0, hid = 0, n_out = 0, max_batch = 0;
  int64_t n_params = 0;
  int64_t oW1, ob1, oW2, ob2, oW3, ob3;
  float *p = nullptr, *g = nullptr, *am = nullptr, *av = nullptr;
  float *h1 = nullptr, *h2 = nullptr, *y = nullptr, *dy = nullptr, *dh1 = nullptr, *dh2 = nullptr;
  float* part = nullptr;
  float *mu = nullptr, *sd = nullptr;  // fixed output affine y = mu + sd * yhat
  float* ws = nullptr;                 // split-K partial products
  int64_t ws_n = 0;                    // its size in floats
  float* cs = nullptr;                 // bias-gradient chunk sums
  int64_t step = 0;
  std::vector<void*> allocs;
  ~admm_mlp() {
    if (!allocs.empty()) {
      hipSetDevice(device);
      for (void* q : allocs) hipFree(q);
    }
  }
};

namespace {

constexpr int LOSS_BLOCKS = 1024;

admm_status mlp_alloc(admm_mlp* n, float** q, int64_t count) {
  ADMM_HIP(hipMalloc((void**)q, (size_t)std::max<int64_t>(count, 1) * sizeof(float)));
  n->allocs.push_back(*q);
  return ADMM_OK;
}

constexpr int MAX_SPLITS = 32;

template <bool TA, bool TB, int EPI>
void gemm(int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C, int ldc,
          const float* bias, const float* mask, int ldm, hipStream_t st,
          const float* mu = nullptr, const float* sd = nullptr, float* ws = nullptr,
          int64_t ws_n = 0) {
  const int gm = (M + BM - 1) / BM, gn = (N + BN - 1) / BN;
  int splits = 1;
  if ((EPI == EPI_PLAIN || EPI == EPI_MASK) && ws != nullptr && ldc == N) {
    // enough workgroups to fill the device, at least 128 of K per split
    splits = std::max(1, std::min(MAX_SPLITS, std::min((1024 + gm * gn - 1) / (gm * gn), K / 128)));
    splits = (int)std::max<int64_t>(1, std::min<int64_t>(splits, ws_n / ((int64_t)M * N)));
  }
  const int kc = ((K + splits - 1) / splits + BK - 1) / BK * BK;
  splits = (K + kc - 1) / kc;
  dim3 grid(gn, gm, splits);
  if (splits > 1) {
    // plain partial products; the reduction applies the mask
    gemm_kernel<TA, TB, EPI_PLAIN><<<grid, GT, 0, st>>>(M, N, K, kc, A, lda, B, ldb, ws, ldc,
                                                         nullptr, nullptr, 0, nullptr, nullptr);
    const int64_t n = (int64_t)M * N;
    if (EPI == EPI_MASK)
      splitk_sum_mask_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, N, splits, ws, mask,
                                                                          ldm, C);
    else
      splitk_sum_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, splits, ws, C);
  } else {
    gemm_kernel<TA, TB, EPI><<<grid, GT, 0, st>>>(M, N, K, kc, A, lda, B, ldb, C, ldc, bias, mask,
                                                   ldm, mu, sd);
  }
}

void colsum(int rows, int cols, const float* dY, float* db, float* cs, hipStream_t st) {
  const int nk = (rows + CS_ROWS - 1) / CS_ROWS;
  colsum_part_kernel<<<dim3((cols + 255) / 256, nk), 256, 0, st>>>(rows, cols, dY, cs);
  splitk_sum_kernel<<<(cols + 255) / 256, 256, 0, st>>>(cols, nk, cs, db);
}

// forward: h1 = relu(x W1^T + b1), h2 = relu(h1 W2^T + b2),
// yhat = h2 W3^T + b3; with denorm, y = mu + sd * yhat.
void forward(admm_mlp* n, const float* x, int batch, float* y, hipStream_t st, bool denorm) {
  gemm<false, true, EPI_BIAS_RELU>(batch, n->hid, n->n_in, x, n->n_in, n->p + n->oW1, n->n_in, n->h1,
                                   n->hid, n->p + n->ob1, nullptr, 0, st);
  gemm<false, true, EPI_BIAS_RELU>(batch, n->hid, n->hid, n->h1, n->hid, n->p + n->oW2, n->hid, n->h2,
                                   n->hid, n->p + n->ob2, nullptr, 0, st);
  if (denorm)
    gemm<false, true, EPI_BIAS_AFFINE>(batch, n->n_out, n->hid, n->h2, n->hid, n->p + n->oW3,
                                       n->hid, y, n->n_out, n->p + n->ob3, nullptr, 0, st, n->mu,
                                       n->sd);
  else
    gemm<false, true, EPI_BIAS>(batch, n->n_out, n->hid, n->h2, n->hid, n->p + n->oW3, n->hid, y,
                                n->n_out, n->p + n->ob3, nullptr, 0, st);
}

// gradients of mean((y - t)^2) into n->g; loss (device scalar) when non-null
void backward(admm_mlp* n, const float* x, const float* tg, int batch, float* loss, hipStream_t st) {
  forward(n, x, batch, n->y, st, false);
  const int64_t ny = (int64_t)batch * n->n_out;
  const float scale = 1.f / (float)ny;
  mse_grad_kernel<<<LOSS_BLOCKS, 256, 0, st>>>(ny, n->n_out, n->y, tg, n->mu, n->sd, scale, n->dy,
                                                n->part);
  if (loss) finish_loss_kernel<<<1, 64, 0, st>>>(LOSS_BLOCKS, n->part, scale, loss);
  float* g = n->g;
  // layer 3
  gemm<true, false, EPI_PLAIN>(n->n_out, n->hid, batch, n->dy, n->n_out, n->h2, n->hid, g + n->oW3,
                               n->hid, nullptr, nullptr, 0, st, nullptr, nullptr, n->ws, n->ws_n);
  colsum(batch, n->n_out, n->dy, g + n->ob3, n->cs, st);
  gemm<false, false, EPI_MASK>(batch, n->hid, n->n_out, n->dy, n->n_out, n->p + n->oW3, n->hid,
                               n->dh2, n->hid, nullptr, n->h2, n->hid, st, nullptr, nullptr, n->ws, n->ws_n);
  // layer 2
  gemm<true, false, EPI_PLAIN>(n->hid, n->hid, batch, n->dh2, n->hid, n->h1, n->hid, g + n->oW2,
                               n->hid, nullptr, nullptr, 0, st, nullptr, nullptr, n->ws, n->ws_n);
  colsum(batch, n->hid, n->dh2, g + n->ob2, n->cs, st);
  gemm<false, false, EPI_MASK>(batch, n->hid, n->hid, n->dh2, n->hid, n->p + n->oW2, n->hid,
                               n->dh1, n->hid, nullptr, n->h1, n->hid, st, nullptr, nullptr, n->ws, n->ws_n);
  // layer 1
  gemm<true, false, EPI_PLAIN>(n->hid, n->n_in, batch, n->dh1, n->hid, x, n->n_in, g + n->oW1,
                               n->n_in, nullptr, nullptr, 0, st, nullptr, nullptr, n->ws, n->ws_n);
  colsum(batch, n->hid, n->dh1, g + n->ob1, n->cs, st);
}

}  // namespace

extern "C" {

admm_status admm_mlp_create(int32_t n_in, int32_t hidden, int32_t n_out, int32_t max_batch,
                            int32_t device, admm_mlp** out) {
  admmi::clear_err();
  if (!out) return admmi::set_err(ADMM_E_ARG, "out is NULL");
  *out = nullptr;
  if (n_in < 1 || hidden < 1 || n_out < 1 || max_batch < 1)
    return admmi::set_err(ADMM_E_ARG, "sizes must be >= 1");
  if ((int64_t)max_batch * std::max(std::max(n_in, hidden), n_out) >= (1LL << 31))
    return admmi::set_err(ADMM_E_UNSUPPORTED, "max_batch x layer width must stay below 2^31");
  std::unique_ptr<admm_mlp> n(new admm_mlp());
  n->device = device;
  n->n_in = n_in;
  n->hid = hidden;
  n->n_out = n_out;
  n->max_batch = max_batch;
  n->oW1 = 0;
  n->ob1 = n->oW1 + (int64_t)hidden * n_in;
  n->oW2 = n->ob1 + hidden;
  n->ob2 = n->oW2 + (int64_t)hidden * hidden;
  n->oW3 = n->ob2 + hidden;
  n->ob3 = n->oW3 + (int64_t)n_out * hidden;
  n->n_params = n->ob3 + n_out;
  if (admm_status s = admmi::probe_device(device)) return s;
  ADMM_HIP(hipSetDevice(device));
  admm_status s;
  const int64_t B = max_batch;
  if ((s = mlp_alloc(n.get(), &n->p, n->n_params))) return s;
  if ((s = mlp_alloc(n.get(), &n->g, n->n_params))) return s;
  if ((s = mlp_alloc(n.get(), &n->am, n->n_params))) return s;
  if ((s = mlp_alloc(n.get(), &n->av, n->n_params))) return s;
  if ((s = mlp_alloc(n.get(), &n->h1, B * hidden))) return s;
  if ((s = mlp_alloc(n.get(), &n->h2, B * hidden))) return s;
  if ((s = mlp_alloc(n.get(), &n->y, B * n_out))) return s;
  if ((s = mlp_alloc(n.get(), &n->dy, B * n_out))) return s;
  if ((s = mlp_alloc(n.get(), &n->dh1, B * hidden))) return s;
  if ((s = mlp_alloc(n.get(), &n->dh2, B * hidden))) return s;
  if ((s = mlp_alloc(n.get(), &n->part, LOSS_BLOCKS))) return s;
  if ((s = mlp_alloc(n.get(), &n->mu, n_out))) return s;
  {
    const int64_t big = std::max<int64_t>((int64_t)n_out * hidden,
                                          std::max<int64_t>((int64_t)hidden * hidden, (int64_t)hidden * n_in));
    n->ws_n = std::max<int64_t>(big, (int64_t)max_batch * hidden) * MAX_SPLITS / 4;
    if ((s = mlp_alloc(n.get(), &n->ws, n->ws_n))) return s;
    const int64_t chunks = (max_batch + CS_ROWS - 1) / CS_ROWS;
    if ((s = mlp_alloc(n.get(), &n->cs, chunks * std::max(n_out, hidden)))) return s;
  }
  if ((s = mlp_alloc(n.get(), &n->sd, n_out))) return s;
  fill_kernel<<<(n_out + 255) / 256, 256>>>(n_out, 0.f, n->mu);
  fill_kernel<<<(n_out + 255) / 256, 256>>>(n_out, 1.f, n->sd);
  ADMM_HIP(hipGetLastError());
  ADMM_HIP(hipDeviceSynchronize());
  ADMM_HIP(hipMemset(n->p, 0, n->n_params * sizeof(float)));
  ADMM_HIP(hipMemset(n->am, 0, n->n_params * sizeof(float)));
  ADMM_HIP(hipMemset(n->av, 0, n->n_params * sizeof(float)));
  *out = n.release();
  return ADMM_OK;
}

int64_t admm_mlp_n_params(const admm_mlp* n) { return n ? n->n_params : -1; }

admm_status admm_mlp_set_params(admm_mlp* n, const float* host) {
  admmi::clear_err();
  if (!n || !host) return admmi::set_err(ADMM_E_ARG, "NULL argument");
  ADMM_HIP(hipSetDevice(n->device));
  ADMM_HIP(hipMemcpy(n->p, host, n->n_params * sizeof(float), hipMemcpyHostToDevice));
  ADMM_HIP(hipMemset(n->am, 0, n->n_params * sizeof(float)));
  ADMM_HIP(hipMemset(n->av, 0, n->n_params * sizeof(float)));
  n->step = 0;
  return ADMM_OK;
}

admm_status admm_mlp_get_params(admm_mlp* n, float* host) {
  admmi::clear_err();
  if (!n || !host) return admmi::set_err(ADMM_E_ARG, "NULL argument");
  ADMM_HIP(hipSetDevice(n->device));
  ADMM_HIP(hipMemcpy(host, n->p, n->n_params * sizeof(float), hipMemcpyDeviceToHost));
  return ADMM_OK;
}

admm_status admm_mlp_forward(admm_mlp* n, const float* x, int32_t batch, float* y, void* stream) {
  admmi::clear_err();
  if (!n || !x || !y) return admmi::set_err(ADMM_E_ARG, "NULL argument");
  if (batch < 1 || batch > n->max_batch) return admmi::set_err(ADMM_E_ARG, "batch out of [1, max_batch]");
  ADMM_HIP(hipSetDevice(n->device));
  forward(n, x, batch, y, (hipStream_t)stream, true);
  ADMM_HIP(hipGetLastError());
  return ADMM_OK;
}

admm_status admm_mlp_grads(admm_mlp* n, const float* x, const float* target, int32_t batch,
                           float* grads, float* loss, void* stream) {
  admmi::clear_err();
  if (!n || !x || !target) return admmi::set_err(ADMM_E_ARG, "NULL argument");
  if (batch < 1 || batch > n->max_batch) return admmi::set_err(ADMM_E_ARG, "batch out of [1, max_batch]");
  ADMM_HIP(hipSetDevice(n->device));
  hipStream_t st = (hipStream_t)stream;
  backward(n, x, target, batch, loss, st);
  if (grads) ADMM_HIP(hipMemcpyAsync(grads, n->g, n->n_params * sizeof(float), hipMemcpyDeviceToDevice, st));
  ADMM_HIP(hipGetLastError());
  return ADMM_OK;
}

admm_status admm_mlp_train_step(admm_mlp* n, const float* x, const float* target, int32_t batch,
                                float lr, float* loss, void* stream) {
  admmi::clear_err();
  if (!n || !x || !target) return admmi::set_err(ADMM_E_ARG, "NULL argument");
  if (batch < 1 || batch > n->max_batch) return admmi::set_err(ADMM_E_ARG, "batch out of [1, max_batch]");
  if (!(lr > 0.f)) return admmi::set_err(ADMM_E_ARG, "lr must be > 0");
  ADMM_HIP(hipSetDevice(n->device));
  hipStream_t st = (hipStream_t)stream;
  backward(n, x, target, batch, loss, st);
  n->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - (float)std::pow(0.9, (double)n->step);
  const float c2 = 1.f - (float)std::pow(0.999, (double)n->step);
  adam_kernel<<<(unsigned)((n->n_params + 255) / 256), 256, 0, st>>>(n->n_params, n->p, n->g, n->am,
                                                                     n->av, lr, b1, b2, 1e-8f, c1, c2);
  ADMM_HIP(hipGetLastError());
  return ADMM_OK;
}

admm_status admm_mlp_fit_output_scaling(admm_mlp* n, const float* targets, int64_t rows,
                                        float sd_min, void* stream) {
  admmi::clear_err();
  if (!n || !targets || rows < 1) return admmi::set_err(ADMM_E_ARG, "bad arguments");
  if (!(sd_min > 0.f)) return admmi::set_err(ADMM_E_ARG, "sd_min must be > 0");
  ADMM_HIP(hipSetDevice(n->device));
  // chunks of at least 256 rows, at most 1024 chunks
  const int64_t nk = std::min<int64_t>(1024, (rows + 255) / 256);
  const int64_t chunk = (rows + nk - 1) / nk;
  const int nkk = (int)((rows + chunk - 1) / chunk);
  double* tmp = nullptr;
  ADMM_HIP(hipMalloc((void**)&tmp, ((size_t)nkk + 1) * n->n_out * sizeof(double)));
  double* mean_d = tmp + (int64_t)nkk * n->n_out;
  hipStream_t st = (hipStream_t)stream;
  const dim3 gp((n->n_out + 255) / 256, nkk);
  const unsigned gf = (n->n_out + 255) / 256;
  colpart_kernel<<<gp, 256, 0, st>>>(rows, n->n_out, chunk, targets, nullptr, 1, tmp);
  colfinish_kernel<<<gf, 256, 0, st>>>(n->n_out, nkk, rows, tmp, 0, mean_d, n->mu, n->sd, sd_min);
  colpart_kernel<<<gp, 256, 0, st>>>(rows, n->n_out, chunk, targets, mean_d, 2, tmp);
  colfinish_kernel<<<gf, 256, 0, st>>>(n->n_out, nkk, rows, tmp, 1, mean_d, n->mu, n->sd, sd_min);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  hipFree(tmp);
  if (e != hipSuccess) return admmi::set_err(ADMM_E_HIP, "output scaling: %s", hipGetErrorString(e));
  ADMM_HIP(hipGetLastError());
  return ADMM_OK;
}

admm_status admm_mlp_fit_output_scaling_noalloc(admm_mlp* n, const float* targets, int64_t rows,
                                                float sd_min, void* stream) {
  admmi::clear_err();
  if (!n || !targets || rows < 1) return admmi::set_err(ADMM_E_ARG, "bad arguments");
  if (!(sd_min > 0.f)) return admmi::set_err(ADMM_E_ARG, "sd_min must be > 0");
  if (2 * (int64_t)n->n_out > SCRATCH_DOUBLES)
    return admmi::set_err(ADMM_E_UNSUPPORTED,
                          "n_out = %d: the fixed workspace holds at most %lld outputs", n->n_out,
                          (long long)(SCRATCH_DOUBLES / 2));
  ADMM_HIP(hipSetDevice(n->device));
  double* ws = nullptr;
  if (admm_status s = scratch_address(n->device, &ws)) return s;
  // the chunking of admm_mlp_fit_output_scaling, with at most as many
  // chunks as the workspace holds partial rows (one more row keeps the mean)
  const int64_t nk = std::min<int64_t>(std::min<int64_t>(1024, (rows + 255) / 256),
                                       SCRATCH_DOUBLES / n->n_out - 1);
  const int64_t chunk = (rows + nk - 1) / nk;
  const int nkk = (int)((rows + chunk - 1) / chunk);
  double* mean_d = ws + (int64_t)nkk * n->n_out;
  hipStream_t st = (hipStream_t)stream;
  const dim3 gp((n->n_out + 255) / 256, nkk);
  const unsigned gf = (n->n_out + 255) / 256;
  colpart_kernel<<<gp, 256, 0, st>>>(rows, n->n_out, chunk, targets, nullptr, 1, ws);
  colfinish_kernel<<<gf, 256, 0, st>>>(n->n_out, nkk, rows, ws, 0, mean_d, n->mu, n->sd, sd_min);
  colpart_kernel<<<gp, 256, 0, st>>>(rows, n->n_out, chunk, targets, mean_d, 2, ws);
  colfinish_kernel<<<gf, 256, 0, st>>>(n->n_out, nkk, rows, ws, 1, mean_d, n->mu, n->sd, sd_min);
  ADMM_HIP(hipGetLastError());
  return ADMM_OK;
}

admm_status admm_mlp_set_output_scaling(admm_mlp* n, const float* mean, const float* sd) {
  admmi::clear_err();
  if (!n || !mean || !sd) return admmi::set_err(ADMM_E_ARG, "NULL argument");
  for (int i = 0; i < n->n_out; ++i)
    if (!(sd[i] > 0.f)) return admmi::set_err(ADMM_E_ARG, "sd must be > 0");
  ADMM_HIP(hipSetDevice(n->device));
  ADMM_HIP(hipMemcpy(n->mu, mean, n->n_out * sizeof(float), hipMemcpyHostToDevice));
  ADMM_HIP(hipMemcpy(n->sd, sd, n->n_out * sizeof(float), hipMemcpyHostToDevice));
  return ADMM_OK;
}

admm_status admm_mlp_get_output_scaling(admm_mlp* n, float* mean, float* sd) {
  admmi::clear_err();
  if (!n || !mean || !sd) return admmi::set_err(ADMM_E_ARG, "NULL argument");
  ADMM_HIP(hipSetDevice(n->device));
  ADMM_HIP(hipMemcpy(mean, n->mu, n->n_out * sizeof(float), hipMemcpyDeviceToHost));
  ADMM_HIP(hipMemcpy(sd, n->sd, n->n_out * sizeof(float), hipMemcpyDeviceToHost));
  return ADMM_OK;
}

admm_status admm_mlp_destroy(admm_mlp* n) {
  admmi::clear_err();
  delete n;
  return ADMM_OK;
}

}  // extern "C"
