// HIP kernels of the two-site H_eff library (gfx950).
//
// The chained block product  out += f * op(L) * op(X) * op(R)  is the task
// of Eq. Hamilton_act_U1sym (L: left-block operator block, X: Psi block,
// op(R): transposed right-block operator block) and also the projection
// A^T (O (x) o) A of the renormalization steps.  Work is output-stationary:
// one work item owns kRows rows of one output block and accumulates all of
// that block's tasks in registers, so no atomics are needed and the sum
// order is fixed (bitwise reproducible).
#include "heff_internal.h"

#include <hip/hip_runtime.h>

namespace heff {

// ------------------------------------------------------------------ helpers
template <typename T>
__device__ __forceinline__ T ld_opL(const T* p, uint32_t fl, int i, int k, int a, int b) {
  return (fl & T_TL) ? p[(int64_t)k * a + i] : p[(int64_t)i * b + k];
}
template <typename T>
__device__ __forceinline__ T ld_opX(const T* p, uint32_t fl, int k, int j, int b, int c) {
  return (fl & T_TX) ? p[(int64_t)j * b + k] : p[(int64_t)k * c + j];
}
template <typename T>
__device__ __forceinline__ T ld_opR(const T* p, uint32_t fl, int j, int n, int c, int e) {
  return (fl & T_TR) ? p[(int64_t)n * c + j] : p[(int64_t)j * e + n];
}

// round-to-nearest-even float -> bf16 bits
__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// ------------------------------------------------------------------ chained product (plain)
// One work-group of 256 threads per work item; T = f * op(L) op(X) rows are
// staged in LDS, then multiplied by op(R).
constexpr int kThreads = 256;
constexpr int kAcc = kRows * kMaxDim / kThreads;

template <typename T>
__global__ __launch_bounds__(kThreads) void chain_plain(const Tile* __restrict__ tiles,
                                                        const Work* __restrict__ work,
                                                        const Task* __restrict__ tasks, Bases<T> B) {
  __shared__ T Ts[kRows * (kMaxDim + 1)];
  const Work w = work[blockIdx.x];
  const Tile tile = tiles[w.tile];
  const int rows = min(kRows, tile.a - w.row0);
  const int E = tile.e;
  const int tid = threadIdx.x;
  T acc[kAcc];
#pragma unroll
  for (int q = 0; q < kAcc; ++q) acc[q] = T(0);
  for (int ti = tile.t0; ti < tile.t1; ++ti) {
    const Task t = tasks[ti];
    const uint32_t fl = t.flags;
    const T* L = B.L[(fl & T_SELL) ? 1 : 0] + t.offL;
    const T* X = B.X[(fl & T_SELX) ? 1 : 0] + t.offX;
    const T* R = B.R[(fl & T_SELR) ? 1 : 0] + t.offR;
    const T f = (T)t.f;
    const int b = t.b, c = t.c;
    // stage 1: Ts[r][j] = f * sum_k op(L)[row0+r][k] op(X)[k][j]
    for (int idx = tid; idx < rows * c; idx += kThreads) {
      const int r = idx / c, j = idx - r * c;
      const int i = w.row0 + r;
      T v = T(0);
      if (fl & T_IDL) {
        v = (fl & T_IDX) ? T(i == j ? 1 : 0) : ld_opX(X, fl, i, j, b, c);
      } else if (fl & T_IDX) {
        v = ld_opL(L, fl, i, j, t.a, b);
      } else {
        for (int k = 0; k < b; ++k) v += ld_opL(L, fl, i, k, t.a, b) * ld_opX(X, fl, k, j, b, c);
      }
      Ts[r * (kMaxDim + 1) + j] = f * v;
    }
    __syncthreads();
    // stage 2: acc[r][n] += sum_j Ts[r][j] op(R)[j][n]
#pragma unroll
    for (int q = 0; q < kAcc; ++q) {
      const int idx = tid + q * kThreads;
      const int r = idx / kMaxDim, n = idx - r * kMaxDim;
      if (r < rows && n < E) {
        if (fl & T_IDR) {
          acc[q] += Ts[r * (kMaxDim + 1) + n];
        } else {
          T v = T(0);
          for (int j = 0; j < c; ++j) v += Ts[r * (kMaxDim + 1) + j] * ld_opR(R, fl, j, n, c, E);
          acc[q] += v;
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kAcc; ++q) {
    const int idx = tid + q * kThreads;
    const int r = idx / kMaxDim, n = idx - r * kMaxDim;
    if (r < rows && n < E) B.out[tile.offOut + (int64_t)(w.row0 + r) * E + n] = acc[q];
  }
}

hipError_t launch_chain_f64(const Tile* tiles, const Work* work, int64_t n_work, const Task* tasks,
                            Bases<double> b, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  hipLaunchKernelGGL(chain_plain<double>, dim3((unsigned)n_work), dim3(kThreads), 0, s, tiles, work, tasks, b);
  return hipGetLastError();
}

hipError_t launch_chain_f32(const Tile* tiles, const Work* work, int64_t n_work, const Task* tasks,
                            Bases<float> b, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  hipLaunchKernelGGL(chain_plain<float>, dim3((unsigned)n_work), dim3(kThreads), 0, s, tiles, work, tasks, b);
  return hipGetLastError();
}

// ------------------------------------------------------------------ chained product, bf16 split
// Products of split operands: a*b ~= ah*bh + ah*bl + al*bh with FP32
// accumulation; Psi and the intermediate T are split on the fly
// (hi = RNE_bf16(x), lo = RNE_bf16(x - hi)).
struct Bf16Args {
  const uint16_t* Lhi[2];
  const uint16_t* Llo[2];
  const uint16_t* Rhi[2];
  const uint16_t* Rlo[2];
  const float* X;
  float* out;
};

__device__ __forceinline__ float mul3(float ah, float al, float bh, float bl) { return ah * bh + (ah * bl + al * bh); }

__global__ __launch_bounds__(kThreads) void chain_bf16x3_plain(const Tile* __restrict__ tiles,
                                                               const Work* __restrict__ work,
                                                               const Task* __restrict__ tasks, Bf16Args B) {
  __shared__ float Ts[kRows * (kMaxDim + 1)];
  const Work w = work[blockIdx.x];
  const Tile tile = tiles[w.tile];
  const int rows = min(kRows, tile.a - w.row0);
  const int E = tile.e;
  const int tid = threadIdx.x;
  float acc[kAcc];
#pragma unroll
  for (int q = 0; q < kAcc; ++q) acc[q] = 0.f;
  for (int ti = tile.t0; ti < tile.t1; ++ti) {
    const Task t = tasks[ti];
    const uint32_t fl = t.flags;
    const int sl = (fl & T_SELL) ? 1 : 0, sr = (fl & T_SELR) ? 1 : 0;
    const uint16_t* Lh = B.Lhi[sl] + t.offL;
    const uint16_t* Ll = B.Llo[sl] + t.offL;
    const uint16_t* Rh = B.Rhi[sr] + t.offR;
    const uint16_t* Rl = B.Rlo[sr] + t.offR;
    const float* X = B.X + t.offX;
    const float f = (float)t.f;
    const int b = t.b, c = t.c;
    for (int idx = tid; idx < rows * c; idx += kThreads) {
      const int r = idx / c, j = idx - r * c;
      const int i = w.row0 + r;
      float v = 0.f;
      if (fl & T_IDL) {
        v = ld_opX(X, fl, i, j, b, c);
      } else {
        for (int k = 0; k < b; ++k) {
          float x = ld_opX(X, fl, k, j, b, c);
          uint16_t xh = f2bf(x);
          uint16_t xl = f2bf(x - bf2f(xh));
          v += mul3(bf2f(ld_opL(Lh, fl, i, k, t.a, b)), bf2f(ld_opL(Ll, fl, i, k, t.a, b)), bf2f(xh), bf2f(xl));
        }
      }
      Ts[r * (kMaxDim + 1) + j] = f * v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kAcc; ++q) {
      const int idx = tid + q * kThreads;
      const int r = idx / kMaxDim, n = idx - r * kMaxDim;
      if (r < rows && n < E) {
        if (fl & T_IDR) {
          acc[q] += Ts[r * (kMaxDim + 1) + n];
        } else {
          float v = 0.f;
          for (int j = 0; j < c; ++j) {
            float tv = Ts[r * (kMaxDim + 1) + j];
            uint16_t th = f2bf(tv);
            uint16_t tl = f2bf(tv - bf2f(th));
            v += mul3(bf2f(th), bf2f(tl), bf2f(ld_opR(Rh, fl, j, n, c, E)), bf2f(ld_opR(Rl, fl, j, n, c, E)));
          }
          acc[q] += v;
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kAcc; ++q) {
    const int idx = tid + q * kThreads;
    const int r = idx / kMaxDim, n = idx - r * kMaxDim;
    if (r < rows && n < E) B.out[tile.offOut + (int64_t)(w.row0 + r) * E + n] = acc[q];
  }
}

hipError_t launch_chain_bf16x3(const Tile* tiles, const Work* work, int64_t n_work, const Task* tasks,
                               const uint16_t* Lhi[2], const uint16_t* Llo[2], const uint16_t* Rhi[2],
                               const uint16_t* Rlo[2], const float* X, float* out, hipStream_t s) {
  if (n_work <= 0) return hipSuccess;
  Bf16Args a;
  for (int i = 0; i < 2; ++i) {
    a.Lhi[i] = Lhi[i];
    a.Llo[i] = Llo[i];
    a.Rhi[i] = Rhi[i];
    a.Rlo[i] = Rlo[i];
  }
  a.X = X;
  a.out = out;
  hipLaunchKernelGGL(chain_bf16x3_plain, dim3((unsigned)n_work), dim3(kThreads), 0, s, tiles, work, tasks, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ diagonal
__global__ __launch_bounds__(256) void diag_kernel(const Tile* __restrict__ tiles, const DiagTask* __restrict__ tasks,
                                                   const double* L0, const double* L1, const double* R0,
                                                   const double* R1, double* out) {
  const Tile tile = tiles[blockIdx.x];
  const int n = tile.a * tile.e;
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
    const int i = idx / tile.e, j = idx - i * tile.e;
    double v = 0.0;
    for (int t = tile.t0; t < tile.t1; ++t) {
      const DiagTask d = tasks[t];
      const double dl = (d.flags & T_IDL) ? 1.0 : ((d.flags & T_SELL) ? L1 : L0)[d.offL + (int64_t)i * (tile.a + 1)];
      const double dr = (d.flags & T_IDR) ? 1.0 : ((d.flags & T_SELR) ? R1 : R0)[d.offR + (int64_t)j * (tile.e + 1)];
      v += d.f * dl * dr;
    }
    out[tile.offOut + idx] = v;
  }
}

hipError_t launch_diag(const Tile* tiles, int64_t n_tiles, const DiagTask* tasks, const double* L0,
                       const double* L1, const double* R0, const double* R1, double* out, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(diag_kernel, dim3((unsigned)n_tiles), dim3(256), 0, s, tiles, tasks, L0, L1, R0, R1, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ FP64 GEMM (operator sums)
// C[m x n] = A[m x k] B[k x n], row-major; 64x64 tiles, 4x4 per thread.
__global__ __launch_bounds__(256) void gemm_f64_kernel(int64_t m, int64_t n, int64_t k, const double* __restrict__ A,
                                                       const double* __restrict__ Bm, double* __restrict__ C) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t row0 = (int64_t)blockIdx.y * 64, col0 = (int64_t)blockIdx.x * 64;
  double acc[4][4] = {};
  for (int64_t k0 = 0; k0 < k; k0 += 16) {
    for (int idx = threadIdx.x; idx < 16 * 64; idx += 256) {
      int kk = idx / 64, rr = idx % 64;
      int64_t gr = row0 + rr, gk = k0 + kk;
      As[kk][rr] = (gr < m && gk < k) ? A[gr * k + gk] : 0.0;
      int64_t gc = col0 + rr;
      Bs[kk][rr] = (gk < k && gc < n) ? Bm[gk * n + gc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * bb[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int64_t gr = row0 + ty + 16 * i, gc = col0 + tx + 16 * j;
      if (gr < m && gc < n) C[gr * n + gc] = acc[i][j];
    }
}

hipError_t launch_gemm_f64(int64_t m, int64_t n, int64_t k, const double* A, const double* B, double* C,
                           hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  dim3 grid((unsigned)((n + 63) / 64), (unsigned)((m + 63) / 64));
  hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, s, m, n, k, A, B, C);
  return hipGetLastError();
}

// ------------------------------------------------------------------ conversions
__global__ void f64_to_f32_kernel(const double* in, float* out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}
__global__ void f32_to_f64_kernel(const float* in, double* out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (double)in[i];
}
__global__ void split_bf16_kernel(const double* in, uint16_t* hi, uint16_t* lo, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float x = (float)in[i];
    uint16_t h = f2bf(x);
    hi[i] = h;
    lo[i] = f2bf(x - bf2f(h));
  }
}

static unsigned grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (unsigned)(g < 65536 ? (g < 1 ? 1 : g) : 65536);
}

hipError_t launch_convert_f32(const double* in, float* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}
hipError_t launch_f64_to_f32(const double* in, float* out, int64_t n, hipStream_t s) {
  return launch_convert_f32(in, out, n, s);
}
hipError_t launch_f32_to_f64(const float* in, double* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(f32_to_f64_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}
hipError_t launch_split_bf16(const double* in, uint16_t* hi, uint16_t* lo, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(split_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, hi, lo, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Davidson vector kernels
// Deterministic two-pass reductions: fixed grid of kRedBlocks partial sums,
// then one work-group folds them in a fixed order.
constexpr int kRedBlocks = 512;

__global__ __launch_bounds__(256) void multidot_partial(const double* A, int64_t lda, int k, const double* x,
                                                        int64_t n, double* part) {
  __shared__ double sh[256];
  for (int i = 0; i < k; ++i) {
    double v = 0.0;
    for (int64_t j = blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) v += A[i * lda + j] * x[j];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)i * gridDim.x + blockIdx.x] = sh[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void multidot_final(const double* part, int k, int nb, double* out) {
  __shared__ double sh[256];
  for (int i = 0; i < k; ++i) {
    double v = 0.0;
    for (int j = threadIdx.x; j < nb; j += 256) v += part[(int64_t)i * nb + j];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = sh[0];
    __syncthreads();
  }
}

hipError_t launch_multidot(const double* A, int64_t lda, int k, const double* x, int64_t n, double* out,
                           double* scratch, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(multidot_partial, dim3(kRedBlocks), dim3(256), 0, s, A, lda, k, x, n, scratch);
  hipLaunchKernelGGL(multidot_final, dim3(1), dim3(256), 0, s, scratch, k, kRedBlocks, out);
  return hipGetLastError();
}

__global__ void multiaxpy_kernel(const double* A, int64_t lda, int k, const double* coef, double cs, double* y,
                                 double alpha, int64_t n) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    double v = alpha == 0.0 ? 0.0 : alpha * y[j];
    for (int i = 0; i < k; ++i) v += cs * coef[i] * A[i * lda + j];
    y[j] = v;
  }
}

hipError_t launch_multiaxpy(const double* A, int64_t lda, int k, const double* coef, double coef_scale, double* y,
                            double alpha, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(multiaxpy_kernel, dim3(grid_for(n)), dim3(256), 0, s, A, lda, k, coef, coef_scale, y, alpha, n);
  return hipGetLastError();
}

}  // namespace heff
