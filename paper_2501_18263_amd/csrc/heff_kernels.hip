// HIP kernels of the two-site H_eff library (gfx950).
//
// The chained block product  out += f * op(L) * op(X) * op(R)  is the task
// of Eq. Hamilton_act_U1sym (L: left-block operator block, X: Psi block,
// op(R): transposed right-block operator block) and also the projection
// A^T (O (x) o) A of the renormalization steps.  Work is output-stationary:
// one work item owns a row range of one output block and accumulates all of
// that block's tasks in registers, so no atomics are needed and the sum
// order is fixed (bitwise reproducible).
#include "heff_internal.h"

#include <hip/hip_runtime.h>

namespace heff {

// ------------------------------------------------------------------ helpers
// elements of op(M) from row-major storage with row stride ld
template <typename T>
__device__ __forceinline__ T ld_op(const T* p, bool trans, int r, int c, int ld) {
  return trans ? p[(int64_t)c * ld + r] : p[(int64_t)r * ld + c];
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

constexpr int kThreads = 256;
constexpr int kAcc = kPlainRows * kMaxDim / kThreads;

// ------------------------------------------------------------------ chained product (MFMA)
// Matrix-core version: one work-group = 4 waves = 64 rows of one output
// block; wave w owns rows [16w, 16w+16).  Per 16-column chunk of c:
//   stage 1  T^T = op(X)^T op(L)^T on v_mfma_*_16x16x4, summing over b with
//            the k order permuted so that lane group g covers the
//            contiguous range [g*ks, (g+1)*ks): its result leaves register i
//            of lane (g, n) holding T[row n][c0 + row(i, g)], which is exactly
//            the A operand of stage 2 for k = c0 + row(i, g) (no LDS round
//            trip);
//   stage 2  acc += T op(R) over the same k order, op(R) row c0 + row(i, g).
// The left operator strip op(L)[row][*] is kept in registers for the whole
// task (it is reused by every chunk).  KS bounds ks = ceil(b/4), NT bounds
// the 16-column output tiles.
// Operand layout of both instructions: lane l holds A[l%16][l/16] and
// B[l/16][l%16].  Result layout differs: register r of lane l holds
// D[row(r, l/16)][l%16] with row = 4r + l/16 for f64 and 4(l/16) + r for f32
// (checked on the device).
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 run(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int g) { return 4 * r + g; }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 run(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int g) { return 4 * g + r; }
};

// One work item (64 rows of one output tile).  Per 16-column chunk of the
// inner dimension c, the X chunk (b x 16) and the R chunk (16 x E) are
// loaded cooperatively by all 256 threads (coalesced, every load of the
// chunk in flight at once) into LDS shared by the four waves; each
// 16-lane group of an MFMA operand read then covers one contiguous 128-byte
// LDS row segment.  Waves whose rows lie outside the tile take part in the
// loads and barriers only.
template <typename T, int KS, int NT>
struct ChainSmem {
  static constexpr int KMAX = 4 * KS;   // largest inner dimension b
  static constexpr int EMAX = 16 * NT;  // largest output width
  T X[KMAX * 16];
  T R[16 * EMAX];
};

template <typename T, int KS, int NT>
__device__ __forceinline__ void chain_item(const Tile& tile, const Work& w, const Task* __restrict__ tasks,
                                           const Bases<T>& B, ChainSmem<T, KS, NT>& sm) {
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int KMAX = 4 * KS;
  constexpr int EMAX = 16 * NT;
  constexpr int XPT = (KMAX * 16 + 255) / 256;
  constexpr int RPT = (16 * EMAX + 255) / 256;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g = lane >> 4, n = lane & 15;
  const int wrow0 = w.row0 + wave * 16;
  const bool wave_on = wrow0 < tile.a;
  const int row = wrow0 + n;
  const bool rowok = row < tile.a;
  const int E = tile.e;
  v4 acc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = v4{0, 0, 0, 0};
  for (int ti = tile.t0; ti < tile.t1; ++ti) {
    const Task t = tasks[ti];
    const uint32_t fl = t.flags;
    const int b = t.b, c = t.c;
    const T* L = B.L[(fl & T_SELL) ? 1 : 0] + t.offL;
    const T* X = B.X[(fl & T_SELX) ? 1 : 0] + t.offX;
    const T* R = B.R[(fl & T_SELR) ? 1 : 0] + t.offR;
    const T f = (T)t.f;
    const int ks = (b + 3) >> 2;
    const bool direct = (fl & (T_IDL | T_IDX)) != 0;
    const bool idr = (fl & T_IDR) != 0;
    const bool tx = (fl & T_TX) != 0, tr = (fl & T_TR) != 0, tl = (fl & T_TL) != 0;
    T Lr[KS];
    if (!direct) {
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int k = g * ks + s;
        T v = T(0);
        if (s < ks && rowok && k < b) v = ld_op(L, tl, row, k, t.ldL);
        Lr[s] = v;
      }
    }
    for (int c0 = 0; c0 < c; c0 += 16) {
      T xr[XPT], rr[RPT];
      if (!direct) {
#pragma unroll
        for (int q = 0; q < XPT; ++q) {
          const int idx = tid + 256 * q;
          const int k = idx >> 4, m = c0 + (idx & 15);
          T v = T(0);
          if (k < b && m < c) v = ld_op(X, tx, k, m, t.ldX);
          xr[q] = v;
        }
      }
      if (!idr) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int idx = tid + 256 * q;
          // transposed storage: consecutive threads walk the stored row (j)
          const int j = tr ? (idx & 15) : (idx / EMAX);
          const int col = tr ? (idx >> 4) : (idx % EMAX);
          T v = T(0);
          if (col < E && c0 + j < c && j < 16) v = ld_op(R, tr, c0 + j, col, t.ldR);
          rr[q] = v;
        }
      }
      __syncthreads();
      if (!direct) {
#pragma unroll
        for (int q = 0; q < XPT; ++q) {
          const int idx = tid + 256 * q;
          if (idx < KMAX * 16) sm.X[idx] = xr[q];
        }
      }
      if (!idr) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int idx = tid + 256 * q;
          const int j = tr ? (idx & 15) : (idx / EMAX);
          const int col = tr ? (idx >> 4) : (idx % EMAX);
          if (j < 16 && col < EMAX) sm.R[j * EMAX + col] = rr[q];
        }
      }
      __syncthreads();
      if (!wave_on) continue;
      v4 Tt = v4{0, 0, 0, 0};
      if (direct) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int col = c0 + M::row(i, g);
          T v = T(0);
          if (rowok && col < c) v = (fl & T_IDL) ? ld_op(X, tx, row, col, t.ldX) : ld_op(L, tl, row, col, t.ldL);
          Tt[i] = v;
        }
      } else {
#pragma unroll
        for (int s = 0; s < KS; ++s)
          if (s < ks) Tt = M::run(sm.X[(g * ks + s) * 16 + n], Lr[s], Tt);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) Tt[i] *= f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = M::row(i, g);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          if (nt * 16 < E) {
            const int col = nt * 16 + n;
            T br;
            if (idr) br = (c0 + j == col) ? T(1) : T(0);
            else br = sm.R[j * EMAX + col];
            acc[nt] = M::run(Tt[i], br, acc[nt]);
          }
        }
      }
    }
  }
  if (!wave_on) return;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int col = nt * 16 + n;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wrow0 + M::row(i, g);
      if (r < tile.a && col < E) B.out[tile.offOut + (int64_t)r * tile.ldOut + col] = acc[nt][i];
    }
  }
}

template <typename T, int KS, int NT>
__global__ __launch_bounds__(256) void chain_mfma(const Tile* __restrict__ tiles, const Work* __restrict__ work,
                                                  const Task* __restrict__ tasks, Bases<T> B) {
  __shared__ ChainSmem<T, KS, NT> sm;
  const Work w = work[blockIdx.x];
  chain_item<T, KS, NT>(tiles[w.tile], w, tasks, B, sm);
}

// Batched, persistent form: a fixed grid strides over the work items of
// many independent problems (tile.prob selects the problem's operator
// stores; Psi and the output of all problems share one base each).
template <typename T, int KS, int NT>
__global__ __launch_bounds__(256) void chain_mfma_batch(const Tile* __restrict__ tiles, const Work* __restrict__ work,
                                                        int64_t n_work, const Task* __restrict__ tasks,
                                                        const ProbBases<T>* __restrict__ pb, const T* X, T* out) {
  __shared__ ChainSmem<T, KS, NT> sm;
  for (int64_t i = blockIdx.x; i < n_work; i += gridDim.x) {
    const Work w = work[i];
    const Tile tile = tiles[w.tile];
    const ProbBases<T> q = pb[tile.prob];
    Bases<T> B;
    B.L[0] = q.L[0];
    B.L[1] = q.L[1];
    B.R[0] = q.R[0];
    B.R[1] = q.R[1];
    B.X[0] = B.X[1] = X;
    B.out = out;
    chain_item<T, KS, NT>(tile, w, tasks, B, sm);
    __syncthreads();  // LDS reuse by the next item
  }
}

hipError_t launch_mfma_batch_f32(const Tile* tiles, const WorkSet& ws, const Task* tasks, const ProbBases<float>* pb,
                                 const float* X, float* out, const int grid[kNumVariants], hipStream_t s) {
  for (int v = kNumVariants - 1; v >= 0; --v) {
    if (ws.n[v] <= 0) continue;
    dim3 gr((unsigned)grid[v]), blk(256);
    switch (v) {
      case 0: hipLaunchKernelGGL((chain_mfma_batch<float, 8, 2>), gr, blk, 0, s, tiles, ws.w[v], ws.n[v], tasks, pb, X, out); break;
      case 1: hipLaunchKernelGGL((chain_mfma_batch<float, 16, 4>), gr, blk, 0, s, tiles, ws.w[v], ws.n[v], tasks, pb, X, out); break;
      case 2: hipLaunchKernelGGL((chain_mfma_batch<float, 32, 8>), gr, blk, 0, s, tiles, ws.w[v], ws.n[v], tasks, pb, X, out); break;
      default: hipLaunchKernelGGL((chain_mfma_batch<float, 64, 16>), gr, blk, 0, s, tiles, ws.w[v], ws.n[v], tasks, pb, X, out); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
static hipError_t launch_mfma_variants(const Tile* tiles, const WorkSet& ws, const Task* tasks, Bases<T> b,
                                       hipStream_t s, hipEvent_t (*ev)[2]) {
  // largest blocks first: their work items are the longest
  for (int v = kNumVariants - 1; v >= 0; --v) {
    if (ws.n[v] <= 0) continue;
    if (ev && ev[v][0]) {
      hipError_t e = hipEventRecord(ev[v][0], s);
      if (e != hipSuccess) return e;
    }
    dim3 grid((unsigned)ws.n[v]), blk(256);
    switch (v) {
      case 0: hipLaunchKernelGGL((chain_mfma<T, 8, 2>), grid, blk, 0, s, tiles, ws.w[v], tasks, b); break;
      case 1: hipLaunchKernelGGL((chain_mfma<T, 16, 4>), grid, blk, 0, s, tiles, ws.w[v], tasks, b); break;
      case 2: hipLaunchKernelGGL((chain_mfma<T, 32, 8>), grid, blk, 0, s, tiles, ws.w[v], tasks, b); break;
      default: hipLaunchKernelGGL((chain_mfma<T, 64, 16>), grid, blk, 0, s, tiles, ws.w[v], tasks, b); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev && ev[v][1]) {
      e = hipEventRecord(ev[v][1], s);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_mfma_f64(const Tile* tiles, const WorkSet& ws, const Task* tasks, Bases<double> b, hipStream_t s,
                           hipEvent_t (*ev)[2]) {
  return launch_mfma_variants<double>(tiles, ws, tasks, b, s, ev);
}
hipError_t launch_mfma_f32(const Tile* tiles, const WorkSet& ws, const Task* tasks, Bases<float> b, hipStream_t s,
                           hipEvent_t (*ev)[2]) {
  return launch_mfma_variants<float>(tiles, ws, tasks, b, s, ev);
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
  __shared__ float Ts[kPlainRows * (kMaxDim + 1)];
  const Work w = work[blockIdx.x];
  const Tile tile = tiles[w.tile];
  const int rows = min(kPlainRows, tile.a - w.row0);
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
        v = ld_op(X, fl & T_TX, i, j, t.ldX);
      } else {
        for (int k = 0; k < b; ++k) {
          float x = ld_op(X, fl & T_TX, k, j, t.ldX);
          uint16_t xh = f2bf(x);
          uint16_t xl = f2bf(x - bf2f(xh));
          v += mul3(bf2f(ld_op(Lh, fl & T_TL, i, k, t.ldL)), bf2f(ld_op(Ll, fl & T_TL, i, k, t.ldL)), bf2f(xh), bf2f(xl));
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
            v += mul3(bf2f(th), bf2f(tl), bf2f(ld_op(Rh, fl & T_TR, j, n, t.ldR)), bf2f(ld_op(Rl, fl & T_TR, j, n, t.ldR)));
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
    if (r < rows && n < E) B.out[tile.offOut + (int64_t)(w.row0 + r) * tile.ldOut + n] = acc[q];
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

// ------------------------------------------------------------------ chained product, bf16 split (MFMA)
// Same output-stationary structure as chain_mfma on v_mfma_f32_16x16x32_bf16
// (K = 32 per instruction; lane l holds A[l%16][8(l/16)+j] and
// B[8(l/16)+j][l%16], j = 0..7; result as the f32 16x16x4 instruction).
// Every product a*b is formed as ah*bh + ah*bl + al*bh (three instructions,
// FP32 accumulation).  Stage 1 sums over b with lane group g covering the
// contiguous k range [8 g ks, 8 (g+1) ks) (ks = ceil(b/32) instructions);
// two 16-column chunks of T = f op(L) op(X) (FP32, re-split into hi/lo)
// form the 32-wide A operand of stage 2.
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __bf16 bits2bf(uint16_t u) { return __builtin_bit_cast(__bf16, u); }

__device__ __forceinline__ void split8(const float (&x)[8], bf8_t& hi, bf8_t& lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    uint16_t h = f2bf(x[j]);
    hi[j] = bits2bf(h);
    lo[j] = bits2bf(f2bf(x[j] - bf2f(h)));
  }
}

__device__ __forceinline__ f4_t mma3(const bf8_t& ah, const bf8_t& al, const bf8_t& bh, const bf8_t& bl, f4_t c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
  return c;
}

template <int KS8, int NT>
__global__ __launch_bounds__(256) void chain_bf16x3_mfma(const Tile* __restrict__ tiles, const Work* __restrict__ work,
                                                         const Task* __restrict__ tasks, Bf16Args B) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4, n = lane & 15;
  const Work w = work[blockIdx.x];
  const Tile tile = tiles[w.tile];
  const int wrow0 = w.row0 + wave * 16;
  if (wrow0 >= tile.a) return;  // no barriers below
  const int row = wrow0 + n;
  const bool rowok = row < tile.a;
  const int E = tile.e;
  f4_t acc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = f4_t{0, 0, 0, 0};
  for (int ti = tile.t0; ti < tile.t1; ++ti) {
    const Task t = tasks[ti];
    const uint32_t fl = t.flags;
    const int b = t.b, c = t.c;
    const int sl = (fl & T_SELL) ? 1 : 0, sr = (fl & T_SELR) ? 1 : 0;
    const uint16_t* Lh = B.Lhi[sl] + t.offL;
    const uint16_t* Ll = B.Llo[sl] + t.offL;
    const uint16_t* Rh = B.Rhi[sr] + t.offR;
    const uint16_t* Rl = B.Rlo[sr] + t.offR;
    const float* X = B.X + t.offX;
    const float f = (float)t.f;
    const int ks = (b + 31) >> 5;
    const bool direct = (fl & (T_IDL | T_IDX)) != 0;
    const bool tl = fl & T_TL, tx = fl & T_TX, tr = fl & T_TR;
    bf8_t Lrh[KS8], Lrl[KS8];
    if (!direct) {
#pragma unroll
      for (int s8 = 0; s8 < KS8; ++s8) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int k = g * 8 * ks + 8 * s8 + j;
          uint16_t vh = 0, vl = 0;
          if (s8 < ks && rowok && k < b) {
            const int64_t o = tl ? (int64_t)k * t.ldL + row : (int64_t)row * t.ldL + k;
            vh = Lh[o];
            vl = Ll[o];
          }
          Lrh[s8][j] = bits2bf(vh);
          Lrl[s8][j] = bits2bf(vl);
        }
      }
    }
    for (int c0 = 0; c0 < c; c0 += 32) {
      f4_t Tc[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int cb = c0 + 16 * h;
        f4_t Tt = f4_t{0, 0, 0, 0};
        if (direct) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int col = cb + 4 * g + r;
            float v = 0.f;
            if (rowok && col < c) {
              if (fl & T_IDL) v = ld_op(X, tx, row, col, t.ldX);
              else {
                const int64_t o = tl ? (int64_t)col * t.ldL + row : (int64_t)row * t.ldL + col;
                v = bf2f(Lh[o]) + bf2f(Ll[o]);
              }
            }
            Tt[r] = v;
          }
        } else if (cb < c) {
          const int m = cb + n;
          const bool mok = m < c;
#pragma unroll
          for (int s8 = 0; s8 < KS8; ++s8) {
            if (s8 < ks) {
              float xv[8];
#pragma unroll
              for (int j = 0; j < 8; ++j) {
                const int k = g * 8 * ks + 8 * s8 + j;
                xv[j] = (mok && k < b) ? ld_op(X, tx, k, m, t.ldX) : 0.f;
              }
              bf8_t xh, xl;
              split8(xv, xh, xl);
              Tt = mma3(xh, xl, Lrh[s8], Lrl[s8], Tt);
            }
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) Tt[r] *= f;
        Tc[h] = Tt;
      }
      float tv[8];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        tv[r] = Tc[0][r];
        tv[4 + r] = Tc[1][r];
      }
      bf8_t th, tlo;
      split8(tv, th, tlo);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        if (nt * 16 < E) {
          const int col = nt * 16 + n;
          bf8_t rh, rl;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int kk = (j < 4) ? c0 + 4 * g + j : c0 + 16 + 4 * g + (j - 4);
            uint16_t vh = 0, vl = 0;
            if (kk < c && col < E) {
              if (fl & T_IDR) {
                vh = (kk == col) ? (uint16_t)0x3f80 : (uint16_t)0;
              } else {
                const int64_t o = tr ? (int64_t)col * t.ldR + kk : (int64_t)kk * t.ldR + col;
                vh = Rh[o];
                vl = Rl[o];
              }
            }
            rh[j] = bits2bf(vh);
            rl[j] = bits2bf(vl);
          }
          acc[nt] = mma3(th, tlo, rh, rl, acc[nt]);
        }
      }
    }
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int col = nt * 16 + n;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = wrow0 + 4 * g + r;
      if (rr < tile.a && col < E) B.out[tile.offOut + (int64_t)rr * tile.ldOut + col] = acc[nt][r];
    }
  }
}

hipError_t launch_bf16x3_mfma(const Tile* tiles, const WorkSet& ws, const Task* tasks, const uint16_t* Lhi[2],
                              const uint16_t* Llo[2], const uint16_t* Rhi[2], const uint16_t* Rlo[2], const float* X,
                              float* out, hipStream_t s, hipEvent_t (*ev)[2]) {
  Bf16Args a;
  for (int i = 0; i < 2; ++i) {
    a.Lhi[i] = Lhi[i];
    a.Llo[i] = Llo[i];
    a.Rhi[i] = Rhi[i];
    a.Rlo[i] = Rlo[i];
  }
  a.X = X;
  a.out = out;
  for (int v = kNumVariants - 1; v >= 0; --v) {
    if (ws.n[v] <= 0) continue;
    if (ev && ev[v][0]) {
      hipError_t e = hipEventRecord(ev[v][0], s);
      if (e != hipSuccess) return e;
    }
    dim3 grid((unsigned)ws.n[v]), blk(256);
    switch (v) {
      case 0: hipLaunchKernelGGL((chain_bf16x3_mfma<1, 2>), grid, blk, 0, s, tiles, ws.w[v], tasks, a); break;
      case 1: hipLaunchKernelGGL((chain_bf16x3_mfma<2, 4>), grid, blk, 0, s, tiles, ws.w[v], tasks, a); break;
      case 2: hipLaunchKernelGGL((chain_bf16x3_mfma<4, 8>), grid, blk, 0, s, tiles, ws.w[v], tasks, a); break;
      default: hipLaunchKernelGGL((chain_bf16x3_mfma<8, 16>), grid, blk, 0, s, tiles, ws.w[v], tasks, a); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev && ev[v][1]) {
      e = hipEventRecord(ev[v][1], s);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
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

// ------------------------------------------------------------------ symmetric eigensolver (truncation)
// One work-group per symmetric matrix A (n x n, row-major in global memory,
// n <= kMaxEig): parallel cyclic Jacobi with the round-robin pair schedule;
// on exit A's diagonal holds the eigenvalues and V the eigenvectors
// (columns).  Sweeps stop when the off-diagonal Frobenius norm is below
// 1e-15 of the total norm (at most 60 sweeps).

__global__ __launch_bounds__(256) void sym_jacobi_kernel(const EigJob* __restrict__ jobs, double* __restrict__ A_all,
                                                         double* __restrict__ V_all) {
  __shared__ double cs[kMaxEig / 2], sn[kMaxEig / 2];
  __shared__ int pp[kMaxEig / 2], qq[kMaxEig / 2];
  __shared__ double red[256];
  __shared__ int done;
  const EigJob J = jobs[blockIdx.x];
  const int n = J.n;
  double* A = A_all + J.off;
  double* V = V_all + J.off;
  const int tid = threadIdx.x;
  for (int64_t idx = tid; idx < (int64_t)n * n; idx += 256) V[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
  __syncthreads();
  const int K = (n + 1) & ~1;
  for (int sweep = 0; sweep < 60 && n > 1; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int64_t idx = tid; idx < (int64_t)n * n; idx += 256) {
      const double a = A[idx];
      tot += a * a;
      if (idx / n != idx % n) off += a * a;
    }
    red[tid] = off;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) red[tid] += red[tid + st];
      __syncthreads();
    }
    const double offs = red[0];
    __syncthreads();
    red[tid] = tot;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) red[tid] += red[tid + st];
      __syncthreads();
    }
    if (tid == 0) done = (offs <= 1e-30 * red[0]) ? 1 : 0;
    __syncthreads();
    if (done) break;
    for (int r = 0; r < K - 1; ++r) {
      for (int pr = tid; pr < K / 2; pr += 256) {
        const int a = (pr == 0) ? 0 : 1 + ((pr - 1 + r) % (K - 1));
        const int bq = 1 + ((K - 1 - pr - 1 + r) % (K - 1));
        const int p = a < bq ? a : bq, q = a < bq ? bq : a;
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[(int64_t)p * n + q];
          if (apq != 0.0) {
            const double th = (A[(int64_t)q * n + q] - A[(int64_t)p * n + p]) / (2.0 * apq);
            const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        cs[pr] = c;
        sn[pr] = s;
        pp[pr] = p;
        qq[pr] = q < n ? q : p;
      }
      __syncthreads();
      for (int64_t idx = tid; idx < (int64_t)(K / 2) * n; idx += 256) {
        const int pr = (int)(idx / n), j = (int)(idx % n);
        const int p = pp[pr], q = qq[pr];
        if (p == q) continue;
        const double c = cs[pr], s = sn[pr];
        const double ap = A[(int64_t)p * n + j], aq = A[(int64_t)q * n + j];
        A[(int64_t)p * n + j] = c * ap - s * aq;
        A[(int64_t)q * n + j] = s * ap + c * aq;
      }
      __syncthreads();
      for (int64_t idx = tid; idx < (int64_t)(K / 2) * n; idx += 256) {
        const int pr = (int)(idx / n), i = (int)(idx % n);
        const int p = pp[pr], q = qq[pr];
        if (p == q) continue;
        const double c = cs[pr], s = sn[pr];
        const double ap = A[(int64_t)i * n + p], aq = A[(int64_t)i * n + q];
        A[(int64_t)i * n + p] = c * ap - s * aq;
        A[(int64_t)i * n + q] = s * ap + c * aq;
        const double vp = V[(int64_t)i * n + p], vq = V[(int64_t)i * n + q];
        V[(int64_t)i * n + p] = c * vp - s * vq;
        V[(int64_t)i * n + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
}

hipError_t launch_sym_jacobi(const EigJob* jobs, int n_jobs, double* A, double* V, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(sym_jacobi_kernel, dim3(n_jobs), dim3(256), 0, s, jobs, A, V);
  return hipGetLastError();
}

// Columns of the new isometry: out[r * ncol + j] = sign_j * V[r * n + col_j]
// with sign_j making the largest-magnitude entry of the column positive.
__global__ __launch_bounds__(256) void gather_columns_kernel(const GatherJob* __restrict__ jobs,
                                                            const double* __restrict__ V_all, double* __restrict__ out) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  const GatherJob J = jobs[blockIdx.x];
  const double* V = V_all + J.v_off;
  const int n = J.n;
  for (int j = 0; j < J.ncol; ++j) {
    const int col = J.cols[j];
    double best = -1.0;
    int idx = 0;
    for (int r = threadIdx.x; r < n; r += 256) {
      const double a = fabs(V[(int64_t)r * n + col]);
      if (a > best) { best = a; idx = r; }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = idx;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st) {
        const double o = bv[threadIdx.x + st];
        const int oi = bi[threadIdx.x + st];
        if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
          bv[threadIdx.x] = o;
          bi[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    const double sg = V[(int64_t)bi[0] * n + col] < 0 ? -1.0 : 1.0;
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += 256) out[J.out_off + (int64_t)r * J.ncol + j] = sg * V[(int64_t)r * n + col];
    __syncthreads();
  }
}

hipError_t launch_gather_columns(const GatherJob* jobs, int n_jobs, const double* V, double* out, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_columns_kernel, dim3(n_jobs), dim3(256), 0, s, jobs, V, out);
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
