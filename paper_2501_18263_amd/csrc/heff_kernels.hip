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

// b if c else a, by integer masking: a conditional choice between two
// members of a private array must not become an indexed access to it
// (that would place the array in scratch memory)
template <typename T>
__device__ __forceinline__ const T* pick(bool c, const T* a, const T* b) {
  const uint64_t x = (uint64_t)a, y = (uint64_t)b, m = 0 - (uint64_t)c;
  return (const T*)(x ^ ((x ^ y) & m));
}

// ------------------------------------------------------------------ chained product (MFMA)
// Matrix-core version: one work-group = 4 waves = 64 rows of one output
// block; wave w owns rows [16w, 16w+16).  A task  f op(L) op(X) op(R)  is
// run as a sequence of steps over 16-wide slices:
//   stage 1, one step per 16 values of the inner index k of op(L) op(X):
//            T[rows][0..c) += op(L)[rows][k..k+16) op(X)[k..k+16)[0..c),
//            with T held in registers as 16x16 MFMA result tiles;
//   stage 2, one step per 16-row slice j of op(R):
//            acc[rows][0..e) += f T[rows][j..j+16) op(R)[j..j+16)[0..e).
// The op(X) and op(R) slices are shared by the four waves and pass through
// LDS; each wave reads its own op(L) values straight into registers.  The
// step loop is software pipelined: the global loads of step s+1 (the next
// task's first slice when the task ends) are issued before the MFMAs of step
// s and land in the other half of a double-buffered LDS area, so one
// barrier per step suffices and the memory latency overlaps the matrix work.
// Identity operands (flags T_IDL/T_IDX/T_IDR) are generated in place of
// loads.  Stage-1 MFMA result registers are the stage-2 A operands without
// any data movement: register i of lane (g, n) of tile cc holds
// T[row n][16 cc + row(i, g)], the A operand for k = 16 cc + row(i, g).
// Operand layout of both instructions: lane l holds A[l%16][l/16] and
// B[l/16][l%16].  Result layout differs: register r of lane l holds
// D[row(r, l/16)][l%16] with row = 4r + l/16 for f64 and 4(l/16) + r for f32
// (checked on the device).  kmin(r) is the smallest row(r, g) over g.
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 run(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int g) { return 4 * r + g; }
  static __device__ __forceinline__ int kmin(int r) { return 4 * r; }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 run(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int g) { return 4 * g + r; }
  static __device__ __forceinline__ int kmin(int r) { return r; }
};

// LDS of one work-group: two step buffers (double buffering), each holding
// one slice of op(X) [16][XST] (k-major) or of op(R) [16][RST], plus the
// matching slice of op(L) [64][LST] for stage-1 steps.  The row strides are
// chosen so that both the slice stores (16 lanes down a column when the
// operand is stored transposed) and the operand reads (16 lanes along a row,
// four row groups) spread over the banks.
template <typename T, int NT>
struct ChainSmem {
  static constexpr int W = 16 * NT;  // largest c and e of the variant
  static constexpr int XST = sizeof(T) == 8 ? W + 17 : W + 20;
  static constexpr int RST = sizeof(T) == 8 ? W + 17 : W + 4;
  static constexpr int LST = 17;
  static constexpr int SL = 16 * (XST > RST ? XST : RST);
  T buf[2][SL];
  T lbuf[2][64 * LST];
};

// Step cursor: task index, stage (0/1) and slice index within the stage.
struct Cursor {
  int ti, ph, s;
};

// advance to the next step; false past the tile's last task.  `pre` holds
// the descriptor of the task after cu.ti (loaded one task ahead).
__device__ __forceinline__ bool next_step(Cursor& cu, Task& t, Task& pre, const Task* __restrict__ tasks, int t1) {
  ++cu.s;
  const int n = cu.ph == 0 ? (t.b + 15) >> 4 : (t.c + 15) >> 4;
  if (cu.s < n) return true;
  if (cu.ph == 0) {
    cu.ph = 1;
    cu.s = 0;
    return true;
  }
  if (++cu.ti >= t1) return false;
  t = pre;
  pre = tasks[min(cu.ti + 1, t1 - 1)];
  cu.ph = 0;
  cu.s = 0;
  return true;
}

// Per-thread coordinates inside the slices.  A 16 x W slice is walked in one
// of two orders, chosen by which index is contiguous in global memory:
//   k-contiguous (operand stored transposed): k = t15, m = t4 + 16 q;
//   m-contiguous:                             k = tW + (256/W) q, m = tm.
// The 64 x 16 op(L) slice: k-contiguous r = t4 + 16 q, k = t15; transposed
// storage r = t63, k = t6 + 4 q.
template <int W>
struct Lane {
  int t15, t4, tW, tm, t6, t63;
  __device__ __forceinline__ explicit Lane(int tid)
      : t15(tid & 15), t4(tid >> 4), tW(tid / W), tm(tid % W), t6(tid >> 6), t63(tid & 63) {}
};

// Staged values of one step for one thread: NT elements of the op(X) or
// op(R) slice and 4 of the op(L) slice (stage 1 only).
template <typename T, int NT>
struct Stage {
  T v[NT];
  T l[4];
};

// Issue the global loads of one step; no loaded value is used here, so they
// stay in flight during the matrix work of the current step.  Indices past
// the operand's extent are clamped to its last row or column: such slice
// entries only meet zeros of the other operand (op(L) columns past b and
// op(R) rows past c are zeroed when stored) or feed rows/columns of the
// result that are never written, so they need only be finite values.
// Identity operands load nothing.
template <typename T, int NT>
__device__ __forceinline__ Stage<T, NT> load_step(const Task& t, const Bases<T>& B, const Cursor& cu,
                                                  const Lane<16 * NT>& ln, int row0) {
  constexpr int KQ = 256 / (16 * NT);
  Stage<T, NT> st;
  const uint32_t fl = t.flags;
  const int base = 16 * cu.s;
  if (cu.ph == 0) {
    const int kmax = t.b - base - 1, cmax = t.c - 1;
    if (!(fl & T_IDX)) {
      const uint32_t ld = t.ldX;
      if (fl & T_TX) {
        const T* X = pick((fl & T_SELX) != 0, B.X[0], B.X[1]) + t.offX + base;
        const uint32_t k = min(ln.t15, kmax);
#pragma unroll
        for (int q = 0; q < NT; ++q) st.v[q] = X[(uint32_t)min(ln.t4 + 16 * q, cmax) * ld + k];
      } else {
        const T* X = pick((fl & T_SELX) != 0, B.X[0], B.X[1]) + t.offX + (int64_t)base * ld;
        const uint32_t m = min(ln.tm, cmax);
#pragma unroll
        for (int q = 0; q < NT; ++q) st.v[q] = X[(uint32_t)min(ln.tW + KQ * q, kmax) * ld + m];
      }
    }
    if (!(fl & T_IDL)) {
      const uint32_t ld = t.ldL;
      const int rmax = t.a - row0 - 1;
      if (fl & T_TL) {
        const T* L = pick((fl & T_SELL) != 0, B.L[0], B.L[1]) + t.offL + row0 + (int64_t)base * ld;
        const uint32_t r = min(ln.t63, rmax);
#pragma unroll
        for (int q = 0; q < 4; ++q) st.l[q] = L[(uint32_t)min(ln.t6 + 4 * q, kmax) * ld + r];
      } else {
        const T* L = pick((fl & T_SELL) != 0, B.L[0], B.L[1]) + t.offL + (int64_t)row0 * ld + base;
        const uint32_t kk = min(ln.t15, kmax);
#pragma unroll
        for (int q = 0; q < 4; ++q) st.l[q] = L[(uint32_t)min(ln.t4 + 16 * q, rmax) * ld + kk];
      }
    }
  } else if (!(fl & T_IDR)) {
    const int jmax = t.c - base - 1, emax = t.e - 1;
    const uint32_t ld = t.ldR;
    if (fl & T_TR) {
      const T* R = pick((fl & T_SELR) != 0, B.R[0], B.R[1]) + t.offR + base;
      const uint32_t j = min(ln.t15, jmax);
#pragma unroll
      for (int q = 0; q < NT; ++q) st.v[q] = R[(uint32_t)min(ln.t4 + 16 * q, emax) * ld + j];
    } else {
      const T* R = pick((fl & T_SELR) != 0, B.R[0], B.R[1]) + t.offR + (int64_t)base * ld;
      const uint32_t col = min(ln.tm, emax);
#pragma unroll
      for (int q = 0; q < NT; ++q) st.v[q] = R[(uint32_t)min(ln.tW + KQ * q, jmax) * ld + col];
    }
  }
  return st;
}

// Write the values of one step to LDS buffer P: generate identity operands,
// scale the op(L) slice by the task factor f and zero its columns past b,
// zero the op(R) rows past c.
template <typename T, int NT, int P>
__device__ __forceinline__ void store_step(const Task& t, const Cursor& cu, const Lane<16 * NT>& ln, int row0,
                                           const Stage<T, NT>& st, ChainSmem<T, NT>& sm) {
  constexpr int W = 16 * NT, KQ = 256 / W;
  using S = ChainSmem<T, NT>;
  const uint32_t fl = t.flags;
  const int base = 16 * cu.s;
  T* buf = sm.buf[P];
  if (cu.ph == 0) {
    const int klim = t.b - base;
    if (fl & T_IDX) {
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const int kk = ln.tW + KQ * q;
        buf[kk * S::XST + ln.tm] = T(base + kk == ln.tm ? 1 : 0);
      }
    } else if (fl & T_TX) {
#pragma unroll
      for (int q = 0; q < NT; ++q) buf[ln.t15 * S::XST + ln.t4 + 16 * q] = st.v[q];
    } else {
#pragma unroll
      for (int q = 0; q < NT; ++q) buf[(ln.tW + KQ * q) * S::XST + ln.tm] = st.v[q];
    }
    T* lb = sm.lbuf[P];
    const T f = (T)t.f;
    if (fl & T_IDL) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = ln.t4 + 16 * q;
        lb[r * S::LST + ln.t15] = (row0 + r == base + ln.t15) ? f : T(0);
      }
    } else if (fl & T_TL) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = ln.t6 + 4 * q;
        lb[ln.t63 * S::LST + kk] = kk < klim ? st.l[q] * f : T(0);
      }
    } else {
      const bool ok = ln.t15 < klim;
#pragma unroll
      for (int q = 0; q < 4; ++q) lb[(ln.t4 + 16 * q) * S::LST + ln.t15] = ok ? st.l[q] * f : T(0);
    }
  } else {
    const int jlim = t.c - base;
    if (fl & T_IDR) {
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const int j = ln.tW + KQ * q;
        buf[j * S::RST + ln.tm] = T(base + j == ln.tm ? 1 : 0);
      }
    } else if (fl & T_TR) {
      const bool ok = ln.t15 < jlim;
#pragma unroll
      for (int q = 0; q < NT; ++q) buf[ln.t15 * S::RST + ln.t4 + 16 * q] = ok ? st.v[q] : T(0);
    } else if (jlim >= 16) {
#pragma unroll
      for (int q = 0; q < NT; ++q) buf[(ln.tW + KQ * q) * S::RST + ln.tm] = st.v[q];
    } else {
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const int j = ln.tW + KQ * q;
        buf[j * S::RST + ln.tm] = j < jlim ? st.v[q] : T(0);
      }
    }
  }
}

// Stage-1 step on the first NC result tiles of T (columns 16 NC), stage-2
// step of T tile CC on the first NE output tiles; NC, CC and NE are
// compile-time so the matrix instructions form straight-line, in-place
// accumulation chains with immediate LDS offsets.
template <typename T, int NT, int NC, int P>
__device__ __forceinline__ void stage1(typename Mfma<T>::v4 (&Tc)[NT], const ChainSmem<T, NT>& sm, int wave, int g,
                                       int n) {
  using S = ChainSmem<T, NT>;
  const T* buf = sm.buf[P] + g * S::XST + n;
  const T* lb = sm.lbuf[P] + (wave * 16 + n) * S::LST + g;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const T lv = lb[4 * j];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) Tc[cc] = Mfma<T>::run(buf[4 * j * S::XST + cc * 16], lv, Tc[cc]);
  }
}
template <typename T, int NT, int NE, int CC, int P>
__device__ __forceinline__ void stage2(typename Mfma<T>::v4 (&acc)[NT], const typename Mfma<T>::v4 (&Tc)[NT],
                                       const ChainSmem<T, NT>& sm, int g, int n) {
  using S = ChainSmem<T, NT>;
  const T* buf = sm.buf[P] + n;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = Mfma<T>::row(i, g);
#pragma unroll
    for (int nt = 0; nt < NE; ++nt) acc[nt] = Mfma<T>::run(Tc[CC][i], buf[j * S::RST + nt * 16], acc[nt]);
  }
}
// Binary-tree dispatch of a runtime count in [LO, HI] to compile-time
// instances (log2 branches instead of a linear chain).
template <typename T, int NT, int LO, int HI, int P>
__device__ __forceinline__ void stage1_sw(int nc, typename Mfma<T>::v4 (&Tc)[NT], const ChainSmem<T, NT>& sm, int wave,
                                          int g, int n) {
  if constexpr (LO == HI) {
    stage1<T, NT, LO, P>(Tc, sm, wave, g, n);
  } else {
    constexpr int MID = (LO + HI) / 2;
    if (nc <= MID) stage1_sw<T, NT, LO, MID, P>(nc, Tc, sm, wave, g, n);
    else stage1_sw<T, NT, MID + 1, HI, P>(nc, Tc, sm, wave, g, n);
  }
}
template <typename T, int NT, int NE, int LO, int HI, int P>
__device__ __forceinline__ void stage2_sw(int s, typename Mfma<T>::v4 (&acc)[NT],
                                          const typename Mfma<T>::v4 (&Tc)[NT], const ChainSmem<T, NT>& sm, int g,
                                          int n) {
  if constexpr (LO == HI) {
    stage2<T, NT, NE, LO, P>(acc, Tc, sm, g, n);
  } else {
    constexpr int MID = (LO + HI) / 2;
    if (s <= MID) stage2_sw<T, NT, NE, LO, MID, P>(s, acc, Tc, sm, g, n);
    else stage2_sw<T, NT, NE, MID + 1, HI, P>(s, acc, Tc, sm, g, n);
  }
}

// One pipeline step on LDS buffer P: loads of step c1 into registers, matrix
// work of step c0, LDS store of step c1 into buffer P^1, barrier.
template <typename T, int NT, int NE, int P>
__device__ __forceinline__ void pipe_step(const Tile& tile, const Task* __restrict__ tasks, const Bases<T>& B,
                                          ChainSmem<T, NT>& sm, const Lane<16 * NT>& ln, int row0, bool wave_on,
                                          int wave, int g, int n, typename Mfma<T>::v4 (&Tc)[NT],
                                          typename Mfma<T>::v4 (&acc)[NT], bool& live, Cursor& c0, Task& t0,
                                          Task& pre) {
  using v4 = typename Mfma<T>::v4;
  Cursor c1 = c0;
  Task t1 = t0;
  const bool more = next_step(c1, t1, pre, tasks, tile.t1);
  Stage<T, NT> st;
  if (more) st = load_step<T, NT>(t1, B, c1, ln, row0);
  if (wave_on) {
    if (c0.ph == 0) {
      if (c0.s == 0) {
#pragma unroll
        for (int cc = 0; cc < NT; ++cc) Tc[cc] = v4{0, 0, 0, 0};
      }
      stage1_sw<T, NT, 1, NT, P>(min(NT, (t0.c + 15) >> 4), Tc, sm, wave, g, n);
    } else {
      stage2_sw<T, NT, NE, 0, NT - 1, P>(c0.s, acc, Tc, sm, g, n);
    }
  }
  if (more) store_step<T, NT, P ^ 1>(t1, c1, ln, row0, st, sm);
  __syncthreads();
  live = more;
  c0 = c1;
  t0 = t1;
}

// One work item (64 rows of one output tile, NE 16-column output tiles).
// Software pipeline: while step s computes from LDS buffer s%2, the global
// loads of step s+1 are in flight and are written to the other buffer after
// the matrix work; one barrier per step.  The loop body is unrolled twice so
// that the buffer index is a compile-time constant.  Waves whose rows lie
// outside the tile take part in the loads and barriers but skip the matrix
// work.
template <typename T, int NT, int NE>
__device__ __forceinline__ void chain_item_e(const Tile& tile, const Work& w, const Task* __restrict__ tasks,
                                             const Bases<T>& B, ChainSmem<T, NT>& sm) {
  using M = Mfma<T>;
  using v4 = typename M::v4;
  const int tid = threadIdx.x;
  const Lane<16 * NT> ln(tid);
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g = lane >> 4, n = lane & 15;
  const int wrow0 = w.row0 + wave * 16;
  const bool wave_on = wrow0 < tile.a;
  const int E = tile.e;
  v4 acc[NT], Tc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = v4{0, 0, 0, 0};
  if (tile.t0 < tile.t1) {
    Cursor c0{tile.t0, 0, 0};
    Task t0 = tasks[tile.t0];
    Task pre = tasks[min(tile.t0 + 1, tile.t1 - 1)];
    {
      const Stage<T, NT> st = load_step<T, NT>(t0, B, c0, ln, w.row0);
      store_step<T, NT, 0>(t0, c0, ln, w.row0, st, sm);
    }
    __syncthreads();
    bool live = true;
    while (live) {
      pipe_step<T, NT, NE, 0>(tile, tasks, B, sm, ln, w.row0, wave_on, wave, g, n, Tc, acc, live, c0, t0, pre);
      if (!live) break;
      pipe_step<T, NT, NE, 1>(tile, tasks, B, sm, ln, w.row0, wave_on, wave, g, n, Tc, acc, live, c0, t0, pre);
    }
  }
  if (!wave_on) return;
#pragma unroll
  for (int nt = 0; nt < NE; ++nt) {
    const int col = nt * 16 + n;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wrow0 + M::row(i, g);
      if (r < tile.a && col < E) B.out[tile.offOut + (int64_t)r * tile.ldOut + col] = acc[nt][i];
    }
  }
}

// Output-width bucket of a tile: the kernel instance holds NE = NT/4, NT/2,
// 3NT/4 or NT output tiles (at least one), the smallest that covers e.
template <int NT, int Q>
struct NeBucket {
  static constexpr int value = (NT * Q) / 4 > 0 ? (NT * Q) / 4 : 1;
};

template <typename T, int NT>
__device__ __forceinline__ void chain_item(const Tile& tile, const Work& w, const Task* __restrict__ tasks,
                                           const Bases<T>& B, ChainSmem<T, NT>& sm) {
  const int ne = (tile.e + 15) >> 4;
  if (ne <= NeBucket<NT, 1>::value)
    chain_item_e<T, NT, NeBucket<NT, 1>::value>(tile, w, tasks, B, sm);
  else if (ne <= NeBucket<NT, 2>::value)
    chain_item_e<T, NT, NeBucket<NT, 2>::value>(tile, w, tasks, B, sm);
  else if (ne <= NeBucket<NT, 3>::value)
    chain_item_e<T, NT, NeBucket<NT, 3>::value>(tile, w, tasks, B, sm);
  else
    chain_item_e<T, NT, NT>(tile, w, tasks, B, sm);
}

// Several work-groups per CU for the variants up to 128 wide (the other
// groups' waves fill the issue gaps and memory waits of the step loop): two
// for FP64 (at 128 wide this costs a few spilled registers and is still much
// faster), three for FP32.
template <typename T, int NT>
__global__ __launch_bounds__(256, NT <= 8 ? (sizeof(T) == 4 ? 3 : 2) : 1) void chain_mfma(
    const Tile* __restrict__ tiles, const Work* __restrict__ work,
                                                  const Task* __restrict__ tasks, Bases<T> B) {
  __shared__ ChainSmem<T, NT> sm;
  const Work w = work[blockIdx.x];
  if (w.row0 < 0) return;  // unused position of the XCD-ordered list
  chain_item<T, NT>(tiles[w.tile], w, tasks, B, sm);
}

// Batched, persistent form: a fixed grid strides over the work items of
// many independent problems (tile.prob selects the problem's operator
// stores; Psi and the output of all problems share one base each).
template <typename T, int NT>
__global__ __launch_bounds__(256) void chain_mfma_batch(const Tile* __restrict__ tiles, const Work* __restrict__ work,
                                                        int64_t n_work, const Task* __restrict__ tasks,
                                                        const ProbBases<T>* __restrict__ pb, const T* X, T* out) {
  __shared__ ChainSmem<T, NT> sm;
  for (int64_t i = blockIdx.x; i < n_work; i += gridDim.x) {
    const Work w = work[i];
    if (w.row0 < 0) continue;  // unused position of the XCD-ordered list
    const Tile tile = tiles[w.tile];
    const ProbBases<T> q = pb[tile.prob];
    Bases<T> B;
    B.L[0] = q.L[0];
    B.L[1] = q.L[1];
    B.R[0] = q.R[0];
    B.R[1] = q.R[1];
    B.X[0] = B.X[1] = X;
    B.out = out;
    chain_item<T, NT>(tile, w, tasks, B, sm);
    __syncthreads();  // LDS reuse by the next item
  }
}

hipError_t launch_mfma_batch_f32(const Tile* tiles, const WorkSet& ws, const Task* tasks, const ProbBases<float>* pb,
                                 const float* X, float* out, const int grid[kNumVariants], const hipStream_t* ss) {
  for (int v = kNumVariants - 1; v >= 0; --v) {
    if (ws.n[v] <= 0) continue;
    hipStream_t s = ss[v];
    dim3 gr((unsigned)grid[v]), blk(256);
    switch (v) {
      case 0: hipLaunchKernelGGL((chain_mfma_batch<float, 2>), gr, blk, 0, s, tiles, ws.w[v], ws.n[v], tasks, pb, X, out); break;
      case 1: hipLaunchKernelGGL((chain_mfma_batch<float, 4>), gr, blk, 0, s, tiles, ws.w[v], ws.n[v], tasks, pb, X, out); break;
      case 2: hipLaunchKernelGGL((chain_mfma_batch<float, 8>), gr, blk, 0, s, tiles, ws.w[v], ws.n[v], tasks, pb, X, out); break;
      default: hipLaunchKernelGGL((chain_mfma_batch<float, 16>), gr, blk, 0, s, tiles, ws.w[v], ws.n[v], tasks, pb, X, out); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------------------------ chained product, LDS-DMA pipeline
// FP64, all output widths.  Same work items, task order and
// per-element arithmetic as chain_mfma (f folded into the op(L) value, the
// same MFMA sequence; results are bitwise identical), but the operand slices
// go straight from global memory to LDS with global_load_lds_dwordx4: each
// wave instruction moves 16 bytes (two consecutive elements of a stored row)
// per lane into 1 KB of consecutive LDS (LDS address = M0 + 16 lane; the
// global address is per lane and only needs 8-byte alignment).  Where a
// pair could reach past the end of its buffer (buffer lengths unknown, or
// the block is the buffer's last), the operand falls back to
// global_load_lds_dword, one dword per lane into 256 bytes.  No staging
// registers are needed, so the slices pass through a ring of three LDS
// buffers: the loads of step s + 2 are in flight while step s computes,
// which hides two steps of memory latency instead of one.  (For FP32, with
// three work-groups per CU hiding the latency already, the register-staged
// kernel measured faster, so FP32 keeps it.)
//
// Every slice is held as 16 x 16 blocks of 256 elements.  Element (k, m) of
// a block (k: contraction index of the step, m: row or column of the other
// operand) sits at
//   N  16 k + m               when the operand is stored with k as its row
//                             index,
//   T  16 m + (k ^ (m & 14))  when it is stored with k contiguous
// (the XOR keeps the two elements of a 16-byte pair adjacent and in order).
// Each layout puts one wave instruction's 256 bytes on 256 contiguous bytes
// of global rows (a permutation inside them) and lets the 64 lanes of every
// operand read hit distinct LDS banks (two lanes per bank pair, the minimum
// for 512 bytes).  Entries past the operand's extent are loaded
// from clamped (in-block) addresses and masked at read time: op(L) values
// with k >= b and stage-2 T values with j >= c are replaced by zero, the
// factor f multiplies the op(L) value.  Identity operands: op(L) = I is
// generated in registers, op(X) = I and op(R) = I are written to the ring
// with LDS stores.
namespace dmak {


// Ring depth and work-groups per CU.  Up to 128 wide, two work-groups per
// CU (the other group's matrix work fills this one's barrier and issue time)
// with a three-slot ring measured faster than one work-group with a
// four-slot ring; the kernel must not spill there (a spill reload waits for
// every outstanding load of the wave, ring loads included).  The 256-wide
// instance (two 256-wide FP64 register tiles) runs one work-group per CU
// with 120 KB of ring; it spills a few registers and is still faster than
// the register-staged kernel (1507 vs 1726 ms at N=40 D=4096 with the wider
// sectors of beta = 1).
template <typename T, int NT>
struct Cfg {
  static_assert(sizeof(T) == 8, "ring kernel is the FP64 path");
  static constexpr int stages = 3;
  static constexpr int groups = NT <= 8 ? 2 : 1;
};
typedef __attribute__((address_space(3))) char lds_char;

__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(const lds_char*)p);
}
__device__ __forceinline__ const char* sgpr_ptr(const char* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (const char*)(((uint64_t)hi << 32) | lo);
}
// LDS[m0 + 4 lane] = dword at sbase + voff (bytes).  A global load into
// LDS needs one wait state after the write of M0.
__device__ __forceinline__ void dma(const char* sbase, uint32_t voff, uint32_t m0) {
  asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dword %0, %1" : : "v"(voff), "s"(sbase), "s"(m0)
               : "memory");
}
// LDS[m0 + 16 lane, + 16) = the 16 bytes at sbase + voff (8-byte aligned)
__device__ __forceinline__ void dma16(const char* sbase, uint32_t voff, uint32_t m0) {
  asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1" : : "v"(voff), "s"(sbase),
               "s"(m0)
               : "memory");
}
template <int N>
__device__ __forceinline__ void wait_vm() {
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}
// wait until at most n vector-memory instructions of this wave are
// outstanding (n rounded down to even, at most 62: waiting for fewer is
// always safe); binary tree over the even counts
template <int LO, int HI>
__device__ __forceinline__ void wait_vm_tree(int n) {
  if constexpr (LO == HI) {
    wait_vm<LO>();
  } else {
    constexpr int MID = ((LO + HI) / 4) * 2;
    if (n <= MID + 1) wait_vm_tree<LO, MID>(n);
    else wait_vm_tree<MID + 2, HI>(n);
  }
}
__device__ __forceinline__ void wait_vm_le(int n) { wait_vm_tree<0, 62>(n < 62 ? n : 62); }
// barrier that orders LDS accesses only (a full __syncthreads would also
// wait for every outstanding global load, including the ring's)
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename T, int NT>
struct Smem {
  static constexpr int S = Cfg<T, NT>::stages;
  T xs[S][NT * 256];  // op(X) or op(R) slice, NT blocks
  T ls[S][4 * 256];   // op(L) slice, one block per wave
};

// What the matrix work of a step needs (filled when its loads are issued),
// packed to keep the three records of the ring in few scalar registers:
// bc = b | c << 16; m = flags (bits 0-8) | ph << 9 | valid << 10 |
// cnt << 11 (ring loads per wave, < 64) | s << 17 (slice index).  A step
// issues at most 2 NT + 8 loads per wave (dword loads of NT op(X) blocks
// and of the wave's op(L) block), so six bits hold the count.
struct Rec {
  double f;
  uint32_t bc, m;
  __device__ __forceinline__ int b() const { return (int)(bc & 0xffff); }
  __device__ __forceinline__ int c() const { return (int)(bc >> 16); }
  __device__ __forceinline__ uint32_t flags() const { return m & 0x1ff; }
  __device__ __forceinline__ int ph() const { return (int)((m >> 9) & 1); }
  __device__ __forceinline__ bool valid() const { return (m >> 10) & 1; }
  __device__ __forceinline__ int cnt() const { return (int)((m >> 11) & 63); }
  __device__ __forceinline__ int s() const { return (int)(m >> 17); }
};
template <typename T, int NT>
using Ring = Rec[Cfg<T, NT>::stages];

// Per-lane constants.  Lane l = 16 g + n.
//   16-byte loads: in 1 KB window q (0, 1) of a block lane l writes
//   elements 128 q + 2 l, + 1, stored at (row, column) = (8 q + r8, c + d)
//   (d = 0, 1) with r8 = l >> 3 and, for N, c = 2 (l & 7) (row = k), for T,
//   c = (2 (l & 7) ^ ((l >> 3) & 6)) ^ 8 q (row = m, column = k).
//   Dword loads: in 256-byte window q (0..7) lane l writes dword l & 1 of
//   element 32 q + l / 2, stored at (row, column) = (2 q + y, mcol) for N and
//   (2 q + y, mcol ^ 2 q) for T.
typedef int i4 __attribute__((ext_vector_type(4)));

template <typename T>
struct LaneC {
  int lane, g, n, y, mcol, h, r8, cn, ct;
  i4 tp;  // T position of (k = 4j + g, m = n)
  __device__ __forceinline__ explicit LaneC(int tid) {
    lane = tid & 63;
    g = lane >> 4;
    n = lane & 15;
    y = lane >> 5;
    mcol = (lane >> 1) & 15;
    h = lane & 1;
    r8 = lane >> 3;
    cn = 2 * (lane & 7);
    ct = cn ^ (r8 & 6);
#pragma unroll
    for (int j = 0; j < 4; ++j) tp[j] = 16 * n + ((4 * j + g) ^ (n & 14));
  }
};

// Clamped scalar start of a slice block: the block's base element offset
// sb (relative to the stored block) is limited to the last stored element
// `end`; rel is how far lanes may reach past it.
struct Span {
  uint32_t sb, rel;
  __device__ __forceinline__ Span(uint32_t sb0, uint32_t end) {
    sb = sb0 < end ? sb0 : end;
    rel = end - sb;
  }
};

// Ring loads of nb 16 x 16 blocks of one operand slice, block i starting at
// element soff + i step of the stored block and landing at LDS m0 + i 2 KB;
// the windows are shared out over the four waves.  Returns the loads this
// wave issued.
template <typename T>
__device__ __forceinline__ int load_blocks(const char* base, uint32_t soff, uint32_t step, uint32_t end, bool x4,
                                           int nb, bool kr, uint32_t ld, uint32_t m0, const LaneC<T>& lc,
                                           int wave) {
  constexpr uint32_t BB = 256 * sizeof(T);
  int cnt = 0;
  if (x4) {
    const uint32_t l0 = (uint32_t)lc.r8 * ld + (uint32_t)(kr ? lc.cn : lc.ct);
    const uint32_t l1 = (uint32_t)(lc.r8 + 8) * ld + (uint32_t)(kr ? lc.cn : (lc.ct ^ 8));
#pragma unroll 1
    for (int v = wave; v < 2 * nb; v += 4) {
      const int i = v >> 1;
      const Span sp(soff + (uint32_t)i * step, end);
      uint32_t off = (v & 1) ? l1 : l0;
      off = off < sp.rel ? off : sp.rel;
      dma16(sgpr_ptr(base + (uint64_t)sp.sb * sizeof(T)), off * (uint32_t)sizeof(T), m0 + i * BB + (v & 1) * 1024);
      ++cnt;
    }
  } else {
#pragma unroll 1
    for (int i = 0; i < nb; ++i) {
      const Span sp(soff + (uint32_t)i * step, end);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int q = 2 * wave + u;
        const uint32_t z = kr ? (uint32_t)lc.mcol : (uint32_t)(lc.mcol ^ (2 * q));
        uint32_t off = (uint32_t)(2 * q + lc.y) * ld + z;
        off = off < sp.rel ? off : sp.rel;
        dma(sgpr_ptr(base + (uint64_t)sp.sb * sizeof(T)), off * (uint32_t)sizeof(T) + 4u * lc.h,
            m0 + i * BB + q * 256);
      }
      cnt += 2;
    }
  }
  return cnt;
}
// Ring loads of one whole block by this wave (its op(L) rows).
template <typename T>
__device__ __forceinline__ int load_own_block(const char* base, const Span& sp, bool x4, bool kr, uint32_t ld,
                                              uint32_t m0, const LaneC<T>& lc) {
  const char* sb = sgpr_ptr(base + (uint64_t)sp.sb * sizeof(T));
  if (x4) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      uint32_t off = (uint32_t)(lc.r8 + 8 * q) * ld + (uint32_t)(kr ? lc.cn : (lc.ct ^ (8 * q)));
      off = off < sp.rel ? off : sp.rel;
      dma16(sb, off * (uint32_t)sizeof(T), m0 + q * 1024);
    }
    return 2;
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const uint32_t z = kr ? (uint32_t)lc.mcol : (uint32_t)(lc.mcol ^ (2 * q));
    uint32_t off = (uint32_t)(2 * q + lc.y) * ld + z;
    off = off < sp.rel ? off : sp.rel;
    dma(sb, off * (uint32_t)sizeof(T) + 4u * lc.h, m0 + q * 256);
  }
  return 8;
}
// whether a 16-byte pair starting at any element of a stored block (at
// element offset off, last element end) stays inside a buffer of lim
// elements
__device__ __forceinline__ bool pairs_fit(int64_t off, uint32_t end, int64_t lim) {
  return off + (int64_t)end + 1 < lim;
}

// Issue the ring loads of the step at cursor (cu, t) into slot KI and fill
// its record; then advance the cursor (ivalid false past the tile's tasks).
template <typename T, int NT, int NE, int KI>
__device__ __forceinline__ void issue(Rec& rec, Cursor& cu, Task& t, Task& pre, bool& ivalid,
                                      const Task* __restrict__ tasks, int t1, const Bases<T>& B, Smem<T, NT>& sm,
                                      const LaneC<T>& lc, int row0, int wave) {
  if (!ivalid) {
    rec.m = 0;
    return;
  }
  const uint32_t fl = t.flags;
  rec.f = t.f;
  rec.bc = (uint32_t)t.b | ((uint32_t)t.c << 16);
  const int s16 = 16 * cu.s;
  const int tid = threadIdx.x;
  int cnt = 0;
  if (cu.ph == 0) {
    const int nc = min(NT, (t.c + 15) >> 4);
    const bool kr = !(fl & T_TX);
    if (fl & T_IDX) {
      const int E = tid;
      const int k = kr ? (E >> 4) : ((E & 15) ^ ((E >> 4) & 14));
      const int m = kr ? (E & 15) : (E >> 4);
#pragma unroll
      for (int cc = 0; cc < NT; ++cc)
        if (cc < nc) sm.xs[KI][cc * 256 + E] = T(s16 + k == 16 * cc + m ? 1 : 0);
    } else {
      const uint32_t ld = t.ldX;
      const int sel = (fl & T_SELX) != 0;
      const char* xb = (const char*)(pick(sel, B.X[0], B.X[1]) + t.offX);
      const uint32_t end = kr ? (uint32_t)(t.b - 1) * ld + (t.c - 1) : (uint32_t)(t.c - 1) * ld + (t.b - 1);
      cnt += load_blocks<T>(xb, kr ? (uint32_t)s16 * ld : (uint32_t)s16, kr ? 16u : 16u * ld, end,
                            pairs_fit(t.offX, end, sel ? B.lim[3] : B.lim[2]), nc, kr, ld, lds_addr(&sm.xs[KI][0]),
                            lc, wave);
    }
    if (!(fl & T_IDL)) {
      const bool klr = (fl & T_TL) != 0;
      const uint32_t ld = t.ldL;
      const int sel = (fl & T_SELL) != 0;
      const char* lb = (const char*)(pick(sel, B.L[0], B.L[1]) + t.offL);
      const int r0 = row0 + 16 * wave;
      const uint32_t end = klr ? (uint32_t)(t.b - 1) * ld + (t.a - 1) : (uint32_t)(t.a - 1) * ld + (t.b - 1);
      const Span sp(klr ? (uint32_t)s16 * ld + r0 : (uint32_t)r0 * ld + s16, end);
      cnt += load_own_block<T>(lb, sp, pairs_fit(t.offL, end, sel ? B.lim[1] : B.lim[0]), klr, ld,
                               lds_addr(&sm.ls[KI][wave * 256]), lc);
    }
  } else {
    const bool kr = !(fl & T_TR);
    if (fl & T_IDR) {
      const int E = tid;
      const int j = kr ? (E >> 4) : ((E & 15) ^ ((E >> 4) & 14));
      const int col = kr ? (E & 15) : (E >> 4);
#pragma unroll
      for (int nt = 0; nt < NE; ++nt) sm.xs[KI][nt * 256 + E] = T(s16 + j == 16 * nt + col ? 1 : 0);
    } else {
      const uint32_t ld = t.ldR;
      const int sel = (fl & T_SELR) != 0;
      const char* rb = (const char*)(pick(sel, B.R[0], B.R[1]) + t.offR);
      const uint32_t end = kr ? (uint32_t)(t.c - 1) * ld + (t.e - 1) : (uint32_t)(t.e - 1) * ld + (t.c - 1);
      cnt += load_blocks<T>(rb, kr ? (uint32_t)s16 * ld : (uint32_t)s16, kr ? 16u : 16u * ld, end,
                            pairs_fit(t.offR, end, sel ? B.lim[5] : B.lim[4]), NE, kr, ld, lds_addr(&sm.xs[KI][0]),
                            lc, wave);
    }
  }
  static_assert(2 * NT + 8 < 64, "ring loads per wave must fit the record's six-bit count");
  rec.m = (fl & 0x1ff) | ((uint32_t)cu.ph << 9) | (1u << 10) | ((uint32_t)cnt << 11) | ((uint32_t)cu.s << 17);
  ivalid = next_step(cu, t, pre, tasks, t1);
}

// Stage-1 matrix work of k-groups J0, J0 + 1 on the first NC tiles of T:
// x positions px, op(L) values lv (already scaled and masked).
template <typename T, int NT, int NC, int K, int J0>
__device__ __forceinline__ void stage1(typename Mfma<T>::v4 (&Tc)[NT], const Smem<T, NT>& sm, const i4 px,
                                       const typename Mfma<T>::v4 lv, int klim) {
  const T* xs = sm.xs[K];
#pragma unroll
  for (int j = J0; j < J0 + 2; ++j) {
    if (j > 0 && 4 * j >= klim) break;  // k-group past b: adds only zeros
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) Tc[cc] = Mfma<T>::run(xs[cc * 256 + px[j]], lv[j], Tc[cc]);
    // keep the operand reads of one k-group next to its matrix instructions
    // (hoisting all of them raises the register peak past the budget)
    __builtin_amdgcn_sched_barrier(0);
  }
}
template <typename T, int NT, int NE, int CC, int K, int J0>
__device__ __forceinline__ void stage2(typename Mfma<T>::v4 (&acc)[NT], const typename Mfma<T>::v4 (&Tc)[NT],
                                       const Smem<T, NT>& sm, const i4 pr, int ok, int jlim) {
  const T* xs = sm.xs[K];
#pragma unroll
  for (int i = J0; i < J0 + 2; ++i) {
    if (i > 0 && Mfma<T>::kmin(i) >= jlim) break;  // rows j past c: adds only zeros
    const T a = ((ok >> i) & 1) ? Tc[CC][i] : T(0);
#pragma unroll
    for (int nt = 0; nt < NE; ++nt) acc[nt] = Mfma<T>::run(a, xs[nt * 256 + pr[i]], acc[nt]);
    __builtin_amdgcn_sched_barrier(0);
  }
}
template <typename T, int NT, int LO, int HI, int K, int J0>
__device__ __forceinline__ void stage1_sw(int nc, typename Mfma<T>::v4 (&Tc)[NT], const Smem<T, NT>& sm,
                                          const i4 px, const typename Mfma<T>::v4 lv, int klim) {
  if constexpr (LO == HI) {
    stage1<T, NT, LO, K, J0>(Tc, sm, px, lv, klim);
  } else {
    constexpr int MID = (LO + HI) / 2;
    if (nc <= MID) stage1_sw<T, NT, LO, MID, K, J0>(nc, Tc, sm, px, lv, klim);
    else stage1_sw<T, NT, MID + 1, HI, K, J0>(nc, Tc, sm, px, lv, klim);
  }
}
template <typename T, int NT, int NE, int LO, int HI, int K, int J0>
__device__ __forceinline__ void stage2_sw(int s, typename Mfma<T>::v4 (&acc)[NT],
                                          const typename Mfma<T>::v4 (&Tc)[NT], const Smem<T, NT>& sm,
                                          const i4 pr, int ok, int jlim) {
  if constexpr (LO == HI) {
    stage2<T, NT, NE, LO, K, J0>(acc, Tc, sm, pr, ok, jlim);
  } else {
    constexpr int MID = (LO + HI) / 2;
    if (s <= MID) stage2_sw<T, NT, NE, LO, MID, K, J0>(s, acc, Tc, sm, pr, ok, jlim);
    else stage2_sw<T, NT, NE, MID + 1, HI, K, J0>(s, acc, Tc, sm, pr, ok, jlim);
  }
}

// Matrix work of half H of the step recorded in rc (k-groups or T-column
// groups 2H, 2H + 1), from ring slot K.
template <typename T, int NT, int NE, int K, int H>
__device__ __forceinline__ void compute(const Rec& rc, typename Mfma<T>::v4 (&Tc)[NT],
                                        typename Mfma<T>::v4 (&acc)[NT], const Smem<T, NT>& sm, const LaneC<T>& lc,
                                        int rabs, int wave) {
  using v4 = typename Mfma<T>::v4;
  const uint32_t fl = rc.flags();
  const int rs = rc.s();
  const int s16 = 16 * rs;
  const int rb = rc.b(), rcc = rc.c();
  if (rc.ph() == 0) {
    if (H == 0 && rs == 0) {
#pragma unroll
      for (int cc = 0; cc < NT; ++cc) Tc[cc] = v4{0, 0, 0, 0};
    }
    const bool krx = !(fl & T_TX), krl = (fl & T_TL) != 0, idl = (fl & T_IDL) != 0;
    const T f = (T)rc.f;
    i4 px;
    v4 lv;
    const T* ls = sm.ls[K] + wave * 256;
#pragma unroll
    for (int j = 2 * H; j < 2 * H + 2; ++j) {
      px[j] = krx ? 64 * j + lc.lane : lc.tp[j];
      const int k = s16 + 4 * j + lc.g;
      const T l = ls[krl ? 64 * j + lc.lane : lc.tp[j]];
      lv[j] = idl ? (rabs == k ? f : T(0)) : (k < rb ? l * f : T(0));
    }
    stage1_sw<T, NT, 1, NT, K, 2 * H>(min(NT, (rcc + 15) >> 4), Tc, sm, px, lv, rb - s16);
  } else {
    const bool kr = !(fl & T_TR);
    i4 pr;
    int ok = 0;
#pragma unroll
    for (int i = 2 * H; i < 2 * H + 2; ++i) {
      pr[i] = kr ? 64 * i + lc.lane : lc.tp[i];
      ok |= (s16 + Mfma<T>::row(i, lc.g) < rcc ? 1 : 0) << i;
    }
    stage2_sw<T, NT, NE, 0, NT - 1, K, 2 * H>(rs, acc, Tc, sm, pr, ok, rcc - s16);
  }
}

// One pipeline iteration with compute slot K of an S-slot ring: wait for
// the step's loads (all but those of the S - 2 steps issued after it),
// barrier, first half of the matrix work, issue of the step S - 1 ahead
// into the slot freed by the previous step (while the matrix instructions
// of the first half execute), second half.
template <typename T, int NT, int NE, int K>
__device__ __forceinline__ bool iter(Ring<T, NT>& r, typename Mfma<T>::v4 (&Tc)[NT],
                                     typename Mfma<T>::v4 (&acc)[NT], Smem<T, NT>& sm, const LaneC<T>& lc,
                                     Cursor& cu, Task& t, Task& pre, bool& ivalid, const Task* __restrict__ tasks,
                                     int t1, const Bases<T>& B, int row0, int wave, int rabs, bool wave_on) {
  constexpr int S = Cfg<T, NT>::stages;
  int pending = 0;
#pragma unroll
  for (int d = 1; d <= S - 2; ++d) pending += r[(K + d) % S].cnt();
  wait_vm_le(pending);
  lds_barrier();
  if (!r[K].valid()) return false;
  if (wave_on) compute<T, NT, NE, K, 0>(r[K], Tc, acc, sm, lc, rabs, wave);
  __builtin_amdgcn_sched_barrier(0);
  issue<T, NT, NE, (K + S - 1) % S>(r[(K + S - 1) % S], cu, t, pre, ivalid, tasks, t1, B, sm, lc, row0, wave);
  __builtin_amdgcn_sched_barrier(0);
  if (wave_on) compute<T, NT, NE, K, 1>(r[K], Tc, acc, sm, lc, rabs, wave);
  return true;
}
// the S iterations of one turn of the ring; false once the tile is done
template <typename T, int NT, int NE, int K>
__device__ __forceinline__ bool turn(Ring<T, NT>& r, typename Mfma<T>::v4 (&Tc)[NT],
                                     typename Mfma<T>::v4 (&acc)[NT], Smem<T, NT>& sm, const LaneC<T>& lc,
                                     Cursor& cu, Task& t, Task& pre, bool& ivalid, const Task* __restrict__ tasks,
                                     int t1, const Bases<T>& B, int row0, int wave, int rabs, bool wave_on) {
  if constexpr (K == Cfg<T, NT>::stages) {
    return true;
  } else {
    if (!iter<T, NT, NE, K>(r, Tc, acc, sm, lc, cu, t, pre, ivalid, tasks, t1, B, row0, wave, rabs, wave_on))
      return false;
    return turn<T, NT, NE, K + 1>(r, Tc, acc, sm, lc, cu, t, pre, ivalid, tasks, t1, B, row0, wave, rabs, wave_on);
  }
}
template <typename T, int NT, int NE, int K>
__device__ __forceinline__ void prologue(Ring<T, NT>& r, Smem<T, NT>& sm, const LaneC<T>& lc,
                                         Cursor& cu, Task& t, Task& pre, bool& ivalid,
                                         const Task* __restrict__ tasks, int t1, const Bases<T>& B, int row0,
                                         int wave) {
  if constexpr (K < Cfg<T, NT>::stages - 1) {
    issue<T, NT, NE, K>(r[K], cu, t, pre, ivalid, tasks, t1, B, sm, lc, row0, wave);
    prologue<T, NT, NE, K + 1>(r, sm, lc, cu, t, pre, ivalid, tasks, t1, B, row0, wave);
  } else {
    r[K].m = 0;
  }
}

template <typename T, int NT, int NE>
__device__ __forceinline__ void item_e(const Tile& tile, const Work& w, const Task* __restrict__ tasks,
                                       const Bases<T>& B, Smem<T, NT>& sm) {
  using M = Mfma<T>;
  using v4 = typename M::v4;
  const int tid = threadIdx.x;
  const LaneC<T> lc(tid);
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wrow0 = w.row0 + wave * 16;
  const bool wave_on = wrow0 < tile.a;
  const int rabs = wrow0 + lc.n;
  v4 acc[NT], Tc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = v4{0, 0, 0, 0};
  if (tile.t0 < tile.t1) {
    Cursor cu{tile.t0, 0, 0};
    Task t = tasks[tile.t0];
    Task pre = tasks[min(tile.t0 + 1, tile.t1 - 1)];
    bool ivalid = true;
    Ring<T, NT> r;
    prologue<T, NT, NE, 0>(r, sm, lc, cu, t, pre, ivalid, tasks, tile.t1, B, w.row0, wave);
    while (turn<T, NT, NE, 0>(r, Tc, acc, sm, lc, cu, t, pre, ivalid, tasks, tile.t1, B, w.row0, wave, rabs, wave_on)) {
    }
  }
  wait_vm<0>();
  if (!wave_on) return;
  const int E = tile.e;
#pragma unroll
  for (int nt = 0; nt < NE; ++nt) {
    const int col = nt * 16 + lc.n;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wrow0 + M::row(i, lc.g);
      if (r < tile.a && col < E) B.out[tile.offOut + (int64_t)r * tile.ldOut + col] = acc[nt][i];
    }
  }
}

}  // namespace dmak

template <typename T, int NT>
__global__ __launch_bounds__(256, (dmak::Cfg<T, NT>::groups)) void chain_dma(const Tile* __restrict__ tiles,
                                                                         const Work* __restrict__ work,
                                                                         const Task* __restrict__ tasks, Bases<T> B) {
  __shared__ dmak::Smem<T, NT> sm;
  const Work w = work[blockIdx.x];
  if (w.row0 < 0) return;  // unused position of the XCD-ordered list
  const Tile tile = tiles[w.tile];
  const int ne = (tile.e + 15) >> 4;
  if (ne <= NeBucket<NT, 1>::value)
    dmak::item_e<T, NT, NeBucket<NT, 1>::value>(tile, w, tasks, B, sm);
  else if (ne <= NeBucket<NT, 2>::value)
    dmak::item_e<T, NT, NeBucket<NT, 2>::value>(tile, w, tasks, B, sm);
  else if (ne <= NeBucket<NT, 3>::value)
    dmak::item_e<T, NT, NeBucket<NT, 3>::value>(tile, w, tasks, B, sm);
  else
    dmak::item_e<T, NT, NT>(tile, w, tasks, B, sm);
}

template <typename T>
static hipError_t launch_mfma_variants(const Tile* tiles, const WorkSet& ws, const Task* tasks, Bases<T> b,
                                       const hipStream_t* ss, hipEvent_t (*ev)[2], int mode) {
  // largest blocks first: their work items are the longest
  for (int v = kNumVariants - 1; v >= 0; --v) {
    if (ws.n[v] <= 0) continue;
    hipStream_t s = ss[v];
    if (ev && ev[v][0]) {
      hipError_t e = hipEventRecord(ev[v][0], s);
      if (e != hipSuccess) return e;
    }
    dim3 grid((unsigned)ws.n[v]), blk(256);
    switch (v) {
      // FP64 128 and 256 wide: LDS-ring kernel.  FP64 32 and 64 wide: the
      // ring kernel while a wider variant runs beside them (sharing the CUs
      // with it they leave it more of the chip), else the register-staged
      // kernel (alone, with few matrix instructions per step, it is faster:
      // 16.0 vs 22.2 ms at N=24 D=1024).  FP32: register-staged kernel.
      // `mode` can force one FP64 family.
      case 0:
        if constexpr (sizeof(T) == 8) {
          if (mode == kFp64Ring || (mode == kFp64Auto && (ws.n[2] > 0 || ws.n[3] > 0))) {
            hipLaunchKernelGGL((chain_dma<T, 2>), grid, blk, 0, s, tiles, ws.w[v], tasks, b);
            break;
          }
        }
        hipLaunchKernelGGL((chain_mfma<T, 2>), grid, blk, 0, s, tiles, ws.w[v], tasks, b);
        break;
      case 1:
        if constexpr (sizeof(T) == 8) {
          if (mode == kFp64Ring || (mode == kFp64Auto && (ws.n[2] > 0 || ws.n[3] > 0))) {
            hipLaunchKernelGGL((chain_dma<T, 4>), grid, blk, 0, s, tiles, ws.w[v], tasks, b);
            break;
          }
        }
        hipLaunchKernelGGL((chain_mfma<T, 4>), grid, blk, 0, s, tiles, ws.w[v], tasks, b);
        break;
      case 2:
        if constexpr (sizeof(T) == 8) {
          if (mode != kFp64Staged) {
            hipLaunchKernelGGL((chain_dma<T, 8>), grid, blk, 0, s, tiles, ws.w[v], tasks, b);
            break;
          }
        }
        hipLaunchKernelGGL((chain_mfma<T, 8>), grid, blk, 0, s, tiles, ws.w[v], tasks, b);
        break;
      default:
        if constexpr (sizeof(T) == 8) {
          if (mode != kFp64Staged) {
            hipLaunchKernelGGL((chain_dma<T, 16>), grid, blk, 0, s, tiles, ws.w[v], tasks, b);
            break;
          }
        }
        hipLaunchKernelGGL((chain_mfma<T, 16>), grid, blk, 0, s, tiles, ws.w[v], tasks, b);
        break;
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

hipError_t launch_mfma_f64(const Tile* tiles, const WorkSet& ws, const Task* tasks, Bases<double> b,
                           const hipStream_t* s, hipEvent_t (*ev)[2], int mode) {
  return launch_mfma_variants<double>(tiles, ws, tasks, b, s, ev, mode);
}
hipError_t launch_mfma_f32(const Tile* tiles, const WorkSet& ws, const Task* tasks, Bases<float> b,
                           const hipStream_t* s, hipEvent_t (*ev)[2]) {
  return launch_mfma_variants<float>(tiles, ws, tasks, b, s, ev, kFp64Auto);
}

// ------------------------------------------------------------------ chained product, bf16 split
// Split precision: every FP32 operand value x is written to LDS as
// hi = RNE_bf16(x) and lo = RNE_bf16(x - hi), and each product a b is
// formed as ah bh + ah bl + al bh on v_mfma_f32_16x16x16_bf16 with FP32
// accumulation (the lo*lo term, of relative size 2^-16, is dropped).  The
// step pipeline, cursors and global loads are those of the FP32 kernel
// (same FP32 operand arenas); the LDS slices hold the split values with k
// contiguous per row or column, so that a lane's four operand values of
// k = 4g..4g+3 are one 8-byte read:
//   op(X) slice  [m][k]  (16 k per column m),
//   op(R) slice  [col][j],
//   op(L) slice  [row][k].
// Stage 1 result layout: register r of lane (g, n) holds
// T[row n][16 cc + 4g + r], which is directly the A operand of stage 2 for
// k = 4g + r of the c-slice (split into hi/lo in registers).
typedef short b3v4 __attribute__((ext_vector_type(4)));
typedef float f32v4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t bf_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float bf_val(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

template <int NT>
struct B3Smem {
  static constexpr int W = 16 * NT;
  static constexpr int KP = 20;  // 16 values + 4 padding (rows stay 8-byte aligned)
  uint16_t sh[2][W * KP], sl[2][W * KP];
  uint16_t lh[2][64 * KP], ll[2][64 * KP];
};

__device__ __forceinline__ void put_split(uint16_t* hi, uint16_t* lo, int pos, float v) {
  const uint16_t h = bf_bits(v);
  hi[pos] = h;
  lo[pos] = bf_bits(v - bf_val(h));
}

template <int NT, int P>
__device__ __forceinline__ void store_step_b3(const Task& t, const Cursor& cu, const Lane<16 * NT>& ln, int row0,
                                              const Stage<float, NT>& st, B3Smem<NT>& sm) {
  constexpr int W = 16 * NT, KQ = 256 / W, KP = B3Smem<NT>::KP;
  const uint32_t fl = t.flags;
  const int base = 16 * cu.s;
  uint16_t* hi = sm.sh[P];
  uint16_t* lo = sm.sl[P];
  if (cu.ph == 0) {
    const int klim = t.b - base;
    if (fl & T_IDX) {
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const int kk = ln.tW + KQ * q;
        put_split(hi, lo, ln.tm * KP + kk, base + kk == ln.tm ? 1.f : 0.f);
      }
    } else if (fl & T_TX) {
#pragma unroll
      for (int q = 0; q < NT; ++q) put_split(hi, lo, (ln.t4 + 16 * q) * KP + ln.t15, st.v[q]);
    } else {
#pragma unroll
      for (int q = 0; q < NT; ++q) put_split(hi, lo, ln.tm * KP + ln.tW + KQ * q, st.v[q]);
    }
    const float f = (float)t.f;
    if (fl & T_IDL) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = ln.t4 + 16 * q;
        put_split(sm.lh[P], sm.ll[P], r * KP + ln.t15, (row0 + r == base + ln.t15) ? f : 0.f);
      }
    } else if (fl & T_TL) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = ln.t6 + 4 * q;
        put_split(sm.lh[P], sm.ll[P], ln.t63 * KP + kk, kk < klim ? st.l[q] * f : 0.f);
      }
    } else {
      const bool ok = ln.t15 < klim;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        put_split(sm.lh[P], sm.ll[P], (ln.t4 + 16 * q) * KP + ln.t15, ok ? st.l[q] * f : 0.f);
    }
  } else {
    const int jlim = t.c - base;
    if (fl & T_IDR) {
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const int j = ln.tW + KQ * q;
        put_split(hi, lo, ln.tm * KP + j, base + j == ln.tm ? 1.f : 0.f);
      }
    } else if (fl & T_TR) {
      const bool ok = ln.t15 < jlim;
#pragma unroll
      for (int q = 0; q < NT; ++q) put_split(hi, lo, (ln.t4 + 16 * q) * KP + ln.t15, ok ? st.v[q] : 0.f);
    } else {
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const int j = ln.tW + KQ * q;
        put_split(hi, lo, ln.tm * KP + j, j < jlim ? st.v[q] : 0.f);
      }
    }
  }
}

__device__ __forceinline__ f32v4 mfma_b3(b3v4 ah, b3v4 al, b3v4 bh, b3v4 bl, f32v4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
}
__device__ __forceinline__ b3v4 ld4(const uint16_t* p) { return *reinterpret_cast<const b3v4*>(p); }

template <int NT, int NC, int P>
__device__ __forceinline__ void stage1_b3(f32v4 (&Tc)[NT], const B3Smem<NT>& sm, int wave, int g, int n) {
  constexpr int KP = B3Smem<NT>::KP;
  const int lo = (wave * 16 + n) * KP + 4 * g;
  const b3v4 bh = ld4(sm.lh[P] + lo), bl = ld4(sm.ll[P] + lo);
#pragma unroll
  for (int cc = 0; cc < NC; ++cc) {
    const int xo = (cc * 16 + n) * KP + 4 * g;
    Tc[cc] = mfma_b3(ld4(sm.sh[P] + xo), ld4(sm.sl[P] + xo), bh, bl, Tc[cc]);
  }
}
template <int NT, int NE, int CC, int P>
__device__ __forceinline__ void stage2_b3(f32v4 (&acc)[NT], const f32v4 (&Tc)[NT], const B3Smem<NT>& sm, int g, int n) {
  constexpr int KP = B3Smem<NT>::KP;
  b3v4 th, tl;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint16_t h = bf_bits(Tc[CC][r]);
    th[r] = (short)h;
    tl[r] = (short)bf_bits(Tc[CC][r] - bf_val(h));
  }
#pragma unroll
  for (int nt = 0; nt < NE; ++nt) {
    const int ro = (nt * 16 + n) * KP + 4 * g;
    acc[nt] = mfma_b3(th, tl, ld4(sm.sh[P] + ro), ld4(sm.sl[P] + ro), acc[nt]);
  }
}
template <int NT, int LO, int HI, int P>
__device__ __forceinline__ void stage1_b3_sw(int nc, f32v4 (&Tc)[NT], const B3Smem<NT>& sm, int wave, int g, int n) {
  if constexpr (LO == HI) {
    stage1_b3<NT, LO, P>(Tc, sm, wave, g, n);
  } else {
    constexpr int MID = (LO + HI) / 2;
    if (nc <= MID) stage1_b3_sw<NT, LO, MID, P>(nc, Tc, sm, wave, g, n);
    else stage1_b3_sw<NT, MID + 1, HI, P>(nc, Tc, sm, wave, g, n);
  }
}
template <int NT, int NE, int LO, int HI, int P>
__device__ __forceinline__ void stage2_b3_sw(int s, f32v4 (&acc)[NT], const f32v4 (&Tc)[NT], const B3Smem<NT>& sm,
                                             int g, int n) {
  if constexpr (LO == HI) {
    stage2_b3<NT, NE, LO, P>(acc, Tc, sm, g, n);
  } else {
    constexpr int MID = (LO + HI) / 2;
    if (s <= MID) stage2_b3_sw<NT, NE, LO, MID, P>(s, acc, Tc, sm, g, n);
    else stage2_b3_sw<NT, NE, MID + 1, HI, P>(s, acc, Tc, sm, g, n);
  }
}

template <int NT, int NE, int P>
__device__ __forceinline__ void pipe_step_b3(const Tile& tile, const Task* __restrict__ tasks, const Bases<float>& B,
                                             B3Smem<NT>& sm, const Lane<16 * NT>& ln, int row0, bool wave_on, int wave,
                                             int g, int n, f32v4 (&Tc)[NT], f32v4 (&acc)[NT], bool& live, Cursor& c0,
                                             Task& t0, Task& pre) {
  Cursor c1 = c0;
  Task t1 = t0;
  const bool more = next_step(c1, t1, pre, tasks, tile.t1);
  Stage<float, NT> st;
  if (more) st = load_step<float, NT>(t1, B, c1, ln, row0);
  if (wave_on) {
    if (c0.ph == 0) {
      if (c0.s == 0) {
#pragma unroll
        for (int cc = 0; cc < NT; ++cc) Tc[cc] = f32v4{0, 0, 0, 0};
      }
      stage1_b3_sw<NT, 1, NT, P>(min(NT, (t0.c + 15) >> 4), Tc, sm, wave, g, n);
    } else {
      stage2_b3_sw<NT, NE, 0, NT - 1, P>(c0.s, acc, Tc, sm, g, n);
    }
  }
  if (more) store_step_b3<NT, P ^ 1>(t1, c1, ln, row0, st, sm);
  __syncthreads();
  live = more;
  c0 = c1;
  t0 = t1;
}

template <int NT, int NE>
__device__ __forceinline__ void chain_item_b3_e(const Tile& tile, const Work& w, const Task* __restrict__ tasks,
                                                const Bases<float>& B, B3Smem<NT>& sm) {
  const int tid = threadIdx.x;
  const Lane<16 * NT> ln(tid);
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g = lane >> 4, n = lane & 15;
  const int wrow0 = w.row0 + wave * 16;
  const bool wave_on = wrow0 < tile.a;
  const int E = tile.e;
  f32v4 acc[NT], Tc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = f32v4{0, 0, 0, 0};
  if (tile.t0 < tile.t1) {
    Cursor c0{tile.t0, 0, 0};
    Task t0 = tasks[tile.t0];
    Task pre = tasks[min(tile.t0 + 1, tile.t1 - 1)];
    {
      const Stage<float, NT> st = load_step<float, NT>(t0, B, c0, ln, w.row0);
      store_step_b3<NT, 0>(t0, c0, ln, w.row0, st, sm);
    }
    __syncthreads();
    bool live = true;
    while (live) {
      pipe_step_b3<NT, NE, 0>(tile, tasks, B, sm, ln, w.row0, wave_on, wave, g, n, Tc, acc, live, c0, t0, pre);
      if (!live) break;
      pipe_step_b3<NT, NE, 1>(tile, tasks, B, sm, ln, w.row0, wave_on, wave, g, n, Tc, acc, live, c0, t0, pre);
    }
  }
  if (!wave_on) return;
#pragma unroll
  for (int nt = 0; nt < NE; ++nt) {
    const int col = nt * 16 + n;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = wrow0 + 4 * g + r;
      if (row < tile.a && col < E) B.out[tile.offOut + (int64_t)row * tile.ldOut + col] = acc[nt][r];
    }
  }
}

template <int NT>
__global__ __launch_bounds__(256, NT <= 8 ? 3 : 1) void chain_b3(const Tile* __restrict__ tiles, const Work* __restrict__ work,
                                                const Task* __restrict__ tasks, Bases<float> B) {
  __shared__ B3Smem<NT> sm;
  const Work w = work[blockIdx.x];
  if (w.row0 < 0) return;  // unused position of the XCD-ordered list
  const Tile tile = tiles[w.tile];
  const int ne = (tile.e + 15) >> 4;
  if (ne <= NeBucket<NT, 1>::value)
    chain_item_b3_e<NT, NeBucket<NT, 1>::value>(tile, w, tasks, B, sm);
  else if (ne <= NeBucket<NT, 2>::value)
    chain_item_b3_e<NT, NeBucket<NT, 2>::value>(tile, w, tasks, B, sm);
  else if (ne <= NeBucket<NT, 3>::value)
    chain_item_b3_e<NT, NeBucket<NT, 3>::value>(tile, w, tasks, B, sm);
  else
    chain_item_b3_e<NT, NT>(tile, w, tasks, B, sm);
}

hipError_t launch_bf16x3(const Tile* tiles, const WorkSet& ws, const Task* tasks, Bases<float> b,
                         const hipStream_t* ss, hipEvent_t (*ev)[2]) {
  for (int v = kNumVariants - 1; v >= 0; --v) {
    if (ws.n[v] <= 0) continue;
    hipStream_t s = ss[v];
    if (ev && ev[v][0]) {
      hipError_t e = hipEventRecord(ev[v][0], s);
      if (e != hipSuccess) return e;
    }
    dim3 grid((unsigned)ws.n[v]), blk(256);
    switch (v) {
      case 0: hipLaunchKernelGGL((chain_b3<2>), grid, blk, 0, s, tiles, ws.w[v], tasks, b); break;
      case 1: hipLaunchKernelGGL((chain_b3<4>), grid, blk, 0, s, tiles, ws.w[v], tasks, b); break;
      case 2: hipLaunchKernelGGL((chain_b3<8>), grid, blk, 0, s, tiles, ws.w[v], tasks, b); break;
      default: hipLaunchKernelGGL((chain_b3<16>), grid, blk, 0, s, tiles, ws.w[v], tasks, b); break;
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

// ------------------------------------------------------------------ split task chains
// One work-group column per job, blockIdx.y strides over its elements; each
// output element is the sum of its parts in the order of p (deterministic).
// The parts and the output may share one buffer (disjoint ranges).
template <typename T>
__global__ __launch_bounds__(256) void reduce_parts_kernel(const RedJob* __restrict__ jobs, const T* part, T* out) {
  const RedJob j = jobs[blockIdx.x];
  const int64_t n = (int64_t)j.a * j.e;
  for (int64_t i = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.y * blockDim.x) {
    const T* p = part + j.part_off + i;
    T s = p[0];
    for (int q = 1; q < j.parts; ++q) s += p[q * n];
    const int64_t r = i / j.e, c = i - r * j.e;
    out[j.out_off + r * j.ld + c] = s;
  }
}

template <typename T>
static hipError_t launch_reduce_parts(const RedJob* jobs, int n_jobs, const T* part, T* out, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_parts_kernel<T>, dim3((unsigned)n_jobs, 16), dim3(256), 0, s, jobs, part, out);
  return hipGetLastError();
}
hipError_t launch_reduce_parts_f64(const RedJob* jobs, int n_jobs, const double* part, double* out, hipStream_t s) {
  return launch_reduce_parts<double>(jobs, n_jobs, part, out, s);
}
hipError_t launch_reduce_parts_f32(const RedJob* jobs, int n_jobs, const float* part, float* out, hipStream_t s) {
  return launch_reduce_parts<float>(jobs, n_jobs, part, out, s);
}

hipError_t launch_diag(const Tile* tiles, int64_t n_tiles, const DiagTask* tasks, const double* L0,
                       const double* L1, const double* R0, const double* R1, double* out, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(diag_kernel, dim3((unsigned)n_tiles), dim3(256), 0, s, tiles, tasks, L0, L1, R0, R1, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ truncation SVD (block one-sided Jacobi)
// One work-group per (sector, block pair) of a round.  The pair's rows
// (at most 2 kBjRows) of B are read in chunks of 64 columns through LDS to
// form their Gram matrix G; G's eigenvectors Q come from a cyclic Jacobi in
// LDS; the rows of B and of W^T are replaced by Q^T times themselves, which
// makes the pair's rows of B mutually orthogonal.  All sums are in a fixed
// order (bitwise reproducible).
namespace bjk {
constexpr int R2 = 2 * kBjRows;  // rows of a pair
constexpr int CH = 64;           // columns per chunk

__device__ __forceinline__ void pair_of(int K, int pr, int r, int& I, int& J) {
  const int a = pr == 0 ? 0 : 1 + ((pr - 1 + r) % (K - 1));
  const int b = 1 + ((K - 1 - pr - 1 + r) % (K - 1));
  I = a < b ? a : b;
  J = a < b ? b : a;
}

// rows: the pair's row indices (nr of them); X: rows of length len at base
// with row stride len; out = Q^T X (in place)
__device__ void rotate_rows(double* base, int64_t len, const int* rows, int nr, const double (*Q)[R2 + 1],
                            double (*buf)[CH + 1]) {
  const int tid = threadIdx.x;
  for (int64_t c0 = 0; c0 < len; c0 += CH) {
    const int w = (int)min<int64_t>(CH, len - c0);
    for (int e = tid; e < nr * CH; e += 256) {
      const int i = e / CH, j = e % CH;
      buf[i][j] = j < w ? base[(int64_t)rows[i] * len + c0 + j] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < nr * CH; e += 256) {
      const int i = e / CH, j = e % CH;
      if (j >= w) continue;
      double v = 0.0;
      for (int k = 0; k < nr; ++k) v += Q[k][i] * buf[k][j];
      base[(int64_t)rows[i] * len + c0 + j] = v;
    }
    __syncthreads();
  }
}
}  // namespace bjk

__global__ __launch_bounds__(256) void bj_round_kernel(const BjJob* __restrict__ jobs, double* __restrict__ Ball,
                                                       double* __restrict__ WTall, unsigned long long* off_max, int r,
                                                       double tol) {
  using namespace bjk;
  __shared__ double G[R2][R2 + 1];
  __shared__ double Q[R2][R2 + 1];
  __shared__ double buf[R2][CH + 1];
  __shared__ double cs[R2 / 2], sn[R2 / 2], dpp[R2 / 2], dqq[R2 / 2];
  __shared__ int pp[R2 / 2], qq[R2 / 2];
  __shared__ int rows[R2];
  __shared__ double red[256];
  __shared__ int flag, rot;
  const BjJob jb = jobs[blockIdx.x];
  if (r >= jb.K - 1) return;
  int I, J;
  pair_of(jb.K, jb.pr, r, I, J);
  const int m = jb.m;
  const int nb = (m + kBjRows - 1) / kBjRows;
  const int tid = threadIdx.x;
  // paired with the padding block of an odd block count (or the only
  // block): block I alone, whose own rows still need orthogonalizing
  const int nI = min(kBjRows, m - kBjRows * I), nJ = J < nb ? min(kBjRows, m - kBjRows * J) : 0;
  const int nr = nI + nJ;
  if (tid < nr) rows[tid] = tid < nI ? kBjRows * I + tid : kBjRows * J + (tid - nI);
  __syncthreads();
  double* B = Ball + jb.b_off;
  double* WT = WTall + jb.w_off;
  // Gram matrix of the pair's rows of B
  double g[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t c0 = 0; c0 < jb.c; c0 += CH) {
    const int w = (int)min<int64_t>(CH, jb.c - c0);
    for (int e = tid; e < nr * CH; e += 256) {
      const int i = e / CH, j = e % CH;
      buf[i][j] = j < w ? B[(int64_t)rows[i] * jb.c + c0 + j] : 0.0;
    }
    __syncthreads();
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;
      if (e >= nr * nr) break;
      const int i = e / nr, j = e % nr;
      double v = 0.0;
      for (int k = 0; k < w; ++k) v += buf[i][k] * buf[j][k];
      g[t] += v;
    }
    __syncthreads();
  }
  for (int t = 0; t < 4; ++t) {
    const int e = tid + 256 * t;
    if (e < nr * nr) G[e / nr][e % nr] = g[t];
  }
  for (int e = tid; e < R2 * R2; e += 256) Q[e / R2][e % R2] = (e / R2 == e % R2) ? 1.0 : 0.0;
  __syncthreads();
  // largest relative off-diagonal entry
  double off = 0.0;
  for (int e = tid; e < nr * nr; e += 256) {
    const int i = e / nr, j = e % nr;
    if (i == j) continue;
    const double d = G[i][i] * G[j][j];
    if (d > 1e-300) off = fmax(off, fabs(G[i][j]) / sqrt(d));
  }
  red[tid] = off;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) red[tid] = fmax(red[tid], red[tid + st]);
    __syncthreads();
  }
  if (tid == 0) {
    atomicMax(off_max + jb.sector, (unsigned long long)__double_as_longlong(red[0]));
    flag = red[0] > tol * sqrt((double)jb.c) ? 1 : 0;
  }
  __syncthreads();
  // (the inner sweeps below keep their own flag: a thread still reading
  // `flag` here must not see a later write)
  if (!flag) return;
  // eigenvectors of G: cyclic Jacobi, round-robin pairs; a pair is rotated
  // while |G_pq| > 1e-15 sqrt(G_pp G_qq) (relative to the pair's own scale,
  // which keeps rows of very different norms accurate), until a sweep
  // rotates nothing (at most 40 sweeps).  The rotated 2 x 2 block is set
  // from the closed form (G_pp - t G_pq, G_qq + t G_pq, 0), so that no
  // rounding residue of the large diagonal entry stays in G_pq.
  const int P = (nr + 1) & ~1;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) rot = 0;
    __syncthreads();
    for (int rr = 0; rr < P - 1; ++rr) {
      if (tid < P / 2) {
        const int a = tid == 0 ? 0 : 1 + ((tid - 1 + rr) % (P - 1));
        const int b = 1 + ((P - 1 - tid - 1 + rr) % (P - 1));
        const int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, sv = 0.0;
        if (q < nr && fabs(G[p][q]) > 1e-15 * sqrt(G[p][p] * G[q][q])) {
          const double th = (G[q][q] - G[p][p]) / (2.0 * G[p][q]);
          const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          sv = t * c;
          dpp[tid] = G[p][p] - t * G[p][q];
          dqq[tid] = G[q][q] + t * G[p][q];
          rot = 1;
        }
        cs[tid] = c;
        sn[tid] = sv;
        pp[tid] = p;
        qq[tid] = (q < nr && sv != 0.0) ? q : p;
      }
      __syncthreads();
      for (int e = tid; e < (P / 2) * nr; e += 256) {  // rows of G
        const int k = e / nr, j = e % nr;
        const int p = pp[k], q = qq[k];
        if (p == q) continue;
        const double gp = G[p][j], gq = G[q][j];
        G[p][j] = cs[k] * gp - sn[k] * gq;
        G[q][j] = sn[k] * gp + cs[k] * gq;
      }
      __syncthreads();
      for (int e = tid; e < (P / 2) * nr; e += 256) {  // columns of G and of Q
        const int k = e / nr, i = e % nr;
        const int p = pp[k], q = qq[k];
        if (p == q) continue;
        const double gp = G[i][p], gq = G[i][q];
        G[i][p] = cs[k] * gp - sn[k] * gq;
        G[i][q] = sn[k] * gp + cs[k] * gq;
        const double vp = Q[i][p], vq = Q[i][q];
        Q[i][p] = cs[k] * vp - sn[k] * vq;
        Q[i][q] = sn[k] * vp + cs[k] * vq;
      }
      __syncthreads();
      if (tid < P / 2) {
        const int p = pp[tid], q = qq[tid];
        if (p != q) {
          G[p][p] = dpp[tid];
          G[q][q] = dqq[tid];
          G[p][q] = 0.0;
          G[q][p] = 0.0;
        }
      }
      __syncthreads();
    }
    if (!rot) break;
    __syncthreads();
  }
  rotate_rows(B, jb.c, rows, nr, Q, buf);
  rotate_rows(WT, m, rows, nr, Q, buf);
}

hipError_t launch_bj_round(const BjJob* jobs, int n_jobs, double* B, double* WT, unsigned long long* off_max, int r,
                           double tol, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(bj_round_kernel, dim3(n_jobs), dim3(256), 0, s, jobs, B, WT, off_max, r, tol);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void copy_blocks_kernel(const CopyJob* __restrict__ jobs, const double* __restrict__ src,
                                                          double* __restrict__ dst) {
  const CopyJob j = jobs[blockIdx.x];
  for (int e = threadIdx.x; e < j.rows * j.cols; e += 256)
    dst[j.dst + (int64_t)(e / j.cols) * j.ld + e % j.cols] = src[j.src + e];
}
hipError_t launch_copy_blocks(const CopyJob* jobs, int n_jobs, const double* src, double* dst, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_blocks_kernel, dim3(n_jobs), dim3(256), 0, s, jobs, src, dst);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void identity_kernel(const int64_t* __restrict__ woff, const int32_t* __restrict__ m,
                                                       double* __restrict__ WT) {
  const int q = blockIdx.x;
  const int n = m[q];
  double* W = WT + woff[q];
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += 256) W[e] = (e / n == e % n) ? 1.0 : 0.0;
}
hipError_t launch_identity(const int64_t* woff, const int32_t* m, int n_sect, double* WT, hipStream_t s) {
  if (n_sect <= 0) return hipSuccess;
  hipLaunchKernelGGL(identity_kernel, dim3(n_sect), dim3(256), 0, s, woff, m, WT);
  return hipGetLastError();
}

// one work-group per sector, one wave per row at a time (fixed-order sums)
__global__ __launch_bounds__(256) void row_norms_kernel(const int64_t* __restrict__ boff, const int32_t* __restrict__ m,
                                                        const int32_t* __restrict__ c, const int64_t* __restrict__ soff,
                                                        const double* __restrict__ B, double* __restrict__ sig) {
  const int q = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = wave; i < m[q]; i += 4) {
    const double* row = B + boff[q] + (int64_t)i * c[q];
    double v = 0.0;
    for (int j = lane; j < c[q]; j += 64) v += row[j] * row[j];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if (lane == 0) sig[soff[q] + i] = sqrt(v);
  }
}
hipError_t launch_row_norms(const int64_t* boff, const int32_t* m, const int32_t* c, const int64_t* soff, int n_sect,
                            const double* B, double* sig, hipStream_t s) {
  if (n_sect <= 0) return hipSuccess;
  hipLaunchKernelGGL(row_norms_kernel, dim3(n_sect), dim3(256), 0, s, boff, m, c, soff, B, sig);
  return hipGetLastError();
}

// kept left singular vectors (rows of W^T) as isometry columns
__global__ __launch_bounds__(256) void gather_rows_kernel(const GatherJob* __restrict__ jobs, const double* __restrict__ WT,
                                                          double* __restrict__ out) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  const GatherJob J = jobs[blockIdx.x];
  const int n = J.n;
  for (int j = 0; j < J.ncol; ++j) {
    const double* u = WT + J.v_off + (int64_t)J.cols[j] * n;
    double best = -1.0;
    int idx = 0;
    for (int r = threadIdx.x; r < n; r += 256) {
      const double a = fabs(u[r]);
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
    const double sg = u[bi[0]] < 0 ? -1.0 : 1.0;
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += 256) out[J.out_off + (int64_t)r * J.ncol + j] = sg * u[r];
  }
}
hipError_t launch_gather_rows(const GatherJob* jobs, int n_jobs, const double* WT, double* out, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_rows_kernel, dim3(n_jobs), dim3(256), 0, s, jobs, WT, out);
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

// One work-group per output block of the pair rotation: out = sum_t c_t in_t
// over the block's elements (contiguous, coalesced; HBM-bound).
__global__ __launch_bounds__(256) void rotate_pair_kernel(const RotJob* __restrict__ jobs, const double* __restrict__ in,
                                                          double* __restrict__ out) {
  const RotJob j = jobs[blockIdx.x];
  for (int i = threadIdx.x; i < j.n; i += 256) {
    double v = 0.0;
    for (int t = 0; t < j.nterm; ++t) v += j.c[t] * in[j.off_in[t] + i];
    out[j.off_out + i] = v;
  }
}

hipError_t launch_rotate_pair(const RotJob* jobs, int64_t n_jobs, const double* in, double* out, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(rotate_pair_kernel, dim3((unsigned)n_jobs), dim3(256), 0, s, jobs, in, out);
  return hipGetLastError();
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

// ------------------------------------------------------------------ Davidson vector kernels
// Deterministic two-pass reductions: fixed grid of kRedBlocks partial sums,
// then one work-group folds them in a fixed order.

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

// out = sum_n x[n] y[n] accumulated in FP64 (fixed reduction order)
template <typename T>
__global__ __launch_bounds__(256) void dot_partial(const T* x, const T* y, int64_t n, double* part) {
  __shared__ double sh[256];
  double v = 0.0;
  for (int64_t j = blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) v += (double)x[j] * (double)y[j];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

template <typename T>
static hipError_t launch_dot_t(const T* x, const T* y, int64_t n, double* out, double* scratch, hipStream_t s) {
  hipLaunchKernelGGL(dot_partial<T>, dim3(kRedBlocks), dim3(256), 0, s, x, y, n, scratch);
  hipLaunchKernelGGL(multidot_final, dim3(1), dim3(256), 0, s, scratch, 1, kRedBlocks, out);
  return hipGetLastError();
}
hipError_t launch_dot_f64(const double* x, const double* y, int64_t n, double* out, double* scratch, hipStream_t s) {
  return launch_dot_t<double>(x, y, n, out, scratch, s);
}
hipError_t launch_dot_f32(const float* x, const float* y, int64_t n, double* out, double* scratch, hipStream_t s) {
  return launch_dot_t<float>(x, y, n, out, scratch, s);
}

template <typename T>
__global__ void scale_kernel(T* x, int64_t n, T a) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    x[j] *= a;
}
hipError_t launch_scale_f64(double* x, int64_t n, double a, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_kernel<double>, dim3(grid_for(n)), dim3(256), 0, s, x, n, a);
  return hipGetLastError();
}
hipError_t launch_scale_f32(float* x, int64_t n, float a, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_kernel<float>, dim3(grid_for(n)), dim3(256), 0, s, x, n, a);
  return hipGetLastError();
}

hipError_t launch_multiaxpy(const double* A, int64_t lda, int k, const double* coef, double coef_scale, double* y,
                            double alpha, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(multiaxpy_kernel, dim3(grid_for(n)), dim3(256), 0, s, A, lda, k, coef, coef_scale, y, alpha, n);
  return hipGetLastError();
}

}  // namespace heff
