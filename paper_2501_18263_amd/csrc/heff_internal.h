// Internal structures shared by the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

namespace heff {

// rows of one output block handled by one work item of the plain kernel
// largest output width and inner dimension one task may have in the
// matrix-core kernels (larger blocks are split into several tasks / tiles)
constexpr int kMaxDim = 256;
// largest output width and middle dimension of the Davidson product's
// tasks: wider output blocks run as column slices and wider middle
// dimensions as consecutive ranges, so the product never needs the
// 256-wide kernel instances (one work-group per CU, register spills)
constexpr int kProductDim = 128;

// One block task of the chained product  out += f * op(L) * op(X) * op(R).
// Shapes: out a x e, op(L) a x b, op(X) b x c, op(R) c x e.  op(M) is M or
// M^T relative to the row-major storage of M.  In the H_eff product L is a
// left-block operator block, X a block of Psi and R^T a right-block
// operator block (Eq. Hamilton_act_U1sym); in the renormalization L = A^T
// and R = A are isometry blocks and X an old operator block.
struct Task {
  double f;
  int64_t offL, offX, offR;  // element offsets into the selected base arrays
  uint16_t a, b, c, e;
  uint16_t ldL, ldX, ldR;    // row strides of the stored L, X, R blocks
  uint16_t flags;
};
static_assert(sizeof(Task) == 48, "task layout");

enum : uint32_t {
  T_TL = 1u << 0,    // L stored as b x a
  T_TX = 1u << 1,    // X stored as c x b
  T_TR = 1u << 2,    // R stored as e x c
  T_IDL = 1u << 3,   // op(L) = identity (a == b)
  T_IDX = 1u << 4,   // op(X) = identity (b == c)
  T_IDR = 1u << 5,   // op(R) = identity (c == e)
  T_SELL = 1u << 6,  // L from base 1 (else base 0)
  T_SELX = 1u << 7,
  T_SELR = 1u << 8,
};

// One output block (or a column slice of one): a x e at offOut with row
// stride ldOut, accumulating tasks [t0, t1).
struct Tile {
  int64_t offOut;
  int32_t a, e;
  int32_t t0, t1;
  int32_t ldOut;
  int32_t prob;  // problem index in a batch (0 for a single problem)
};
static_assert(sizeof(Tile) == 32, "tile layout");

// Fixed-order sum of the parts of one split task chain: out block (a x e at
// out_off, row stride ld) = sum over p < parts of the part p (a x e, row
// stride e) at part_off + p a e, added in the order of p (the parts are
// written by tiles of their own, like any output block, behind psi').
struct RedJob {
  int64_t out_off, part_off;
  int32_t a, e, ld, parts;
};

// One work-group's share: rows [row0, row0 + ROWS) of tile `tile`.
struct Work {
  int32_t tile;
  int32_t row0;
};

// Diagonal task: out[i*e + j] += f * dL[i] * dR[j] with dL the diagonal of
// an a x a block (stride a+1) and dR of an e x e block; identity -> ones.
struct DiagTask {
  double f;
  int64_t offL, offR;
  uint32_t flags;  // T_IDL, T_IDR, T_SELL, T_SELR
  uint32_t pad;
};

template <typename T>
struct ProbBases {  // operator stores of one problem of a batch
  const T* L[2];
  const T* R[2];
};

template <typename T>
struct Bases {
  const T* L[2];
  const T* X[2];
  const T* R[2];
  T* out;
  // elements readable at L[0], L[1], X[0], X[1], R[0], R[1] (0: unknown).
  // The FP64 ring kernel moves operand pairs with 16-byte loads, which may
  // read one element past a block; it does so only where that element lies
  // inside the buffer by these lengths, else it loads single dwords.
  int64_t lim[6];
};

// Work items of the matrix-core kernels: kTileRows rows of one output block,
// grouped into kNumVariants lists by the largest dimension D of the block
// (output columns and every task's inner dimension b): D <= 32, 64, 128, 256.
constexpr int kTileRows = 64;
constexpr int kNumVariants = 4;
inline int variant_of(int d) { return d <= 32 ? 0 : d <= 64 ? 1 : d <= 128 ? 2 : 3; }
struct WorkSet {
  const Work* w[kNumVariants];
  int64_t n[kNumVariants];
};

// ---- launchers (heff_kernels.hip) ----
// ev: optional [kNumVariants][2] start/stop events recorded around each launch
// s[v]: stream of variant v (the variants touch disjoint outputs and may run
// concurrently); the single-stream forms launch all variants on one stream
// mode (FP64 only): which kernel family runs the variants, kFp64Auto (LDS
// ring for the 128- and 256-wide variants and, while one of them runs, for
// the narrower ones; register staging otherwise), kFp64Staged (register
// staging everywhere) or kFp64Ring (the ring for every width).  The
// families give bitwise identical results.
// kFp64RingDword runs the ring kernel with its 16-byte loads switched off
// (every slice moves by dword loads; the same sums in the same order).
enum { kFp64Auto = 0, kFp64Staged = 1, kFp64Ring = 2, kFp64RingDword = 3 };
hipError_t launch_mfma_f64(const Tile* tiles, const WorkSet& ws, const Task* tasks, Bases<double> b,
                           const hipStream_t* s, hipEvent_t (*ev)[2] = nullptr, int mode = kFp64Auto);
hipError_t launch_mfma_f32(const Tile* tiles, const WorkSet& ws, const Task* tasks, Bases<float> b,
                           const hipStream_t* s, hipEvent_t (*ev)[2] = nullptr);
inline hipError_t launch_mfma_f64(const Tile* tiles, const WorkSet& ws, const Task* tasks, Bases<double> b,
                                  hipStream_t s, hipEvent_t (*ev)[2] = nullptr) {
  const hipStream_t a[kNumVariants] = {s, s, s, s};
  return launch_mfma_f64(tiles, ws, tasks, b, a, ev);
}
inline hipError_t launch_mfma_f32(const Tile* tiles, const WorkSet& ws, const Task* tasks, Bases<float> b,
                                  hipStream_t s, hipEvent_t (*ev)[2] = nullptr) {
  const hipStream_t a[kNumVariants] = {s, s, s, s};
  return launch_mfma_f32(tiles, ws, tasks, b, a, ev);
}
// grid[v]: persistent work-groups of variant v
// s[v]: stream of variant v (the variants may run concurrently)
hipError_t launch_mfma_batch_f32(const Tile* tiles, const WorkSet& ws, const Task* tasks, const ProbBases<float>* pb,
                                 const float* X, float* out, const int grid[kNumVariants], const hipStream_t* s);
// split-precision (bf16 hi+lo, FP32 accumulation) product on the FP32 operand arenas
hipError_t launch_bf16x3(const Tile* tiles, const WorkSet& ws, const Task* tasks, Bases<float> b,
                         const hipStream_t* s, hipEvent_t (*ev)[2] = nullptr);
// Rotation of the two middle orbitals on a two-site vector: every output
// block is a combination of at most four input blocks of the same shape
// (the middle states of one (n_up, n_dn) sector of the two sites).
struct RotJob {
  int64_t off_out;
  int64_t off_in[4];
  double c[4];
  int32_t n, nterm;  // elements of the block, terms used
};
hipError_t launch_rotate_pair(const RotJob* jobs, int64_t n_jobs, const double* in, double* out, hipStream_t s);
struct GatherJob {
  int64_t v_off, out_off;
  const int32_t* cols;  // device array of ncol row indices of W^T
  int32_t n, ncol;
};
// Truncation SVD by block one-sided (Hestenes) Jacobi: per sector the rows
// of B (m x c, row-major, a copy of M) and of W^T (m x m, starting as the
// identity) are rotated together, two blocks of kBjRows rows at a time,
// until the rows of B are mutually orthogonal; then M = W B, the singular
// values are the row norms of B and the left singular vectors the rows of
// W^T.  One job = one block pair of one sector in every round of the
// round-robin schedule over the sector's K (even) blocks.
constexpr int kBjRows = 16;
struct BjJob {
  int64_t b_off, w_off;  // element offsets of the sector's B and W^T
  int32_t m, c;          // rows, columns of M
  int32_t K, pr;         // blocks of the schedule (even), pair index in a round
  int32_t sector, pad;
};
// one round r of every job's schedule; off_max[sector] receives (as bits of
// a non-negative double, atomic max) the largest |G_ij| / sqrt(G_ii G_jj)
// of the round's Gram matrices; pairs already below tol * sqrt(c) are left unrotated
hipError_t launch_bj_round(const BjJob* jobs, int n_jobs, double* B, double* WT, unsigned long long* off_max, int r,
                           double tol, hipStream_t s);
// B blocks of the truncation: copy psi block (rows x cols, contiguous) to
// dst (row stride ld)
struct CopyJob {
  int64_t src, dst;
  int32_t rows, cols, ld, pad;
};
hipError_t launch_copy_blocks(const CopyJob* jobs, int n_jobs, const double* src, double* dst, hipStream_t s);
// W^T = identity for every sector (n_sect sectors: offsets woff, sizes m)
hipError_t launch_identity(const int64_t* woff, const int32_t* m, int n_sect, double* WT, hipStream_t s);
// sig[soff[q] + i] = norm of row i of sector q's B
hipError_t launch_row_norms(const int64_t* boff, const int32_t* m, const int32_t* c, const int64_t* soff, int n_sect,
                            const double* B, double* sig, hipStream_t s);
// out[out_off + r * ncol + j] = sign_j * WT[w_off + rows_j * n + r]: kept
// left singular vectors as isometry columns, each signed so that its
// largest-magnitude entry is positive (GatherJob.cols holds row indices of W^T)
hipError_t launch_gather_rows(const GatherJob* jobs, int n_jobs, const double* WT, double* out, hipStream_t s);
hipError_t launch_reduce_parts_f64(const RedJob* jobs, int n_jobs, const double* part, double* out, hipStream_t s);
hipError_t launch_reduce_parts_f32(const RedJob* jobs, int n_jobs, const float* part, float* out, hipStream_t s);
hipError_t launch_diag(const Tile* tiles, int64_t n_tiles, const DiagTask* tasks, const double* L0,
                       const double* L1, const double* R0, const double* R1, double* out,
                       hipStream_t s);
// C[m x n] = A[m x k] * B[k x n], all row-major, FP64.
hipError_t launch_gemm_f64(int64_t m, int64_t n, int64_t k, const double* A, const double* B,
                           double* C, hipStream_t s);
hipError_t launch_convert_f32(const double* in, float* out, int64_t n, hipStream_t s);
hipError_t launch_f64_to_f32(const double* in, float* out, int64_t n, hipStream_t s);
hipError_t launch_f32_to_f64(const float* in, double* out, int64_t n, hipStream_t s);

// ---- Davidson vector kernels ----
// out[i] = sum_n A[i*lda + n] * x[n], i < k   (FP64, deterministic)
hipError_t launch_multidot(const double* A, int64_t lda, int k, const double* x, int64_t n,
                           double* out, double* scratch, hipStream_t s);
// y[n] = alpha*y[n] + sum_i coef[i] * A[i*lda + n]  (coef on the device)
hipError_t launch_multiaxpy(const double* A, int64_t lda, int k, const double* coef,
                            double coef_scale, double* y, double alpha, int64_t n, hipStream_t s);
// out[0] = sum x[n] y[n] in FP64; scratch holds kRedBlocks doubles
constexpr int kRedBlocks = 512;
hipError_t launch_dot_f64(const double* x, const double* y, int64_t n, double* out, double* scratch, hipStream_t s);
hipError_t launch_dot_f32(const float* x, const float* y, int64_t n, double* out, double* scratch, hipStream_t s);
hipError_t launch_scale_f64(double* x, int64_t n, double a, hipStream_t s);
hipError_t launch_scale_f32(float* x, int64_t n, float a, hipStream_t s);
}  // namespace heff

struct heff_blocks;
namespace heff {
// whether every later product on b writes only one shard's output blocks
bool blocks_sharded(const heff_blocks* b);
// elements of b's two-site vector
int64_t blocks_n_elem(const heff_blocks* b);
// records the device address of the allocation-free energy's static
// scratch array on `device` (current); called once per context creation
hipError_t noalloc_setup(int device);
}  // namespace heff

namespace heff {
// Device memory provider (the heff_alloc callbacks of a context, or
// hipMalloc / hipFree when fa is null).  Every object keeps the provider its
// memory came from and frees through it.
struct Alloc {
  void* (*fa)(size_t, void*) = nullptr;
  void (*ff)(void*, void*) = nullptr;
  void* user = nullptr;
};
// provider of the context whose C-ABI call runs on this thread (contexts
// are used by one host thread at a time)
extern thread_local Alloc tl_alloc;
// nullptr when the provider refuses (or hipMalloc fails)
void* dev_alloc(size_t bytes, const Alloc& a);
void dev_free(void* p, const Alloc& a);
}  // namespace heff

// context object behind the opaque heff_ctx handle of the C ABI
struct heff_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  heff::Alloc alloc;  // device memory provider of every object made on it
  std::string err;
  // per-variant kernel timing of the product (HIP events on the variant's stream)
  bool timing = false;
  std::vector<hipEvent_t> ev_start[heff::kNumVariants], ev_stop[heff::kNumVariants];
  // streams of the product's kernel variants (default priority, forked from
  // and joined back into `stream` by events); created on first use
  hipStream_t vs[heff::kNumVariants] = {};
  hipEvent_t fork = nullptr, join[heff::kNumVariants] = {};
  int fp64_kernel = heff::kFp64Auto;  // kernel family of the FP64 product
};
