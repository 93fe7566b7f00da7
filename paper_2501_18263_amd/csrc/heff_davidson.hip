// Davidson eigensolver of the Diag_H step (the lowest eigenpair of H_eff).
// The solver choices (one product per step, restart to the current and
// previous Ritz vectors, preconditioner r/(theta - diag) with |theta - d|
// floored at 1e-8, classical Gram-Schmidt twice, ||r|| <= tol |theta|) are
// fixed so that the iterates are comparable step by step.  Everything but
// the H_eff product is FP64 on the device; the subspace eigenproblem is a
// one-work-group parallel (round-robin) Jacobi method.
#include "heff_internal.h"
#include "../../include/heff.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>


namespace heff {
constexpr int kMaxBasis = 32;

// ---------------------------------------------------------------- small kernels
// G[i][k-1] = G[k-1][i] = col[i]
__global__ void set_gcol(double* G, const double* col, int k) {
  int i = threadIdx.x;
  if (i < k) {
    G[i * kMaxBasis + (k - 1)] = col[i];
    G[(k - 1) * kMaxBasis + i] = col[i];
  }
}

// Lowest eigenpair of the symmetric k x k matrix G (ld kMaxBasis):
// small[0] = theta, y[0..k) eigenvector with its largest |entry| positive.
__global__ __launch_bounds__(256) void jacobi_lowest(const double* G, int k, double* small, double* y) {
  __shared__ double A[kMaxBasis][kMaxBasis + 1];
  __shared__ double Vm[kMaxBasis][kMaxBasis + 1];
  __shared__ double cs[kMaxBasis / 2], sn[kMaxBasis / 2];
  __shared__ int pp[kMaxBasis / 2], qq[kMaxBasis / 2];
  __shared__ double red[256];
  __shared__ int done;
  const int tid = threadIdx.x;
  const int K = (k + 1) & ~1;  // even number of players (a padded index never rotates)
  for (int idx = tid; idx < kMaxBasis * kMaxBasis; idx += 256) {
    int i = idx / kMaxBasis, j = idx % kMaxBasis;
    A[i][j] = (i < k && j < k) ? G[i * kMaxBasis + j] : 0.0;
    Vm[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int idx = tid; idx < k * k; idx += 256) {
      int i = idx / k, j = idx % k;
      double a2 = A[i][j] * A[i][j];
      tot += a2;
      if (i != j) off += a2;
    }
    red[tid] = off;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) red[tid] += red[tid + st];
      __syncthreads();
    }
    double offs = red[0];
    __syncthreads();
    red[tid] = tot;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) red[tid] += red[tid + st];
      __syncthreads();
    }
    if (tid == 0) done = (offs <= 1e-32 * red[0]) ? 1 : 0;
    __syncthreads();
    if (done) break;
    for (int r = 0; r < K - 1; ++r) {
      if (tid < K / 2) {
        // circle method: player 0 fixed, players 1..K-1 rotate
        auto pos = [&](int j) { return j == 0 ? 0 : 1 + ((j - 1 + r) % (K - 1)); };
        int a = pos(tid), b = pos(K - 1 - tid);
        int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, s = 0.0;
        if (q < k && A[p][q] != 0.0) {
          double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
          double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
        }
        cs[tid] = c;
        sn[tid] = s;
        pp[tid] = p;
        qq[tid] = q;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int idx = tid; idx < (K / 2) * K; idx += 256) {
        int pr = idx / K, j = idx % K;
        int p = pp[pr], q = qq[pr];
        double c = cs[pr], s = sn[pr];
        double ap = A[p][j], aq = A[q][j];
        A[p][j] = c * ap - s * aq;
        A[q][j] = s * ap + c * aq;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int idx = tid; idx < (K / 2) * K; idx += 256) {
        int pr = idx / K, i = idx % K;
        int p = pp[pr], q = qq[pr];
        double c = cs[pr], s = sn[pr];
        double ap = A[i][p], aq = A[i][q];
        A[i][p] = c * ap - s * aq;
        A[i][q] = s * ap + c * aq;
        double vp = Vm[i][p], vq = Vm[i][q];
        Vm[i][p] = c * vp - s * vq;
        Vm[i][q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    int best = 0;
    for (int i = 1; i < k; ++i)
      if (A[i][i] < A[best][best]) best = i;
    int im = 0;
    for (int i = 1; i < k; ++i)
      if (fabs(Vm[i][best]) > fabs(Vm[im][best])) im = i;
    double sg = Vm[im][best] < 0 ? -1.0 : 1.0;
    small[0] = A[best][best];
    for (int i = 0; i < kMaxBasis; ++i) y[i] = (i < k) ? sg * Vm[i][best] : 0.0;
  }
}

// t = r / (theta - d), |theta - d| floored at 1e-8 (sign kept, zero positive)
__global__ void precondition(const double* r, const double* d, const double* small, double* t, int64_t n) {
  const double th = small[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double den = th - d[i];
    if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
    t[i] = r[i] / den;
  }
}

// x *= 1/sqrt(nrm2[0])
__global__ void normalize(double* x, const double* nrm2, int64_t n) {
  const double s = 1.0 / sqrt(nrm2[0]);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] *= s;
}

// restart coefficients: Y[:,0] = y, Y[:,1] = z/||z||, z = yp - (y.yp) y twice;
// small[2] = ||z||.  Y stored column-major with ld kMaxBasis.
__global__ void restart_coef(const double* y, const double* yp, int k, double* Y, double* small) {
  if (threadIdx.x != 0) return;
  double z[kMaxBasis];
  double d = 0.0;
  for (int i = 0; i < k; ++i) d += y[i] * yp[i];
  for (int i = 0; i < k; ++i) z[i] = yp[i] - d * y[i];
  d = 0.0;
  for (int i = 0; i < k; ++i) d += y[i] * z[i];
  double nz = 0.0;
  for (int i = 0; i < k; ++i) {
    z[i] -= d * y[i];
    nz += z[i] * z[i];
  }
  nz = sqrt(nz);
  small[2] = nz;
  for (int i = 0; i < kMaxBasis; ++i) {
    Y[i] = i < k ? y[i] : 0.0;
    Y[kMaxBasis + i] = (i < k && nz > 0) ? z[i] / nz : 0.0;
  }
}

// G_new = Y^T G Y for kk columns; y_prev = Y^T y (= e_0)
__global__ void restart_g(double* G, const double* Y, int k, int kk, double* yprev) {
  __shared__ double T[kMaxBasis][2];
  int i = threadIdx.x;
  if (i < k) {
    for (int c = 0; c < kk; ++c) {
      double v = 0.0;
      for (int j = 0; j < k; ++j) v += G[i * kMaxBasis + j] * Y[c * kMaxBasis + j];
      T[i][c] = v;
    }
  }
  __syncthreads();
  double out[2][2] = {};
  if (i == 0) {
    for (int a = 0; a < kk; ++a)
      for (int c = 0; c < kk; ++c) {
        double v = 0.0;
        for (int j = 0; j < k; ++j) v += Y[a * kMaxBasis + j] * T[j][c];
        out[a][c] = v;
      }
  }
  __syncthreads();
  if (i == 0) {
    for (int a = 0; a < kMaxBasis * kMaxBasis; ++a) G[a] = 0.0;
    for (int a = 0; a < kk; ++a)
      for (int c = 0; c < kk; ++c) G[a * kMaxBasis + c] = out[a][c];
    for (int a = 0; a < kMaxBasis; ++a) yprev[a] = (a == 0) ? 1.0 : 0.0;
  }
}

__global__ void copy_small(const double* src, double* dst, int n) {
  int i = threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// index of the largest |x_i| (first on ties) -> flip sign of x so it is positive
__global__ __launch_bounds__(256) void fix_sign(double* x, int64_t n) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  double best = -1.0;
  int64_t idx = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    double a = fabs(x[i]);
    if (a > best) { best = a; idx = i; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      double o = bv[threadIdx.x + st];
      int64_t oi = bi[threadIdx.x + st];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const double sg = x[bi[0]] < 0 ? -1.0 : 1.0;
  __syncthreads();
  if (sg < 0)
    for (int64_t i = threadIdx.x; i < n; i += 256) x[i] = -x[i];
}

static unsigned g1d(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace heff

using namespace heff;

struct heff_dav {
  heff_ctx* ctx = nullptr;  // creating context (not used by heff_dav_free)
  hipStream_t stream = nullptr;
  const heff_blocks* blocks = nullptr;
  int m_max = 24;
  double tol = 1e-10;
  int64_t n = 0;
  int k = 1;               // basis vectors present (the newest has no product yet)
  bool converged = false;
  bool started = false;
  double* V = nullptr;     // (m_max + 3) x n
  double* W = nullptr;     // (m_max + 3) x n
  double* d = nullptr;     // diag(H_eff)
  double* r = nullptr;
  double* u = nullptr;
  double* t = nullptr;
  float* x32 = nullptr;    // reduced-precision product buffers
  float* y32 = nullptr;
  double* scratch = nullptr;  // reduction partials
  double* G = nullptr;        // kMaxBasis^2
  double* small = nullptr;    // [0] theta, [1] ||r||^2, [2] ||z||, [3] ||t||^2
  double* y = nullptr;        // kMaxBasis
  double* yprev = nullptr;    // kMaxBasis
  double* col = nullptr;      // kMaxBasis
  double* Y = nullptr;        // 2*kMaxBasis
  double* cvec = nullptr;     // kMaxBasis
  double* minus1 = nullptr;   // constant
  Alloc al;                   // provider of the buffers above
};

extern "C" int heff_diag(heff_ctx* ctx, const heff_blocks* b, double* diag);

#define DCHECK(x)                                                      \
  do {                                                                 \
    hipError_t e_ = (x);                                               \
    if (e_ != hipSuccess) {                                            \
      ctx->err = std::string(#x) + ": " + hipGetErrorString(e_);       \
      return HEFF_EHIP;                                                \
    }                                                                  \
  } while (0)

static void dav_release(heff_dav* d) {
  double* ptrs[] = {d->V, d->W, d->d, d->r, d->u, d->t, d->scratch, d->G, d->small, d->y, d->yprev, d->col, d->Y, d->cvec, d->minus1};
  for (double* p : ptrs) dev_free(p, d->al);
  dev_free(d->x32, d->al);
  dev_free(d->y32, d->al);
}

extern "C" int heff_dav_create(heff_ctx* ctx, const heff_blocks* b, int32_t m_max, double tol, const double* psi0,
                               heff_dav** out) {
  if (!ctx) return HEFF_EINVAL;
  if (!b || !psi0 || !out || m_max < 3 || m_max > 29 || !(tol > 0)) {
    ctx->err = "heff_dav_create: bad argument (m_max in [3, 29], tol > 0)";
    return HEFF_EINVAL;
  }
  *out = nullptr;
  if (blocks_sharded(b)) {
    ctx->err = "heff_dav_create: the product is restricted to one shard's output blocks";
    return HEFF_ESTATE;
  }
  int64_t n = 0;
  heff_psi_layout(b, &n, nullptr, nullptr, nullptr);
  heff_dav* D = new (std::nothrow) heff_dav;
  if (!D) return HEFF_ENOMEM;
  D->ctx = ctx;
  D->stream = ctx->stream;
  D->blocks = b;
  D->m_max = m_max;
  D->tol = tol;
  D->n = n;
  hipStream_t s = ctx->stream;
  D->al = ctx->alloc;
  auto A = [&](double** p, size_t cnt) { return (*p = (double*)dev_alloc(std::max<size_t>(cnt, 1) * sizeof(double), D->al)) != nullptr; };
  auto F = [&](float** p, size_t cnt) { return (*p = (float*)dev_alloc(std::max<size_t>(cnt, 1) * sizeof(float), D->al)) != nullptr; };
  size_t slots = (size_t)(m_max + 3);
  if (!A(&D->V, slots * n) || !A(&D->W, slots * n) || !A(&D->d, n) || !A(&D->r, n) || !A(&D->u, n) ||
      !A(&D->t, n) || !A(&D->scratch, 512 * kMaxBasis) || !A(&D->G, kMaxBasis * kMaxBasis) || !A(&D->small, 8) ||
      !A(&D->y, kMaxBasis) || !A(&D->yprev, kMaxBasis) || !A(&D->col, kMaxBasis) || !A(&D->Y, 2 * kMaxBasis) ||
      !A(&D->cvec, kMaxBasis) || !A(&D->minus1, 1) || !F(&D->x32, n) || !F(&D->y32, n)) {
    dav_release(D);
    delete D;
    ctx->err = "heff_dav_create: device allocation failed";
    return HEFF_ENOMEM;
  }
  DCHECK(hipMemsetAsync(D->G, 0, kMaxBasis * kMaxBasis * sizeof(double), s));
  DCHECK(hipMemsetAsync(D->yprev, 0, kMaxBasis * sizeof(double), s));
  const double m1 = -1.0;
  DCHECK(hipMemcpyAsync(D->minus1, &m1, sizeof(double), hipMemcpyHostToDevice, s));
  DCHECK(hipMemcpyAsync(D->V, psi0, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  DCHECK(launch_multidot(D->V, n, 1, D->V, n, D->small + 3, D->scratch, s));
  hipLaunchKernelGGL(normalize, dim3(g1d(n)), dim3(256), 0, s, D->V, D->small + 3, n);
  int rc = heff_diag(ctx, b, D->d);
  if (rc != HEFF_OK) {
    dav_release(D);
    delete D;
    return rc;
  }
  DCHECK(hipStreamSynchronize(s));
  *out = D;
  return HEFF_OK;
}

extern "C" int heff_davidson_step(heff_ctx* ctx, heff_dav* D, int prec, double* theta, double* resid) {
  if (!ctx) return HEFF_EINVAL;
  if (!D) { ctx->err = "null solver"; return HEFF_EINVAL; }
  if (D->converged) { ctx->err = "Davidson already converged"; return HEFF_ESTATE; }
  if (blocks_sharded(D->blocks)) {
    ctx->err = "the product is restricted to one shard's output blocks";
    return HEFF_ESTATE;
  }
  hipStream_t s = ctx->stream;
  const int64_t n = D->n;
  const int k = D->k;
  double* vk = D->V + (int64_t)(k - 1) * n;
  double* wk = D->W + (int64_t)(k - 1) * n;
  // 1. w = H v
  int rc;
  if (prec == HEFF_FP64) {
    rc = heff_apply(ctx, D->blocks, prec, vk, wk);
  } else {
    DCHECK(launch_f64_to_f32(vk, D->x32, n, s));
    rc = heff_apply(ctx, D->blocks, prec, D->x32, D->y32);
    if (rc == HEFF_OK) DCHECK(launch_f32_to_f64(D->y32, wk, n, s));
  }
  if (rc != HEFF_OK) return rc;
  // 2. Rayleigh matrix column
  DCHECK(launch_multidot(D->V, n, k, wk, n, D->col, D->scratch, s));
  hipLaunchKernelGGL(set_gcol, dim3(1), dim3(kMaxBasis), 0, s, D->G, D->col, k);
  // 3. lowest eigenpair of G
  hipLaunchKernelGGL(jacobi_lowest, dim3(1), dim3(256), 0, s, D->G, k, D->small, D->y);
  // 4. u = V y, r = W y - theta u, ||r||^2
  DCHECK(launch_multiaxpy(D->V, n, k, D->y, 1.0, D->u, 0.0, n, s));
  DCHECK(launch_multiaxpy(D->W, n, k, D->y, 1.0, D->r, 0.0, n, s));
  DCHECK(launch_multiaxpy(D->u, n, 1, D->small, -1.0, D->r, 1.0, n, s));
  DCHECK(launch_multidot(D->r, n, 1, D->r, n, D->small + 1, D->scratch, s));
  double hs[2];
  DCHECK(hipMemcpyAsync(hs, D->small, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  DCHECK(hipStreamSynchronize(s));
  const double th = hs[0], rn = std::sqrt(std::max(hs[1], 0.0));
  if (theta) *theta = th;
  if (resid) *resid = rn;
  D->started = true;
  if (!std::isfinite(th) || !std::isfinite(rn)) {
    ctx->err = "Davidson breakdown: non-finite Ritz value or residual";
    return HEFF_ENOCONV;
  }
  if (rn <= D->tol * std::fabs(th)) {
    D->converged = true;
    hipLaunchKernelGGL(copy_small, dim3(1), dim3(kMaxBasis), 0, s, D->y, D->yprev, kMaxBasis);
    return HEFF_OK;
  }
  // 5. correction
  hipLaunchKernelGGL(precondition, dim3(g1d(n)), dim3(256), 0, s, D->r, D->d, D->small, D->t, n);
  int kn = k;
  if (k >= D->m_max) {
    hipLaunchKernelGGL(restart_coef, dim3(1), dim3(1), 0, s, D->y, D->yprev, k, D->Y, D->small);
    double nz = 0.0;
    DCHECK(hipMemcpyAsync(&nz, D->small + 2, sizeof(double), hipMemcpyDeviceToHost, s));
    DCHECK(hipStreamSynchronize(s));
    int kk = nz > 1e-8 ? 2 : 1;
    double* Vt = D->V + (int64_t)(D->m_max + 1) * n;
    double* Wt = D->W + (int64_t)(D->m_max + 1) * n;
    for (int c = 0; c < kk; ++c) {
      DCHECK(launch_multiaxpy(D->V, n, k, D->Y + c * kMaxBasis, 1.0, Vt + (int64_t)c * n, 0.0, n, s));
      DCHECK(launch_multiaxpy(D->W, n, k, D->Y + c * kMaxBasis, 1.0, Wt + (int64_t)c * n, 0.0, n, s));
    }
    DCHECK(hipMemcpyAsync(D->V, Vt, (size_t)kk * n * sizeof(double), hipMemcpyDeviceToDevice, s));
    DCHECK(hipMemcpyAsync(D->W, Wt, (size_t)kk * n * sizeof(double), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(restart_g, dim3(1), dim3(kMaxBasis), 0, s, D->G, D->Y, k, kk, D->yprev);
    kn = kk;
  } else {
    hipLaunchKernelGGL(copy_small, dim3(1), dim3(kMaxBasis), 0, s, D->y, D->yprev, kMaxBasis);
  }
  // 6. classical Gram-Schmidt twice, normalize, append
  for (int pass = 0; pass < 2; ++pass) {
    DCHECK(launch_multidot(D->V, n, kn, D->t, n, D->cvec, D->scratch, s));
    DCHECK(launch_multiaxpy(D->V, n, kn, D->cvec, -1.0, D->t, 1.0, n, s));
  }
  DCHECK(launch_multidot(D->t, n, 1, D->t, n, D->small + 3, D->scratch, s));
  double* vnew = D->V + (int64_t)kn * n;
  DCHECK(hipMemcpyAsync(vnew, D->t, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(normalize, dim3(g1d(n)), dim3(256), 0, s, vnew, D->small + 3, n);
  D->k = kn + 1;
  return HEFF_OK;
}

extern "C" int heff_dav_ritz(heff_ctx* ctx, heff_dav* D, double* psi) {
  if (!ctx) return HEFF_EINVAL;
  if (!D || !psi) { ctx->err = "null argument"; return HEFF_EINVAL; }
  if (!D->started) { ctx->err = "no Davidson step taken yet"; return HEFF_ESTATE; }
  hipStream_t s = ctx->stream;
  DCHECK(hipMemcpyAsync(psi, D->u, D->n * sizeof(double), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(fix_sign, dim3(1), dim3(256), 0, s, psi, D->n);
  DCHECK(hipGetLastError());
  return HEFF_OK;
}

extern "C" int heff_dav_free(heff_dav* D) {
  if (!D) return HEFF_OK;
  (void)hipStreamSynchronize(D->stream);
  dav_release(D);
  delete D;
  return HEFF_OK;
}
