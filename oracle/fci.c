/* Test infrastructure: reference (oracle) code.  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may use it.
 *
 * Plain determinant-space action of the second-quantized Hamiltonian
 * (Sec. II.A, Eq. ``Hamiltonian``), written straight from its definition:
 *
 *   H = sum_{pq} t_pq a+_p a_q + 1/2 sum_{pqrs} g_pqrs a+_p a+_q a_s a_r
 *
 * with spin-orbital p = (i, sigma), t_pq = h[i_p][i_q] delta(sigma_p,sigma_q)
 * and g_pqrs = V[i_p][i_r][i_q][i_s] delta(sigma_p,sigma_r)
 * delta(sigma_q,sigma_s)  (chemist's (ij|kl) = V[i][j][k][l]).
 *
 * A determinant is a bit string over 2N modes, mode m = 2 i + sigma
 * (sigma 0 = up, 1 = down); the state is the product of creation operators
 * in ascending mode order acting on the vacuum.  The sign of a+_m / a_m is
 * (-1)^(number of occupied modes below m).  128-bit strings cover N <= 64.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

static inline int bit(u128 d, int m) { return (int)((d >> m) & 1); }

static inline int popc(u128 x) {
  return __builtin_popcountll((uint64_t)x) + __builtin_popcountll((uint64_t)(x >> 64));
}

/* parity sign of the occupied modes strictly below m */
static inline double jw(u128 d, int m) {
  u128 mask = (m == 0) ? (u128)0 : ((((u128)1) << m) - 1);
  return (popc(d & mask) & 1) ? -1.0 : 1.0;
}

static inline u128 ld(const uint64_t* p) { return ((u128)p[1] << 64) | (u128)p[0]; }
static inline void st(uint64_t* p, u128 d) { p[0] = (uint64_t)d; p[1] = (uint64_t)(d >> 64); }

/* Callback-style accumulation: emit(ctx, det_out, value). */
typedef void (*emit_fn)(void* ctx, u128 d, double v);

static void apply_h(int n, const double* h, const double* V, u128 d, emit_fn emit, void* ctx) {
  const int nm = 2 * n;
  /* one-body: t_pq a+_p a_q */
  for (int q = 0; q < nm; ++q) {
    if (!bit(d, q)) continue;
    double s1 = jw(d, q);
    u128 d1 = d & ~(((u128)1) << q);
    for (int p = (q & 1); p < nm; p += 2) { /* same spin as q */
      if (bit(d1, p)) continue;
      double s2 = jw(d1, p);
      double t = h[(p >> 1) * n + (q >> 1)];
      if (t == 0.0) continue;
      emit(ctx, d1 | (((u128)1) << p), t * s1 * s2);
    }
  }
  /* two-body: 1/2 g_pqrs a+_p a+_q a_s a_r  (a_r acts first) */
  for (int r = 0; r < nm; ++r) {
    if (!bit(d, r)) continue;
    double s1 = jw(d, r);
    u128 d1 = d & ~(((u128)1) << r);
    for (int s = 0; s < nm; ++s) {
      if (!bit(d1, s)) continue;
      double s2 = jw(d1, s);
      u128 d2 = d1 & ~(((u128)1) << s);
      for (int q = (s & 1); q < nm; q += 2) { /* sigma_q == sigma_s */
        if (bit(d2, q)) continue;
        double s3 = jw(d2, q);
        u128 d3 = d2 | (((u128)1) << q);
        for (int p = (r & 1); p < nm; p += 2) { /* sigma_p == sigma_r */
          if (bit(d3, p)) continue;
          double s4 = jw(d3, p);
          int ip = p >> 1, ir = r >> 1, iq = q >> 1, is = s >> 1;
          double g = V[(((size_t)ip * n + ir) * n + iq) * n + is];
          if (g == 0.0) continue;
          emit(ctx, d3 | (((u128)1) << p), 0.5 * g * s1 * s2 * s3 * s4);
        }
      }
    }
  }
}

/* ---- binary search in a sorted basis ---- */
static int64_t find(const uint64_t* basis, int64_t nb, u128 d) {
  int64_t lo = 0, hi = nb - 1;
  while (lo <= hi) {
    int64_t mid = (lo + hi) >> 1;
    u128 v = ld(basis + 2 * mid);
    if (v == d) return mid;
    if (v < d) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

/* ---- H|det> as a list ---- */
typedef struct { u128* d; double* v; int64_t n, cap; } listctx;
static void emit_list(void* c, u128 d, double v) {
  listctx* L = (listctx*)c;
  if (L->n < L->cap) { L->d[L->n] = d; L->v[L->n] = v; }
  L->n++;
}

/* Writes the (unsummed) terms of H|det> into out_det (2 words each) and
 * out_val; returns the number of terms (larger than cap means truncated). */
int64_t fci_apply_det(int n, const double* h, const double* V, const uint64_t* det,
                      uint64_t* out_det, double* out_val, int64_t cap) {
  listctx L;
  L.cap = cap; L.n = 0;
  L.d = (u128*)malloc(sizeof(u128) * (size_t)(cap > 0 ? cap : 1));
  L.v = out_val;
  apply_h(n, h, V, ld(det), emit_list, &L);
  int64_t m = L.n < cap ? L.n : cap;
  for (int64_t i = 0; i < m; ++i) st(out_det + 2 * i, L.d[i]);
  free(L.d);
  return L.n;
}

/* ---- <det'|H|det> summed against a vector on a sorted basis ---- */
typedef struct { const uint64_t* basis; int64_t nb; const double* x; double acc; } dotctx;
static void emit_dot(void* c, u128 d, double v) {
  dotctx* D = (dotctx*)c;
  int64_t j = find(D->basis, D->nb, d);
  if (j >= 0) D->acc += v * D->x[j];
}

/* returns sum_{j} <basis_j| H |det> x_j  ( = (H x)[det] since H is real symmetric) */
double fci_row_dot(int n, const double* h, const double* V, const uint64_t* det,
                   int64_t nb, const uint64_t* basis, const double* x) {
  dotctx D = {basis, nb, x, 0.0};
  apply_h(n, h, V, ld(det), emit_dot, &D);
  return D.acc;
}

/* ---- sparse H on a sorted sector basis: COO triplets (duplicates allowed) ---- */
typedef struct { const uint64_t* basis; int64_t nb, col; int64_t *ri, *ci; double* v; int64_t n, cap; } cooctx;
static void emit_coo(void* c, u128 d, double v) {
  cooctx* C = (cooctx*)c;
  int64_t j = find(C->basis, C->nb, d);
  if (j < 0) return;
  if (C->n < C->cap) { C->ri[C->n] = j; C->ci[C->n] = C->col; C->v[C->n] = v; }
  C->n++;
}

int64_t fci_build_coo(int n, const double* h, const double* V, int64_t nb, const uint64_t* basis,
                      int64_t* rows, int64_t* cols, double* vals, int64_t cap) {
  cooctx C = {basis, nb, 0, rows, cols, vals, 0, cap};
  for (int64_t i = 0; i < nb; ++i) {
    C.col = i;
    apply_h(n, h, V, ld(basis + 2 * i), emit_coo, &C);
  }
  return C.n;
}
