// Host runtime of the two-site H_eff library: problem validation, sector
// tables, renormalized operator stores, the factorized term list and the
// block task tables (Sec. II.C, Eqs. Hamilton_act_nonsym / _U1sym).
//
// Operator algebra (mode m = 2*site + spin, spin 0 = up, 1 = down):
//   H = sum t_pq a+_p a_q + 1/2 sum g_pqrs a+_p a+_q a_s a_r,
//   t_pq = h[i_p][i_q] d(s_p,s_q),  g_pqrs = (i_p i_r | i_q i_s) d(s_p,s_r) d(s_q,s_s).
// Split X | Y (all X modes before Y modes, products written X-op then Y-op):
//   H = H_X + H_Y + sum_{p in X} (a+_p S^Y_p - a_p S^Y+_p)
//       + sum_{r in Y} (T^X_r a_r - T^X+_r a+_r)
//       + sum_{p<q in X} (A_pq P_pq + h.c.) + sum_{p,r in X} B_pr Q_pr
//   S^Y_p = sum_q t_pq a_q + sum g_pqrs a+_q a_s a_r   (q,r,s in Y)
//   T^X_r = sum g_pqrs a+_p a+_q a_s                    (p,q,s in X)
//   A_pq = a+_p a+_q,  P_pq = sum_{r,s in Y} g_pqrs a_s a_r
//   B_pr = a+_p a_r,   Q_pr = sum_{q,s in Y} (g_pqrs - g_pqsr) a+_q a_s
// The left block keeps a+_p, A_pq, B_pq, T_x (x outside L) and H_L; the
// right block keeps a_r, a_s a_r, a+_q a_s, S_x (x outside R) and H_R.
// A product l (x) m (x) r acting on |l>|mid>|r> carries
// (-1)^(|m| n(l) + |r| (n(l) + n(mid))) for the input particle numbers.
#include "heff_host_common.h"

namespace heff {

// ------------------------------------------------------------------ device memory
thread_local Alloc tl_alloc;

void* dev_alloc(size_t bytes, const Alloc& a) {
  void* p = nullptr;
  if (a.fa) {
    p = a.fa(bytes, a.user);
    if (p && (reinterpret_cast<uintptr_t>(p) & 255)) {  // the provider broke its alignment promise
      a.ff(p, a.user);
      p = nullptr;
    }
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  return p;
}
void dev_free(void* p, const Alloc& a) {
  if (!p) return;
  if (a.fa) a.ff(p, a.user);
  else (void)hipFree(p);
}

// ------------------------------------------------------------------ sectors
static const int SQU[4] = {0, 0, 1, 1};  // site state (0, dn, up, updn): n_up
static const int SQD[4] = {0, 1, 0, 1};  //                                n_dn
static inline int site_n(int s) { return SQU[s] + SQD[s]; }

struct Bond {
  std::vector<int> nu, nd, dim;
  std::map<std::pair<int, int>, int> index;
  int n() const { return (int)dim.size(); }
  int find(int u, int d) const {
    auto it = index.find({u, d});
    return it == index.end() ? -1 : it->second;
  }
  int par(int i) const { return (nu[i] + nd[i]) & 1; }
};

static Bond make_bond(const heff_bond& b, const char* what) {
  Bond r;
  if (b.n_sect <= 0 || !b.nup || !b.ndn || !b.dim) throw Error(HEFF_EINVAL, std::string(what) + ": empty table");
  for (int i = 0; i < b.n_sect; ++i) {
    if (b.dim[i] <= 0) throw Error(HEFF_EINVAL, std::string(what) + ": non-positive dimension");
    if (b.dim[i] > 65535) throw Error(HEFF_EINVAL, std::string(what) + ": sector dimension above 65535");
    if (i > 0 && std::make_pair(b.nup[i - 1], b.ndn[i - 1]) >= std::make_pair(b.nup[i], b.ndn[i]))
      throw Error(HEFF_EINVAL, std::string(what) + ": sectors not strictly sorted");
    r.nu.push_back(b.nup[i]);
    r.nd.push_back(b.ndn[i]);
    r.dim.push_back(b.dim[i]);
    r.index[{b.nup[i], b.ndn[i]}] = i;
  }
  return r;
}

// ------------------------------------------------------------------ integrals
struct Ints {
  int n = 0;
  std::vector<double> h, V;
  double t(int p, int q) const {
    if ((p & 1) != (q & 1)) return 0.0;
    return h[(size_t)(p >> 1) * n + (q >> 1)];
  }
  double g(int p, int q, int r, int s) const {
    if ((p & 1) != (r & 1) || (q & 1) != (s & 1)) return 0.0;
    int ip = p >> 1, ir = r >> 1, iq = q >> 1, is = s >> 1;
    return V[(((size_t)ip * n + ir) * n + iq) * n + is];
  }
};

// ------------------------------------------------------------------ site matrices
using Mat4 = std::array<double, 16>;   // [out*4 + in]
using Mat16 = std::array<double, 256>; // [out*16 + in], middle state 4*s_k + s_k1

static Mat4 m4zero() { Mat4 m{}; return m; }
static Mat4 m4eye() { Mat4 m{}; for (int i = 0; i < 4; ++i) m[i * 5] = 1.0; return m; }
static Mat4 m4mul(const Mat4& a, const Mat4& b) {
  Mat4 c{};
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 4; ++k)
      if (a[i * 4 + k] != 0.0)
        for (int j = 0; j < 4; ++j) c[i * 4 + j] += a[i * 4 + k] * b[k * 4 + j];
  return c;
}
static Mat4 m4t(const Mat4& a) { Mat4 c{}; for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) c[i * 4 + j] = a[j * 4 + i]; return c; }
static void m4axpy(Mat4& y, double a, const Mat4& x) { for (int i = 0; i < 16; ++i) y[i] += a * x[i]; }
static bool m4nz(const Mat4& a) { for (double v : a) if (v != 0.0) return true; return false; }

static Mat4 CDAG4(int spin) {  // basis (0, dn, up, updn), |updn> = c+_up c+_dn |0>
  Mat4 m{};
  if (spin == 0) { m[2 * 4 + 0] = 1.0; m[3 * 4 + 1] = 1.0; }
  else { m[1 * 4 + 0] = 1.0; m[3 * 4 + 2] = -1.0; }
  return m;
}
static Mat4 C4(int spin) { return m4t(CDAG4(spin)); }

static Mat16 m16zero() { Mat16 m{}; return m; }
static Mat16 m16eye() { Mat16 m{}; for (int i = 0; i < 16; ++i) m[i * 17] = 1.0; return m; }
static Mat16 m16mul(const Mat16& a, const Mat16& b) {
  Mat16 c{};
  for (int i = 0; i < 16; ++i)
    for (int k = 0; k < 16; ++k)
      if (a[i * 16 + k] != 0.0)
        for (int j = 0; j < 16; ++j) c[i * 16 + j] += a[i * 16 + k] * b[k * 16 + j];
  return c;
}
static Mat16 m16t(const Mat16& a) { Mat16 c{}; for (int i = 0; i < 16; ++i) for (int j = 0; j < 16; ++j) c[i * 16 + j] = a[j * 16 + i]; return c; }
static void m16axpy(Mat16& y, double a, const Mat16& x) { for (int i = 0; i < 256; ++i) y[i] += a * x[i]; }
static bool m16nz(const Mat16& a) { for (double v : a) if (v != 0.0) return true; return false; }
static Mat16 kron44(const Mat4& a, const Mat4& b) {
  Mat16 c{};
  for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j)
    for (int k = 0; k < 4; ++k) for (int l = 0; l < 4; ++l)
      c[(i * 4 + k) * 16 + (j * 4 + l)] = a[i * 4 + j] * b[k * 4 + l];
  return c;
}

// parity of a site / middle operator from its first non-zero entry
static int par4(const Mat4& o) {
  for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) if (o[i * 4 + j] != 0.0) return (site_n(i) + site_n(j)) & 1;
  return 0;
}
static int mid_n(int m) { return site_n(m >> 2) + site_n(m & 3); }
static int par16(const Mat16& o) {
  for (int i = 0; i < 16; ++i) for (int j = 0; j < 16; ++j) if (o[i * 16 + j] != 0.0) return (mid_n(i) + mid_n(j)) & 1;
  return 0;
}

// sector change of one creation (+1) / annihilation (-1) of mode m
struct DQ { int u = 0, d = 0; };
static inline DQ mdq(int m, int sgn) { DQ q; if ((m & 1) == 0) q.u = sgn; else q.d = sgn; return q; }
static inline DQ operator+(DQ a, DQ b) { return {a.u + b.u, a.d + b.d}; }
static inline DQ operator-(DQ a, DQ b) { return {a.u - b.u, a.d - b.d}; }
static inline DQ operator-(DQ a) { return {-a.u, -a.d}; }

// ------------------------------------------------------------------ operator stores
struct Layout {
  DQ dq;
  std::vector<int> qin, qout, rows, cols;
  std::vector<int64_t> off;
  std::vector<int> blk_in, blk_out;  // sector index -> block index or -1
  int64_t size = 0;
};

static Layout make_layout(const Bond& b, DQ dq) {
  Layout L;
  L.dq = dq;
  L.blk_in.assign(b.n(), -1);
  L.blk_out.assign(b.n(), -1);
  for (int i = 0; i < b.n(); ++i) {
    int o = b.find(b.nu[i] + dq.u, b.nd[i] + dq.d);
    if (o < 0) continue;
    L.blk_in[i] = (int)L.qin.size();
    L.blk_out[o] = (int)L.qin.size();
    L.qin.push_back(i);
    L.qout.push_back(o);
    L.rows.push_back(b.dim[o]);
    L.cols.push_back(b.dim[i]);
    L.off.push_back(L.size);
    L.size += (int64_t)b.dim[o] * b.dim[i];
  }
  return L;
}

struct Key {
  int kind, i, j, k;
  bool operator<(const Key& o) const {
    if (kind != o.kind) return kind < o.kind;
    if (i != o.i) return i < o.i;
    if (j != o.j) return j < o.j;
    return k < o.k;
  }
};
enum Kind { K_H, K_C, K_A, K_B, K_T, K_D, K_DD, K_BB, K_S, K_TMP };

struct OpId {
  int cls = -1, idx = -1;
  bool valid() const { return cls >= 0; }
};

struct Store {
  const Bond* bond = nullptr;
  std::vector<Layout> cls;
  std::map<std::pair<int, int>, int> cls_of;
  std::vector<std::vector<Key>> keys;   // per class, per op
  std::vector<std::vector<int>> par;    // per class, per op
  std::vector<int64_t> base;
  int64_t total = 0;
  DevBuf dev;
  std::map<Key, OpId> names;

  int class_for(DQ dq) {
    auto it = cls_of.find({dq.u, dq.d});
    if (it != cls_of.end()) return it->second;
    int c = (int)cls.size();
    cls.push_back(make_layout(*bond, dq));
    keys.emplace_back();
    par.emplace_back();
    cls_of[{dq.u, dq.d}] = c;
    return c;
  }
  OpId add(const Key& k, DQ dq, int parity) {
    int c = class_for(dq);
    OpId id{c, (int)keys[c].size()};
    keys[c].push_back(k);
    par[c].push_back(parity);
    names[k] = id;
    return id;
  }
  OpId get(const Key& k) const {
    auto it = names.find(k);
    return it == names.end() ? OpId{} : it->second;
  }
  void allocate(hipStream_t s, bool zero) {
    base.assign(cls.size(), 0);
    total = 0;
    for (size_t c = 0; c < cls.size(); ++c) {
      base[c] = total;
      total += cls[c].size * (int64_t)keys[c].size();
    }
    dev.alloc((size_t)std::max<int64_t>(total, 1) * sizeof(double));
    if (zero) HCHECK(hipMemsetAsync(dev.p, 0, (size_t)std::max<int64_t>(total, 1) * sizeof(double), s));
  }
  int64_t offset(OpId id) const { return base[id.cls] + (int64_t)id.idx * cls[id.cls].size; }
  const Layout& lay(OpId id) const { return cls[id.cls]; }
  int parity(OpId id) const { return par[id.cls][id.idx]; }
};

// reference to an operator as used in a term / projection source
struct Ref {
  int where = -1;  // -1 identity, 0 main store, 1 temp store
  OpId id;
  bool trans = false;
};

// ------------------------------------------------------------------ isometries (device)
struct Iso {
  const Bond* old = nullptr;
  const Bond* nw = nullptr;
  std::vector<int64_t> qoff;                 // per new sector: offset of stacked matrix
  std::vector<std::array<int64_t, 4>> rowoff;  // per new sector, per s: first row
  DevBuf dev;
  int64_t size = 0;
  // offset of block (s, q_out) stored D_old(q_in) x D_new(q_out), or -1
  int64_t block(int s, int qo) const {
    int qi = old->find(nw->nu[qo] - SQU[s], nw->nd[qo] - SQD[s]);
    if (qi < 0) return -1;
    return qoff[qo] + rowoff[qo][s] * nw->dim[qo];
  }
};

static void make_iso(Iso& iso, const Bond& old, const Bond& nw, const double* host, hipStream_t s,
                     const char* what) {
  iso.old = &old;
  iso.nw = &nw;
  iso.qoff.resize(nw.n());
  iso.rowoff.resize(nw.n());
  int64_t off = 0;
  for (int q = 0; q < nw.n(); ++q) {
    int64_t r = 0;
    for (int st = 0; st < 4; ++st) {
      iso.rowoff[q][st] = r;
      int qi = old.find(nw.nu[q] - SQU[st], nw.nd[q] - SQD[st]);
      if (qi >= 0) r += old.dim[qi];
    }
    if (r < nw.dim[q]) throw Error(HEFF_EINVAL, std::string(what) + ": more kept states than reachable states");
    iso.qoff[q] = off;  // (orthonormality is checked by validate_problem)
    off += r * (int64_t)nw.dim[q];
  }
  iso.size = off;
  iso.dev.alloc((size_t)std::max<int64_t>(off, 1) * sizeof(double));
  HCHECK(hipMemcpyAsync(iso.dev.p, host, (size_t)off * sizeof(double), hipMemcpyHostToDevice, s));
}

// ------------------------------------------------------------------ step plans
struct Src {
  double coef;
  Ref x;
  Mat4 o;
};
struct NewDef {
  OpId out;
  std::vector<Src> src;
};
struct LinDef {
  int in_cls;                                 // class in the main store
  OpId out;                                   // op in the temp store (same dq)
  std::vector<std::pair<int, double>> coefs;  // (op index in in_cls, coefficient)
};

// temp ops are linear combinations of main-store ops of one class
struct LinPlan {
  Store* main = nullptr;
  Store tmp;
  std::vector<LinDef> defs;
  Ref make(DQ dq, int parity, const std::function<double(const Key&)>& coef) {
    auto it = main->cls_of.find({dq.u, dq.d});
    if (it == main->cls_of.end()) return Ref{};
    int c = it->second;
    LinDef d;
    d.in_cls = c;
    for (size_t i = 0; i < main->keys[c].size(); ++i) {
      double v = coef(main->keys[c][i]);
      if (v != 0.0) d.coefs.push_back({(int)i, v});
    }
    if (d.coefs.empty()) return Ref{};
    Key k{K_TMP, (int)defs.size(), 0, 0};
    d.out = tmp.add(k, dq, parity);
    defs.push_back(std::move(d));
    Ref r;
    r.where = 1;
    r.id = d.out;
    r.id = tmp.names[k];
    return r;
  }
  // run all lincombs as one GEMM per class
  void run(hipStream_t s) {
    tmp.allocate(s, false);
    std::map<int, std::vector<const LinDef*>> by_cls;
    for (auto& d : defs) by_cls[d.in_cls].push_back(&d);
    for (auto& kv : by_cls) {
      int c = kv.first;
      auto& v = kv.second;
      int n_in = (int)main->keys[c].size();
      int n_out = (int)v.size();
      const Layout& L = main->cls[c];
      if (L.size == 0) continue;
      // temps of this input class are consecutive in the temp class of the same dq
      OpId first = v.front()->out;
      for (int i = 0; i < n_out; ++i)
        if (v[i]->out.cls != first.cls || v[i]->out.idx != first.idx + i)
          throw Error(HEFF_EINVAL, "internal: temp ops not contiguous");
      std::vector<double> C((size_t)n_out * n_in, 0.0);
      for (int i = 0; i < n_out; ++i)
        for (auto& pc : v[i]->coefs) C[(size_t)i * n_in + pc.first] = pc.second;
      DevBuf dC;
      upload(dC, C, s);
      HCHECK(launch_gemm_f64(n_out, L.size, n_in, dC.as<double>(), main->dev.as<double>() + main->base[c],
                             tmp.dev.as<double>() + tmp.offset(first), s));
      HCHECK(hipStreamSynchronize(s));
    }
  }
};

// projection tasks of one renormalization step
struct ChainPlan {
  std::vector<Tile> tiles;
  std::vector<Task> tasks;
};

// Restrict a task to the range [m0, m0 + w) of its middle index c.  An
// identity op(X) (b == c) keeps only the rows k in the same range, so b and
// the columns of op(L) shrink with it; an identity op(R) stays the identity.
static Task restrict_c(Task s, int m0, int w) {
  if (s.flags & T_IDX) {
    s.b = (uint16_t)w;
    s.offL += (s.flags & T_TL) ? (int64_t)m0 * s.ldL : m0;
  } else {
    s.offX += (s.flags & T_TX) ? (int64_t)m0 * s.ldX : m0;
  }
  if (!(s.flags & T_IDR)) s.offR += (s.flags & T_TR) ? m0 : (int64_t)m0 * s.ldR;
  s.c = (uint16_t)w;
  return s;
}

// Split output tiles wider than max_dim into column slices and tasks whose
// middle dimension c exceeds max_dim into ranges of c (the partial products
// add up in the output-stationary accumulation, in the order the unsplit
// task adds them, so every output element gets the same sum in the same
// order), so that every task fits the register budget of a kernel instance
// (it holds T = op(L) op(X) with c columns and the output rows' e columns;
// the inner dimension b is streamed and unbounded).  The slices of one tile
// are consecutive; parent, if given, receives each new tile's original
// index.  Returns whether anything was split.
bool split_large(std::vector<Tile>& tiles, std::vector<Task>& tasks, int max_dim, std::vector<int>* parent) {
  bool any = false;
  for (auto& t : tiles) any |= t.e > max_dim;
  for (auto& k : tasks) any |= k.c > max_dim;
  if (parent) {
    parent->resize(tiles.size());
    for (size_t i = 0; i < tiles.size(); ++i) (*parent)[i] = (int)i;
  }
  if (!any) return false;
  std::vector<Tile> nt;
  std::vector<Task> nk;
  nk.reserve(tasks.size() + tasks.size() / 4);
  if (parent) parent->clear();
  for (size_t ti = 0; ti < tiles.size(); ++ti) {
    const Tile& t = tiles[ti];
    for (int n0 = 0; n0 < std::max(t.e, 1); n0 += max_dim) {
      Tile u = t;
      const int ew = std::max(std::min(max_dim, t.e - n0), 0);
      u.offOut = t.offOut + n0;
      u.e = ew;
      u.t0 = (int32_t)nk.size();
      for (int q = t.t0; q < t.t1; ++q) {
        Task s = tasks[q];
        if (s.flags & T_IDR) {
          // identity op(R) (c == e): the column slice [n0, n0 + ew) of the
          // output takes the same range of c
          if (s.c != t.e) throw Error(HEFF_EINVAL, "internal: identity right operand with c != e");
          s = restrict_c(s, n0, ew);
          s.e = (uint16_t)ew;
          nk.push_back(s);
          continue;
        }
        if (n0 > 0) s.offR += (s.flags & T_TR) ? (int64_t)n0 * s.ldR : n0;
        s.e = (uint16_t)ew;
        if (s.c <= max_dim) {
          nk.push_back(s);
          continue;
        }
        for (int m0 = 0; m0 < s.c; m0 += max_dim) nk.push_back(restrict_c(s, m0, std::min(max_dim, s.c - m0)));
      }
      u.t1 = (int32_t)nk.size();
      nt.push_back(u);
      if (parent) parent->push_back((int)ti);
    }
  }
  if (nk.size() > (size_t)INT32_MAX) throw Error(HEFF_EINVAL, "task table too large");
  tiles.swap(nt);
  tasks.swap(nk);
  return true;
}

// Largest dimension a tile's kernels hold in registers: the output width e
// and the middle dimension c of its tasks (T = op(L) op(X) has c columns).
int tile_dim(const Tile& t, const std::vector<Task>& tasks) {
  int d = t.e;
  for (int k = t.t0; k < t.t1; ++k) d = std::max<int>(d, tasks[k].c);
  return d;
}

// Work items of the matrix-core kernels, one list per variant.  Work-groups
// are dispatched round-robin over the eight XCDs (list position p runs on
// XCD p % 8), each with its own L2.  The 64-row items of one tile share the
// op(X) and op(R) slices of every step, so they are placed on the same XCD.
// Tiles with the same key form a group that goes to one XCD; groups go,
// largest first, to the XCD with the least work so far.  Without keys every
// tile is its own group (grouping the product's output blocks by their
// right sector, which share the sequence of op(R) blocks, raised the HBM
// traffic: it separated the blocks that share op(L) and psi).  Each XCD then
// starts its longest items first (a longest-processing-time order; items of
// one tile have the same estimate and stay adjacent, so they run side by
// side).  Unused positions hold row0 = -1 (the kernels skip them).
double task_flops(const Task& t);

// Kernel variant that runs a tile.  When a task table has tiles for the
// 128- or 256-wide kernels, its narrower tiles join the 128-wide kernel's
// queue instead of running in kernels of their own beside it: one
// longest-first queue keeps every CU on the wide work and fills the gaps
// with the short narrow items (concurrent narrow kernels took CU slots
// from the wide one's tail; N=40 D=4096: FP64 317 -> 300 ms, FP32 169 ->
// 150 ms, bf16 split 136 -> 124 ms on one box).
int launch_variant(const Tile& t, const std::vector<Task>& tasks, bool wide) {
  const int v = variant_of(tile_dim(t, tasks));
  return wide ? std::max(v, 2) : v;
}
bool has_wide(const std::vector<Tile>& tiles, const std::vector<Task>& tasks) {
  for (const Tile& t : tiles)
    if (variant_of(tile_dim(t, tasks)) >= 2) return true;
  return false;
}

// Estimated run time of one 64-row work item of a tile, in units of one
// 16x16x4 matrix instruction per wave: every pipeline step costs a fixed
// overhead (loads, LDS traffic, barrier) of about kStepCost instructions
// plus its matrix work, 4 ceil(c/16) instructions per stage-1 step and 4 NE
// per stage-2 step (NE = the output-width bucket of the kernel instance).
static int width_bucket(const Tile& tile, int nt) {
  const int ne = (tile.e + 15) / 16;
  for (int q = 1; q <= 3; ++q)
    if (ne <= std::max(1, nt * q / 4)) return std::max(1, nt * q / 4);
  return nt;
}
static double task_cost(const Task& t, int nt, int neb) {
  constexpr double kStepCost = 8.0;
  const int nb = (t.b + 15) / 16, nc = (t.c + 15) / 16;
  return nb * (kStepCost + 4.0 * std::min(nc, nt)) + nc * (kStepCost + 4.0 * neb);
}
static double item_cost(const Tile& tile, const std::vector<Task>& tasks, int v) {
  const int nt = 2 << v, neb = width_bucket(tile, nt);
  double cost = 0.0;
  for (int k = tile.t0; k < tile.t1; ++k) cost += task_cost(tasks[k], nt, neb);
  return cost;
}

// Split the task chains of the tiles whose work items would each take
// longer than the average work-group slot (total estimated work over
// `slots` concurrent work-groups): such a tile's tasks are cut into P <=
// max_parts contiguous ranges of about equal estimated time, each range a
// tile of its own that writes its partial sum (a x e, row stride e) into
// the output buffer at part_base and beyond; jobs then add the parts into
// the tile's output block in order.  The longest chain no longer bounds the
// product's time, at the price of P partial blocks and one small
// reduction.  Returns the number of part elements after part_base.
int64_t split_chains(std::vector<Tile>& tiles, const std::vector<Task>& tasks, int slots, int max_parts,
                     int64_t part_base, std::vector<RedJob>& jobs) {
  jobs.clear();
  const bool wide = has_wide(tiles, tasks);
  const size_t n = tiles.size();
  std::vector<double> cost(n);
  double total = 0.0;
  for (size_t t = 0; t < n; ++t) {
    cost[t] = item_cost(tiles[t], tasks, launch_variant(tiles[t], tasks, wide));
    total += cost[t] * std::max(1, (tiles[t].a + kTileRows - 1) / kTileRows);
  }
  const double target = total / std::max(1, slots);
  std::vector<Tile> nt;
  nt.reserve(n);
  int64_t part_elems = 0;
  for (size_t t = 0; t < n; ++t) {
    const Tile& tl = tiles[t];
    const int ntask = tl.t1 - tl.t0;
    const int P = std::min(ntask, (int)std::min<double>(max_parts, std::ceil(cost[t] / std::max(target, 1.0))));
    if (P < 2 || tl.a <= 0 || tl.e <= 0) {
      nt.push_back(tl);
      continue;
    }
    const int v = launch_variant(tl, tasks, wide), ntv = 2 << v, neb = width_bucket(tl, ntv);
    const int64_t blk = (int64_t)tl.a * tl.e;
    RedJob j{};
    j.out_off = tl.offOut;
    j.part_off = part_base + part_elems;
    j.a = tl.a;
    j.e = tl.e;
    j.ld = tl.ldOut;
    int k = tl.t0;
    double done = 0.0;
    int made = 0;
    for (int p = 0; p < P; ++p) {
      Tile u = tl;
      u.t0 = k;
      if (p == P - 1) {
        k = tl.t1;
      } else {
        // at least one task per part, and leave one for each later part
        const double goal = cost[t] * (p + 1) / P;
        do done += task_cost(tasks[k], ntv, neb), ++k;
        while (k < tl.t1 - (P - 1 - p) && done + 0.5 * task_cost(tasks[k], ntv, neb) < goal);
      }
      u.t1 = k;
      u.offOut = part_base + part_elems + (int64_t)made * blk;
      u.ldOut = tl.e;
      nt.push_back(u);
      ++made;
    }
    j.parts = made;
    part_elems += (int64_t)made * blk;
    jobs.push_back(j);
  }
  tiles.swap(nt);
  return part_elems;
}

void split_work(const std::vector<Tile>& tiles, const std::vector<Task>& tasks, const std::vector<int>& order,
                std::vector<Work> (&lists)[kNumVariants], const std::vector<int>* key) {
  constexpr int kXcd = 8;
  const bool wide = has_wide(tiles, tasks);
  std::vector<double> icost(tiles.size(), 0.0);
  for (size_t t = 0; t < tiles.size(); ++t) icost[t] = item_cost(tiles[t], tasks, launch_variant(tiles[t], tasks, wide));
  // groups per variant, in first-appearance order of `order`
  std::vector<std::vector<int>> groups[kNumVariants];
  std::vector<double> gcost[kNumVariants];
  std::map<std::pair<int, int>, int> gid;
  for (int t : order) {
    const int v = launch_variant(tiles[t], tasks, wide);
    const double cost = icost[t] * std::max(1, (tiles[t].a + kTileRows - 1) / kTileRows);
    int g;
    if (key) {
      auto it = gid.find({v, (*key)[t]});
      if (it == gid.end()) {
        g = (int)groups[v].size();
        gid[{v, (*key)[t]}] = g;
        groups[v].emplace_back();
        gcost[v].push_back(0.0);
      } else {
        g = it->second;
      }
    } else {
      g = (int)groups[v].size();
      groups[v].emplace_back();
      gcost[v].push_back(0.0);
    }
    groups[v][g].push_back(t);
    gcost[v][g] += cost;
  }
  for (int v = 0; v < kNumVariants; ++v) {
    std::vector<int> gorder(groups[v].size());
    for (size_t i = 0; i < gorder.size(); ++i) gorder[i] = (int)i;
    std::stable_sort(gorder.begin(), gorder.end(), [&](int a, int b) { return gcost[v][a] > gcost[v][b]; });
    std::vector<Work> q[kXcd];
    double load[kXcd] = {};
    for (int g : gorder) {
      int x = 0;
      for (int j = 1; j < kXcd; ++j)
        if (load[j] < load[x]) x = j;
      for (int t : groups[v][g])
        for (int r = 0; r < tiles[t].a; r += kTileRows) q[x].push_back({t, r});
      load[x] += gcost[v][g];
    }
    for (int x = 0; x < kXcd; ++x)
      std::stable_sort(q[x].begin(), q[x].end(),
                       [&](const Work& a, const Work& b) { return icost[a.tile] > icost[b.tile]; });
    size_t m = 0;
    for (int x = 0; x < kXcd; ++x) m = std::max(m, q[x].size());
    lists[v].clear();
    for (size_t i = 0; i < m; ++i)
      for (int x = 0; x < kXcd; ++x) lists[v].push_back(i < q[x].size() ? q[x][i] : Work{0, -1});
  }
}

// Readable element counts of the FP64 operand buffers (the ring kernel's
// 16-byte loads stay inside them).
int64_t elems64(const DevBuf& d) { return (int64_t)(d.bytes / sizeof(double)); }
static void set_limits(Bases<double>& b, const DevBuf& l0, const DevBuf& l1, const DevBuf& x0, const DevBuf& x1,
                       const DevBuf& r0, const DevBuf& r1) {
  b.lim[0] = elems64(l0);
  b.lim[1] = elems64(l1);
  b.lim[2] = elems64(x0);
  b.lim[3] = elems64(x1);
  b.lim[4] = elems64(r0);
  b.lim[5] = elems64(r1);
}
void set_limits(Bases<double>& b, const DevBuf& l0, const DevBuf& l1, int64_t x, const DevBuf& r0,
                       const DevBuf& r1) {
  b.lim[0] = elems64(l0);
  b.lim[1] = elems64(l1);
  b.lim[2] = b.lim[3] = x;
  b.lim[4] = elems64(r0);
  b.lim[5] = elems64(r1);
}

static void run_chain(ChainPlan& P, Bases<double> b, hipStream_t s) {
  if (P.tiles.empty()) return;
  // (the renormalization keeps tasks up to 256 wide: capped at 128 as the
  // product is, the block build at N=40, D=4096 took 5.5 instead of 5.7 s
  // with beta=1/2 and 5.8 instead of 6.8 s with beta=1, but the sweep
  // step's Ren_l 1.03 instead of 0.98 s)
  split_large(P.tiles, P.tasks, kMaxDim);
  DevBuf dt, dk;
  upload(dt, P.tiles, s);
  upload(dk, P.tasks, s);
  std::vector<int> order(P.tiles.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::vector<Work> lists[kNumVariants];
  split_work(P.tiles, P.tasks, order, lists);
  DevWorkSet dws;
  dws.upload_lists(lists, s);
  HCHECK(launch_mfma_f64(dt.as<Tile>(), dws.ws, dk.as<Task>(), b, s));
  HCHECK(hipStreamSynchronize(s));
}

// Generate the tasks new[q'<-q] += sum coef * o[s',s] * sign * A_{s'}^T X[q'-s' <- q-s] A_s
// for all new ops.  left: sign (-1)^{|o| n(q-s)}; right: (-1)^{|X| n(s)}.
static void plan_projection(const std::vector<NewDef>& defs, Store& nw, const Store& old, const Store* tmp,
                            const Iso& iso, bool left, ChainPlan& P) {
  const Bond& ob = *iso.old;
  const Bond& nb = *iso.nw;
  for (const NewDef& d : defs) {
    const Layout& NL = nw.lay(d.out);
    int64_t obase = nw.offset(d.out);
    for (size_t bi = 0; bi < NL.qin.size(); ++bi) {
      int qo_new = NL.qout[bi], qi_new = NL.qin[bi];
      Tile tile{};
      tile.offOut = obase + NL.off[bi];
      tile.a = NL.rows[bi];
      tile.e = NL.cols[bi];
      tile.ldOut = NL.cols[bi];
      tile.t0 = (int32_t)P.tasks.size();
      for (const Src& sr : d.src) {
        const Store* st = sr.x.where == 1 ? tmp : &old;
        int xpar = sr.x.where < 0 ? 0 : st->parity(sr.x.id);
        int opar = par4(sr.o);
        if (bi == 0) {  // every source must carry the sector change of the new operator
          DQ dx{};
          if (sr.x.where >= 0) dx = sr.x.trans ? -st->lay(sr.x.id).dq : st->lay(sr.x.id).dq;
          DQ ds{};
          for (int k = 0; k < 16; ++k)
            if (sr.o[k] != 0.0) { ds = DQ{SQU[k >> 2] - SQU[k & 3], SQD[k >> 2] - SQD[k & 3]}; break; }
          DQ tot = dx + ds;
          if (tot.u != NL.dq.u || tot.d != NL.dq.d || ((xpar + opar) & 1) != nw.parity(d.out))
            throw Error(HEFF_EINVAL, "internal: inconsistent renormalization source");
        }
        for (int so = 0; so < 4; ++so) {
          int qa = ob.find(nb.nu[qo_new] - SQU[so], nb.nd[qo_new] - SQD[so]);
          if (qa < 0) continue;
          for (int si = 0; si < 4; ++si) {
            double w = sr.o[so * 4 + si];
            if (w == 0.0) continue;
            int qb = ob.find(nb.nu[qi_new] - SQU[si], nb.nd[qi_new] - SQD[si]);
            if (qb < 0) continue;
            Task t{};
            uint32_t fl = T_TL;
            if (sr.x.where < 0) {
              if (qa != qb) continue;
              fl |= T_IDX;
            } else {
              const Layout& XL = st->lay(sr.x.id);
              int blk;
              if (!sr.x.trans) {
                blk = XL.blk_in[qb];
                if (blk < 0 || XL.qout[blk] != qa) continue;
              } else {
                blk = XL.blk_in[qa];
                if (blk < 0 || XL.qout[blk] != qb) continue;
                fl |= T_TX;
              }
              t.offX = st->offset(sr.x.id) + XL.off[blk];
              t.ldX = (uint16_t)XL.cols[blk];
              if (sr.x.where == 1) fl |= T_SELX;
            }
            t.ldL = (uint16_t)nb.dim[qo_new];
            t.ldR = (uint16_t)nb.dim[qi_new];
            int sgn = left ? ((opar && ob.par(qb)) ? -1 : 1) : ((xpar && (site_n(si) & 1)) ? -1 : 1);
            t.f = sr.coef * w * sgn;
            t.offL = iso.block(so, qo_new);
            t.offR = iso.block(si, qi_new);
            t.a = (uint16_t)nb.dim[qo_new];
            t.b = (uint16_t)ob.dim[qa];
            t.c = (uint16_t)ob.dim[qb];
            t.e = (uint16_t)nb.dim[qi_new];
            t.flags = (uint16_t)fl;
            P.tasks.push_back(t);
          }
        }
      }
      tile.t1 = (int32_t)P.tasks.size();
      P.tiles.push_back(tile);
    }
  }
}

// ------------------------------------------------------------------ block growth
static Mat4 site_ham(const Ints& I, int u) {
  int site[2] = {u, u + 1};
  Mat4 H = m4zero();
  for (int a : site) for (int b : site) m4axpy(H, I.t(a, b), m4mul(CDAG4(a & 1), C4(b & 1)));
  for (int a : site) for (int b : site) for (int c : site) for (int d : site) {
    double g = I.g(a, b, c, d);
    if (g != 0.0) m4axpy(H, 0.5 * g, m4mul(m4mul(CDAG4(a & 1), CDAG4(b & 1)), m4mul(C4(d & 1), C4(c & 1))));
  }
  return H;
}

struct Block {
  Bond bond;       // copy of the current bond table
  Store store;
};

static std::unique_ptr<Block> initial_block(bool left, int nmode, hipStream_t s) {
  auto B = std::make_unique<Block>();
  B->bond.nu = {0};
  B->bond.nd = {0};
  B->bond.dim = {1};
  B->bond.index[{0, 0}] = 0;
  B->store.bond = &B->bond;
  B->store.add({K_H, 0, 0, 0}, DQ{}, 0);
  for (int x = 0; x < nmode; ++x) {
    if (left) B->store.add({K_T, x, 0, 0}, mdq(x, +1), 1);
    else B->store.add({K_S, x, 0, 0}, mdq(x, -1), 1);
  }
  B->store.allocate(s, true);
  return B;
}

static Ref R_(const Store& st, const Key& k, bool trans = false) {
  Ref r;
  r.id = st.get(k);
  if (!r.id.valid()) throw Error(HEFF_EINVAL, "internal: missing operator");
  r.where = 0;
  r.trans = trans;
  return r;
}
static Ref RI() { return Ref{}; }

// one left step: L_old (sites 0..j-1) -> L_new (sites 0..j) with site j
static std::unique_ptr<Block> grow_left(Block& old, const Bond& nb, const Iso& iso, int j, int nmode,
                                        const Ints& I, hipStream_t s) {
  auto B = std::make_unique<Block>();
  B->bond = nb;
  B->store.bond = &B->bond;
  Store& os = old.store;
  Store& ns = B->store;
  LinPlan lp;
  lp.main = &os;
  lp.tmp.bond = &old.bond;
  std::vector<NewDef> defs;
  const int u = 2 * j, dn = 2 * j + 1;
  const int site[2] = {u, dn};
  Mat4 I4 = m4eye();
  auto def = [&](Key k, DQ dq, int parity) -> NewDef& {
    NewDef d;
    d.out = ns.add(k, dq, parity);
    defs.push_back(d);
    return defs.back();
  };
  std::vector<int> oldm;  // old modes
  for (int m = 0; m < 2 * j; ++m) oldm.push_back(m);
  // creators
  for (int p : oldm) def({K_C, p, 0, 0}, mdq(p, 1), 1).src.push_back({1.0, R_(os, {K_C, p, 0, 0}), I4});
  for (int m : site) def({K_C, m, 0, 0}, mdq(m, 1), 1).src.push_back({1.0, RI(), CDAG4(m & 1)});
  // pairs a+_p a+_q, p < q
  for (int p : oldm) for (int q : oldm) if (p < q)
    def({K_A, p, q, 0}, mdq(p, 1) + mdq(q, 1), 0).src.push_back({1.0, R_(os, {K_A, p, q, 0}), I4});
  for (int p : oldm) for (int m : site)
    def({K_A, p, m, 0}, mdq(p, 1) + mdq(m, 1), 0).src.push_back({1.0, R_(os, {K_C, p, 0, 0}), CDAG4(m & 1)});
  def({K_A, u, dn, 0}, mdq(u, 1) + mdq(dn, 1), 0).src.push_back({1.0, RI(), m4mul(CDAG4(0), CDAG4(1))});
  // a+_p a_q
  for (int p : oldm) for (int q : oldm)
    def({K_B, p, q, 0}, mdq(p, 1) + mdq(q, -1), 0).src.push_back({1.0, R_(os, {K_B, p, q, 0}), I4});
  for (int p : oldm) for (int m : site) {
    def({K_B, p, m, 0}, mdq(p, 1) + mdq(m, -1), 0).src.push_back({1.0, R_(os, {K_C, p, 0, 0}), C4(m & 1)});
    def({K_B, m, p, 0}, mdq(m, 1) + mdq(p, -1), 0).src.push_back({-1.0, R_(os, {K_C, p, 0, 0}, true), CDAG4(m & 1)});
  }
  for (int m : site) for (int n : site)
    def({K_B, m, n, 0}, mdq(m, 1) + mdq(n, -1), 0).src.push_back({1.0, RI(), m4mul(CDAG4(m & 1), C4(n & 1))});
  // T_x = sum_{p,q,s in L} g_pqxs a+_p a+_q a_s for x outside the new block
  for (int x = 2 * j + 2; x < nmode; ++x) {
    DQ dqx = mdq(x, 1);
    NewDef& d = def({K_T, x, 0, 0}, dqx, 1);
    d.src.push_back({1.0, R_(os, {K_T, x, 0, 0}), I4});
    for (int m : site) {
      Ref U = lp.make(dqx - mdq(m, -1), 0, [&](const Key& k) {
        return k.kind == K_A ? I.g(k.i, k.j, x, m) - I.g(k.j, k.i, x, m) : 0.0; });
      if (U.where >= 0) d.src.push_back({1.0, U, C4(m & 1)});
      Ref W = lp.make(dqx - mdq(m, 1), 0, [&](const Key& k) {
        return k.kind == K_B ? I.g(m, k.i, x, k.j) - I.g(k.i, m, x, k.j) : 0.0; });
      if (W.where >= 0) d.src.push_back({1.0, W, CDAG4(m & 1)});
    }
    for (int m : site) for (int n : site) {
      Ref Y = lp.make(dqx - mdq(m, 1) - mdq(n, -1), 1, [&](const Key& k) {
        return k.kind == K_C ? I.g(k.i, m, x, n) - I.g(m, k.i, x, n) : 0.0; });
      if (Y.where >= 0) d.src.push_back({1.0, Y, m4mul(CDAG4(m & 1), C4(n & 1))});
      if (m != n) {
        // sum_s g_{m n x s} a_s (x) a+_m a+_n, stored untransposed as sum g c_s
        Ref Z = lp.make(-(dqx - mdq(m, 1) - mdq(n, 1)), 1, [&](const Key& k) {
          return k.kind == K_C ? I.g(m, n, x, k.i) : 0.0; });
        if (Z.where >= 0) { Z.trans = true; d.src.push_back({1.0, Z, m4mul(CDAG4(m & 1), CDAG4(n & 1))}); }
      }
    }
    Mat4 o3 = m4zero();
    for (int a : site) for (int b : site) for (int c : site) {
      double g = I.g(a, b, x, c);
      if (g != 0.0) m4axpy(o3, g, m4mul(m4mul(CDAG4(a & 1), CDAG4(b & 1)), C4(c & 1)));
    }
    if (m4nz(o3)) d.src.push_back({1.0, RI(), o3});
  }
  // H_new
  {
    NewDef& d = def({K_H, 0, 0, 0}, DQ{}, 0);
    d.src.push_back({1.0, R_(os, {K_H, 0, 0, 0}), I4});
    d.src.push_back({1.0, RI(), site_ham(I, u)});
    for (int p : oldm) {
      Mat4 S = m4zero();
      for (int q : site) if (I.t(p, q) != 0.0) m4axpy(S, I.t(p, q), C4(q & 1));
      for (int q : site) for (int r : site) for (int t : site) {
        double g = I.g(p, q, r, t);
        if (g != 0.0) m4axpy(S, g, m4mul(m4mul(CDAG4(q & 1), C4(t & 1)), C4(r & 1)));
      }
      if (!m4nz(S)) continue;
      d.src.push_back({1.0, R_(os, {K_C, p, 0, 0}), S});
      d.src.push_back({-1.0, R_(os, {K_C, p, 0, 0}, true), m4t(S)});
    }
    for (int r : site) {
      d.src.push_back({1.0, R_(os, {K_T, r, 0, 0}), C4(r & 1)});
      d.src.push_back({-1.0, R_(os, {K_T, r, 0, 0}, true), CDAG4(r & 1)});
    }
    Ref PL = lp.make(DQ{1, 1}, 0, [&](const Key& k) {
      return k.kind == K_A ? I.g(k.i, k.j, u, dn) - I.g(k.i, k.j, dn, u) : 0.0; });
    if (PL.where >= 0) {
      Mat4 op = m4mul(C4(1), C4(0));
      d.src.push_back({1.0, PL, op});
      Ref PT = PL;
      PT.trans = true;
      d.src.push_back({1.0, PT, m4t(op)});
    }
    for (int q : site) for (int t : site) {
      Ref QL = lp.make(mdq(t, 1) - mdq(q, 1), 0, [&](const Key& k) {
        return k.kind == K_B ? I.g(k.i, q, k.j, t) - I.g(k.i, q, t, k.j) : 0.0; });
      if (QL.where >= 0) d.src.push_back({1.0, QL, m4mul(CDAG4(q & 1), C4(t & 1))});
    }
  }
  lp.run(s);
  ns.allocate(s, false);
  ChainPlan P;
  plan_projection(defs, ns, os, &lp.tmp, iso, true, P);
  Bases<double> b{};
  b.L[0] = b.L[1] = iso.dev.as<double>();
  b.R[0] = b.R[1] = iso.dev.as<double>();
  b.X[0] = os.dev.as<double>();
  b.X[1] = lp.tmp.dev.as<double>();
  b.out = ns.dev.as<double>();
  set_limits(b, iso.dev, iso.dev, os.dev, lp.tmp.dev, iso.dev, iso.dev);
  run_chain(P, b, s);
  return B;
}

// one right step: R_old (sites j+1..N-1) -> R_new (sites j..N-1) with site j
static std::unique_ptr<Block> grow_right(Block& old, const Bond& nb, const Iso& iso, int j, int nmode,
                                         const Ints& I, hipStream_t s) {
  auto B = std::make_unique<Block>();
  B->bond = nb;
  B->store.bond = &B->bond;
  Store& os = old.store;
  Store& ns = B->store;
  LinPlan lp;
  lp.main = &os;
  lp.tmp.bond = &old.bond;
  std::vector<NewDef> defs;
  const int u = 2 * j, dn = 2 * j + 1;
  const int site[2] = {u, dn};
  Mat4 I4 = m4eye();
  auto def = [&](Key k, DQ dq, int parity) -> NewDef& {
    NewDef d;
    d.out = ns.add(k, dq, parity);
    defs.push_back(d);
    return defs.back();
  };
  std::vector<int> oldm;
  for (int m = 2 * j + 2; m < nmode; ++m) oldm.push_back(m);
  // annihilators a_r
  for (int m : site) def({K_D, m, 0, 0}, mdq(m, -1), 1).src.push_back({1.0, RI(), C4(m & 1)});
  for (int r : oldm) def({K_D, r, 0, 0}, mdq(r, -1), 1).src.push_back({1.0, R_(os, {K_D, r, 0, 0}), I4});
  // a_s a_r, r < s
  def({K_DD, u, dn, 0}, mdq(u, -1) + mdq(dn, -1), 0).src.push_back({1.0, RI(), m4mul(C4(1), C4(0))});
  for (int m : site) for (int t : oldm)
    def({K_DD, m, t, 0}, mdq(m, -1) + mdq(t, -1), 0).src.push_back({-1.0, R_(os, {K_D, t, 0, 0}), C4(m & 1)});
  for (int r : oldm) for (int t : oldm) if (r < t)
    def({K_DD, r, t, 0}, mdq(r, -1) + mdq(t, -1), 0).src.push_back({1.0, R_(os, {K_DD, r, t, 0}), I4});
  // a+_q a_s
  for (int m : site) for (int n : site)
    def({K_BB, m, n, 0}, mdq(m, 1) + mdq(n, -1), 0).src.push_back({1.0, RI(), m4mul(CDAG4(m & 1), C4(n & 1))});
  for (int m : site) for (int t : oldm) {
    def({K_BB, m, t, 0}, mdq(m, 1) + mdq(t, -1), 0).src.push_back({1.0, R_(os, {K_D, t, 0, 0}), CDAG4(m & 1)});
    def({K_BB, t, m, 0}, mdq(t, 1) + mdq(m, -1), 0).src.push_back({-1.0, R_(os, {K_D, t, 0, 0}, true), C4(m & 1)});
  }
  for (int q : oldm) for (int t : oldm)
    def({K_BB, q, t, 0}, mdq(q, 1) + mdq(t, -1), 0).src.push_back({1.0, R_(os, {K_BB, q, t, 0}), I4});
  // S_x for x outside the new block
  for (int x = 0; x < 2 * j; ++x) {
    DQ dqx = mdq(x, -1);
    NewDef& d = def({K_S, x, 0, 0}, dqx, 1);
    d.src.push_back({1.0, R_(os, {K_S, x, 0, 0}), I4});
    for (int m : site) {
      if (I.t(x, m) != 0.0) d.src.push_back({I.t(x, m), RI(), C4(m & 1)});
      Ref D = lp.make(dqx - mdq(m, 1), 0, [&](const Key& k) {
        return k.kind == K_DD ? I.g(x, m, k.i, k.j) - I.g(x, m, k.j, k.i) : 0.0; });
      if (D.where >= 0) d.src.push_back({1.0, D, CDAG4(m & 1)});
      Ref Bq = lp.make(dqx - mdq(m, -1), 0, [&](const Key& k) {
        return k.kind == K_BB ? I.g(x, k.i, m, k.j) - I.g(x, k.i, k.j, m) : 0.0; });
      if (Bq.where >= 0) d.src.push_back({1.0, Bq, C4(m & 1)});
    }
    for (int m : site) for (int n : site) {
      Ref Yd = lp.make(dqx - mdq(m, 1) - mdq(n, -1), 1, [&](const Key& k) {
        return k.kind == K_D ? I.g(x, m, k.i, n) - I.g(x, m, n, k.i) : 0.0; });
      if (Yd.where >= 0) d.src.push_back({1.0, Yd, m4mul(CDAG4(m & 1), C4(n & 1))});
      if (m != n) {
        // (q outside site; r = m, s = n): a_n a_m (x) a+_q, stored as sum g d_q
        Ref Zd = lp.make(-(dqx - mdq(m, -1) - mdq(n, -1)), 1, [&](const Key& k) {
          return k.kind == K_D ? I.g(x, k.i, m, n) : 0.0; });
        if (Zd.where >= 0) { Zd.trans = true; d.src.push_back({1.0, Zd, m4mul(C4(n & 1), C4(m & 1))}); }
      }
    }
    Mat4 o3 = m4zero();
    for (int a : site) for (int b : site) for (int c : site) {
      double g = I.g(x, a, b, c);
      if (g != 0.0) m4axpy(o3, g, m4mul(m4mul(CDAG4(a & 1), C4(c & 1)), C4(b & 1)));
    }
    if (m4nz(o3)) d.src.push_back({1.0, RI(), o3});
  }
  // H_new
  {
    NewDef& d = def({K_H, 0, 0, 0}, DQ{}, 0);
    d.src.push_back({1.0, R_(os, {K_H, 0, 0, 0}), I4});
    d.src.push_back({1.0, RI(), site_ham(I, u)});
    for (int p : site) {
      d.src.push_back({1.0, R_(os, {K_S, p, 0, 0}), CDAG4(p & 1)});
      d.src.push_back({-1.0, R_(os, {K_S, p, 0, 0}, true), C4(p & 1)});
    }
    for (int r : oldm) {
      Mat4 Ts = m4zero();
      for (int a : site) for (int b : site) for (int c : site) {
        double g = I.g(a, b, r, c);
        if (g != 0.0) m4axpy(Ts, g, m4mul(m4mul(CDAG4(a & 1), CDAG4(b & 1)), C4(c & 1)));
      }
      if (!m4nz(Ts)) continue;
      d.src.push_back({1.0, R_(os, {K_D, r, 0, 0}), Ts});
      d.src.push_back({-1.0, R_(os, {K_D, r, 0, 0}, true), m4t(Ts)});
    }
    Ref P = lp.make(DQ{-1, -1}, 0, [&](const Key& k) {
      return k.kind == K_DD ? I.g(u, dn, k.i, k.j) - I.g(u, dn, k.j, k.i) : 0.0; });
    if (P.where >= 0) {
      Mat4 op = m4mul(CDAG4(0), CDAG4(1));
      d.src.push_back({1.0, P, op});
      Ref PT = P;
      PT.trans = true;
      d.src.push_back({1.0, PT, m4t(op)});
    }
    for (int p : site) for (int r : site) {
      Ref Q = lp.make(mdq(r, 1) - mdq(p, 1), 0, [&](const Key& k) {
        return k.kind == K_BB ? I.g(p, k.i, r, k.j) - I.g(p, k.i, k.j, r) : 0.0; });
      if (Q.where >= 0) d.src.push_back({1.0, Q, m4mul(CDAG4(p & 1), C4(r & 1))});
    }
  }
  lp.run(s);
  ns.allocate(s, false);
  ChainPlan P;
  plan_projection(defs, ns, os, &lp.tmp, iso, false, P);
  Bases<double> b{};
  b.L[0] = b.L[1] = iso.dev.as<double>();
  b.R[0] = b.R[1] = iso.dev.as<double>();
  b.X[0] = os.dev.as<double>();
  b.X[1] = lp.tmp.dev.as<double>();
  b.out = ns.dev.as<double>();
  set_limits(b, iso.dev, iso.dev, os.dev, lp.tmp.dev, iso.dev, iso.dev);
  run_chain(P, b, s);
  return B;
}

// ------------------------------------------------------------------ the two-site terms
struct Term {
  double coef;
  Ref l;    // left-block operator (where 0: L store, 1: L temps)
  Mat16 mu; // middle-site operator
  Ref r;    // right-block operator (where 0: R store, 1: R temps)
};

// What the sweep steps after a build need (kept when the build is asked to
// keep its environment): the integrals, and the right blocks of every
// length with the isometries that grew them (the right part shrinks by one
// site per step of a left-to-right sweep).  Shared by every heff_blocks
// object of one sweep.
struct Env {
  Ints I;
  int nmode = 0;
  std::vector<Bond> rb;                       // rb[m]: bond table of the right block of m sites
  std::vector<std::shared_ptr<Block>> right;  // right[m]
  std::vector<std::shared_ptr<Iso>> riso;     // riso[m]: isometry of site N-m (m >= 1), old = &rb[m-1]
};

}  // namespace heff

// ====================================================================== public objects

struct heff_blocks {
  heff_ctx* ctx = nullptr;  // context that built it (not used after the build)
  int device = 0;
  hipStream_t stream = nullptr;
  int n_orb = 0, n_up = 0, n_dn = 0, k0 = 0;
  uint32_t prec_mask = 0;
  std::shared_ptr<heff::Block> L, R;
  std::shared_ptr<heff::Env> env;  // kept for sweeps (HEFF_KEEP_ENV), else null
  heff::DevBuf start;              // start vector made by the sweep step that built these blocks
  heff::LinPlan Ltmp, Rtmp;
  std::vector<heff::Term> terms;
  // two-site layout
  std::vector<int32_t> blk_desc;
  std::vector<int64_t> blk_off;
  std::vector<int> blk_qa, blk_qb;
  std::map<std::array<int, 3>, int> blk_index;  // (qa index, s_k, s_k1) -> block
  int64_t n_elem = 0;
  // product task table
  heff::DevBuf d_tiles, d_tasks, d_dtiles, d_dtasks;
  heff::DevWorkSet mwork;  // matrix-core work lists
  std::vector<heff::Tile> h_tiles;  // host copies (shards, batches)
  std::vector<heff::Task> h_tasks;
  // when the product splits wide output blocks: the table with one tile
  // per output block (the operand gradients use it) and each product
  // tile's output block (empty: the tables coincide)
  std::vector<heff::Tile> blk_tiles;
  std::vector<heff::Task> blk_tasks;
  std::vector<int> tile_blk;
  int64_t n_tiles = 0, n_tasks = 0, n_dtasks = 0;
  // ranks of the output-block shard the product is restricted to (1: the
  // full product); while > 1 the calls that need every output element
  // (energies, gradients, Davidson) refuse with HEFF_ESTATE
  int32_t shard_nranks = 1;
  double flops = 0.0, bytes[3] = {0, 0, 0};
  double vflops[heff::kNumVariants] = {0, 0, 0, 0};  // algorithmic flops per kernel variant
  double vissued[heff::kNumVariants] = {0, 0, 0, 0};  // matrix-instruction flops of the FP64/FP32 kernel
  int64_t vsteps[heff::kNumVariants] = {0, 0, 0, 0};  // pipeline steps summed over work-groups
  int64_t vmaxsteps[heff::kNumVariants] = {0, 0, 0, 0};  // pipeline steps of the longest work-group
  // FP32 operand copies (FP32 and split-bf16 products): [L store, L temps,
  // R store, R temps]
  heff::DevBuf f32[4];
  // backward: task tables of the operand gradients (0: left, 1: right
  // operator arenas), built on first use; scratch of heff_energy
  struct GradPlan {
    heff::DevBuf tiles, tasks;
    heff::DevWorkSet work;
    bool ready = false;
  };
  mutable GradPlan grad[2];
  mutable heff::DevBuf escratch;
};

namespace heff {

static Mat16 mid_c(int m, bool dag, int k0) {
  int sp = m & 1;
  Mat4 op = dag ? CDAG4(sp) : C4(sp);
  Mat4 F = m4zero();
  F[0] = 1; F[5] = -1; F[10] = -1; F[15] = 1;
  if ((m >> 1) == k0) return kron44(op, m4eye());
  return kron44(F, op);
}

static void add_term(std::vector<Term>& T, double c, Ref l, const Mat16& mu, Ref r, bool hc,
                     const Store& Ls, const Store& Lt, const Store& Rs, const Store& Rt) {
  if (c == 0.0 || !m16nz(mu)) return;
  T.push_back({c, l, mu, r});
  if (hc) {
    int pl = l.where < 0 ? 0 : (l.where == 0 ? Ls : Lt).parity(l.id);
    int pr = r.where < 0 ? 0 : (r.where == 0 ? Rs : Rt).parity(r.id);
    int pm = par16(mu);
    int sgn = ((pl * pm + pl * pr + pm * pr) & 1) ? -1 : 1;
    Ref l2 = l, r2 = r;
    if (l2.where >= 0) l2.trans = !l2.trans;
    if (r2.where >= 0) r2.trans = !r2.trans;
    T.push_back({c * sgn, l2, m16t(mu), r2});
  }
}

static void build_terms(heff_blocks& B, const Ints& I) {
  Store& Ls = B.L->store;
  Store& Rs = B.R->store;
  LinPlan& lt = B.Ltmp;
  LinPlan& rt = B.Rtmp;
  lt.main = &Ls;
  lt.tmp.bond = &B.L->bond;
  rt.main = &Rs;
  rt.tmp.bond = &B.R->bond;
  const int k0 = B.k0;
  const int nmode = 2 * B.n_orb;
  std::vector<int> Lm, M, Rm, X;
  for (int m = 0; m < 2 * k0; ++m) Lm.push_back(m);
  for (int m = 2 * k0; m < 2 * k0 + 4; ++m) M.push_back(m);
  for (int m = 2 * k0 + 4; m < nmode; ++m) Rm.push_back(m);
  X = Lm;
  X.insert(X.end(), M.begin(), M.end());
  std::map<int, Mat16> cd, cc;
  for (int m : M) { cd[m] = mid_c(m, true, k0); cc[m] = mid_c(m, false, k0); }
  const Mat16 I16 = m16eye();
  std::vector<Term>& T = B.terms;
  auto add = [&](double c, Ref l, const Mat16& mu, Ref r, bool hc) {
    add_term(T, c, l, mu, r, hc, Ls, lt.tmp, Rs, rt.tmp);
  };
  auto isL = [&](int m) { return m < 2 * k0; };
  // --- all lincombs first (temps must be created before the stores run)
  std::map<std::pair<int, int>, Ref> PL, QL, U, W;
  std::map<std::array<int, 3>, Ref> Y, Z;
  std::map<std::pair<int, int>, Ref> P, Q;
  for (size_t i = 0; i < M.size(); ++i) for (size_t k = i + 1; k < M.size(); ++k) {
    int r = M[i], s = M[k];
    PL[{r, s}] = lt.make(mdq(r, 1) + mdq(s, 1), 0, [&](const Key& key) {
      return key.kind == K_A ? I.g(key.i, key.j, r, s) - I.g(key.i, key.j, s, r) : 0.0; });
  }
  for (int q : M) for (int s : M)
    QL[{q, s}] = lt.make(mdq(s, 1) - mdq(q, 1), 0, [&](const Key& key) {
      return key.kind == K_B ? I.g(key.i, q, key.j, s) - I.g(key.i, q, s, key.j) : 0.0; });
  for (int r : Rm) {
    DQ dqr = mdq(r, 1);
    for (int m : M) {
      U[{r, m}] = lt.make(dqr - mdq(m, -1), 0, [&](const Key& key) {
        return key.kind == K_A ? I.g(key.i, key.j, r, m) - I.g(key.j, key.i, r, m) : 0.0; });
      W[{r, m}] = lt.make(dqr - mdq(m, 1), 0, [&](const Key& key) {
        return key.kind == K_B ? I.g(m, key.i, r, key.j) - I.g(key.i, m, r, key.j) : 0.0; });
    }
    for (int m : M) for (int n : M) {
      Y[{r, m, n}] = lt.make(dqr - mdq(m, 1) - mdq(n, -1), 1, [&](const Key& key) {
        return key.kind == K_C ? I.g(key.i, m, r, n) - I.g(m, key.i, r, n) : 0.0; });
      if (m != n) {
        Ref z = lt.make(-(dqr - mdq(m, 1) - mdq(n, 1)), 1, [&](const Key& key) {
          return key.kind == K_C ? I.g(m, n, r, key.i) : 0.0; });
        if (z.where >= 0) z.trans = true;
        Z[{r, m, n}] = z;
      }
    }
  }
  for (size_t i = 0; i < X.size(); ++i) for (size_t k = i + 1; k < X.size(); ++k) {
    int a = X[i], b = X[k];
    P[{a, b}] = rt.make(-(mdq(a, 1) + mdq(b, 1)), 0, [&](const Key& key) {
      return key.kind == K_DD ? I.g(a, b, key.i, key.j) - I.g(a, b, key.j, key.i) : 0.0; });
  }
  for (int a : X) for (int b : X)
    Q[{a, b}] = rt.make(mdq(b, 1) - mdq(a, 1), 0, [&](const Key& key) {
      return key.kind == K_BB ? I.g(a, key.i, b, key.j) - I.g(a, key.i, key.j, b) : 0.0; });

  // --- H^X (x) I_R with X = L + M
  add(1.0, R_(Ls, {K_H, 0, 0, 0}), I16, RI(), false);
  Mat16 HM = m16zero();
  for (int a : M) for (int b : M) if (I.t(a, b) != 0.0) m16axpy(HM, I.t(a, b), m16mul(cd[a], cc[b]));
  for (int a : M) for (int b : M) for (int c : M) for (int d : M) {
    double g = I.g(a, b, c, d);
    if (g != 0.0) m16axpy(HM, 0.5 * g, m16mul(m16mul(cd[a], cd[b]), m16mul(cc[d], cc[c])));
  }
  add(1.0, RI(), HM, RI(), false);
  for (int p : Lm) {
    Mat16 S = m16zero();
    for (int q : M) if (I.t(p, q) != 0.0) m16axpy(S, I.t(p, q), cc[q]);
    for (int q : M) for (int r : M) for (int s : M) {
      double g = I.g(p, q, r, s);
      if (g != 0.0) m16axpy(S, g, m16mul(m16mul(cd[q], cc[s]), cc[r]));
    }
    add(1.0, R_(Ls, {K_C, p, 0, 0}), S, RI(), true);
  }
  for (int m : M) add(1.0, R_(Ls, {K_T, m, 0, 0}), cc[m], RI(), true);
  for (auto& kv : PL) if (kv.second.where >= 0)
    add(1.0, kv.second, m16mul(cc[kv.first.second], cc[kv.first.first]), RI(), true);
  for (auto& kv : QL) if (kv.second.where >= 0)
    add(1.0, kv.second, m16mul(cd[kv.first.first], cc[kv.first.second]), RI(), false);
  // --- I (x) I (x) H^R
  add(1.0, RI(), I16, R_(Rs, {K_H, 0, 0, 0}), false);
  // --- sum_{p in X} a+_p S^R_p + h.c.
  for (int p : Lm) add(1.0, R_(Ls, {K_C, p, 0, 0}), I16, R_(Rs, {K_S, p, 0, 0}), true);
  for (int m : M) add(1.0, RI(), cd[m], R_(Rs, {K_S, m, 0, 0}), true);
  // --- sum_{r in R} T^X_r a_r + h.c.
  for (int r : Rm) {
    Ref rho = R_(Rs, {K_D, r, 0, 0});
    add(1.0, R_(Ls, {K_T, r, 0, 0}), I16, rho, true);
    for (int m : M) {
      if (U[{r, m}].where >= 0) add(1.0, U[{r, m}], cc[m], rho, true);
      if (W[{r, m}].where >= 0) add(1.0, W[{r, m}], cd[m], rho, true);
    }
    for (int m : M) for (int n : M) {
      if (Y[{r, m, n}].where >= 0) add(1.0, Y[{r, m, n}], m16mul(cd[m], cc[n]), rho, true);
      if (m != n && Z[{r, m, n}].where >= 0) add(1.0, Z[{r, m, n}], m16mul(cd[m], cd[n]), rho, true);
    }
    Mat16 tau = m16zero();
    for (int a : M) for (int b : M) for (int d : M) {
      double g = I.g(a, b, r, d);
      if (g != 0.0) m16axpy(tau, g, m16mul(m16mul(cd[a], cd[b]), cc[d]));
    }
    add(1.0, RI(), tau, rho, true);
  }
  // --- sum_{p<q in X} A^X_pq P^R_pq + h.c.
  for (size_t i = 0; i < X.size(); ++i) for (size_t k = i + 1; k < X.size(); ++k) {
    int a = X[i], b = X[k];
    Ref Pr = P[{a, b}];
    if (Pr.where < 0) continue;
    if (isL(a) && isL(b)) add(1.0, R_(Ls, {K_A, a, b, 0}), I16, Pr, true);
    else if (isL(a)) add(1.0, R_(Ls, {K_C, a, 0, 0}), cd[b], Pr, true);
    else add(1.0, RI(), m16mul(cd[a], cd[b]), Pr, true);
  }
  // --- sum_{p,r in X} B^X_pr Q^R_pr
  for (int a : X) for (int b : X) {
    Ref Qr = Q[{a, b}];
    if (Qr.where < 0) continue;
    if (isL(a) && isL(b)) add(1.0, R_(Ls, {K_B, a, b, 0}), I16, Qr, false);
    else if (isL(a)) add(1.0, R_(Ls, {K_C, a, 0, 0}), cc[b], Qr, false);
    else if (isL(b)) add(-1.0, R_(Ls, {K_C, b, 0, 0}, true), cd[a], Qr, false);
    else add(1.0, RI(), m16mul(cd[a], cc[b]), Qr, false);
  }
}

// ------------------------------------------------------------------ product tasks
static void build_psi_layout(heff_blocks& B) {
  const Bond& bl = B.L->bond;
  const Bond& br = B.R->bond;
  int64_t off = 0;
  for (int qa = 0; qa < bl.n(); ++qa)
    for (int sk = 0; sk < 4; ++sk)
      for (int sk1 = 0; sk1 < 4; ++sk1) {
        int u = B.n_up - bl.nu[qa] - SQU[sk] - SQU[sk1];
        int d = B.n_dn - bl.nd[qa] - SQD[sk] - SQD[sk1];
        int qb = br.find(u, d);
        if (qb < 0) continue;
        int idx = (int)B.blk_off.size();
        B.blk_index[{qa, sk, sk1}] = idx;
        B.blk_desc.insert(B.blk_desc.end(), {bl.nu[qa], bl.nd[qa], sk, sk1, bl.dim[qa], br.dim[qb]});
        B.blk_off.push_back(off);
        B.blk_qa.push_back(qa);
        B.blk_qb.push_back(qb);
        off += (int64_t)bl.dim[qa] * br.dim[qb];
      }
  B.n_elem = off;
  if (B.blk_off.empty()) throw Error(HEFF_ESECTOR, "no two-site block in the target sector");
}

double task_flops(const Task& t) {
  double a = t.a, b = t.b, c = t.c, e = t.e;
  bool idl = t.flags & T_IDL, idr = t.flags & T_IDR;
  if (idl && idr) return 2.0 * a * e;
  if (idl) return 2.0 * a * c * e;
  if (idr) return 2.0 * a * b * c;
  return std::min(2 * a * b * c + 2 * a * c * e, 2 * b * c * e + 2 * a * b * e);
}

static void build_tasks(heff_blocks& B, hipStream_t s) {
  const Bond& bl = B.L->bond;
  const Bond& br = B.R->bond;
  for (int d : bl.dim)
    if (d > kMaxDim) throw Error(HEFF_EINVAL, "middle-bond sector dimension above " + std::to_string(kMaxDim));
  for (int d : br.dim)
    if (d > kMaxDim) throw Error(HEFF_EINVAL, "middle-bond sector dimension above " + std::to_string(kMaxDim));
  const Store& Ls = B.L->store;
  const Store& Lt = B.Ltmp.tmp;
  const Store& Rs = B.R->store;
  const Store& Rt = B.Rtmp.tmp;
  const int nb = (int)B.blk_off.size();
  std::vector<std::vector<Task>> per(nb);
  std::vector<std::vector<DiagTask>> dper(nb);
  // referenced operator blocks: store (0, 1 left store and temporaries; 2,
  // 3 right) in the top bits, element offset below
  std::unordered_set<uint64_t> seen;
  seen.reserve(1u << 16);
  auto first_use = [&](int store, int64_t off) { return seen.insert(((uint64_t)store << 60) | (uint64_t)off).second; };
  double op_elems = 0.0;
  for (const Term& tm : B.terms) {
    const Store* lst = tm.l.where < 0 ? nullptr : (tm.l.where == 0 ? &Ls : &Lt);
    const Store* rst = tm.r.where < 0 ? nullptr : (tm.r.where == 0 ? &Rs : &Rt);
    int pm = par16(tm.mu);
    int pr = rst ? rst->parity(tm.r.id) : 0;
    for (int x = 0; x < nb; ++x) {
      int qa = B.blk_qa[x], qb = B.blk_qb[x];
      int sk = B.blk_desc[6 * x + 2], sk1 = B.blk_desc[6 * x + 3];
      int mid = 4 * sk + sk1;
      // left block
      int qa2 = qa, lblk = -1;
      if (lst) {
        const Layout& LL = lst->lay(tm.l.id);
        if (!tm.l.trans) { lblk = LL.blk_in[qa]; if (lblk < 0) continue; qa2 = LL.qout[lblk]; }
        else { lblk = LL.blk_out[qa]; if (lblk < 0) continue; qa2 = LL.qin[lblk]; }
      }
      int qb2 = qb, rblk = -1;
      if (rst) {
        const Layout& RL = rst->lay(tm.r.id);
        if (!tm.r.trans) { rblk = RL.blk_in[qb]; if (rblk < 0) continue; qb2 = RL.qout[rblk]; }
        else { rblk = RL.blk_out[qb]; if (rblk < 0) continue; qb2 = RL.qin[rblk]; }
      }
      int nl = bl.par(qa), nmid = mid_n(mid) & 1;
      int sgn = ((pm * nl + pr * (nl + nmid)) & 1) ? -1 : 1;
      for (int mid2 = 0; mid2 < 16; ++mid2) {
        double w = tm.mu[mid2 * 16 + mid];
        if (w == 0.0) continue;
        auto it = B.blk_index.find({qa2, mid2 >> 2, mid2 & 3});
        if (it == B.blk_index.end()) continue;
        int y = it->second;
        if (B.blk_qb[y] != qb2) throw Error(HEFF_EINVAL, "internal: term violates sector conservation");
        Task t{};
        t.f = tm.coef * w * sgn;
        t.a = (uint16_t)bl.dim[qa2];
        t.b = (uint16_t)bl.dim[qa];
        t.c = (uint16_t)br.dim[qb];
        t.e = (uint16_t)br.dim[qb2];
        t.offX = B.blk_off[x];
        t.ldX = (uint16_t)br.dim[qb];
        uint32_t fl = 0;
        if (!lst) fl |= T_IDL;
        else {
          t.offL = lst->offset(tm.l.id) + lst->lay(tm.l.id).off[lblk];
          t.ldL = (uint16_t)lst->lay(tm.l.id).cols[lblk];
          if (tm.l.trans) fl |= T_TL;
          if (tm.l.where == 1) fl |= T_SELL;
          if (first_use(tm.l.where, t.offL)) op_elems += (double)t.a * t.b;
        }
        if (!rst) fl |= T_IDR;
        else {
          t.offR = rst->offset(tm.r.id) + rst->lay(tm.r.id).off[rblk];
          t.ldR = (uint16_t)rst->lay(tm.r.id).cols[rblk];
          if (!tm.r.trans) fl |= T_TR;
          if (tm.r.where == 1) fl |= T_SELR;
          if (first_use(2 + tm.r.where, t.offR)) op_elems += (double)t.c * t.e;
        }
        t.flags = (uint16_t)fl;
        per[y].push_back(t);
        B.flops += task_flops(t);
        if (mid2 == mid && qa2 == qa && qb2 == qb) {
          DiagTask dt{};
          dt.f = t.f;
          dt.flags = fl & (T_IDL | T_IDR | T_SELL | T_SELR);
          dt.offL = t.offL;
          dt.offR = t.offR;
          dper[y].push_back(dt);
        }
      }
    }
  }
  std::vector<Tile> tiles(nb), dtiles(nb);
  std::vector<Task> tasks;
  std::vector<DiagTask> dtasks;
  for (int y = 0; y < nb; ++y) {
    Tile t{};
    t.offOut = B.blk_off[y];
    t.a = B.blk_desc[6 * y + 4];
    t.e = B.blk_desc[6 * y + 5];
    t.ldOut = t.e;
    t.t0 = (int32_t)tasks.size();
    tasks.insert(tasks.end(), per[y].begin(), per[y].end());
    t.t1 = (int32_t)tasks.size();
    tiles[y] = t;
    Tile d = t;
    d.t0 = (int32_t)dtasks.size();
    dtasks.insert(dtasks.end(), dper[y].begin(), dper[y].end());
    d.t1 = (int32_t)dtasks.size();
    dtiles[y] = d;
  }
  // The product runs output blocks and middle dimensions of at most 128
  // columns (column slices, ranges of c), so it never needs the 256-wide
  // kernel instances, which hold one work-group per CU and spill (N=40,
  // D=4096, beta=1, blocks up to 229 wide: FP64 1406 -> 924 ms, FP32 699 ->
  // 464 ms, bf16 split 670 -> 372 ms on one box).  The operand gradients
  // take every output block whole: they keep the unsplit table.
  B.n_tasks = (int64_t)tasks.size();
  bool wide_any = false;
  for (const Tile& t : tiles) wide_any |= t.e > kProductDim;
  for (const Task& k : tasks) wide_any |= k.c > kProductDim;
  if (wide_any) {
    B.blk_tiles = tiles;
    B.blk_tasks = tasks;
    split_large(tiles, tasks, kProductDim, &B.tile_blk);
  }
  const int nt_ = (int)tiles.size();
  // largest output blocks first (longest work items start early)
  std::vector<int> order(nt_);
  for (int i = 0; i < nt_; ++i) order[i] = i;
  std::vector<double> rowfl(nt_, 0.0);
  for (int y = 0; y < nt_; ++y)
    for (int k = tiles[y].t0; k < tiles[y].t1; ++k) rowfl[y] += task_flops(tasks[k]) / std::max(1, tiles[y].a);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return rowfl[a] > rowfl[b]; });
  std::vector<Work> lists[kNumVariants];
  split_work(tiles, tasks, order, lists);
  B.mwork.upload_lists(lists, s);
  const bool wide = has_wide(tiles, tasks);
  // algorithmic flops per variant: an output block's unsplit tasks, counted
  // with its first slice (the slices of a block run in one variant: a split
  // product has wide tiles, so every tile runs on the 128-wide kernel)
  std::vector<double> blk_fl(B.tile_blk.empty() ? 0 : B.blk_tiles.size(), 0.0);
  for (size_t y = 0; y < blk_fl.size(); ++y)
    for (int k = B.blk_tiles[y].t0; k < B.blk_tiles[y].t1; ++k) blk_fl[y] += task_flops(B.blk_tasks[k]);
  for (int y = 0; y < nt_; ++y) {
    double fl = 0.0;
    if (B.tile_blk.empty()) {
      for (int k = tiles[y].t0; k < tiles[y].t1; ++k) fl += task_flops(tasks[k]);
    } else if (y == 0 || B.tile_blk[y] != B.tile_blk[y - 1]) {
      fl = blk_fl[B.tile_blk[y]];
    }
    const int v = launch_variant(tiles[y], tasks, wide);
    B.vflops[v] += fl;
    // what the FP64/FP32 kernel issues: per active 16-row wave, 4 ceil(c/16)
    // MFMAs per stage-1 step (ceil(b/16) steps) and 4 ceil(e/16) per stage-2
    // step (ceil(c/16) steps); every 64-row work-group takes every step
    const int64_t waves = (tiles[y].a + 15) / 16, groups = (tiles[y].a + kTileRows - 1) / kTileRows;
    const int64_t ne = (tiles[y].e + 15) / 16;
    int64_t item_steps = 0;
    for (int k = tiles[y].t0; k < tiles[y].t1; ++k) {
      const int64_t nb = (tasks[k].b + 15) / 16, nc = (tasks[k].c + 15) / 16;
      B.vissued[v] += 2048.0 * 4.0 * (double)waves * (double)(nb * nc + nc * ne);
      item_steps += nb + nc;
    }
    B.vsteps[v] += groups * item_steps;
    B.vmaxsteps[v] = std::max(B.vmaxsteps[v], item_steps);
  }
  if (tasks.size() > (size_t)INT32_MAX) throw Error(HEFF_EINVAL, "task table too large");
  B.n_tiles = nb;
  B.n_dtasks = (int64_t)dtasks.size();
  double psi_elems = (double)B.n_elem;
  B.bytes[0] = 8.0 * (op_elems + 2 * psi_elems);
  B.bytes[1] = 4.0 * (op_elems + 2 * psi_elems);
  B.bytes[2] = 4.0 * op_elems + 4.0 * 2 * psi_elems;
  upload(B.d_tiles, tiles, s);
  upload(B.d_tasks, tasks, s);
  B.h_tiles = tiles;
  B.h_tasks = tasks;
  upload(B.d_dtiles, dtiles, s);
  upload(B.d_dtasks, dtasks, s);
  HCHECK(hipStreamSynchronize(s));
}

static void validate_ints(const heff_problem* p, Ints& I) {
  int n = p->n_orb;
  I.n = n;
  I.h.assign(p->h, p->h + (size_t)n * n);
  I.V.assign(p->V, p->V + (size_t)n * n * n * n);
  double hs = 0, vs = 0;
  for (double v : I.h) hs = std::max(hs, std::fabs(v));
  for (double v : I.V) vs = std::max(vs, std::fabs(v));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (std::fabs(I.h[i * n + j] - I.h[j * n + i]) > 1e-12 * std::max(1.0, hs))
        throw Error(HEFF_EINVAL, "h is not symmetric");
  auto v = [&](int i, int j, int k, int l) { return I.V[(((size_t)i * n + j) * n + k) * n + l]; };
  double tol = 1e-12 * std::max(1.0, vs);
  for (int i = 0; i < n; ++i) for (int j = 0; j < n; ++j) for (int k = 0; k < n; ++k) for (int l = 0; l < n; ++l) {
    double a = v(i, j, k, l);
    if (std::fabs(a - v(j, i, k, l)) > tol || std::fabs(a - v(i, j, l, k)) > tol || std::fabs(a - v(k, l, i, j)) > tol)
      throw Error(HEFF_EINVAL, "V lacks the 8-fold (ij|kl) symmetry");
  }
}

// Largest |(M^T M - I)_ij| of an r x d row-major matrix (rank-one updates
// row by row over the upper triangle).
static double gram_defect(const double* M, int64_t r, int d) {
  std::vector<double> G((size_t)d * d, 0.0);
  for (int64_t i = 0; i < r; ++i) {
    const double* row = M + i * d;
    for (int a = 0; a < d; ++a) {
      const double x = row[a];
      if (x == 0.0) continue;
      double* g = G.data() + (size_t)a * d;
      for (int b = a; b < d; ++b) g[b] += x * row[b];
    }
  }
  double worst = 0.0;
  for (int a = 0; a < d; ++a)
    for (int b = a; b < d; ++b) worst = std::max(worst, std::fabs(G[(size_t)a * d + b] - (a == b ? 1.0 : 0.0)));
  return worst;
}

// Every check heff_build_blocks makes before it touches the device: sizes,
// symmetric integrals, sorted bond tables with the empty blocks' single
// sector, isometry shapes (no more kept than reachable states), orthonormal
// isometry columns (the whole Gram matrix of every out-sector block, 1e-10)
// and a non-empty target sector.  Host only.
static void validate_problem(const heff_problem* p, Ints* ints) {
  if (!p || !p->h || !p->V || !p->left || !p->right || !p->iso_left || !p->iso_right)
    throw Error(HEFF_EINVAL, "null argument");
  const int n = p->n_orb;
  if (n < 4 || n > 64) throw Error(HEFF_EINVAL, "n_orb must be in [4, 64]");
  if (p->n_up < 0 || p->n_dn < 0 || p->n_up > n || p->n_dn > n) throw Error(HEFF_EINVAL, "bad electron numbers");
  Ints local;
  Ints& I = ints ? *ints : local;
  validate_ints(p, I);
  const int k0 = n / 2 - 1, mR = n - k0 - 2;
  std::vector<Bond> lb, rb;
  for (int l = 0; l <= k0; ++l) lb.push_back(make_bond(p->left[l], "left bond table"));
  for (int m = 0; m <= mR; ++m) rb.push_back(make_bond(p->right[m], "right bond table"));
  if (lb[0].n() != 1 || lb[0].nu[0] != 0 || lb[0].nd[0] != 0 || lb[0].dim[0] != 1 ||
      rb[0].n() != 1 || rb[0].nu[0] != 0 || rb[0].nd[0] != 0 || rb[0].dim[0] != 1)
    throw Error(HEFF_EINVAL, "empty blocks must have the single sector (0,0) of dimension 1");
  // isometry blocks: (host pointer, rows, kept columns, description)
  struct Job { const double* M; int64_t r; int d; int site; bool left; };
  std::vector<Job> jobs;
  auto shapes = [&](const Bond& old, const Bond& nw, const double* host, int site, bool left) {
    if (!host) throw Error(HEFF_EINVAL, left ? "null left isometry" : "null right isometry");
    int64_t off = 0;
    for (int q = 0; q < nw.n(); ++q) {
      int64_t r = 0;
      for (int st = 0; st < 4; ++st) {
        int qi = old.find(nw.nu[q] - SQU[st], nw.nd[q] - SQD[st]);
        if (qi >= 0) r += old.dim[qi];
      }
      if (r < nw.dim[q])
        throw Error(HEFF_EINVAL, std::string(left ? "left" : "right") + " isometry of site " + std::to_string(site) +
                                     ": more kept states than reachable states");
      jobs.push_back({host + off, r, nw.dim[q], site, left});
      off += r * (int64_t)nw.dim[q];
    }
  };
  for (int l = 0; l < k0; ++l) shapes(lb[l], lb[l + 1], p->iso_left[l], l, true);
  for (int m = 1; m <= mR; ++m) shapes(rb[m - 1], rb[m], p->iso_right[m - 1], n - m, false);
  // Gram matrices, spread over host threads (largest blocks first)
  std::vector<size_t> order(jobs.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
    return (double)jobs[a].r * jobs[a].d * jobs[a].d > (double)jobs[b].r * jobs[b].d * jobs[b].d;
  });
  std::vector<double> defect(jobs.size(), 0.0);
  std::atomic<size_t> next{0};
  auto worker = [&]() {
    for (size_t i; (i = next.fetch_add(1)) < order.size();) {
      const Job& j = jobs[order[i]];
      defect[order[i]] = gram_defect(j.M, j.r, j.d);
    }
  };
  const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (unsigned t = 1; t < nth; ++t) pool.emplace_back(worker);
  worker();
  for (auto& t : pool) t.join();
  for (size_t i = 0; i < jobs.size(); ++i)
    if (!(defect[i] <= 1e-10))
      throw Error(HEFF_EINVAL, std::string(jobs[i].left ? "left" : "right") + " isometry of site " +
                                   std::to_string(jobs[i].site) + ": columns not orthonormal (|M^T M - I| = " +
                                   std::to_string(defect[i]) + ")");
  // the target sector must meet at least one two-site block
  const Bond& bl = lb[k0];
  const Bond& br = rb[mR];
  bool any = false;
  for (int qa = 0; qa < bl.n() && !any; ++qa)
    for (int sk = 0; sk < 4 && !any; ++sk)
      for (int sk1 = 0; sk1 < 4 && !any; ++sk1)
        any = br.find(p->n_up - bl.nu[qa] - SQU[sk] - SQU[sk1], p->n_dn - bl.nd[qa] - SQD[sk] - SQD[sk1]) >= 0;
  if (!any) throw Error(HEFF_ESECTOR, "no two-site block in the target sector");
}

}  // namespace heff

// ====================================================================== C ABI
using namespace heff;

extern "C" int heff_validate_problem(const heff_problem* prob, char* msg, int32_t msg_len) {
  try {
    validate_problem(prob, nullptr);
  } catch (const Error& e) {
    if (msg && msg_len > 0) std::snprintf(msg, (size_t)msg_len, "%s", e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    if (msg && msg_len > 0) std::snprintf(msg, (size_t)msg_len, "host allocation failed");
    return HEFF_ENOMEM;
  }
  if (msg && msg_len > 0) msg[0] = 0;
  return HEFF_OK;
}

namespace heff {
// Streams of the product's kernel variants, forked from the context stream
// (so the variants run concurrently: the small-block variants are bound by
// their longest work item and fill the chip while the large one runs) and
// joined back into it.  All default priority.
static hipError_t make_variant_streams(heff_ctx* c) {
  if (c->fork) return hipSuccess;
  hipError_t e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
  for (int v = 0; v < kNumVariants && e == hipSuccess; ++v) {
    e = hipStreamCreateWithFlags(&c->vs[v], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join[v], hipEventDisableTiming);
  }
  return e;
}
void fork_variants(heff_ctx* c, hipStream_t out[kNumVariants]) {
  HCHECK(make_variant_streams(c));
  HCHECK(hipEventRecord(c->fork, c->stream));
  for (int v = 0; v < kNumVariants; ++v) {
    HCHECK(hipStreamWaitEvent(c->vs[v], c->fork, 0));
    out[v] = c->vs[v];
  }
}
void join_variants(heff_ctx* c) {
  for (int v = 0; v < kNumVariants; ++v) {
    HCHECK(hipEventRecord(c->join[v], c->vs[v]));
    HCHECK(hipStreamWaitEvent(c->stream, c->join[v], 0));
  }
}
}  // namespace heff

extern "C" int heff_create(heff_ctx** out, int device, void* stream, const heff_alloc* alloc) {
  if (!out) return HEFF_EINVAL;
  *out = nullptr;
  if (alloc && (!alloc->alloc || !alloc->free)) return HEFF_EINVAL;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return HEFF_EHIP;
  if (hipSetDevice(device) != hipSuccess) return HEFF_EHIP;
  heff_ctx* c = new (std::nothrow) heff_ctx;
  if (!c) return HEFF_ENOMEM;
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  if (alloc) c->alloc = Alloc{alloc->alloc, alloc->free, alloc->user};
  // the product's variant streams exist from here on (no product call
  // creates runtime objects); the allocation-free energy's scratch address
  // on this device is recorded
  if (make_variant_streams(c) != hipSuccess || noalloc_setup(device) != hipSuccess) {
    heff_destroy(c);
    return HEFF_EHIP;
  }
  *out = c;
  return HEFF_OK;
}

extern "C" int heff_destroy(heff_ctx* c) {
  if (c) {
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (int v = 0; v < kNumVariants; ++v) {
      if (c->vs[v]) (void)hipStreamSynchronize(c->vs[v]);
      for (hipEvent_t e : c->ev_start[v]) (void)hipEventDestroy(e);
      for (hipEvent_t e : c->ev_stop[v]) (void)hipEventDestroy(e);
      if (c->vs[v]) (void)hipStreamDestroy(c->vs[v]);
      if (c->join[v]) (void)hipEventDestroy(c->join[v]);
    }
    if (c->fork) (void)hipEventDestroy(c->fork);
  }
  delete c;
  return HEFF_OK;
}

extern "C" const char* heff_last_error(const heff_ctx* c) { return c ? c->err.c_str() : "null context"; }

extern "C" int heff_build_blocks(heff_ctx* ctx, const heff_problem* p, uint32_t prec_mask, heff_blocks** out) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!out) throw Error(HEFF_EINVAL, "null argument");
  *out = nullptr;
  if (prec_mask & ~((1u << HEFF_FP32) | (1u << HEFF_BF16X3) | 1u | HEFF_KEEP_ENV))
    throw Error(HEFF_EINVAL, "bad prec_mask");
  Ints I;
  validate_problem(p, &I);
  const int n = p->n_orb;
  HCHECK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  auto B = std::make_unique<heff_blocks>();
  B->ctx = ctx;
  B->device = ctx->device;
  B->stream = ctx->stream;
  B->n_orb = n;
  B->n_up = p->n_up;
  B->n_dn = p->n_dn;
  B->k0 = n / 2 - 1;
  B->prec_mask = prec_mask;
  const int k0 = B->k0, mR = n - k0 - 2, nmode = 2 * n;
  std::vector<Bond> lb, rb;
  for (int l = 0; l <= k0; ++l) lb.push_back(make_bond(p->left[l], "left bond table"));
  for (int m = 0; m <= mR; ++m) rb.push_back(make_bond(p->right[m], "right bond table"));
  if (lb[0].n() != 1 || lb[0].nu[0] != 0 || lb[0].nd[0] != 0 || lb[0].dim[0] != 1 ||
      rb[0].n() != 1 || rb[0].nu[0] != 0 || rb[0].nd[0] != 0 || rb[0].dim[0] != 1)
    throw Error(HEFF_EINVAL, "empty blocks must have the single sector (0,0) of dimension 1");
  // left block
  auto L = initial_block(true, nmode, s);
  for (int l = 0; l < k0; ++l) {
    if (!p->iso_left[l]) throw Error(HEFF_EINVAL, "null left isometry");
    Iso iso;
    make_iso(iso, lb[l], lb[l + 1], p->iso_left[l], s, "left isometry");
    L->bond = lb[l];  // (same table; keeps the pointer of the store valid)
    auto Ln = grow_left(*L, lb[l + 1], iso, l, nmode, I, s);
    L = std::move(Ln);
  }
  // right block; with HEFF_KEEP_ENV every length and its isometry stay
  std::shared_ptr<Env> env;
  if (prec_mask & HEFF_KEEP_ENV) {
    env = std::make_shared<Env>();
    env->I = I;
    env->nmode = nmode;
    env->rb = rb;
    env->right.resize(mR + 1);
    env->riso.resize(mR + 1);
  }
  const std::vector<Bond>& rbv = env ? env->rb : rb;
  std::shared_ptr<Block> R = initial_block(false, nmode, s);
  if (env) env->right[0] = R;
  for (int m = 1; m <= mR; ++m) {
    if (!p->iso_right[m - 1]) throw Error(HEFF_EINVAL, "null right isometry");
    auto iso = std::make_shared<Iso>();
    make_iso(*iso, rbv[m - 1], rbv[m], p->iso_right[m - 1], s, "right isometry");
    std::shared_ptr<Block> Rn = grow_right(*R, rbv[m], *iso, n - m, nmode, I, s);
    R = Rn;
    if (env) {
      env->right[m] = R;
      env->riso[m] = iso;
    }
  }
  B->env = env;
  B->L = std::move(L);
  B->R = R;
  build_psi_layout(*B);
  build_terms(*B, I);
  B->Ltmp.run(s);
  B->Rtmp.run(s);
  build_tasks(*B, s);
  // reduced-precision operand copies
  const double* srcs[4] = {B->L->store.dev.as<double>(), B->Ltmp.tmp.dev.as<double>(),
                           B->R->store.dev.as<double>(), B->Rtmp.tmp.dev.as<double>()};
  int64_t sizes[4] = {B->L->store.total, B->Ltmp.tmp.total, B->R->store.total, B->Rtmp.tmp.total};
  if (prec_mask & ((1u << HEFF_FP32) | (1u << HEFF_BF16X3))) {
    for (int i = 0; i < 4; ++i) {
      B->f32[i].alloc((size_t)std::max<int64_t>(sizes[i], 1) * sizeof(float));
      if (sizes[i]) HCHECK(launch_convert_f32(srcs[i], B->f32[i].as<float>(), sizes[i], s));
    }
  }
  HCHECK(hipStreamSynchronize(s));
  *out = B.release();
  ABI_END(ctx)
}

extern "C" int heff_blocks_free(heff_blocks* b) {
  if (!b) return HEFF_OK;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  delete b;
  return HEFF_OK;
}

extern "C" int heff_psi_layout(const heff_blocks* b, int64_t* n_elem, int32_t* n_blk, const int32_t** desc,
                               const int64_t** off) {
  if (!b) return HEFF_EINVAL;
  if (n_elem) *n_elem = b->n_elem;
  if (n_blk) *n_blk = (int32_t)b->blk_off.size();
  if (desc) *desc = b->blk_desc.data();
  if (off) *off = b->blk_off.data();
  return HEFF_OK;
}

extern "C" int heff_task_stats(const heff_blocks* b, int64_t* n_tasks, double* flops, double* bytes3) {
  if (!b) return HEFF_EINVAL;
  if (n_tasks) *n_tasks = b->n_tasks;
  if (flops) *flops = b->flops;
  if (bytes3) for (int i = 0; i < 3; ++i) bytes3[i] = b->bytes[i];
  return HEFF_OK;
}

// One GPU's share of the product when the output blocks are spread over
// nranks GPUs (Sec. II.D: the product is distributed over devices; here by
// output blocks, so no reduction is needed and each block keeps its own
// summation order).  Output blocks go, largest algorithmic work first, to
// the rank with the least work so far; the product's work lists are rebuilt
// from this rank's blocks in the same order and placement rules as the
// full product (nranks = 1 restores exactly the full lists).
extern "C" int heff_blocks_shard(heff_ctx* ctx, heff_blocks* b, int32_t rank, int32_t nranks, double* shard_flops) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!b || nranks < 1 || rank < 0 || rank >= nranks) throw Error(HEFF_EINVAL, "bad shard (rank, nranks)");
  HCHECK(hipSetDevice(ctx->device));
  const std::vector<Tile>& tiles = b->h_tiles;
  const std::vector<Task>& tasks = b->h_tasks;
  // owners per output block (a block split into column slices for the
  // product stays on one rank), weighed by its unsplit tasks
  const bool sliced = !b->blk_tiles.empty();
  const std::vector<Tile>& btiles = sliced ? b->blk_tiles : tiles;
  const std::vector<Task>& btasks = sliced ? b->blk_tasks : tasks;
  const int nblk = (int)btiles.size(), nt = (int)tiles.size();
  std::vector<double> fl(nblk, 0.0);
  for (int y = 0; y < nblk; ++y)
    for (int k = btiles[y].t0; k < btiles[y].t1; ++k) fl[y] += task_flops(btasks[k]);
  std::vector<int> byfl(nblk);
  for (int i = 0; i < nblk; ++i) byfl[i] = i;
  std::stable_sort(byfl.begin(), byfl.end(), [&](int x, int y) { return fl[x] > fl[y]; });
  std::vector<double> load(nranks, 0.0);
  std::vector<int> owner(nblk, 0);
  for (int y : byfl) {
    int r = 0;
    for (int j = 1; j < nranks; ++j)
      if (load[j] < load[r]) r = j;
    owner[y] = r;
    load[r] += fl[y];
  }
  // the full product's tile order (largest per-row work first), restricted
  std::vector<double> rowfl(nt, 0.0);
  for (int y = 0; y < nt; ++y)
    for (int k = tiles[y].t0; k < tiles[y].t1; ++k) rowfl[y] += task_flops(tasks[k]) / std::max(1, tiles[y].a);
  std::vector<int> order(nt);
  for (int i = 0; i < nt; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return rowfl[x] > rowfl[y]; });
  std::vector<int> mine;
  for (int y : order)
    if (owner[sliced ? b->tile_blk[y] : y] == rank) mine.push_back(y);
  std::vector<Work> lists[kNumVariants];
  split_work(tiles, tasks, mine, lists);
  HCHECK(hipStreamSynchronize(ctx->stream));  // no product still reads the old lists
  b->mwork.upload_lists(lists, ctx->stream);
  HCHECK(hipStreamSynchronize(ctx->stream));
  b->shard_nranks = nranks;
  if (shard_flops) *shard_flops = load[rank];
  ABI_END(ctx)
}

bool heff::blocks_sharded(const heff_blocks* b) { return b && b->shard_nranks > 1; }
int64_t heff::blocks_n_elem(const heff_blocks* b) { return b ? b->n_elem : 0; }

namespace heff {
void run_product(heff_ctx* ctx, const Tile* tl, const Task* tk, const WorkSet& ws, int prec, uint32_t prec_mask,
                 Bases<double> b64, Bases<float> b32, const void* psi, void* out) {
  hipEvent_t evbuf[kNumVariants][2] = {};
  hipEvent_t(*ev)[2] = nullptr;
  if (ctx->timing) {
    for (int v = 0; v < kNumVariants; ++v) {
      if (ws.n[v] <= 0) continue;
      HCHECK(hipEventCreate(&evbuf[v][0]));
      HCHECK(hipEventCreate(&evbuf[v][1]));
      ctx->ev_start[v].push_back(evbuf[v][0]);
      ctx->ev_stop[v].push_back(evbuf[v][1]);
    }
    ev = evbuf;
  }
  hipStream_t vs[kNumVariants];
  if (prec == HEFF_FP64) {
    b64.X[0] = b64.X[1] = static_cast<const double*>(psi);
    b64.out = static_cast<double*>(out);
    int mode = ctx->fp64_kernel;
    if (mode == kFp64RingDword) {  // no buffer lengths known: the ring kernel moves single dwords
      for (int i = 0; i < 6; ++i) b64.lim[i] = 0;
      mode = kFp64Ring;
    }
    fork_variants(ctx, vs);
    HCHECK(launch_mfma_f64(tl, ws, tk, b64, vs, ev, mode));
    join_variants(ctx);
  } else if (prec == HEFF_FP32 || prec == HEFF_BF16X3) {
    if (!(prec_mask & (1u << prec)))
      throw Error(HEFF_ENOTSUP, prec == HEFF_FP32 ? "FP32 operands were not built" : "BF16X3 operands were not built");
    b32.X[0] = b32.X[1] = static_cast<const float*>(psi);
    b32.out = static_cast<float*>(out);
    fork_variants(ctx, vs);
    if (prec == HEFF_FP32) HCHECK(launch_mfma_f32(tl, ws, tk, b32, vs, ev));
    else HCHECK(launch_bf16x3(tl, ws, tk, b32, vs, ev));
    join_variants(ctx);
  } else {
    throw Error(HEFF_EINVAL, "unknown precision");
  }
}
}  // namespace heff

extern "C" int heff_apply(heff_ctx* ctx, const heff_blocks* b, int prec, const void* psi, void* out) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!b || !psi || !out) throw Error(HEFF_EINVAL, "null argument");
  if (psi == out) throw Error(HEFF_EINVAL, "psi and out alias");
  HCHECK(hipSetDevice(ctx->device));
  Bases<double> b64{};
  b64.L[0] = b->L->store.dev.as<double>();
  b64.L[1] = b->Ltmp.tmp.dev.as<double>();
  b64.R[0] = b->R->store.dev.as<double>();
  b64.R[1] = b->Rtmp.tmp.dev.as<double>();
  set_limits(b64, b->L->store.dev, b->Ltmp.tmp.dev, b->n_elem, b->R->store.dev, b->Rtmp.tmp.dev);
  Bases<float> b32{};
  b32.L[0] = b->f32[0].as<float>();
  b32.L[1] = b->f32[1].as<float>();
  b32.R[0] = b->f32[2].as<float>();
  b32.R[1] = b->f32[3].as<float>();
  run_product(ctx, b->d_tiles.as<Tile>(), b->d_tasks.as<Task>(), b->mwork.ws, prec, b->prec_mask, b64, b32, psi, out);
  ABI_END(ctx)
}

static void drop_events(heff_ctx* c) {
  for (int v = 0; v < kNumVariants; ++v) {
    for (hipEvent_t e : c->ev_start[v]) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_stop[v]) (void)hipEventDestroy(e);
    c->ev_start[v].clear();
    c->ev_stop[v].clear();
  }
}

extern "C" int heff_timing(heff_ctx* ctx, int enable) {
  if (!ctx) return HEFF_EINVAL;
  (void)hipStreamSynchronize(ctx->stream);
  drop_events(ctx);
  ctx->timing = enable != 0;
  return HEFF_OK;
}

extern "C" int heff_timing_read(heff_ctx* ctx, double* ms, int64_t* launches) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  HCHECK(hipStreamSynchronize(ctx->stream));
  for (int v = 0; v < kNumVariants; ++v) {
    double tot = 0.0;
    for (size_t i = 0; i < ctx->ev_start[v].size(); ++i) {
      float t = 0.f;
      HCHECK(hipEventElapsedTime(&t, ctx->ev_start[v][i], ctx->ev_stop[v][i]));
      tot += t;
    }
    if (ms) ms[v] = tot;
    if (launches) launches[v] = (int64_t)ctx->ev_start[v].size();
  }
  drop_events(ctx);
  ABI_END(ctx)
}

extern "C" int heff_task_stats_variant(const heff_blocks* b, int v, double* flops, int64_t* work_items) {
  if (!b || v < 0 || v >= kNumVariants) return HEFF_EINVAL;
  if (flops) *flops = b->vflops[v];
  if (work_items) *work_items = b->mwork.ws.n[v];
  return HEFF_OK;
}

extern "C" int heff_task_stats_issued(const heff_blocks* b, int v, double* mfma_flops, int64_t* steps,
                                      int64_t* max_steps) {
  if (!b || v < 0 || v >= kNumVariants) return HEFF_EINVAL;
  if (mfma_flops) *mfma_flops = b->vissued[v];
  if (steps) *steps = b->vsteps[v];
  if (max_steps) *max_steps = b->vmaxsteps[v];
  return HEFF_OK;
}

extern "C" int heff_diag(heff_ctx* ctx, const heff_blocks* b, double* diag) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!b || !diag) throw Error(HEFF_EINVAL, "null argument");
  HCHECK(hipSetDevice(ctx->device));
  HCHECK(launch_diag(b->d_dtiles.as<Tile>(), b->n_tiles, b->d_dtasks.as<DiagTask>(),
                     b->L->store.dev.as<double>(), b->Ltmp.tmp.dev.as<double>(), b->R->store.dev.as<double>(),
                     b->Rtmp.tmp.dev.as<double>(), diag, ctx->stream));
  ABI_END(ctx)
}

// ---------------------------------------------------------------- batches of problems
// Many independent two-site problems in one persistent launch per kernel
// variant: the task tables are concatenated (Psi and output offsets shifted
// into one concatenated FP32 vector each, tile.prob selects the problem's
// operator stores), and the launch sequence is captured once in a HIP graph
// on an internal stream and replayed by every heff_batch_apply.
struct heff_batch {
  int device = 0;
  int n = 0;
  std::vector<int64_t> off;
  int64_t n_total = 0;
  double flops = 0.0;
  float* x = nullptr;  // caller-owned concatenated input / output
  float* y = nullptr;
  heff::DevBuf tiles, tasks, pb;
  heff::DevWorkSet work;
  int grid[heff::kNumVariants] = {0, 0, 0, 0};
  hipStream_t gs = nullptr;
  hipStream_t vs[heff::kNumVariants] = {};  // captured branches, one per variant
  hipEvent_t cfork = nullptr, cjoin[heff::kNumVariants] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~heff_batch() {
    if (gs) (void)hipStreamSynchronize(gs);
    drop_graph();
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    for (int v = 0; v < heff::kNumVariants; ++v) {
      if (vs[v]) (void)hipStreamDestroy(vs[v]);
      if (cjoin[v]) (void)hipEventDestroy(cjoin[v]);
    }
    if (cfork) (void)hipEventDestroy(cfork);
    if (gs) (void)hipStreamDestroy(gs);
  }
};

extern "C" int heff_batch_create(heff_ctx* ctx, const heff_blocks* const* probs, int32_t n, float* x_dev,
                                 float* y_dev, heff_batch** out) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!probs || !out || n <= 0 || !x_dev || !y_dev || x_dev == y_dev) throw Error(HEFF_EINVAL, "bad argument");
  *out = nullptr;
  HCHECK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  auto Bt = std::make_unique<heff_batch>();
  Bt->device = ctx->device;
  Bt->n = n;
  std::vector<Tile> tiles;
  std::vector<Task> tasks;
  std::vector<ProbBases<float>> pb(n);
  for (int i = 0; i < n; ++i) {
    const heff_blocks* b = probs[i];
    if (!b) throw Error(HEFF_EINVAL, "null problem");
    if (!(b->prec_mask & (1u << HEFF_FP32))) throw Error(HEFF_ENOTSUP, "batched problems need FP32 operands");
    Bt->off.push_back(Bt->n_total);
    const int64_t xo = Bt->n_total;
    const int32_t tb = (int32_t)tasks.size();
    for (Tile t : b->h_tiles) {
      t.offOut += xo;
      t.t0 += tb;
      t.t1 += tb;
      t.prob = i;
      tiles.push_back(t);
    }
    for (Task k : b->h_tasks) {
      k.offX += xo;
      tasks.push_back(k);
    }
    pb[i].L[0] = b->f32[0].as<float>();
    pb[i].L[1] = b->f32[1].as<float>();
    pb[i].R[0] = b->f32[2].as<float>();
    pb[i].R[1] = b->f32[3].as<float>();
    Bt->n_total += b->n_elem;
    Bt->flops += b->flops;
  }
  if (tasks.size() > (size_t)INT32_MAX) throw Error(HEFF_EINVAL, "batch task table too large");
  std::vector<double> cost(tiles.size(), 0.0);
  for (size_t t = 0; t < tiles.size(); ++t)
    for (int k = tiles[t].t0; k < tiles[t].t1; ++k) cost[t] += task_flops(tasks[k]) / std::max(1, tiles[t].a);
  std::vector<int> order(tiles.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<Work> lists[kNumVariants];
  split_work(tiles, tasks, order, lists);
  Bt->work.upload_lists(lists, s);
  upload(Bt->tiles, tiles, s);
  upload(Bt->tasks, tasks, s);
  upload(Bt->pb, pb, s);
  Bt->x = x_dev;
  Bt->y = y_dev;
  for (int v = 0; v < kNumVariants; ++v) Bt->grid[v] = (int)std::min<int64_t>(Bt->work.ws.n[v], 512);
  HCHECK(hipStreamCreateWithFlags(&Bt->gs, hipStreamNonBlocking));
  HCHECK(hipEventCreateWithFlags(&Bt->ev_in, hipEventDisableTiming));
  HCHECK(hipEventCreateWithFlags(&Bt->ev_out, hipEventDisableTiming));
  HCHECK(hipStreamSynchronize(s));
  *out = Bt.release();
  ABI_END(ctx)
}

extern "C" int heff_batch_layout(const heff_blocks* const* probs, int32_t n, int64_t* offsets, int64_t* n_total) {
  if (!probs || n <= 0) return HEFF_EINVAL;
  int64_t o = 0;
  for (int i = 0; i < n; ++i) {
    if (!probs[i]) return HEFF_EINVAL;
    if (offsets) offsets[i] = o;
    o += probs[i]->n_elem;
  }
  if (n_total) *n_total = o;
  return HEFF_OK;
}

extern "C" int heff_batch_io(const heff_batch* b, const int64_t** offsets, int64_t* n_total) {
  if (!b) return HEFF_EINVAL;
  if (offsets) *offsets = b->off.data();
  if (n_total) *n_total = b->n_total;
  return HEFF_OK;
}

extern "C" int heff_batch_set_grid(heff_batch* b, const int32_t* grid) {
  if (!b || !grid) return HEFF_EINVAL;
  for (int v = 0; v < kNumVariants; ++v) {
    if (grid[v] <= 0) return HEFF_EINVAL;
    b->grid[v] = (int)std::min<int64_t>(grid[v], std::max<int64_t>(b->work.ws.n[v], 1));
  }
  (void)hipStreamSynchronize(b->gs);
  b->drop_graph();
  return HEFF_OK;
}

extern "C" int heff_batch_stats(const heff_batch* b, double* flops, int32_t* grid, int64_t* work_items) {
  if (!b) return HEFF_EINVAL;
  if (flops) *flops = b->flops;
  for (int v = 0; v < kNumVariants; ++v) {
    if (grid) grid[v] = b->grid[v];
    if (work_items) work_items[v] = b->work.ws.n[v];
  }
  return HEFF_OK;
}

// y = H_eff x for every problem (FP32).  use_graph: 1 = capture on first use
// and replay, 0 = plain launches on the context stream.
extern "C" int heff_batch_apply(heff_ctx* ctx, heff_batch* b, int use_graph) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!b) throw Error(HEFF_EINVAL, "null batch");
  HCHECK(hipSetDevice(ctx->device));
  const Tile* tl = b->tiles.as<Tile>();
  const Task* tk = b->tasks.as<Task>();
  const ProbBases<float>* pb = b->pb.as<ProbBases<float>>();
  if (!use_graph) {
    hipStream_t vs[kNumVariants];
    fork_variants(ctx, vs);
    HCHECK(launch_mfma_batch_f32(tl, b->work.ws, tk, pb, b->x, b->y, b->grid, vs));
    join_variants(ctx);
  } else {
    if (!b->exec) {
      if (!b->cfork) {
        HCHECK(hipEventCreateWithFlags(&b->cfork, hipEventDisableTiming));
        for (int v = 0; v < kNumVariants; ++v) {
          HCHECK(hipStreamCreateWithFlags(&b->vs[v], hipStreamNonBlocking));
          HCHECK(hipEventCreateWithFlags(&b->cjoin[v], hipEventDisableTiming));
        }
      }
      // the variant launches form parallel branches of the captured graph
      HCHECK(hipStreamBeginCapture(b->gs, hipStreamCaptureModeThreadLocal));
      hipError_t e = hipEventRecord(b->cfork, b->gs);
      for (int v = 0; v < kNumVariants && e == hipSuccess; ++v) e = hipStreamWaitEvent(b->vs[v], b->cfork, 0);
      if (e == hipSuccess) e = launch_mfma_batch_f32(tl, b->work.ws, tk, pb, b->x, b->y, b->grid, b->vs);
      for (int v = 0; v < kNumVariants && e == hipSuccess; ++v) {
        e = hipEventRecord(b->cjoin[v], b->vs[v]);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->gs, b->cjoin[v], 0);
      }
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(b->gs, &g);
      HCHECK(e);
      HCHECK(e2);
      b->graph = g;
      HCHECK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    HCHECK(hipEventRecord(b->ev_in, ctx->stream));
    HCHECK(hipStreamWaitEvent(b->gs, b->ev_in, 0));
    HCHECK(hipGraphLaunch(b->exec, b->gs));
    HCHECK(hipEventRecord(b->ev_out, b->gs));
    HCHECK(hipStreamWaitEvent(ctx->stream, b->ev_out, 0));
  }
  ABI_END(ctx)
}

extern "C" int heff_batch_free(heff_batch* b) {
  if (b) (void)hipSetDevice(b->device);
  delete b;
  return HEFF_OK;
}

// ---------------------------------------------------------------- truncation (SVD step)
// The two-site vector is reshaped, per sector Q' of the enlarged left block
// L + {k}, into M_Q'[(s_k, alpha), (s_k+1, beta)]; its left singular vectors
// and squared singular values are the eigenpairs of rho_Q' = M M^T (the
// reduced density matrix of L + {k}).  rho is assembled from Psi blocks by
// the chained-product kernel, diagonalized by Jacobi in FP64, and the D
// largest singular values over all sectors are kept (Sec. II.A).
struct heff_trunc {
  int32_t n_kept = 0;
  double discarded = 0.0;
  std::vector<double> sing;
  std::vector<int32_t> nup, ndn, dim;
  heff::DevBuf iso;
  int64_t iso_len = 0;
};

extern "C" int heff_truncate(heff_ctx* ctx, const heff_blocks* b, const double* psi, int32_t d_keep, heff_trunc** out) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!b || !psi || !out || d_keep <= 0) throw Error(HEFF_EINVAL, "bad argument");
  *out = nullptr;
  HCHECK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const Bond& bl = b->L->bond;
  // enlarged sectors and their row blocks (s_k, q_alpha)
  std::map<std::pair<int, int>, int> qidx;
  std::vector<std::pair<int, int>> qlist;
  for (int qa = 0; qa < bl.n(); ++qa)
    for (int sk = 0; sk < 4; ++sk) qidx[{bl.nu[qa] + SQU[sk], bl.nd[qa] + SQD[sk]}] = 0;
  for (auto& kv : qidx) { kv.second = (int)qlist.size(); qlist.push_back(kv.first); }
  const int nq = (int)qlist.size();
  std::vector<std::array<int, 4>> roff(nq), rq(nq);  // per sector, per s: row offset / q_alpha index
  std::vector<int> nrow(nq, 0);
  for (int q = 0; q < nq; ++q)
    for (int sk = 0; sk < 4; ++sk) {
      int qa = bl.find(qlist[q].first - SQU[sk], qlist[q].second - SQD[sk]);
      rq[q][sk] = qa;
      roff[q][sk] = nrow[q];
      if (qa >= 0) nrow[q] += bl.dim[qa];
    }
  // columns of M_Q' (s_k+1, q_beta); M has rank at most min(rows, columns),
  // so the remaining eigenvalues of M M^T are zero by dimension (their
  // computed values are rounding, about 1e-17, whose square roots would
  // otherwise enter the singular values at the 1e-9 level)
  const Bond& br = b->R->bond;
  std::vector<int> ncol(nq, 0);
  for (int q = 0; q < nq; ++q)
    for (int s1 = 0; s1 < 4; ++s1) {
      const int qb = br.find(b->n_up - qlist[q].first - SQU[s1], b->n_dn - qlist[q].second - SQD[s1]);
      if (qb >= 0) ncol[q] += br.dim[qb];
    }
  // dense M_Q' (B, m x c) and W^T = I (m x m) per sector
  std::vector<int64_t> boff(nq), woff(nq), soff(nq);
  int64_t btot = 0, wtot = 0, stot = 0;
  for (int q = 0; q < nq; ++q) {
    boff[q] = btot;
    woff[q] = wtot;
    soff[q] = stot;
    btot += (int64_t)nrow[q] * ncol[q];
    wtot += (int64_t)nrow[q] * nrow[q];
    stot += nrow[q];
  }
  std::vector<std::array<int, 4>> coff(nq);  // per sector, per s_k+1: column offset
  for (int q = 0; q < nq; ++q) {
    int c = 0;
    for (int s1 = 0; s1 < 4; ++s1) {
      coff[q][s1] = c;
      const int qb = br.find(b->n_up - qlist[q].first - SQU[s1], b->n_dn - qlist[q].second - SQD[s1]);
      if (qb >= 0) c += br.dim[qb];
    }
  }
  std::vector<CopyJob> cj;
  for (int q = 0; q < nq; ++q)
    for (int sk = 0; sk < 4; ++sk) {
      const int qa = rq[q][sk];
      if (qa < 0) continue;
      for (int s1 = 0; s1 < 4; ++s1) {
        auto it = b->blk_index.find({qa, sk, s1});
        if (it == b->blk_index.end()) continue;
        const int x = it->second;
        CopyJob j{};
        j.src = b->blk_off[x];
        j.dst = boff[q] + (int64_t)roff[q][sk] * ncol[q] + coff[q][s1];
        j.rows = b->blk_desc[6 * x + 4];
        j.cols = b->blk_desc[6 * x + 5];
        j.ld = ncol[q];
        cj.push_back(j);
      }
    }
  DevBuf Bm, WT, dcj, dwoff, dboff, dsoff, dm, dc, doff, dsig;
  Bm.alloc((size_t)std::max<int64_t>(btot, 1) * sizeof(double));
  WT.alloc((size_t)std::max<int64_t>(wtot, 1) * sizeof(double));
  // columns of M without a psi block stay zero
  if (btot) HCHECK(hipMemsetAsync(Bm.p, 0, (size_t)btot * sizeof(double), s));
  upload(dcj, cj, s);
  HCHECK(launch_copy_blocks(dcj.as<CopyJob>(), (int)cj.size(), psi, Bm.as<double>(), s));
  upload(dwoff, woff, s);
  upload(dboff, boff, s);
  upload(dsoff, soff, s);
  upload(dm, nrow, s);
  upload(dc, ncol, s);
  HCHECK(launch_identity(dwoff.as<int64_t>(), dm.as<int32_t>(), nq, WT.as<double>(), s));
  dsig.alloc((size_t)std::max<int64_t>(stot, 1) * sizeof(double));
  // rounds of the block pair schedule, sweeps until every sector's rows are
  // orthogonal to rounding: |G_ij| <= eps sqrt(c) sqrt(G_ii G_jj), c the
  // length of a row (the one-sided Jacobi threshold of Demmel and Veselic)
  std::vector<BjJob> bj;
  int maxK = 0;
  for (int q = 0; q < nq; ++q) {
    if (nrow[q] < 2 || ncol[q] == 0) continue;
    const int nbk = (nrow[q] + kBjRows - 1) / kBjRows;
    const int K = nbk + (nbk & 1);
    if (K < 2) continue;
    maxK = std::max(maxK, K);
    for (int pr = 0; pr < K / 2; ++pr) {
      BjJob j{};
      j.b_off = boff[q];
      j.w_off = woff[q];
      j.m = nrow[q];
      j.c = ncol[q];
      j.K = K;
      j.pr = pr;
      j.sector = q;
      bj.push_back(j);
    }
  }
  DevBuf dbj;
  upload(dbj, bj, s);
  doff.alloc((size_t)std::max(nq, 1) * sizeof(unsigned long long));
  const double tol = 2.220446049250313e-16;
  std::vector<unsigned long long> offbits(nq);
  for (int sweep = 0; sweep < 40 && !bj.empty(); ++sweep) {
    HCHECK(hipMemsetAsync(doff.p, 0, (size_t)nq * sizeof(unsigned long long), s));
    for (int r = 0; r < maxK - 1; ++r)
      HCHECK(launch_bj_round(dbj.as<BjJob>(), (int)bj.size(), Bm.as<double>(), WT.as<double>(),
                             doff.as<unsigned long long>(), r, tol, s));
    HCHECK(hipMemcpyAsync(offbits.data(), doff.p, (size_t)nq * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HCHECK(hipStreamSynchronize(s));
    bool done = true;
    for (int q = 0; q < nq; ++q) {
      double d;
      std::memcpy(&d, &offbits[q], sizeof(d));
      if (d > tol * std::sqrt((double)ncol[q])) done = false;
    }
    if (done) break;
  }
  // singular values: row norms of B (at most min(rows, columns) non-zero)
  HCHECK(launch_row_norms(dboff.as<int64_t>(), dm.as<int32_t>(), dc.as<int32_t>(), dsoff.as<int64_t>(), nq,
                          Bm.as<double>(), dsig.as<double>(), s));
  std::vector<double> sig(stot);
  if (stot) HCHECK(hipMemcpyAsync(sig.data(), dsig.p, (size_t)stot * sizeof(double), hipMemcpyDeviceToHost, s));
  HCHECK(hipStreamSynchronize(s));
  std::vector<std::vector<double>> lam(nq);
  for (int q = 0; q < nq; ++q) {
    lam[q].resize(nrow[q]);
    for (int i = 0; i < nrow[q]; ++i) lam[q][i] = sig[soff[q] + i] * sig[soff[q] + i];
  }
  // descending order inside each sector, then the global selection
  std::vector<std::vector<int>> ord(nq);
  struct Cand { double lam; int q, rank; };
  std::vector<Cand> all;
  for (int q = 0; q < nq; ++q) {
    ord[q].resize(nrow[q]);
    for (int i = 0; i < nrow[q]; ++i) ord[q][i] = i;
    std::stable_sort(ord[q].begin(), ord[q].end(), [&](int x, int y) { return lam[q][x] > lam[q][y]; });
    for (int r = std::min(nrow[q], ncol[q]); r < nrow[q]; ++r) lam[q][ord[q][r]] = 0.0;
    for (int r = 0; r < nrow[q]; ++r) all.push_back({lam[q][ord[q][r]], q, r});
  }
  std::stable_sort(all.begin(), all.end(), [](const Cand& x, const Cand& y) {
    if (x.lam != y.lam) return x.lam > y.lam;
    if (x.q != y.q) return x.q < y.q;
    return x.rank < y.rank;
  });
  auto T = std::make_unique<heff_trunc>();
  const int nk = std::min<int>(d_keep, (int)all.size());
  std::vector<int> kept(nq, 0);
  for (int i = 0; i < (int)all.size(); ++i) {
    if (i < nk) {
      T->sing.push_back(std::sqrt(std::max(all[i].lam, 0.0)));
      kept[all[i].q]++;
    } else {
      T->discarded += std::max(all[i].lam, 0.0);
    }
  }
  T->n_kept = nk;
  // new isometry: kept left singular vectors (descending) of every kept sector
  std::vector<GatherJob> gj;
  std::vector<int32_t> cols;
  std::vector<size_t> col_start;
  int64_t ioff = 0;
  for (int q = 0; q < nq; ++q) {
    if (nrow[q] == 0 || kept[q] == 0) continue;
    T->nup.push_back(qlist[q].first);
    T->ndn.push_back(qlist[q].second);
    T->dim.push_back(kept[q]);
    col_start.push_back(cols.size());
    for (int r = 0; r < kept[q]; ++r) cols.push_back(ord[q][r]);
    GatherJob g{};
    g.v_off = woff[q];
    g.out_off = ioff;
    g.n = nrow[q];
    g.ncol = kept[q];
    gj.push_back(g);
    ioff += (int64_t)nrow[q] * kept[q];
  }
  DevBuf dcols, dg;
  upload(dcols, cols, s);
  for (size_t j = 0; j < gj.size(); ++j) gj[j].cols = dcols.as<int32_t>() + col_start[j];
  upload(dg, gj, s);
  T->iso.alloc((size_t)std::max<int64_t>(ioff, 1) * sizeof(double));
  T->iso_len = ioff;
  HCHECK(launch_gather_rows(dg.as<GatherJob>(), (int)gj.size(), WT.as<double>(), T->iso.as<double>(), s));
  HCHECK(hipStreamSynchronize(s));
  *out = T.release();
  ABI_END(ctx)
}

extern "C" int heff_trunc_info(const heff_trunc* t, int32_t* n_kept, double* discarded, int32_t* n_sect, int64_t* iso_len) {
  if (!t) return HEFF_EINVAL;
  if (n_kept) *n_kept = t->n_kept;
  if (discarded) *discarded = t->discarded;
  if (n_sect) *n_sect = (int32_t)t->dim.size();
  if (iso_len) *iso_len = t->iso_len;
  return HEFF_OK;
}

extern "C" int heff_trunc_get(heff_ctx* ctx, const heff_trunc* t, double* sing, int32_t* nup, int32_t* ndn,
                              int32_t* dim, double* iso_dev) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!t) throw Error(HEFF_EINVAL, "null truncation");
  if (sing) std::copy(t->sing.begin(), t->sing.end(), sing);
  if (nup) std::copy(t->nup.begin(), t->nup.end(), nup);
  if (ndn) std::copy(t->ndn.begin(), t->ndn.end(), ndn);
  if (dim) std::copy(t->dim.begin(), t->dim.end(), dim);
  if (iso_dev && t->iso_len) {
    HCHECK(hipMemcpyAsync(iso_dev, t->iso.p, (size_t)t->iso_len * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    HCHECK(hipStreamSynchronize(ctx->stream));
  }
  ABI_END(ctx)
}

extern "C" int heff_trunc_free(heff_trunc* t) {
  delete t;
  return HEFF_OK;
}

// ---------------------------------------------------------------- sweep step (Ren_l, StVec)
// One step of a left-to-right sweep (Sec. II.A: the MPS is optimized bond by
// bond; Sec. IV.A names the phases SVD, Ren_l and StVec around Diag_H).  The
// optimized two-site vector of the pair (k, k+1) is truncated; the left
// block grows by site k with the truncated isometry A (the same blocking and
// projection as the build's own left steps); the right part loses site k+2
// (its block of one site fewer was kept by the build); the pair (k+1, k+2)
// gets its terms and task table; and the start vector of the new pair is the
// old state expressed in the new two-site basis,
//   psi'[a', s1, s2, g] = sum_{s, a, b} A[(s, a), a'] psi[a, s, s1, b] B[(s2, g), b],
// with B the right isometry of site k+2.  The basis change keeps the mode
// order (block modes, then the sites in order), so no fermionic sign enters.
// Every term is one chained block product on the same kernels as H_eff psi.
static void make_iso_from_device(Iso& iso, const Bond& old, const Bond& nw, const double* dev, int64_t len,
                                 hipStream_t s) {
  iso.old = &old;
  iso.nw = &nw;
  iso.qoff.resize(nw.n());
  iso.rowoff.resize(nw.n());
  int64_t off = 0;
  for (int q = 0; q < nw.n(); ++q) {
    int64_t r = 0;
    for (int st = 0; st < 4; ++st) {
      iso.rowoff[q][st] = r;
      int qi = old.find(nw.nu[q] - SQU[st], nw.nd[q] - SQD[st]);
      if (qi >= 0) r += old.dim[qi];
    }
    iso.qoff[q] = off;
    off += r * (int64_t)nw.dim[q];
  }
  if (off != len) throw Error(HEFF_EINVAL, "internal: truncated isometry length does not match its bond");
  iso.size = off;
  iso.dev.alloc((size_t)std::max<int64_t>(off, 1) * sizeof(double));
  if (off) HCHECK(hipMemcpyAsync(iso.dev.p, dev, (size_t)off * sizeof(double), hipMemcpyDeviceToDevice, s));
}

extern "C" int heff_sweep_right(heff_ctx* ctx, const heff_blocks* b, const double* psi, int32_t d_keep,
                                uint32_t prec_mask, heff_blocks** out, heff_trunc** trunc_out) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!b || !psi || !out || d_keep <= 0) throw Error(HEFF_EINVAL, "bad argument");
  *out = nullptr;
  if (trunc_out) *trunc_out = nullptr;
  if (prec_mask & ~((1u << HEFF_FP32) | (1u << HEFF_BF16X3) | 1u | HEFF_KEEP_ENV))
    throw Error(HEFF_EINVAL, "bad prec_mask");
  if (!b->env) throw Error(HEFF_ESTATE, "the blocks were built without HEFF_KEEP_ENV");
  if (b->shard_nranks > 1) throw Error(HEFF_ESTATE, "the product is restricted to one shard's output blocks");
  const int n = b->n_orb, k0 = b->k0, mR = n - k0 - 2;
  if (mR < 1) throw Error(HEFF_ESTATE, "the pair is already at the right end");
  HCHECK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  std::shared_ptr<Env> env = b->env;
  // SVD step: truncated isometry of site k
  heff_trunc* tr_raw = nullptr;
  if (int rc = heff_truncate(ctx, b, psi, d_keep, &tr_raw)) throw Error(rc, ctx->err);
  std::unique_ptr<heff_trunc> tr(tr_raw);
  Bond nb;
  for (size_t i = 0; i < tr->dim.size(); ++i) {
    nb.nu.push_back(tr->nup[i]);
    nb.nd.push_back(tr->ndn[i]);
    nb.dim.push_back(tr->dim[i]);
    nb.index[{tr->nup[i], tr->ndn[i]}] = (int)i;
  }
  if (nb.n() == 0) throw Error(HEFF_ESECTOR, "truncation kept no state");
  // Ren_l: the left block of k+1 sites
  Block& Lold = *b->L;
  Iso isoA;
  make_iso_from_device(isoA, Lold.bond, nb, tr->iso.as<double>(), tr->iso_len, s);
  std::shared_ptr<Block> Lnew = grow_left(Lold, nb, isoA, k0, env->nmode, env->I, s);
  // the two-site problem of the pair (k+1, k+2)
  auto B = std::make_unique<heff_blocks>();
  B->ctx = ctx;
  B->device = ctx->device;
  B->stream = ctx->stream;
  B->n_orb = n;
  B->n_up = b->n_up;
  B->n_dn = b->n_dn;
  B->k0 = k0 + 1;
  B->prec_mask = prec_mask;
  B->env = env;
  B->L = Lnew;
  B->R = env->right[mR - 1];
  build_psi_layout(*B);
  build_terms(*B, env->I);
  B->Ltmp.run(s);
  B->Rtmp.run(s);
  build_tasks(*B, s);
  if (prec_mask & ((1u << HEFF_FP32) | (1u << HEFF_BF16X3))) {
    const double* srcs[4] = {B->L->store.dev.as<double>(), B->Ltmp.tmp.dev.as<double>(),
                             B->R->store.dev.as<double>(), B->Rtmp.tmp.dev.as<double>()};
    int64_t sizes[4] = {B->L->store.total, B->Ltmp.tmp.total, B->R->store.total, B->Rtmp.tmp.total};
    for (int i = 0; i < 4; ++i) {
      B->f32[i].alloc((size_t)std::max<int64_t>(sizes[i], 1) * sizeof(float));
      if (sizes[i]) HCHECK(launch_convert_f32(srcs[i], B->f32[i].as<float>(), sizes[i], s));
    }
  }
  // StVec: one task per (new block, s_k)
  const Iso& isoB = *env->riso[mR];  // site k+2: (site, right block of mR-1 sites) -> right block of mR sites
  const Bond& blo = b->L->bond;      // old left bond (k sites)
  const Bond& bro = b->R->bond;      // old right bond (mR sites)
  const Bond& brn = B->R->bond;      // new right bond (mR - 1 sites)
  ChainPlan P;
  const int nbk = (int)B->blk_off.size();
  for (int y = 0; y < nbk; ++y) {
    const int qa2 = B->blk_qa[y], qg = B->blk_qb[y];
    const int s1 = B->blk_desc[6 * y + 2], s2 = B->blk_desc[6 * y + 3];
    const int qb = bro.find(brn.nu[qg] + SQU[s2], brn.nd[qg] + SQD[s2]);
    Tile t{};
    t.offOut = B->blk_off[y];
    t.a = nb.dim[qa2];
    t.e = brn.dim[qg];
    t.ldOut = t.e;
    t.t0 = (int32_t)P.tasks.size();
    if (qb >= 0) {
      const int64_t offR = isoB.block(s2, qb);
      for (int sk = 0; sk < 4; ++sk) {
        const int qa = blo.find(nb.nu[qa2] - SQU[sk], nb.nd[qa2] - SQD[sk]);
        if (qa < 0) continue;
        auto it = b->blk_index.find({qa, sk, s1});
        if (it == b->blk_index.end()) continue;
        const int x = it->second;
        if (b->blk_qb[x] != qb) throw Error(HEFF_EINVAL, "internal: start vector block violates sector conservation");
        const int64_t offL = isoA.block(sk, qa2);
        if (offL < 0 || offR < 0) throw Error(HEFF_EINVAL, "internal: missing isometry block");
        Task k{};
        k.f = 1.0;
        k.a = (uint16_t)nb.dim[qa2];
        k.b = (uint16_t)blo.dim[qa];
        k.c = (uint16_t)bro.dim[qb];
        k.e = (uint16_t)brn.dim[qg];
        k.offL = offL;  // A block stored D(q_a) x D'(q_a'): op(L) = A^T
        k.ldL = (uint16_t)nb.dim[qa2];
        k.offX = b->blk_off[x];
        k.ldX = (uint16_t)bro.dim[qb];
        k.offR = offR;  // B block stored D(q_g) x D(q_b) = e x c
        k.ldR = (uint16_t)bro.dim[qb];
        k.flags = (uint16_t)(T_TL | T_TR);
        P.tasks.push_back(k);
      }
    }
    t.t1 = (int32_t)P.tasks.size();
    P.tiles.push_back(t);
  }
  B->start.alloc((size_t)std::max<int64_t>(B->n_elem, 1) * sizeof(double));
  Bases<double> bs{};
  bs.L[0] = bs.L[1] = isoA.dev.as<double>();
  bs.X[0] = bs.X[1] = psi;
  bs.R[0] = bs.R[1] = isoB.dev.as<double>();
  bs.out = B->start.as<double>();
  set_limits(bs, isoA.dev, isoA.dev, b->n_elem, isoB.dev, isoB.dev);
  run_chain(P, bs, s);
  HCHECK(hipStreamSynchronize(s));
  *out = B.release();
  if (trunc_out) *trunc_out = tr.release();
  ABI_END(ctx)
}

extern "C" int heff_start_vector(const heff_blocks* b, const double** psi) {
  if (!b || !psi) return HEFF_EINVAL;
  if (!b->start.p) return HEFF_ESTATE;
  *psi = b->start.as<double>();
  return HEFF_OK;
}

// ---------------------------------------------------------------- mode rotation of the pair
// The micro-iteration of the mode optimization (Sec. II.B, Fig. microiter):
// the orbitals k and k+1 of the pair are rotated by
// U = exp(theta (E_k,k+1 - E_k+1,k)) (the identity except for the 2 x 2
// block), the new orbitals being c'+_i = sum_a U_ai c+_a.  The same
// physical state then has the coefficients exp(-K) phi with K the
// many-body generator sum_s (c+_ks c_k+1,s - c+_k+1,s c_ks); K acts on the
// two middle sites only (the parity strings of the left block cancel in a
// bilinear), so on the two-site vector it is one 16 x 16 matrix G(theta) =
// exp(-theta K) on the middle index, block diagonal over the (n_up, n_dn)
// of the two sites.  The integrals transform as h' = U^T h U and
// V'_ijkl = sum U_ai U_bj U_ck U_dl V_abcd (heff_rotate_integrals), which
// leaves <psi|H_eff|psi> unchanged.

// matrix exponential of a 16 x 16 matrix by scaling and squaring with a
// truncated Taylor series (the norm is scaled below 1/2; 20 terms)
static Mat16 expm16(const Mat16& A) {
  double nrm = 0.0;
  for (int i = 0; i < 16; ++i) {
    double r = 0.0;
    for (int j = 0; j < 16; ++j) r += std::fabs(A[i * 16 + j]);
    nrm = std::max(nrm, r);
  }
  int sq = 0;
  while (nrm > 0.5) {
    nrm *= 0.5;
    ++sq;
  }
  Mat16 X = A;
  const double sc = std::ldexp(1.0, -sq);
  for (double& v : X) v *= sc;
  Mat16 E = m16eye(), term = m16eye();
  for (int k = 1; k <= 20; ++k) {
    term = m16mul(term, X);
    for (double& v : term) v /= (double)k;
    m16axpy(E, 1.0, term);
  }
  for (int i = 0; i < sq; ++i) E = m16mul(E, E);
  return E;
}

// G(theta) on the middle index 4 s_k + s_k+1
static Mat16 pair_rotation(double theta, int k0) {
  Mat16 K = m16zero();
  for (int sg = 0; sg < 2; ++sg) {
    const int a = 2 * k0 + sg, b = 2 * (k0 + 1) + sg;
    m16axpy(K, 1.0, m16mul(mid_c(a, true, k0), mid_c(b, false, k0)));
    m16axpy(K, -1.0, m16mul(mid_c(b, true, k0), mid_c(a, false, k0)));
  }
  for (double& v : K) v *= -theta;
  Mat16 G = expm16(K);
  // exact zeros outside the (n_up, n_dn) blocks of the two sites
  for (int i = 0; i < 16; ++i)
    for (int j = 0; j < 16; ++j) {
      const int ui = SQU[i >> 2] + SQU[i & 3], di = SQD[i >> 2] + SQD[i & 3];
      const int uj = SQU[j >> 2] + SQU[j & 3], dj = SQD[j >> 2] + SQD[j & 3];
      if (ui != uj || di != dj) G[i * 16 + j] = 0.0;
    }
  return G;
}

static void rotate_pair(const heff_blocks* b, double theta, const double* psi, double* out, hipStream_t s) {
  const Mat16 G = pair_rotation(theta, b->k0);
  std::vector<RotJob> jobs;
  const int nb = (int)b->blk_off.size();
  for (int y = 0; y < nb; ++y) {
    const int qa = b->blk_qa[y];
    const int m2 = 4 * b->blk_desc[6 * y + 2] + b->blk_desc[6 * y + 3];
    RotJob j{};
    j.off_out = b->blk_off[y];
    j.n = b->blk_desc[6 * y + 4] * b->blk_desc[6 * y + 5];
    for (int m = 0; m < 16; ++m) {
      const double g = G[m2 * 16 + m];
      if (g == 0.0) continue;
      auto it = b->blk_index.find({qa, m >> 2, m & 3});
      if (it == b->blk_index.end()) continue;
      if (j.nterm >= 4) throw Error(HEFF_EINVAL, "internal: more than four middle states in one sector");
      if (b->blk_qb[it->second] != b->blk_qb[y]) throw Error(HEFF_EINVAL, "internal: rotation leaves the sector");
      j.off_in[j.nterm] = b->blk_off[it->second];
      j.c[j.nterm] = g;
      ++j.nterm;
    }
    jobs.push_back(j);
  }
  DevBuf dj;
  upload(dj, jobs, s);
  HCHECK(launch_rotate_pair(dj.as<RotJob>(), (int64_t)jobs.size(), psi, out, s));
  HCHECK(hipStreamSynchronize(s));
}

// S_1/2 = 2 ln sum sigma and S_1 = -sum lambda ln lambda of the normalized
// state over the cut (left part | rest), from every singular value
static void pair_entropies(heff_ctx* ctx, const heff_blocks* b, const double* psi, double* s_half, double* s_vn) {
  heff_trunc* tr = nullptr;
  if (int rc = heff_truncate(ctx, b, psi, INT32_MAX, &tr)) throw Error(rc, ctx->err);
  std::unique_ptr<heff_trunc> t(tr);
  double nrm2 = 0.0;
  for (double v : t->sing) nrm2 += v * v;
  if (!(nrm2 > 0.0)) throw Error(HEFF_EINVAL, "zero vector");
  double sum = 0.0, svn = 0.0;
  for (double v : t->sing) {
    const double l = v * v / nrm2;
    sum += v;
    if (l > 0.0) svn -= l * std::log(l);
  }
  if (s_half) *s_half = 2.0 * std::log(sum / std::sqrt(nrm2));
  if (s_vn) *s_vn = svn;
}

extern "C" int heff_rotate_pair(heff_ctx* ctx, const heff_blocks* b, double theta, const double* psi, double* out) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!b || !psi || !out) throw Error(HEFF_EINVAL, "null argument");
  if (psi == out) throw Error(HEFF_EINVAL, "psi and out alias");
  if (!std::isfinite(theta)) throw Error(HEFF_EINVAL, "non-finite angle");
  HCHECK(hipSetDevice(ctx->device));
  rotate_pair(b, theta, psi, out, ctx->stream);
  ABI_END(ctx)
}

extern "C" int heff_pair_entropy(heff_ctx* ctx, const heff_blocks* b, const double* psi, double* s_half, double* s_vn) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!b || !psi) throw Error(HEFF_EINVAL, "null argument");
  HCHECK(hipSetDevice(ctx->device));
  pair_entropies(ctx, b, psi, s_half, s_vn);
  ABI_END(ctx)
}

extern "C" int heff_optimize_pair(heff_ctx* ctx, const heff_blocks* b, const double* psi, double* out, double* theta,
                                  double* s_before, double* s_after, int32_t* n_evals) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!b || !psi || !out || !theta) throw Error(HEFF_EINVAL, "null argument");
  if (psi == out) throw Error(HEFF_EINVAL, "psi and out alias");
  HCHECK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  int evals = 0;
  auto f = [&](double t) {
    rotate_pair(b, t, psi, out, s);
    double sh = 0.0;
    pair_entropies(ctx, b, out, &sh, nullptr);
    ++evals;
    return sh;
  };
  // S_1/2 has period pi in theta: 16 angles of [-pi/2, pi/2), then golden
  // section on the bracket around the best one
  const double pi = 3.14159265358979323846;
  const int ng = 16;
  double best_t = 0.0, best = 0.0;
  for (int i = 0; i < ng; ++i) {
    const double t = -pi / 2 + pi * i / ng, v = f(t);
    if (i == 0 || v < best) {
      best = v;
      best_t = t;
    }
  }
  const double hw = pi / ng, g = (std::sqrt(5.0) - 1.0) / 2.0;
  double a = best_t - hw, bb = best_t + hw;
  double c = bb - g * (bb - a), d = a + g * (bb - a);
  double fc = f(c), fd = f(d);
  while (bb - a > 1e-8) {
    if (fc < fd) {
      bb = d;
      d = c;
      fd = fc;
      c = bb - g * (bb - a);
      fc = f(c);
    } else {
      a = c;
      c = d;
      fc = fd;
      d = a + g * (bb - a);
      fd = f(d);
    }
  }
  double t = 0.5 * (a + bb), st = f(t);
  if (best < st) {
    t = best_t;
    st = f(t);
  }
  if (s_before) pair_entropies(ctx, b, psi, s_before, nullptr);
  *theta = t;
  if (s_after) *s_after = st;
  if (n_evals) *n_evals = evals;
  ABI_END(ctx)
}

extern "C" int heff_rotate_integrals(int32_t n, const double* h, const double* V, int32_t x, int32_t y, double theta,
                                     double* h_out, double* V_out) {
  if (n <= 0 || !h || !V || !h_out || !V_out || x < 0 || y < 0 || x >= n || y >= n || x == y) return HEFF_EINVAL;
  if (!std::isfinite(theta)) return HEFF_EINVAL;
  const double c = std::cos(theta), sn = std::sin(theta);
  // U_aa = 1 (a != x, y); U_xx = U_yy = c, U_xy = s, U_yx = -s; new index i
  // mixes old x and y through column i of U
  auto mix = [&](double vx, double vy, int i) -> double {  // sum_a U_ai v_a over a in {x, y}
    return i == x ? c * vx - sn * vy : sn * vx + c * vy;
  };
  const size_t N = (size_t)n;
  std::vector<double> H(h, h + N * N);
  for (int pass = 0; pass < 2; ++pass)  // h' = U^T h U: rotate the row, then the column index
    for (size_t o = 0; o < N; ++o) {
      auto at = [&](int i) -> double& { return pass == 0 ? H[(size_t)i * N + o] : H[o * N + (size_t)i]; };
      const double vx = at(x), vy = at(y);
      at(x) = mix(vx, vy, x);
      at(y) = mix(vx, vy, y);
    }
  std::copy(H.begin(), H.end(), h_out);
  std::vector<double> W(V, V + N * N * N * N);
  const size_t st[4] = {N * N * N, N * N, N, 1};
  for (int ax = 0; ax < 4; ++ax)  // one index of V at a time
    for (size_t r = 0; r < N * N * N; ++r) {
      // r enumerates the other three indices
      size_t rem = r, base = 0;
      for (int o = 3; o >= 0; --o) {
        if (o == ax) continue;
        base += (rem % N) * st[o];
        rem /= N;
      }
      double& ex = W[base + (size_t)x * st[ax]];
      double& ey = W[base + (size_t)y * st[ax]];
      const double vx = ex, vy = ey;
      ex = mix(vx, vy, x);
      ey = mix(vx, vy, y);
    }
  std::copy(W.begin(), W.end(), V_out);
  return HEFF_OK;
}

// ---------------------------------------------------------------- introspection for tests
// Copies the blocks of a named renormalized operator to host memory, blocks
// ordered by in-sector, each row-major.  side 0 = L, 1 = R; kind per the
// internal Kind enum (H=0, C=1, A=2, B=3, T=4, D=5, DD=6, BB=7, S=8).
// Returns the number of elements (0 if the operator does not exist).
extern "C" int64_t heff_debug_op(const heff_blocks* b, int side, int kind, int i, int j, double* host,
                                 int64_t cap) {
  if (!b) return -1;
  const Store& st = side == 0 ? b->L->store : b->R->store;
  OpId id = st.get({kind, i, j, 0});
  if (!id.valid()) return 0;
  const Layout& L = st.lay(id);
  if (host && cap >= L.size) {
    (void)hipStreamSynchronize(b->stream);
    if (hipMemcpy(host, st.dev.as<double>() + st.offset(id), L.size * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
      return -2;
  }
  return L.size;
}

// ====================================================================== backward
namespace heff {

// Task tables of dE/d(operator arena) for E = <psi|H_eff|psi>.  Every product
// task  out_y += f op(L) op(X) op(R)  (X a block of psi) contributes
// E_t = f <psi_y, op(L) op(X) op(R)>, whose gradient is
//   d/d op(L) = f psi_y op(R)^T op(X)^T,   d/d op(R) = f op(X)^T op(L)^T psi_y,
// taken back to the storage orientation of the operand block.  Each stored
// block becomes one output tile (all tasks that use it, in either
// orientation, accumulate into it), and each contribution is again a
// chained product, so the forward kernels run it.  Launch bases:
// L[*] = R[*] = psi; X[0..1] = the other side's store and temporaries.
static void make_grad_plan(const heff_blocks& B, int side, hipStream_t s) {
  auto& G = B.grad[side];
  const bool left = side == 0;
  const int64_t n0 = left ? B.L->store.total : B.R->store.total;
  std::map<std::pair<int, int64_t>, int> tile_of;
  std::vector<Tile> tiles;
  std::vector<std::vector<Task>> per;
  const std::vector<Tile>& btiles = B.blk_tiles.empty() ? B.h_tiles : B.blk_tiles;
  const std::vector<Task>& btasks = B.blk_tiles.empty() ? B.h_tasks : B.blk_tasks;
  const int nb = (int)btiles.size();
  for (int y = 0; y < nb; ++y) {
    const Tile& ty = btiles[y];
    const int64_t py = ty.offOut;  // psi_y block (a x e, row stride e)
    for (int k = ty.t0; k < ty.t1; ++k) {
      const Task& t = btasks[k];
      const uint32_t fl = t.flags;
      const bool tl = fl & T_TL, tx = fl & T_TX, tr = fl & T_TR;
      if (left ? (fl & T_IDL) : (fl & T_IDR)) continue;
      const int sel = left ? ((fl & T_SELL) ? 1 : 0) : ((fl & T_SELR) ? 1 : 0);
      const int64_t off = left ? t.offL : t.offR;
      int rows, cols, ld;
      if (left) {
        rows = tl ? t.b : t.a;
        cols = tl ? t.a : t.b;
        ld = t.ldL;
      } else {
        rows = tr ? t.e : t.c;
        cols = tr ? t.c : t.e;
        ld = t.ldR;
      }
      auto key = std::make_pair(sel, off);
      auto it = tile_of.find(key);
      int id;
      if (it == tile_of.end()) {
        id = (int)tiles.size();
        tile_of[key] = id;
        Tile u{};
        u.offOut = off + (sel ? n0 : 0);
        u.a = rows;
        u.e = cols;
        u.ldOut = ld;
        tiles.push_back(u);
        per.emplace_back();
      } else {
        id = it->second;
        if (tiles[id].a != rows || tiles[id].e != cols || tiles[id].ldOut != ld)
          throw Error(HEFF_EINVAL, "internal: one operator block used with two shapes");
      }
      Task g{};
      g.f = t.f;
      uint32_t gf = 0;
      if (left) {
        // middle operand: op(R) or its transpose, from the right arenas
        gf |= (fl & T_SELR) ? T_SELX : 0u;
        gf |= (fl & T_IDR) ? T_IDX : 0u;
        g.offX = t.offR;
        g.ldX = t.ldR;
        if (!tl) {  // (a x b) += f psi_y op(R)^T op(X)^T
          g.a = t.a; g.b = t.e; g.c = t.c; g.e = t.b;
          g.offL = py; g.ldL = t.e;
          if (!tr) gf |= T_TX;
          g.offR = t.offX; g.ldR = t.ldX;
          if (!tx) gf |= T_TR;
          if (fl & T_IDX) gf |= T_IDR;
        } else {  // (b x a) += f op(X) op(R) psi_y^T
          g.a = t.b; g.b = t.c; g.c = t.e; g.e = t.a;
          g.offL = t.offX; g.ldL = t.ldX;
          if (tx) gf |= T_TL;
          if (fl & T_IDX) gf |= T_IDL;
          if (tr) gf |= T_TX;
          g.offR = py; g.ldR = t.e;
          gf |= T_TR;
        }
      } else {
        gf |= (fl & T_SELL) ? T_SELX : 0u;
        gf |= (fl & T_IDL) ? T_IDX : 0u;
        g.offX = t.offL;
        g.ldX = t.ldL;
        if (!tr) {  // (c x e) += f op(X)^T op(L)^T psi_y
          g.a = t.c; g.b = t.b; g.c = t.a; g.e = t.e;
          g.offL = t.offX; g.ldL = t.ldX;
          if (!tx) gf |= T_TL;
          if (fl & T_IDX) gf |= T_IDL;
          if (!tl) gf |= T_TX;
          g.offR = py; g.ldR = t.e;
        } else {  // (e x c) += f psi_y^T op(L) op(X)
          g.a = t.e; g.b = t.a; g.c = t.b; g.e = t.c;
          g.offL = py; g.ldL = t.e;
          gf |= T_TL;
          if (tl) gf |= T_TX;
          g.offR = t.offX; g.ldR = t.ldX;
          if (tx) gf |= T_TR;
          if (fl & T_IDX) gf |= T_IDR;
        }
      }
      g.flags = (uint16_t)gf;
      per[id].push_back(g);
    }
  }
  std::vector<Task> tasks;
  for (size_t i = 0; i < tiles.size(); ++i) {
    tiles[i].t0 = (int32_t)tasks.size();
    tasks.insert(tasks.end(), per[i].begin(), per[i].end());
    tiles[i].t1 = (int32_t)tasks.size();
  }
  if (tasks.size() > (size_t)INT32_MAX) throw Error(HEFF_EINVAL, "gradient task table too large");
  split_large(tiles, tasks, kMaxDim);
  std::vector<int> order(tiles.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::vector<double> cost(tiles.size(), 0.0);
  for (size_t i = 0; i < tiles.size(); ++i)
    for (int k = tiles[i].t0; k < tiles[i].t1; ++k) cost[i] += task_flops(tasks[k]) / std::max(1, tiles[i].a);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<Work> lists[kNumVariants];
  split_work(tiles, tasks, order, lists);
  upload(G.tiles, tiles, s);
  upload(G.tasks, tasks, s);
  G.work.upload_lists(lists, s);
  HCHECK(hipStreamSynchronize(s));
  G.ready = true;
}

// device pointers of the four operand arenas [L store, L temps, R store,
// R temps] in the given precision, and their element counts
static void arenas(const heff_blocks& B, int prec, void* p[4], int64_t n[4]) {
  n[0] = B.L->store.total;
  n[1] = B.Ltmp.tmp.total;
  n[2] = B.R->store.total;
  n[3] = B.Rtmp.tmp.total;
  if (prec == HEFF_FP64) {
    p[0] = B.L->store.dev.p;
    p[1] = B.Ltmp.tmp.dev.p;
    p[2] = B.R->store.dev.p;
    p[3] = B.Rtmp.tmp.dev.p;
  } else if (prec == HEFF_FP32) {
    if (!(B.prec_mask & (1u << HEFF_FP32))) throw Error(HEFF_ENOTSUP, "FP32 operands were not built");
    for (int i = 0; i < 4; ++i) p[i] = B.f32[i].p;
  } else {
    throw Error(HEFF_ENOTSUP, "gradients are available in FP64 and FP32");
  }
}

template <typename T>
static void run_grad(const heff_blocks& B, int side, void* const ar[4], const void* psi, void* dout, hipStream_t s) {
  const auto& G = B.grad[side];
  Bases<T> bs{};
  bs.L[0] = bs.L[1] = static_cast<const T*>(psi);
  bs.R[0] = bs.R[1] = static_cast<const T*>(psi);
  bs.X[0] = static_cast<const T*>(ar[side == 0 ? 2 : 0]);
  bs.X[1] = static_cast<const T*>(ar[side == 0 ? 3 : 1]);
  bs.out = static_cast<T*>(dout);
  if constexpr (sizeof(T) == 8)
    HCHECK(launch_mfma_f64(G.tiles.as<Tile>(), G.work.ws, G.tasks.as<Task>(), bs, s));
  else
    HCHECK(launch_mfma_f32(G.tiles.as<Tile>(), G.work.ws, G.tasks.as<Task>(), bs, s));
}


// first-order change of the integrals under the orbital rotation generated
// by K = E_xy - E_yx: dh = K^T h + h K, dV_ijkl = sum over the four index
// positions of K_ai V_(i -> a)
static void rotation_derivative(const Ints& I, int x, int y, std::vector<double>& dh, std::vector<double>& dV) {
  const int n = I.n;
  auto K = [&](int a, int i) { return (a == x && i == y) ? 1.0 : (a == y && i == x) ? -1.0 : 0.0; };
  dh.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = 0.0;
      for (int a : {x, y}) v += K(a, i) * I.h[(size_t)a * n + j] + I.h[(size_t)i * n + a] * K(a, j);
      dh[(size_t)i * n + j] = v;
    }
  auto V = [&](int i, int j, int k, int l) { return I.V[(((size_t)i * n + j) * n + k) * n + l]; };
  dV.assign((size_t)n * n * n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k)
        for (int l = 0; l < n; ++l) {
          double v = 0.0;
          for (int a : {x, y}) {
            v += K(a, i) * V(a, j, k, l) + K(a, j) * V(i, a, k, l) + K(a, k) * V(i, j, a, l) + K(a, l) * V(i, j, k, a);
          }
          dV[(((size_t)i * n + j) * n + k) * n + l] = v;
        }
}

}  // namespace heff

extern "C" int heff_op_arena(const heff_blocks* b, int prec, void* ptr[4], int64_t n_elem[4]) {
  if (!b || !ptr || !n_elem) return HEFF_EINVAL;
  try {
    heff::arenas(*b, prec, ptr, n_elem);
  } catch (const heff::Error& e) {
    return e.code;
  }
  return HEFF_OK;
}

extern "C" int heff_energy(heff_ctx* ctx, const heff_blocks* b, int prec, const void* psi, double* E) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!b || !psi || !E) throw Error(HEFF_EINVAL, "null argument");
  if (b->shard_nranks > 1) throw Error(HEFF_ESTATE, "the product is restricted to one shard's output blocks");
  if (prec != HEFF_FP64 && prec != HEFF_FP32) throw Error(HEFF_ENOTSUP, "energy is available in FP64 and FP32");
  HCHECK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const size_t es = prec == HEFF_FP64 ? 8 : 4;
  const size_t hbytes = ((b->n_elem * es + 255) / 256) * 256;  // H psi, then the reduction partials
  const size_t need = hbytes + (kRedBlocks + 1) * sizeof(double);
  if (b->escratch.bytes < need) b->escratch.alloc(need);
  char* base = b->escratch.as<char>();
  void* hp = base;
  double* red = reinterpret_cast<double*>(base + hbytes);
  if (int rc = heff_apply(ctx, b, prec, psi, hp)) throw Error(rc, ctx->err);
  if (prec == HEFF_FP64)
    HCHECK(launch_dot_f64(static_cast<const double*>(psi), static_cast<const double*>(hp), b->n_elem, red + kRedBlocks,
                          red, s));
  else
    HCHECK(launch_dot_f32(static_cast<const float*>(psi), static_cast<const float*>(hp), b->n_elem, red + kRedBlocks,
                          red, s));
  HCHECK(hipMemcpyAsync(E, red + kRedBlocks, sizeof(double), hipMemcpyDeviceToHost, s));
  HCHECK(hipStreamSynchronize(s));
  ABI_END(ctx)
}

extern "C" int heff_energy_backward(heff_ctx* ctx, const heff_blocks* b, int prec, const void* psi, double gE,
                                    void* dpsi, void* dL, void* dR) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!b || !psi) throw Error(HEFF_EINVAL, "null argument");
  if (b->shard_nranks > 1) throw Error(HEFF_ESTATE, "the product is restricted to one shard's output blocks");
  if (prec != HEFF_FP64 && prec != HEFF_FP32) throw Error(HEFF_ENOTSUP, "gradients are available in FP64 and FP32");
  if (dpsi == psi) throw Error(HEFF_EINVAL, "psi and dpsi alias");
  HCHECK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  void* ar[4];
  int64_t n[4];
  arenas(*b, prec, ar, n);
  const bool f64 = prec == HEFF_FP64;
  const size_t es = f64 ? 8 : 4;
  if (dpsi) {
    // E is a symmetric quadratic form: dE/dpsi = 2 H_eff psi
    if (int rc = heff_apply(ctx, b, prec, psi, dpsi)) throw Error(rc, ctx->err);
    if (f64) HCHECK(launch_scale_f64(static_cast<double*>(dpsi), b->n_elem, 2.0 * gE, s));
    else HCHECK(launch_scale_f32(static_cast<float*>(dpsi), b->n_elem, (float)(2.0 * gE), s));
  }
  void* douts[2] = {dL, dR};
  for (int side = 0; side < 2; ++side) {
    void* d = douts[side];
    if (!d) continue;
    if (!b->grad[side].ready) make_grad_plan(*b, side, s);
    const int64_t tot = n[2 * side] + n[2 * side + 1];
    HCHECK(hipMemsetAsync(d, 0, tot * es, s));
    if (f64) run_grad<double>(*b, side, ar, psi, d, s);
    else run_grad<float>(*b, side, ar, psi, d, s);
    if (f64) HCHECK(launch_scale_f64(static_cast<double*>(d), tot, gE, s));
    else HCHECK(launch_scale_f32(static_cast<float*>(d), tot, (float)gE, s));
  }
  ABI_END(ctx)
}

extern "C" int heff_set_fp64_kernel(heff_ctx* ctx, int32_t mode) {
  if (!ctx) return HEFF_EINVAL;
  if (mode < kFp64Auto || mode > kFp64RingDword) {
    ctx->err = "unknown FP64 kernel family";
    return HEFF_EINVAL;
  }
  ctx->fp64_kernel = mode;
  return HEFF_OK;
}

// dE/dh and dE/dV of E = <psi|H_eff(h, V)|psi> (isometries and psi fixed),
// as symmetric tensors.  E is linear in the integrals, so each component is
// an energy: E with the indicator of one symmetry orbit of indices as the
// integrals equals the orbit size times the common component.
extern "C" int heff_integral_gradient(heff_ctx* ctx, const heff_problem* p, const double* psi, double* gh,
                                      double* gV) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!p || !psi) throw Error(HEFF_EINVAL, "null argument");
  Ints I;
  validate_ints(p, I);
  const int n = p->n_orb;
  const size_t n2 = (size_t)n * n;
  std::vector<double> dh(n2, 0.0), dV(n2 * n2, 0.0);
  auto energy_at = [&](double* e) {
    heff_problem q = *p;
    q.h = dh.data();
    q.V = dV.data();
    heff_blocks* bq = nullptr;
    int rc = heff_build_blocks(ctx, &q, 0u, &bq);
    if (rc != HEFF_OK) return rc;
    rc = heff_energy(ctx, bq, HEFF_FP64, psi, e);
    heff_blocks_free(bq);
    return rc;
  };
  if (gh) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j <= i; ++j) {
        dh[(size_t)i * n + j] = dh[(size_t)j * n + i] = 1.0;
        double e = 0.0;
        const int rc = energy_at(&e);
        dh[(size_t)i * n + j] = dh[(size_t)j * n + i] = 0.0;
        if (rc != HEFF_OK) return rc;
        gh[(size_t)i * n + j] = gh[(size_t)j * n + i] = i == j ? e : 0.5 * e;
      }
  }
  if (gV) {
    auto at = [&](int i, int j, int k, int l) { return ((size_t)(i * n + j) * n + k) * n + l; };
    for (int i = 0; i < n; ++i)
      for (int j = 0; j <= i; ++j)
        for (int k = 0; k <= i; ++k)
          for (int l = 0; l <= (k == i ? j : k); ++l) {
            // orbit of (ij|kl): pairs unordered, the two pairs exchangeable
            const size_t m[8] = {at(i, j, k, l), at(j, i, k, l), at(i, j, l, k), at(j, i, l, k),
                                 at(k, l, i, j), at(l, k, i, j), at(k, l, j, i), at(l, k, j, i)};
            std::vector<size_t> orb(m, m + 8);
            std::sort(orb.begin(), orb.end());
            orb.erase(std::unique(orb.begin(), orb.end()), orb.end());
            for (size_t x : orb) dV[x] = 1.0;
            double e = 0.0;
            const int rc = energy_at(&e);
            for (size_t x : orb) dV[x] = 0.0;
            if (rc != HEFF_OK) return rc;
            for (size_t x : orb) gV[x] = e / (double)orb.size();
          }
  }
  ABI_END(ctx)
}

extern "C" int heff_kappa_gradient(heff_ctx* ctx, const heff_problem* p, const double* psi, int32_t n_pairs,
                                   const int32_t* pairs, double* g) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!p || !psi || !g || (n_pairs > 0 && !pairs) || n_pairs < 0) throw Error(HEFF_EINVAL, "null argument");
  Ints I;
  validate_ints(p, I);
  const int n = p->n_orb;
  for (int i = 0; i < n_pairs; ++i) {
    const int x = pairs[2 * i], y = pairs[2 * i + 1];
    if (x < 0 || y < 0 || x >= n || y >= n || x == y) throw Error(HEFF_EINVAL, "bad orbital pair");
  }
  std::vector<double> dh, dV;
  for (int i = 0; i < n_pairs; ++i) {
    rotation_derivative(I, pairs[2 * i], pairs[2 * i + 1], dh, dV);
    heff_problem q = *p;
    q.h = dh.data();
    q.V = dV.data();
    heff_blocks* bq = nullptr;
    int rc = heff_build_blocks(ctx, &q, 0u, &bq);
    if (rc != HEFF_OK) return rc;
    double e = 0.0;
    rc = heff_energy(ctx, bq, HEFF_FP64, psi, &e);
    heff_blocks_free(bq);
    if (rc != HEFF_OK) return rc;
    g[i] = e;
  }
  ABI_END(ctx)
}
