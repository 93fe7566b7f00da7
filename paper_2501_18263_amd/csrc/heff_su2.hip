// Host runtime of the SU(2) spin-adapted two-site product (Sec. II.C,
// Eq. Hamilton_act_su2): validation of the multiplet problem, the factor
// table F (rescaled Wigner 9j symbols), the task table with one scalar
// prefactor per task, and the product on the matrix-core kernels of the
// U(1) path.
#include "heff_host_common.h"

#include <mutex>
#include <unordered_map>

namespace heff {
namespace su2 {

// ------------------------------------------------------------------ angular momentum
// Spins are doubled integers.  6j symbols by Racah's single-sum formula in
// long double; 9j symbols as the sum over x of (-1)^{2x} (2x+1) times three
// 6j symbols.
static bool tri(int a, int b, int c) { return std::abs(a - b) <= c && c <= a + b && ((a + b + c) & 1) == 0; }

static long double lfact(int n) {
  static std::vector<long double> t;
  static std::once_flag once;
  std::call_once(once, [] {
    t.resize(200);
    t[0] = 0.0L;
    for (int i = 1; i < 200; ++i) t[i] = t[i - 1] + std::log((long double)i);
  });
  if (n < 0 || n >= 200) throw Error(HEFF_EINVAL, "spin too large for the factor table");
  return t[n];
}

// log of Delta(abc) = (a+b-c)!(a-b+c)!(-a+b+c)!/(a+b+c+1)! (all halved)
static long double ldelta(int a, int b, int c) {
  return lfact((a + b - c) / 2) + lfact((a - b + c) / 2) + lfact((-a + b + c) / 2) - lfact((a + b + c) / 2 + 1);
}

static double sixj(int a, int b, int c, int d, int e, int f) {
  if (!tri(a, b, c) || !tri(a, e, f) || !tri(d, b, f) || !tri(d, e, c)) return 0.0;
  const long double pre = 0.5L * (ldelta(a, b, c) + ldelta(a, e, f) + ldelta(d, b, f) + ldelta(d, e, c));
  const int lo = std::max(std::max(a + b + c, a + e + f), std::max(d + b + f, d + e + c)) / 2;
  const int hi = std::min(std::min(a + b + d + e, b + c + e + f), c + a + f + d) / 2;
  long double s = 0.0L;
  for (int t = lo; t <= hi; ++t) {
    const long double l = lfact(t + 1) - lfact(t - (a + b + c) / 2) - lfact(t - (a + e + f) / 2) -
                          lfact(t - (d + b + f) / 2) - lfact(t - (d + e + c) / 2) - lfact((a + b + d + e) / 2 - t) -
                          lfact((b + c + e + f) / 2 - t) - lfact((c + a + f + d) / 2 - t);
    const long double v = std::exp(l + pre);
    s += (t & 1) ? -v : v;
  }
  return (double)s;
}

static double ninej(int a, int b, int c, int d, int e, int f, int g, int h, int i) {
  const int lo = std::max(std::max(std::abs(a - i), std::abs(h - d)), std::abs(b - f));
  const int hi = std::min(std::min(a + i, h + d), b + f);
  long double s = 0.0L;
  for (int x = lo; x <= hi; x += 2) {
    const long double v = (long double)(x + 1) * sixj(a, d, g, h, i, x) * sixj(b, e, h, d, x, f) * sixj(c, f, i, x, a, b);
    s += (x & 1) ? -v : v;
  }
  return (double)s;
}

// F(a, b, c; ka, kb, kc; a', b', c'): reduced element of [A^ka x B^kb]^kc
// between the coupled states (a b)c -> (a' b')c' over <a'||A||a><b'||B||b>.
// Values below 1e-13 are rounding of a structural zero and read as zero.
static double factor_value(const int j[9]) {
  if (!tri(j[0], j[1], j[2]) || !tri(j[3], j[4], j[5]) || !tri(j[6], j[7], j[8]) || !tri(j[0], j[3], j[6]) ||
      !tri(j[1], j[4], j[7]) || !tri(j[2], j[5], j[8]))
    return 0.0;
  const double w = ninej(j[0], j[1], j[2], j[3], j[4], j[5], j[6], j[7], j[8]);
  const double f = std::sqrt((double)(j[6] + 1) * (j[7] + 1) * (j[2] + 1) * (j[5] + 1)) * w;
  return std::fabs(f) < 1e-13 ? 0.0 : f;
}

// lookup table of F, keyed by the nine doubled spins (7 bits each)
struct FactorTable {
  std::unordered_map<uint64_t, double> map;
  double get(const int j[9]) {
    uint64_t key = 0;
    for (int i = 0; i < 9; ++i) {
      if (j[i] < 0 || j[i] > 127) throw Error(HEFF_EINVAL, "spin out of range");
      key = (key << 7) | (uint64_t)j[i];
    }
    auto it = map.find(key);
    if (it != map.end()) return it->second;
    const double v = factor_value(j);
    map.emplace(key, v);
    return v;
  }
};

// ------------------------------------------------------------------ site multiplets and operators
constexpr int kSiteN[3] = {0, 1, 2};
constexpr int kSiteS[3] = {0, 1, 0};
constexpr int kNumSiteOps = 7;
constexpr int kSiteOpK[kNumSiteOps] = {0, 1, 1, 0, 2, 0, 0};
constexpr int kSiteOpDn[kNumSiteOps] = {0, 1, -1, 0, 0, 2, -2};
// reduced elements <m_out||O||m_in> of the site operators (rows m_out,
// columns m_in), from their matrices in the states |0>, |up>, |down>,
// |up down> = c+_up c+_down |0> by the Wigner-Eckart convention above
static const double kSqrt2 = 1.4142135623730951, kSqrt3h = 0.8660254037844386;
static const double kSiteRed[kNumSiteOps][3][3] = {
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},           // identity
    {{0, 0, 0}, {1, 0, 0}, {0, -kSqrt2, 0}},     // creation: <d||a+||0> = 1, <2||a+||d> = -sqrt2
    {{0, -kSqrt2, 0}, {0, 0, -1}, {0, 0, 0}},    // annihilation: <0||a~||d> = -sqrt2, <d||a~||2> = -1
    {{0, 0, 0}, {0, 1, 0}, {0, 0, 2}},           // number
    {{0, 0, 0}, {0, kSqrt3h, 0}, {0, 0, 0}},     // spin vector: <d||T^1||d> = sqrt3 / 2
    {{0, 0, 0}, {0, 0, 0}, {1, 0, 0}},           // pair creation
    {{0, 0, 1}, {0, 0, 0}, {0, 0, 0}},           // pair annihilation
};

struct Sector {
  int n, ts, dim;
};
struct OpBlock {
  int out;
  int64_t off;  // element offset in the block's FP64 arena
};
struct BlockDef {
  std::vector<Sector> sect;
  std::vector<int> two_k, dn;
  // per operator, per input sector: the operator's blocks leaving it
  std::vector<std::vector<std::vector<OpBlock>>> from;
  std::vector<double> data;  // concatenated reduced blocks (arena order)
};

static void check_block(const heff_su2_block& b, const char* what, BlockDef& B) {
  const std::string w(what);
  if (b.n_sect <= 0 || !b.n || !b.two_s || !b.dim) throw Error(HEFF_EINVAL, w + ": no sectors");
  std::set<std::pair<int, int>> seen;
  for (int i = 0; i < b.n_sect; ++i) {
    Sector s{b.n[i], b.two_s[i], b.dim[i]};
    if (s.n < 0 || s.ts < 0 || ((s.n - s.ts) & 1)) throw Error(HEFF_EINVAL, w + ": sector " + std::to_string(i) + " has a spin of the wrong parity");
    if (s.dim <= 0 || s.dim > kMaxDim)
      throw Error(HEFF_EINVAL, w + ": sector " + std::to_string(i) + " dimension outside 1.." + std::to_string(kMaxDim));
    if (!seen.insert({s.n, s.ts}).second) throw Error(HEFF_EINVAL, w + ": repeated sector (n, 2S)");
    B.sect.push_back(s);
  }
  if (b.n_ops < 0 || (b.n_ops > 0 && (!b.two_k || !b.dn))) throw Error(HEFF_EINVAL, w + ": operator table");
  for (int j = 0; j < b.n_ops; ++j) {
    if (b.two_k[j] < 0 || ((b.two_k[j] - b.dn[j]) & 1))
      throw Error(HEFF_EINVAL, w + ": operator " + std::to_string(j) + " rank and particle change of different parity");
    B.two_k.push_back(b.two_k[j]);
    B.dn.push_back(b.dn[j]);
  }
  B.from.assign(b.n_ops, std::vector<std::vector<OpBlock>>(b.n_sect));
  if (b.n_blk < 0 || (b.n_blk > 0 && (!b.blk_op || !b.blk_out || !b.blk_in || !b.blk_off || !b.data)))
    throw Error(HEFF_EINVAL, w + ": block table");
  std::set<std::array<int, 3>> have;
  int64_t total = 0;
  for (int64_t k = 0; k < b.n_blk; ++k) {
    const int j = b.blk_op[k], o = b.blk_out[k], i = b.blk_in[k];
    if (j < 0 || j >= b.n_ops || o < 0 || o >= b.n_sect || i < 0 || i >= b.n_sect)
      throw Error(HEFF_EINVAL, w + ": block " + std::to_string(k) + " index out of range");
    if (B.sect[o].n != B.sect[i].n + B.dn[j] || !tri(B.sect[i].ts, B.two_k[j], B.sect[o].ts))
      throw Error(HEFF_EINVAL, w + ": block " + std::to_string(k) + " violates particle or spin selection");
    if (!have.insert({j, o, i}).second) throw Error(HEFF_EINVAL, w + ": repeated block");
    const int64_t len = (int64_t)B.sect[o].dim * B.sect[i].dim;
    if (b.blk_off[k] < 0 || b.blk_off[k] + len > b.data_len)
      throw Error(HEFF_EINVAL, w + ": block " + std::to_string(k) + " outside the data");
    total += len;
  }
  B.data.reserve((size_t)total + 1);
  for (int64_t k = 0; k < b.n_blk; ++k) {
    const int j = b.blk_op[k], o = b.blk_out[k], i = b.blk_in[k];
    const int64_t len = (int64_t)B.sect[o].dim * B.sect[i].dim;
    for (int64_t e = 0; e < len; ++e) {
      const double v = b.data[b.blk_off[k] + e];
      if (!std::isfinite(v)) throw Error(HEFF_EINVAL, w + ": non-finite operator element");
    }
    B.from[j][i].push_back({o, (int64_t)B.data.size()});
    B.data.insert(B.data.end(), b.data + b.blk_off[k], b.data + b.blk_off[k] + len);
  }
  // output sectors in ascending order (a fixed task order)
  for (auto& per : B.from)
    for (auto& v : per) std::sort(v.begin(), v.end(), [](const OpBlock& x, const OpBlock& y) { return x.out < y.out; });
}

static int ts_of(const BlockDef& B, int op) { return op < 0 ? 0 : B.two_k[op]; }
static int dn_of(const BlockDef& B, int op) { return op < 0 ? 0 : B.dn[op]; }

}  // namespace su2
}  // namespace heff

struct heff_su2 {
  int device = 0;
  uint32_t prec_mask = 0;
  int64_t n_elem = 0;
  std::vector<int32_t> desc;  // 8 per block: il, mk, tsg, mk1, ir, tsd, rows, cols
  std::vector<int64_t> off;
  heff::DevBuf dL, dR, fL, fR;  // FP64 arenas and FP32 copies of the reduced operator blocks
  heff::DevBuf d_tiles, d_tasks;
  heff::DevWorkSet mwork;
  // split task chains: the product writes psi' and then the chains' partial
  // sums into a work vector (FP64; FP32 for the FP32 and bf16-split
  // products), the jobs add the parts into psi', which is copied out
  heff::DevBuf d_red, work64, work32;
  int n_red = 0;
  int64_t n_tasks = 0;
  double flops = 0.0, n_resolved = 0.0;
};

namespace heff {
namespace su2 {

static void to_f32(const DevBuf& src, DevBuf& dst, int64_t n, hipStream_t s) {
  dst.alloc((size_t)std::max<int64_t>(n, 1) * sizeof(float));
  if (n > 0) HCHECK(launch_f64_to_f32(src.as<double>(), dst.as<float>(), n, s));
}

static void build(heff_ctx* ctx, const heff_su2_problem* p, uint32_t prec_mask, heff_su2& H) {
  BlockDef L, R;
  check_block(p->left, "left block", L);
  check_block(p->right, "right block", R);
  if (p->n_terms < 0 || (p->n_terms > 0 && (!p->term_l || !p->term_site_k || !p->term_site_k1 || !p->term_r ||
                                             !p->term_two_s || !p->term_coef)))
    throw Error(HEFF_EINVAL, "term table");
  if (p->two_s_tot < 0 || ((p->n_tot - p->two_s_tot) & 1)) throw Error(HEFF_EINVAL, "total spin of the wrong parity");
  const int nL = (int)L.sect.size(), nR = (int)R.sect.size();
  for (int t = 0; t < p->n_terms; ++t) {
    const int l = p->term_l[t], r = p->term_r[t], sk = p->term_site_k[t], sk1 = p->term_site_k1[t];
    const std::string w = "term " + std::to_string(t);
    if (l < -1 || l >= (int)L.two_k.size() || r < -1 || r >= (int)R.two_k.size())
      throw Error(HEFF_EINVAL, w + ": operator index out of range");
    if (sk < 0 || sk >= kNumSiteOps || sk1 < 0 || sk1 >= kNumSiteOps) throw Error(HEFF_EINVAL, w + ": site operator code");
    if (dn_of(L, l) + kSiteOpDn[sk] + kSiteOpDn[sk1] + dn_of(R, r) != 0)
      throw Error(HEFF_EINVAL, w + ": does not conserve the particle number");
    const int tc = p->term_two_s[t];
    if (!tri(ts_of(L, l), kSiteOpK[sk], tc) || !tri(kSiteOpK[sk1], ts_of(R, r), tc))
      throw Error(HEFF_EINVAL, w + ": rank coupling violates the triangle rule");
    if (!std::isfinite(p->term_coef[t])) throw Error(HEFF_EINVAL, w + ": non-finite coefficient");
  }
  // reduced two-site layout
  std::map<std::array<int, 6>, int> index;
  for (int il = 0; il < nL; ++il)
    for (int mk = 0; mk < 3; ++mk)
      for (int tsg = std::abs(L.sect[il].ts - kSiteS[mk]); tsg <= L.sect[il].ts + kSiteS[mk]; tsg += 2)
        for (int mk1 = 0; mk1 < 3; ++mk1)
          for (int ir = 0; ir < nR; ++ir) {
            if (L.sect[il].n + kSiteN[mk] + kSiteN[mk1] + R.sect[ir].n != p->n_tot) continue;
            for (int tsd = std::abs(kSiteS[mk1] - R.sect[ir].ts); tsd <= kSiteS[mk1] + R.sect[ir].ts; tsd += 2) {
              if (!tri(tsg, tsd, p->two_s_tot)) continue;
              index[{il, mk, tsg, mk1, ir, tsd}] = (int)H.off.size();
              H.desc.insert(H.desc.end(), {il, mk, tsg, mk1, ir, tsd, L.sect[il].dim, R.sect[ir].dim});
              H.off.push_back(H.n_elem);
              H.n_elem += (int64_t)L.sect[il].dim * R.sect[ir].dim;
            }
          }
  if (H.off.empty()) throw Error(HEFF_ESECTOR, "no reduced two-site block has this particle number and spin");
  // magnetic-resolved amplitudes at M = S_tot with the same multiplets
  for (int il = 0; il < nL; ++il)
    for (int sk = 0; sk < 4; ++sk)
      for (int sk1 = 0; sk1 < 4; ++sk1)
        for (int ir = 0; ir < nR; ++ir) {
          const int nk = (sk == 0) ? 0 : (sk == 3 ? 2 : 1), nk1 = (sk1 == 0) ? 0 : (sk1 == 3 ? 2 : 1);
          if (L.sect[il].n + nk + nk1 + R.sect[ir].n != p->n_tot) continue;
          const int mk = (sk == 1) ? 1 : (sk == 2 ? -1 : 0), mk1 = (sk1 == 1) ? 1 : (sk1 == 2 ? -1 : 0);
          int cnt = 0;
          for (int ml = -L.sect[il].ts; ml <= L.sect[il].ts; ml += 2) {
            const int mr = p->two_s_tot - ml - mk - mk1;
            if (std::abs(mr) <= R.sect[ir].ts && ((R.sect[ir].ts - mr) & 1) == 0) ++cnt;
          }
          H.n_resolved += (double)cnt * L.sect[il].dim * R.sect[ir].dim;
        }
  // tasks, Eq. Hamilton_act_su2
  const int nb = (int)H.off.size();
  std::vector<std::vector<Task>> per(nb);
  FactorTable F;
  for (int x = 0; x < nb; ++x) {
    const int* d = &H.desc[8 * x];
    const int il = d[0], mk = d[1], tsg = d[2], mk1 = d[3], ir = d[4], tsd = d[5];
    const int nl = L.sect[il].n;
    for (int t = 0; t < p->n_terms; ++t) {
      const int l = p->term_l[t], r = p->term_r[t], sk = p->term_site_k[t], sk1 = p->term_site_k1[t];
      const int tc = p->term_two_s[t], tA = ts_of(L, l), tD = ts_of(R, r);
      const int oB = kSiteOpDn[sk] & 1, oC = kSiteOpDn[sk1] & 1, oD = dn_of(R, r) & 1;
      const int par = oB * nl + oC * (nl + kSiteN[mk]) + oD * (nl + kSiteN[mk] + kSiteN[mk1]);
      const double base = p->term_coef[t] * ((par & 1) ? -1.0 : 1.0);
      if (base == 0.0) continue;
      std::vector<OpBlock> idl{{il, -1}}, idr{{ir, -1}};
      const std::vector<OpBlock>& lo = l < 0 ? idl : L.from[l][il];
      const std::vector<OpBlock>& ro = r < 0 ? idr : R.from[r][ir];
      for (const OpBlock& lb : lo) {
        const int il2 = lb.out;
        for (int mk2 = 0; mk2 < 3; ++mk2) {
          const double rb = kSiteRed[sk][mk2][mk];
          if (rb == 0.0) continue;
          for (int mk12 = 0; mk12 < 3; ++mk12) {
            const double rc = kSiteRed[sk1][mk12][mk1];
            if (rc == 0.0) continue;
            for (const OpBlock& rbk : ro) {
              const int ir2 = rbk.out;
              const int tl2 = L.sect[il2].ts, tr2 = R.sect[ir2].ts;
              for (int tsg2 = std::abs(tl2 - kSiteS[mk2]); tsg2 <= tl2 + kSiteS[mk2]; tsg2 += 2)
                for (int tsd2 = std::abs(kSiteS[mk12] - tr2); tsd2 <= kSiteS[mk12] + tr2; tsd2 += 2) {
                  auto it = index.find({il2, mk2, tsg2, mk12, ir2, tsd2});
                  if (it == index.end()) continue;
                  const int jl[9] = {L.sect[il].ts, kSiteS[mk], tsg, tA, kSiteOpK[sk], tc, tl2, kSiteS[mk2], tsg2};
                  const double fl = F.get(jl);
                  if (fl == 0.0) continue;
                  const int jr[9] = {kSiteS[mk1], R.sect[ir].ts, tsd, kSiteOpK[sk1], tD, tc, kSiteS[mk12], tr2, tsd2};
                  const double fr = F.get(jr);
                  if (fr == 0.0) continue;
                  const int jt[9] = {tsg, tsd, p->two_s_tot, tc, tc, 0, tsg2, tsd2, p->two_s_tot};
                  const double ft = F.get(jt);
                  if (ft == 0.0) continue;
                  const int y = it->second;
                  Task k{};
                  k.f = base * rb * rc * fl * fr * ft;
                  k.a = (uint16_t)L.sect[il2].dim;
                  k.b = (uint16_t)L.sect[il].dim;
                  k.c = (uint16_t)R.sect[ir].dim;
                  k.e = (uint16_t)R.sect[ir2].dim;
                  k.offX = H.off[x];
                  k.ldX = (uint16_t)R.sect[ir].dim;
                  uint32_t fl_ = 0;
                  if (l < 0) fl_ |= T_IDL;
                  else {
                    k.offL = lb.off;
                    k.ldL = (uint16_t)L.sect[il].dim;
                  }
                  if (r < 0) fl_ |= T_IDR;
                  else {
                    k.offR = rbk.off;  // stored dim_out x dim_in = e x c
                    k.ldR = (uint16_t)R.sect[ir].dim;
                    fl_ |= T_TR;
                  }
                  k.flags = (uint16_t)fl_;
                  per[y].push_back(k);
                }
            }
          }
        }
      }
    }
  }
  std::vector<Tile> tiles(nb);
  std::vector<Task> tasks;
  for (int y = 0; y < nb; ++y) {
    Tile t{};
    t.offOut = H.off[y];
    t.a = H.desc[8 * y + 6];
    t.e = H.desc[8 * y + 7];
    t.ldOut = t.e;
    t.t0 = (int32_t)tasks.size();
    tasks.insert(tasks.end(), per[y].begin(), per[y].end());
    t.t1 = (int32_t)tasks.size();
    tiles[y] = t;
  }
  if (tasks.size() > (size_t)INT32_MAX) throw Error(HEFF_EINVAL, "task table too large");
  for (const Task& k : tasks) H.flops += task_flops(k);
  H.n_tasks = (int64_t)tasks.size();
  // output blocks and middle dimensions of at most 128 columns (column
  // slices, ranges of c), as in the U(1) product: the 256-wide kernel
  // instances hold one work-group per CU and spill (benchmark problem,
  // right sectors up to 256 wide: FP64 233 -> 140 ms, FP32 110 -> 88 ms,
  // bf16 split 112 -> 79 ms on one box)
  split_large(tiles, tasks, kProductDim);
  // the longest output blocks gather thousands of tasks: their chains are
  // split over several work-groups (partial sums, then a fixed-order sum)
  // into parts of at most a quarter of the average work-group slot of the
  // 128-wide kernel (256 CUs, two work-groups each), which leaves the
  // longest-first queues room to balance (benchmark problem, FP64 / FP32 /
  // bf16 split: 512 slots and 8 parts 105 / 60 / 53 ms, 1024 and 8 100 /
  // 51 / 41 ms, 2048 and 16 99 / 50 / 42 ms on one box)
  std::vector<RedJob> jobs;
  const int64_t part_elems = split_chains(tiles, tasks, 2048, 16, H.n_elem, jobs);
  const int nt_ = (int)tiles.size();
  std::vector<int> order(nt_);
  for (int i = 0; i < nt_; ++i) order[i] = i;
  std::vector<Work> lists[kNumVariants];
  split_work(tiles, tasks, order, lists);
  hipStream_t s = ctx->stream;
  H.mwork.upload_lists(lists, s);
  upload(H.d_tiles, tiles, s);
  upload(H.d_tasks, tasks, s);
  H.n_red = (int)jobs.size();
  if (H.n_red) {
    upload(H.d_red, jobs, s);
    const size_t nw = (size_t)(H.n_elem + part_elems);
    H.work64.alloc(nw * sizeof(double));
    if (prec_mask & ((1u << HEFF_FP32) | (1u << HEFF_BF16X3))) H.work32.alloc(nw * sizeof(float));
  }
  upload(H.dL, L.data, s);
  upload(H.dR, R.data, s);
  H.prec_mask = prec_mask | (1u << HEFF_FP64);
  if (prec_mask & ((1u << HEFF_FP32) | (1u << HEFF_BF16X3))) {
    to_f32(H.dL, H.fL, (int64_t)L.data.size(), s);
    to_f32(H.dR, H.fR, (int64_t)R.data.size(), s);
  }
  HCHECK(hipStreamSynchronize(s));
}

}  // namespace su2
}  // namespace heff

using namespace heff;

extern "C" int heff_su2_create(heff_ctx* ctx, const heff_su2_problem* p, uint32_t prec_mask, heff_su2** out) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!p || !out) throw Error(HEFF_EINVAL, "null argument");
  *out = nullptr;
  if (prec_mask & ~((1u << HEFF_FP64) | (1u << HEFF_FP32) | (1u << HEFF_BF16X3)))
    throw Error(HEFF_EINVAL, "unknown precision bits");
  HCHECK(hipSetDevice(ctx->device));
  auto H = std::make_unique<heff_su2>();
  H->device = ctx->device;
  su2::build(ctx, p, prec_mask, *H);
  *out = H.release();
  ABI_END(ctx)
}

extern "C" int heff_su2_layout(const heff_su2* h, int64_t* n_elem, int32_t* n_blk, const int32_t** desc,
                               const int64_t** off) {
  if (!h) return HEFF_EINVAL;
  if (n_elem) *n_elem = h->n_elem;
  if (n_blk) *n_blk = (int32_t)h->off.size();
  if (desc) *desc = h->desc.data();
  if (off) *off = h->off.data();
  return HEFF_OK;
}

extern "C" int heff_su2_stats(const heff_su2* h, int64_t* n_tasks, double* flops, double* n_resolved) {
  if (!h) return HEFF_EINVAL;
  if (n_tasks) *n_tasks = h->n_tasks;
  if (flops) *flops = h->flops;
  if (n_resolved) *n_resolved = h->n_resolved;
  return HEFF_OK;
}

extern "C" int heff_su2_apply(heff_ctx* ctx, const heff_su2* h, int prec, const void* psi, void* out) {
  if (!ctx) return HEFF_EINVAL;
  ABI_BEGIN
  if (!h || !psi || !out) throw Error(HEFF_EINVAL, "null argument");
  if (psi == out) throw Error(HEFF_EINVAL, "psi and out alias");
  if (h->device != ctx->device) throw Error(HEFF_EINVAL, "built on another device");
  HCHECK(hipSetDevice(ctx->device));
  Bases<double> b64{};
  b64.L[0] = b64.L[1] = h->dL.as<double>();
  b64.R[0] = b64.R[1] = h->dR.as<double>();
  set_limits(b64, h->dL, h->dL, h->n_elem, h->dR, h->dR);
  Bases<float> b32{};
  b32.L[0] = b32.L[1] = h->fL.as<float>();
  b32.R[0] = b32.R[1] = h->fR.as<float>();
  if (!h->n_red) {
    run_product(ctx, h->d_tiles.as<Tile>(), h->d_tasks.as<Task>(), h->mwork.ws, prec, h->prec_mask, b64, b32, psi, out);
  } else {
    // into the work vector; after the variants joined the context stream,
    // the parts are added into psi' and psi' is copied out
    const bool f64 = prec == HEFF_FP64;
    void* w = f64 ? h->work64.p : h->work32.p;
    if (!w) throw Error(HEFF_ENOTSUP, "precision not built for this SU(2) problem");
    run_product(ctx, h->d_tiles.as<Tile>(), h->d_tasks.as<Task>(), h->mwork.ws, prec, h->prec_mask, b64, b32, psi, w);
    if (f64)
      HCHECK(launch_reduce_parts_f64(h->d_red.as<RedJob>(), h->n_red, h->work64.as<double>(), h->work64.as<double>(),
                                     ctx->stream));
    else
      HCHECK(launch_reduce_parts_f32(h->d_red.as<RedJob>(), h->n_red, h->work32.as<float>(), h->work32.as<float>(),
                                     ctx->stream));
    HCHECK(hipMemcpyAsync(out, w, (size_t)h->n_elem * (f64 ? sizeof(double) : sizeof(float)), hipMemcpyDeviceToDevice,
                          ctx->stream));
  }
  ABI_END(ctx)
}

extern "C" int heff_su2_free(heff_su2* h) {
  if (!h) return HEFF_EINVAL;
  (void)hipSetDevice(h->device);
  delete h;
  return HEFF_OK;
}

extern "C" int heff_su2_factor(const int32_t two_j[9], double* F) {
  if (!two_j || !F) return HEFF_EINVAL;
  try {
    int j[9];
    for (int i = 0; i < 9; ++i) {
      if (two_j[i] < 0 || two_j[i] > 127) return HEFF_EINVAL;
      j[i] = two_j[i];
    }
    *F = su2::factor_value(j);
  } catch (const Error& e) {
    return e.code;
  }
  return HEFF_OK;
}
