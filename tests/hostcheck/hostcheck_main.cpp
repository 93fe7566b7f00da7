// Driver of the CPU host check (test infrastructure only): reads two-site
// problems from a file written by tests/test_hostcheck.py, runs the
// library's C ABI on them with the host-only runtime (build of the blocks
// and task tables with FP32 operands, single products in every precision,
// the diagonal, a sweep step to the next pair with its product and the mode
// rotation of that pair (rotation, entropies, angle search), and a batch
// of all problems with plain and graph-replayed launches), and reports what
// the launch checkers found.
//
// Problem file (little endian): "HEFFPRB1", int32 count, then per problem
// int32 n_orb, n_up, n_dn; double h[n^2]; double V[n^4];
// int32 n_left; per left bond: int32 n_sect, int32 nup[], ndn[], dim[];
// int32 n_right; per right bond likewise;
// int32 n_iso_left; per isometry: int64 len, double[len];
// int32 n_iso_right; per isometry likewise.
//
// SU(2) mode (``--su2 file``): "HEFFSU21", int32 count, then per problem two
// blocks (int32 n_sect; int32 n[], two_s[], dim[]; int32 n_ops; int32
// two_k[], dn[]; int64 n_blk; int32 op[], out[], in[]; int64 off[]; int64
// data_len; double data[]), int32 n_terms; int32 l[], site_k[], site_k1[],
// r[], two_s[]; double coef[]; int32 n_tot, two_s_tot.  Each problem is
// created with FP32 operands and applied in every precision.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "heff.h"
#include "hip/hip_runtime.h"

extern "C" void hostcheck_report(long* violations, long* launches, long* items, long* tasks, size_t* peak_bytes,
                                 size_t* live_bytes, long* live_allocs);

namespace {

struct BondData {
  std::vector<int32_t> nup, ndn, dim;
};

struct ProblemData {
  int32_t n, nu, nd;
  std::vector<double> h, V;
  std::vector<BondData> left, right;
  std::vector<std::vector<double>> iso_l, iso_r;
  std::vector<heff_bond> lb, rb;
  std::vector<const double*> il, ir;
  heff_problem p{};
};

struct Reader {
  FILE* f;
  template <typename T>
  T get() {
    T v;
    if (std::fread(&v, sizeof(T), 1, f) != 1) { std::fprintf(stderr, "truncated problem file\n"); std::exit(2); }
    return v;
  }
  template <typename T>
  void arr(std::vector<T>& v, size_t n) {
    v.resize(n);
    if (n && std::fread(v.data(), sizeof(T), n, f) != n) { std::fprintf(stderr, "truncated problem file\n"); std::exit(2); }
  }
  void bonds(std::vector<BondData>& out) {
    out.resize(get<int32_t>());
    for (auto& b : out) {
      const int32_t ns = get<int32_t>();
      arr(b.nup, ns);
      arr(b.ndn, ns);
      arr(b.dim, ns);
    }
  }
  void isos(std::vector<std::vector<double>>& out) {
    out.resize(get<int32_t>());
    for (auto& a : out) arr(a, (size_t)get<int64_t>());
  }
};

void finish(ProblemData& d) {
  for (auto& b : d.left) d.lb.push_back({(int32_t)b.dim.size(), b.nup.data(), b.ndn.data(), b.dim.data()});
  for (auto& b : d.right) d.rb.push_back({(int32_t)b.dim.size(), b.nup.data(), b.ndn.data(), b.dim.data()});
  for (auto& a : d.iso_l) d.il.push_back(a.data());
  for (auto& a : d.iso_r) d.ir.push_back(a.data());
  d.p.n_orb = d.n;
  d.p.n_up = d.nu;
  d.p.n_dn = d.nd;
  d.p.h = d.h.data();
  d.p.V = d.V.data();
  d.p.left = d.lb.data();
  d.p.right = d.rb.data();
  d.p.iso_left = d.il.data();
  d.p.iso_right = d.ir.data();
}

int fail(heff_ctx* ctx, const char* what, int rc) {
  std::fprintf(stderr, "%s failed: %d (%s)\n", what, rc, ctx ? heff_last_error(ctx) : "");
  return 1;
}

struct Su2Block {
  std::vector<int32_t> n, ts, dim, two_k, dn, op, out, in;
  std::vector<int64_t> off;
  std::vector<double> data;
  heff_su2_block b{};
};

void read_su2_block(Reader& r, Su2Block& d) {
  const int32_t ns = r.get<int32_t>();
  r.arr(d.n, ns);
  r.arr(d.ts, ns);
  r.arr(d.dim, ns);
  const int32_t no = r.get<int32_t>();
  r.arr(d.two_k, no);
  r.arr(d.dn, no);
  const int64_t nb = r.get<int64_t>();
  r.arr(d.op, nb);
  r.arr(d.out, nb);
  r.arr(d.in, nb);
  r.arr(d.off, nb);
  r.arr(d.data, (size_t)r.get<int64_t>());
  d.b = {ns, d.n.data(), d.ts.data(), d.dim.data(), no, d.two_k.data(), d.dn.data(), nb, d.op.data(), d.out.data(),
         d.in.data(), d.off.data(), d.data.data(), (int64_t)d.data.size()};
}

int run_su2(const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) { std::perror(path); return 2; }
  Reader r{f};
  char magic[8];
  if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, "HEFFSU21", 8) != 0) {
    std::fprintf(stderr, "not an SU(2) problem file\n");
    return 2;
  }
  heff_ctx* ctx = nullptr;
  int rc = heff_create(&ctx, 0, nullptr, nullptr);
  if (rc) return fail(nullptr, "heff_create", rc);
  const int32_t count = r.get<int32_t>();
  long long n_tasks = 0;
  double flops = 0.0;
  for (int i = 0; i < count; ++i) {
    Su2Block L, R;
    read_su2_block(r, L);
    read_su2_block(r, R);
    const int32_t nt = r.get<int32_t>();
    std::vector<int32_t> tl, tk, tk1, tr, tts;
    std::vector<double> tc;
    r.arr(tl, nt);
    r.arr(tk, nt);
    r.arr(tk1, nt);
    r.arr(tr, nt);
    r.arr(tts, nt);
    r.arr(tc, nt);
    heff_su2_problem p{};
    p.left = L.b;
    p.right = R.b;
    p.n_terms = nt;
    p.term_l = tl.data();
    p.term_site_k = tk.data();
    p.term_site_k1 = tk1.data();
    p.term_r = tr.data();
    p.term_two_s = tts.data();
    p.term_coef = tc.data();
    p.n_tot = r.get<int32_t>();
    p.two_s_tot = r.get<int32_t>();
    heff_su2* h = nullptr;
    if ((rc = heff_su2_create(ctx, &p, (1u << HEFF_FP32) | (1u << HEFF_BF16X3), &h))) return fail(ctx, "heff_su2_create", rc);
    int64_t ne = 0, tasks = 0;
    double fl = 0.0, nres = 0.0;
    heff_su2_layout(h, &ne, nullptr, nullptr, nullptr);
    heff_su2_stats(h, &tasks, &fl, &nres);
    n_tasks += tasks;
    flops += fl;
    void *x = nullptr, *y = nullptr;
    hipMalloc(&x, (size_t)ne * 8);
    hipMalloc(&y, (size_t)ne * 8);
    for (int prec : {HEFF_FP64, HEFF_FP32, HEFF_BF16X3})
      if ((rc = heff_su2_apply(ctx, h, prec, x, y))) return fail(ctx, "heff_su2_apply", rc);
    hipFree(x);
    hipFree(y);
    heff_su2_free(h);
  }
  std::fclose(f);
  heff_destroy(ctx);
  long viol, launches, items, tasks, live_allocs;
  size_t peak, live;
  hostcheck_report(&viol, &launches, &items, &tasks, &peak, &live, &live_allocs);
  std::printf("{\"problems\": %d, \"tasks\": %lld, \"flops\": %.6e, \"launches\": %ld, \"work_items_checked\": %ld, "
              "\"tasks_checked\": %ld, \"violations\": %ld, \"peak_device_bytes\": %zu, \"leaked_bytes\": %zu, "
              "\"leaked_allocations\": %ld}\n",
              count, n_tasks, flops, launches, items, tasks, viol, peak, live, live_allocs);
  return viol ? 1 : 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc == 3 && std::strcmp(argv[1], "--su2") == 0) return run_su2(argv[2]);
  if (argc < 2) {
    std::fprintf(stderr, "usage: %s problems.bin [--no-single]\n", argv[0]);
    return 2;
  }
  const bool single = !(argc > 2 && std::strcmp(argv[2], "--no-single") == 0);
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) { std::perror(argv[1]); return 2; }
  Reader r{f};
  char magic[8];
  if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, "HEFFPRB1", 8) != 0) {
    std::fprintf(stderr, "not a problem file\n");
    return 2;
  }
  const int32_t count = r.get<int32_t>();
  std::vector<std::unique_ptr<ProblemData>> probs;
  for (int i = 0; i < count; ++i) {
    auto d = std::make_unique<ProblemData>();
    d->n = r.get<int32_t>();
    d->nu = r.get<int32_t>();
    d->nd = r.get<int32_t>();
    r.arr(d->h, (size_t)d->n * d->n);
    r.arr(d->V, (size_t)d->n * d->n * d->n * d->n);
    r.bonds(d->left);
    r.bonds(d->right);
    r.isos(d->iso_l);
    r.isos(d->iso_r);
    finish(*d);
    probs.push_back(std::move(d));
  }
  std::fclose(f);

  heff_ctx* ctx = nullptr;
  int rc = heff_create(&ctx, 0, nullptr, nullptr);
  if (rc) return fail(nullptr, "heff_create", rc);
  std::vector<heff_blocks*> blocks;
  std::vector<int64_t> n_elem;
  double flops = 0.0;
  int64_t n_tasks = 0;
  for (int i = 0; i < count; ++i) {
    heff_blocks* b = nullptr;
    rc = heff_build_blocks(ctx, &probs[i]->p, (1u << HEFF_FP32) | (1u << HEFF_BF16X3) | (single ? HEFF_KEEP_ENV : 0u),
                           &b);
    if (rc) return fail(ctx, ("heff_build_blocks of problem " + std::to_string(i)).c_str(), rc);
    int64_t ne = 0, nt = 0;
    int32_t nb = 0;
    const int32_t* desc = nullptr;
    const int64_t* off = nullptr;
    double fl = 0.0;
    heff_psi_layout(b, &ne, &nb, &desc, &off);
    heff_task_stats(b, &nt, &fl, nullptr);
    flops += fl;
    n_tasks += nt;
    std::printf("problem %d: N=%d (%d up, %d down), psi %lld, tasks %lld\n", i, probs[i]->n, probs[i]->nu,
                probs[i]->nd, (long long)ne, (long long)nt);
    std::fflush(stdout);
    if (single) {
      void *x = nullptr, *y = nullptr;
      hipMalloc(&x, (size_t)ne * 8);
      hipMalloc(&y, (size_t)ne * 8);
      if ((rc = heff_apply(ctx, b, HEFF_FP64, x, y))) return fail(ctx, "heff_apply FP64", rc);
      if ((rc = heff_apply(ctx, b, HEFF_FP32, x, y))) return fail(ctx, "heff_apply FP32", rc);
      if ((rc = heff_apply(ctx, b, HEFF_BF16X3, x, y))) return fail(ctx, "heff_apply BF16X3", rc);
      if ((rc = heff_diag(ctx, b, (double*)y))) return fail(ctx, "heff_diag", rc);
      // each rank's share of a three-way output-block shard, then the full
      // product's lists again
      for (int rk = 0; rk < 3; ++rk) {
        double sf = 0.0;
        if ((rc = heff_blocks_shard(ctx, b, rk, 3, &sf))) return fail(ctx, "heff_blocks_shard", rc);
        if ((rc = heff_apply(ctx, b, HEFF_FP64, x, y))) return fail(ctx, "heff_apply of a shard", rc);
      }
      if ((rc = heff_blocks_shard(ctx, b, 0, 1, nullptr))) return fail(ctx, "heff_blocks_shard (full)", rc);
      {  // operand gradients (their task tables take the output blocks whole)
        void* ap[4] = {};
        int64_t an[4] = {};
        if ((rc = heff_op_arena(b, HEFF_FP64, ap, an))) return fail(ctx, "heff_op_arena", rc);
        void *dL = nullptr, *dR = nullptr, *dpsi = nullptr;
        hipMalloc(&dL, (size_t)std::max<int64_t>(an[0] + an[1], 1) * 8);
        hipMalloc(&dR, (size_t)std::max<int64_t>(an[2] + an[3], 1) * 8);
        hipMalloc(&dpsi, (size_t)ne * 8);
        if ((rc = heff_energy_backward(ctx, b, HEFF_FP64, x, 1.0, dpsi, dL, dR)))
          return fail(ctx, "heff_energy_backward", rc);
        hipFree(dL);
        hipFree(dR);
        hipFree(dpsi);
      }
      if (probs[i]->n - (probs[i]->n / 2 - 1) - 2 >= 1) {  // a sweep step to the next pair, then its product
        heff_blocks* b2 = nullptr;
        heff_trunc* tr = nullptr;
        if ((rc = heff_sweep_right(ctx, b, (const double*)x, 24, 1u, &b2, &tr))) return fail(ctx, "heff_sweep_right", rc);
        const double* st = nullptr;
        if ((rc = heff_start_vector(b2, &st))) return fail(ctx, "heff_start_vector", rc);
        int64_t ne2 = 0;
        int32_t nb2 = 0;
        heff_psi_layout(b2, &ne2, &nb2, &desc, &off);
        void* y2 = nullptr;
        hipMalloc(&y2, (size_t)ne2 * 8);
        if ((rc = heff_apply(ctx, b2, HEFF_FP64, st, y2))) return fail(ctx, "heff_apply after the sweep step", rc);
        double th = 0.0, sb = 0.0, sa = 0.0, sh = 0.0, sv = 0.0;
        int32_t ne_ = 0;
        if ((rc = heff_rotate_pair(ctx, b2, 0.3, st, (double*)y2))) return fail(ctx, "heff_rotate_pair", rc);
        // no arithmetic runs here, so the vectors are zero and the entropies
        // refuse them (HEFF_EINVAL) after the rotation and SVD launches
        if ((rc = heff_pair_entropy(ctx, b2, st, &sh, &sv)) && rc != HEFF_EINVAL) return fail(ctx, "heff_pair_entropy", rc);
        if ((rc = heff_optimize_pair(ctx, b2, st, (double*)y2, &th, &sb, &sa, &ne_)) && rc != HEFF_EINVAL)
          return fail(ctx, "heff_optimize_pair", rc);
        hipFree(y2);
        heff_trunc_free(tr);
        heff_blocks_free(b2);
      }
      hipFree(x);
      hipFree(y);
    }
    blocks.push_back(b);
    n_elem.push_back(ne);
  }
  int64_t total = 0;
  std::vector<int64_t> offs(count);
  if ((rc = heff_batch_layout(blocks.data(), count, offs.data(), &total))) return fail(ctx, "heff_batch_layout", rc);
  void *x = nullptr, *y = nullptr;
  hipMalloc(&x, (size_t)std::max<int64_t>(total, 1) * 4);
  hipMalloc(&y, (size_t)std::max<int64_t>(total, 1) * 4);
  heff_batch* bt = nullptr;
  if ((rc = heff_batch_create(ctx, blocks.data(), count, (float*)x, (float*)y, &bt))) return fail(ctx, "heff_batch_create", rc);
  if ((rc = heff_batch_apply(ctx, bt, 0))) return fail(ctx, "heff_batch_apply (plain)", rc);
  const int grids[4] = {256, 512, 1024, 2048};
  for (int g : grids) {  // the autotuner's sweep: every grid drops and recaptures the graph
    const int32_t gg[4] = {g, g, g, g};
    if ((rc = heff_batch_set_grid(bt, gg))) return fail(ctx, "heff_batch_set_grid", rc);
    for (int rep = 0; rep < 2; ++rep)
      if ((rc = heff_batch_apply(ctx, bt, 1))) return fail(ctx, "heff_batch_apply (graph)", rc);
  }
  heff_batch_free(bt);
  hipFree(x);
  hipFree(y);
  for (auto* b : blocks) heff_blocks_free(b);
  heff_destroy(ctx);
  long viol, launches, items, tasks, live_allocs;
  size_t peak, live;
  hostcheck_report(&viol, &launches, &items, &tasks, &peak, &live, &live_allocs);
  std::printf("{\"problems\": %d, \"tasks\": %lld, \"flops\": %.6e, \"launches\": %ld, \"work_items_checked\": %ld, "
              "\"tasks_checked\": %ld, \"violations\": %ld, \"peak_device_bytes\": %zu, \"leaked_bytes\": %zu, "
              "\"leaked_allocations\": %ld}\n",
              count, (long long)n_tasks, flops, launches, items, tasks, viol, peak, live, live_allocs);
  return viol ? 1 : 0;
}
