// CPU host check of the library's host code (test infrastructure only).
//
// Implements the HIP runtime calls of hip/hip_runtime.h over host memory and
// replaces every kernel launcher of csrc/heff_internal.h by a checker: a
// launch computes nothing; it verifies, for every work item, tile and task
// it would run, that each operand block, output block and table entry lies
// inside one live allocation, that identity operands have matching
// dimensions and that blocks fit the kernel variant they are queued on.
// Launches issued while a stream is being captured are recorded and run
// (checked) again at every graph launch, with the arguments captured then.
//
// "Device" allocations are anonymous private mappings reserved without
// backing, so operator arenas that no stub ever writes cost no memory;
// fills with zero are checked but not performed (fresh mappings are zero).
// Violations are counted and printed; HOSTCHECK_ABORT=1 aborts at the first.
#include "heff_internal.h"

#include <sys/mman.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <unordered_set>
#include <vector>

struct hc_stream { int id; };
struct hc_event { int id; };
struct hc_graph { std::vector<std::function<void()>> ops; };
struct hc_graph_exec { std::vector<std::function<void()>> ops; };

namespace hc {

struct Region { size_t bytes, mapped; };
static std::map<uintptr_t, Region> g_allocs;
static std::mutex g_mu;
static long g_violations = 0, g_launches = 0, g_items = 0, g_tasks = 0;
static size_t g_live = 0, g_peak = 0;
static thread_local hc_graph* g_capture = nullptr;

static void violation(const char* fmt, ...) {
  ++g_violations;
  if (g_violations <= 50) {
    va_list ap;
    va_start(ap, fmt);
    std::fprintf(stderr, "hostcheck violation: ");
    std::vfprintf(stderr, fmt, ap);
    std::fprintf(stderr, "\n");
    va_end(ap);
  }
  const char* a = std::getenv("HOSTCHECK_ABORT");
  if (a && a[0] == '1') std::abort();
}

// allocation containing address p (nullptr if none)
static const std::pair<const uintptr_t, Region>* find(const void* p) {
  std::lock_guard<std::mutex> lk(g_mu);
  const uintptr_t a = (uintptr_t)p;
  auto it = g_allocs.upper_bound(a);
  if (it == g_allocs.begin()) return nullptr;
  --it;
  if (a >= it->first + it->second.bytes) return nullptr;
  return &*it;
}

// [p, p + bytes) inside one live allocation
static bool inside(const void* p, size_t bytes) {
  if (bytes == 0) return true;
  const auto* r = find(p);
  return r && (uintptr_t)p + bytes <= r->first + r->second.bytes;
}

static bool check_range(const void* p, size_t bytes, const char* what) {
  if (inside(p, bytes)) return true;
  violation("%s: [%p, +%zu bytes) is not inside one device allocation", what, p, bytes);
  return false;
}

// elements of size es from p to the end of its allocation (-1: none)
static int64_t elems_to_end(const void* p, size_t es) {
  const auto* r = find(p);
  if (!r) return -1;
  return (int64_t)((r->first + r->second.bytes - (uintptr_t)p) / es);
}

static hipError_t run(std::function<void()> f) {
  ++g_launches;
  if (g_capture) g_capture->ops.push_back(std::move(f));
  else f();
  return hipSuccess;
}

// stored block: `rows` x `cols` (row stride ld) at base + off
template <typename T>
static void check_block(const T* base, int64_t off, int64_t rows, int64_t cols, int64_t ld, const char* what,
                        int64_t task) {
  if (rows <= 0 || cols <= 0) return;
  if (!base) { violation("%s of task %lld: null base", what, (long long)task); return; }
  if (ld < cols) violation("%s of task %lld: row stride %lld below %lld columns", what, (long long)task, (long long)ld,
                           (long long)cols);
  if (off < 0) { violation("%s of task %lld: negative offset", what, (long long)task); return; }
  const int64_t last = off + (rows - 1) * ld + cols;
  if (!inside(base, (size_t)last * sizeof(T)))
    violation("%s of task %lld: elements [%lld, %lld) of a %lld-element buffer", what, (long long)task,
              (long long)off, (long long)last, (long long)elems_to_end(base, sizeof(T)));
}

template <typename T>
static void check_task(const heff::Task& t, int64_t k, const heff::Tile& tile, const heff::Bases<T>& b, int wmax) {
  using namespace heff;
  ++g_tasks;
  const uint32_t f = t.flags;
  if (t.a != tile.a || t.e != tile.e)
    violation("task %lld: %dx%d output part in a %dx%d tile", (long long)k, t.a, t.e, tile.a, tile.e);
  if (t.c > wmax) violation("task %lld: middle dimension %d above the variant's %d", (long long)k, t.c, wmax);
  if ((f & T_IDL) && t.a != t.b) violation("task %lld: identity op(L) with a=%d b=%d", (long long)k, t.a, t.b);
  if ((f & T_IDX) && t.b != t.c) violation("task %lld: identity op(X) with b=%d c=%d", (long long)k, t.b, t.c);
  if ((f & T_IDR) && t.c != t.e) violation("task %lld: identity op(R) with c=%d e=%d", (long long)k, t.c, t.e);
  if (!(f & T_IDL)) {
    const T* base = b.L[(f & T_SELL) ? 1 : 0];
    if (f & T_TL) check_block(base, t.offL, t.b, t.a, t.ldL, "op(L)", k);
    else check_block(base, t.offL, t.a, t.b, t.ldL, "op(L)", k);
  }
  if (!(f & T_IDX)) {
    const T* base = b.X[(f & T_SELX) ? 1 : 0];
    if (f & T_TX) check_block(base, t.offX, t.c, t.b, t.ldX, "op(X)", k);
    else check_block(base, t.offX, t.b, t.c, t.ldX, "op(X)", k);
  }
  if (!(f & T_IDR)) {
    const T* base = b.R[(f & T_SELR) ? 1 : 0];
    if (f & T_TR) check_block(base, t.offR, t.e, t.c, t.ldR, "op(R)", k);
    else check_block(base, t.offR, t.c, t.e, t.ldR, "op(R)", k);
  }
}

// lim[j]: elements readable at the j-th base (L0, L1, X0, X1, R0, R1) as the
// host declares them to the 16-byte loads of the FP64 ring kernel
template <typename T>
static void check_limits(const heff::Bases<T>& b) {
  const T* base[6] = {b.L[0], b.L[1], b.X[0], b.X[1], b.R[0], b.R[1]};
  for (int j = 0; j < 6; ++j) {
    if (b.lim[j] <= 0 || !base[j]) continue;
    const int64_t real = elems_to_end(base[j], sizeof(T));
    if (b.lim[j] > real)
      violation("declared length %lld of base %d exceeds the %lld elements of its allocation", (long long)b.lim[j],
                j, (long long)real);
  }
}

// every work item of every variant; bases_of(tile) gives the operand bases
template <typename T, typename F>
static void check_chain(const heff::Tile* tiles, const heff::WorkSet& ws, const heff::Task* tasks, F bases_of) {
  using namespace heff;
  for (int v = 0; v < kNumVariants; ++v) {
    if (ws.n[v] <= 0) continue;
    if (!check_range(ws.w[v], (size_t)ws.n[v] * sizeof(Work), "work list")) continue;
    const int wmax = 32 << v;
    std::unordered_set<int> seen;
    for (int64_t i = 0; i < ws.n[v]; ++i) {
      const Work w = ws.w[v][i];
      if (w.row0 < 0) continue;
      ++g_items;
      if (w.tile < 0 || !check_range(tiles + w.tile, sizeof(Tile), "tile of a work item")) continue;
      const Tile tile = tiles[w.tile];
      if (w.row0 % kTileRows != 0 || w.row0 >= tile.a)
        violation("work item %lld of variant %d: first row %d of a %d-row tile", (long long)i, v, w.row0, tile.a);
      if (!seen.insert(w.tile).second) continue;
      const Bases<T> b = bases_of(tile);
      if (tile.e > wmax) violation("tile %d: width %d on the %d-wide variant", w.tile, tile.e, wmax);
      if (tile.ldOut < tile.e) violation("tile %d: output stride %d below width %d", w.tile, tile.ldOut, tile.e);
      if (tile.a > 0 && tile.e > 0) {
        const int64_t last = tile.offOut + (int64_t)(tile.a - 1) * tile.ldOut + tile.e;
        if (!b.out || tile.offOut < 0 || !inside(b.out, (size_t)last * sizeof(T)))
          violation("tile %d: output elements [%lld, %lld) outside the output buffer", w.tile,
                    (long long)tile.offOut, (long long)last);
      }
      if (tile.t0 < 0 || tile.t1 < tile.t0) { violation("tile %d: task range [%d, %d)", w.tile, tile.t0, tile.t1); continue; }
      if (tile.t1 > tile.t0 && !check_range(tasks + tile.t0, (size_t)(tile.t1 - tile.t0) * sizeof(Task), "task range"))
        continue;
      for (int k = tile.t0; k < tile.t1; ++k) check_task<T>(tasks[k], k, tile, b, wmax);
    }
  }
}

}  // namespace hc

// ------------------------------------------------------------------ runtime
hipError_t hipMalloc(void** p, size_t bytes) {
  if (!p) return hipErrorInvalidValue;
  const size_t pg = 4096, mapped = std::max<size_t>((bytes + pg - 1) / pg * pg, pg);
  void* m = mmap(nullptr, mapped, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
  if (m == MAP_FAILED) { *p = nullptr; return hipErrorOutOfMemory; }
  std::lock_guard<std::mutex> lk(hc::g_mu);
  hc::g_allocs[(uintptr_t)m] = {std::max<size_t>(bytes, 1), mapped};
  hc::g_live += bytes;
  hc::g_peak = std::max(hc::g_peak, hc::g_live);
  *p = m;
  return hipSuccess;
}

hipError_t hipFree(void* p) {
  if (!p) return hipSuccess;
  std::lock_guard<std::mutex> lk(hc::g_mu);
  auto it = hc::g_allocs.find((uintptr_t)p);
  if (it == hc::g_allocs.end()) {
    hc::g_mu.unlock();
    hc::violation("hipFree of %p, which is not the start of a live allocation", p);
    hc::g_mu.lock();
    return hipErrorInvalidValue;
  }
  munmap(p, it->second.mapped);
  hc::g_live -= std::min(hc::g_live, it->second.bytes);
  hc::g_allocs.erase(it);
  return hipSuccess;
}

hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  if (bytes == 0) return hipSuccess;
  if ((kind == hipMemcpyHostToDevice || kind == hipMemcpyDeviceToDevice) && !hc::check_range(dst, bytes, "copy destination"))
    return hipErrorInvalidValue;
  if ((kind == hipMemcpyDeviceToHost || kind == hipMemcpyDeviceToDevice) && !hc::check_range(src, bytes, "copy source"))
    return hipErrorInvalidValue;
  std::memmove(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t) {
  return hipMemcpy(dst, src, bytes, kind);
}
hipError_t hipMemcpy2DAsync(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width, size_t height,
                            hipMemcpyKind kind, hipStream_t) {
  if (height == 0 || width == 0) return hipSuccess;
  const size_t dspan = (height - 1) * dpitch + width, sspan = (height - 1) * spitch + width;
  if ((kind == hipMemcpyHostToDevice || kind == hipMemcpyDeviceToDevice) && !hc::check_range(dst, dspan, "2D copy destination"))
    return hipErrorInvalidValue;
  if ((kind == hipMemcpyDeviceToHost || kind == hipMemcpyDeviceToDevice) && !hc::check_range(src, sspan, "2D copy source"))
    return hipErrorInvalidValue;
  for (size_t r = 0; r < height; ++r) std::memmove((char*)dst + r * dpitch, (const char*)src + r * spitch, width);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t) {
  if (!hc::check_range(dst, bytes, "fill")) return hipErrorInvalidValue;
  if (value != 0) std::memset(dst, value, bytes);
  return hipSuccess;
}
hipError_t hipSetDevice(int device) { return device == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetDevice(int* device) { if (device) *device = 0; return hipSuccess; }
hipError_t hipGetDeviceCount(int* n) { if (n) *n = 1; return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new hc_stream{1}; return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned) { return e ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = new hc_event{1}; return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = new hc_event{1}; return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { return e ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipEventSynchronize(hipEvent_t e) { return e ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { if (ms) *ms = 0.f; return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) {
  if (hc::g_capture) return hipErrorInvalidValue;
  hc::g_capture = new hc_graph;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  if (!hc::g_capture) return hipErrorInvalidValue;
  *g = hc::g_capture;
  hc::g_capture = nullptr;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  if (!g) return hipErrorInvalidValue;
  *x = new hc_graph_exec{g->ops};
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t) {
  if (!x) return hipErrorInvalidValue;
  for (auto& f : x->ops) f();
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t x) { delete x; return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "host-check runtime error"; }

// ------------------------------------------------------------------ launch checkers
namespace heff {

template <typename T>
static hipError_t checked_chain(const Tile* tiles, const WorkSet& ws, const Task* tasks, Bases<T> b) {
  return hc::run([=]() {
    hc::check_limits(b);
    hc::check_chain<T>(tiles, ws, tasks, [&](const Tile&) { return b; });
  });
}

hipError_t launch_mfma_f64(const Tile* tiles, const WorkSet& ws, const Task* tasks, Bases<double> b,
                           const hipStream_t*, hipEvent_t (*)[2], int) {
  return checked_chain(tiles, ws, tasks, b);
}
hipError_t launch_mfma_f32(const Tile* tiles, const WorkSet& ws, const Task* tasks, Bases<float> b,
                           const hipStream_t*, hipEvent_t (*)[2]) {
  return checked_chain(tiles, ws, tasks, b);
}
hipError_t launch_bf16x3(const Tile* tiles, const WorkSet& ws, const Task* tasks, Bases<float> b,
                         const hipStream_t*, hipEvent_t (*)[2]) {
  return checked_chain(tiles, ws, tasks, b);
}

hipError_t launch_mfma_batch_f32(const Tile* tiles, const WorkSet& ws, const Task* tasks, const ProbBases<float>* pb,
                                 const float* X, float* out, const int grid[kNumVariants], const hipStream_t*) {
  int g[kNumVariants];
  for (int v = 0; v < kNumVariants; ++v) g[v] = grid[v];
  return hc::run([=]() {
    for (int v = 0; v < kNumVariants; ++v)
      if (ws.n[v] > 0 && g[v] <= 0) hc::violation("batched variant %d: persistent grid %d", v, g[v]);
    hc::check_chain<float>(tiles, ws, tasks, [&](const Tile& t) {
      Bases<float> b{};
      if (t.prob < 0 || !hc::check_range(pb + t.prob, sizeof(ProbBases<float>), "problem bases")) return b;
      b.L[0] = pb[t.prob].L[0];
      b.L[1] = pb[t.prob].L[1];
      b.R[0] = pb[t.prob].R[0];
      b.R[1] = pb[t.prob].R[1];
      b.X[0] = b.X[1] = X;
      b.out = out;
      return b;
    });
  });
}

template <typename T>
static hipError_t checked_reduce(const RedJob* jobs, int n_jobs, const T* part, T* out) {
  return hc::run([=]() {
    if (n_jobs <= 0) return;
    if (!hc::check_range(jobs, (size_t)n_jobs * sizeof(RedJob), "reduction jobs")) return;
    for (int i = 0; i < n_jobs; ++i) {
      const RedJob j = jobs[i];
      ++hc::g_items;
      if (j.a <= 0 || j.e <= 0 || j.parts < 2 || j.ld < j.e || j.out_off < 0 || j.part_off < 0) {
        hc::violation("reduction job %d: a=%d e=%d ld=%d parts=%d", i, j.a, j.e, j.ld, j.parts);
        continue;
      }
      const int64_t last = j.out_off + (int64_t)(j.a - 1) * j.ld + j.e;
      if (!out || !hc::inside(out, (size_t)last * sizeof(T))) hc::violation("reduction job %d: output outside", i);
      const int64_t plast = j.part_off + (int64_t)j.parts * j.a * j.e;
      if (!part || !hc::inside(part, (size_t)plast * sizeof(T))) hc::violation("reduction job %d: parts outside", i);
    }
  });
}
hipError_t launch_reduce_parts_f64(const RedJob* jobs, int n_jobs, const double* part, double* out, hipStream_t) {
  return checked_reduce(jobs, n_jobs, part, out);
}
hipError_t launch_reduce_parts_f32(const RedJob* jobs, int n_jobs, const float* part, float* out, hipStream_t) {
  return checked_reduce(jobs, n_jobs, part, out);
}

hipError_t launch_diag(const Tile* tiles, int64_t n_tiles, const DiagTask* tasks, const double* L0, const double* L1,
                       const double* R0, const double* R1, double* out, hipStream_t) {
  return hc::run([=]() {
    if (!hc::check_range(tiles, (size_t)n_tiles * sizeof(Tile), "diagonal tiles")) return;
    for (int64_t i = 0; i < n_tiles; ++i) {
      const Tile t = tiles[i];
      if (t.a > 0 && t.e > 0 && !hc::inside(out, (size_t)(t.offOut + (int64_t)(t.a - 1) * t.ldOut + t.e) * 8))
        hc::violation("diagonal tile %lld: output outside the buffer", (long long)i);
      if (t.t1 > t.t0 && !hc::check_range(tasks + t.t0, (size_t)(t.t1 - t.t0) * sizeof(DiagTask), "diagonal tasks"))
        continue;
      for (int k = t.t0; k < t.t1; ++k) {
        const DiagTask d = tasks[k];
        if (!(d.flags & T_IDL)) hc::check_block((d.flags & T_SELL) ? L1 : L0, d.offL, t.a, t.a, t.a, "diag(L)", k);
        if (!(d.flags & T_IDR)) hc::check_block((d.flags & T_SELR) ? R1 : R0, d.offR, t.e, t.e, t.e, "diag(R)", k);
      }
    }
  });
}

hipError_t launch_rotate_pair(const RotJob* jobs, int64_t n_jobs, const double* in, double* out, hipStream_t) {
  return hc::run([=]() {
    if (!hc::check_range(jobs, (size_t)n_jobs * sizeof(RotJob), "rotation jobs")) return;
    for (int64_t i = 0; i < n_jobs; ++i) {
      const RotJob j = jobs[i];
      if (j.nterm < 0 || j.nterm > 4) hc::violation("rotation job %lld: %d terms", (long long)i, j.nterm);
      hc::check_range(out + j.off_out, (size_t)j.n * 8, "rotation output block");
      for (int t = 0; t < j.nterm && t < 4; ++t) hc::check_range(in + j.off_in[t], (size_t)j.n * 8, "rotation input block");
    }
  });
}

hipError_t launch_gemm_f64(int64_t m, int64_t n, int64_t k, const double* A, const double* B, double* C,
                           hipStream_t) {
  return hc::run([=]() {
    hc::check_range(A, (size_t)(m * k) * 8, "gemm A");
    hc::check_range(B, (size_t)(k * n) * 8, "gemm B");
    hc::check_range(C, (size_t)(m * n) * 8, "gemm C");
  });
}

hipError_t launch_bj_round(const BjJob* jobs, int n_jobs, double* B, double* WT, unsigned long long* off_max, int r,
                           double, hipStream_t) {
  return hc::run([=]() {
    if (!hc::check_range(jobs, (size_t)n_jobs * sizeof(BjJob), "block-Jacobi jobs")) return;
    for (int i = 0; i < n_jobs; ++i) {
      const BjJob j = jobs[i];
      if (j.K % 2 || j.pr < 0 || j.pr >= j.K / 2) hc::violation("block-Jacobi job %d: pair %d of %d blocks", i, j.pr, j.K);
      if ((j.K - 1) * kBjRows >= j.m + kBjRows * 2) hc::violation("block-Jacobi job %d: %d blocks for %d rows", i, j.K, j.m);
      hc::check_range(B + j.b_off, (size_t)j.m * j.c * 8, "block-Jacobi rows of B");
      hc::check_range(WT + j.w_off, (size_t)j.m * j.m * 8, "block-Jacobi rows of W^T");
      hc::check_range(off_max + j.sector, 8, "block-Jacobi convergence slot");
    }
    (void)r;
  });
}

hipError_t launch_copy_blocks(const CopyJob* jobs, int n_jobs, const double* src, double* dst, hipStream_t) {
  return hc::run([=]() {
    if (!hc::check_range(jobs, (size_t)n_jobs * sizeof(CopyJob), "copy jobs")) return;
    for (int i = 0; i < n_jobs; ++i) {
      const CopyJob j = jobs[i];
      if (j.cols > j.ld) hc::violation("copy job %d: %d columns into stride %d", i, j.cols, j.ld);
      hc::check_range(src + j.src, (size_t)j.rows * j.cols * 8, "copy source block");
      if (j.rows > 0) hc::check_range(dst + j.dst, (size_t)((j.rows - 1) * (int64_t)j.ld + j.cols) * 8, "copy destination block");
    }
  });
}

hipError_t launch_identity(const int64_t* woff, const int32_t* m, int n_sect, double* WT, hipStream_t) {
  return hc::run([=]() {
    if (!hc::check_range(woff, (size_t)n_sect * 8, "identity offsets") || !hc::check_range(m, (size_t)n_sect * 4, "identity sizes"))
      return;
    for (int q = 0; q < n_sect; ++q) hc::check_range(WT + woff[q], (size_t)m[q] * m[q] * 8, "identity matrix");
  });
}

hipError_t launch_row_norms(const int64_t* boff, const int32_t* m, const int32_t* c, const int64_t* soff, int n_sect,
                            const double* B, double* sig, hipStream_t) {
  return hc::run([=]() {
    for (int q = 0; q < n_sect; ++q) {
      hc::check_range(B + boff[q], (size_t)m[q] * c[q] * 8, "row-norm rows");
      hc::check_range(sig + soff[q], (size_t)m[q] * 8, "row norms");
    }
  });
}

hipError_t launch_gather_rows(const GatherJob* jobs, int n_jobs, const double* WT, double* out, hipStream_t) {
  return hc::run([=]() {
    if (!hc::check_range(jobs, (size_t)n_jobs * sizeof(GatherJob), "gather jobs")) return;
    for (int i = 0; i < n_jobs; ++i) {
      const GatherJob g = jobs[i];
      if (!hc::check_range(g.cols, (size_t)g.ncol * 4, "gather rows")) continue;
      for (int c = 0; c < g.ncol; ++c) {
        if (g.cols[c] < 0 || g.cols[c] >= g.n) hc::violation("gather job %d: row %d of %d", i, g.cols[c], g.n);
        else hc::check_range(WT + g.v_off + (int64_t)g.cols[c] * g.n, (size_t)g.n * 8, "gathered row");
      }
      hc::check_range(out + g.out_off, (size_t)g.n * g.ncol * 8, "gather destination");
    }
  });
}

hipError_t launch_convert_f32(const double* in, float* out, int64_t n, hipStream_t) {
  return hc::run([=]() { hc::check_range(in, (size_t)n * 8, "convert source"); hc::check_range(out, (size_t)n * 4, "convert destination"); });
}
hipError_t launch_f64_to_f32(const double* in, float* out, int64_t n, hipStream_t s) { return launch_convert_f32(in, out, n, s); }
hipError_t launch_f32_to_f64(const float* in, double* out, int64_t n, hipStream_t) {
  return hc::run([=]() { hc::check_range(in, (size_t)n * 4, "convert source"); hc::check_range(out, (size_t)n * 8, "convert destination"); });
}
hipError_t launch_multidot(const double* A, int64_t lda, int k, const double* x, int64_t n, double* out, double* scratch,
                           hipStream_t) {
  return hc::run([=]() {
    if (k > 0) hc::check_range(A, (size_t)((k - 1) * lda + n) * 8, "multidot A");
    hc::check_range(x, (size_t)n * 8, "multidot x");
    hc::check_range(out, (size_t)k * 8, "multidot out");
    (void)scratch;
  });
}
hipError_t launch_multiaxpy(const double* A, int64_t lda, int k, const double* coef, double, double* y, double, int64_t n,
                            hipStream_t) {
  return hc::run([=]() {
    if (k > 0) hc::check_range(A, (size_t)((k - 1) * lda + n) * 8, "multiaxpy A");
    hc::check_range(coef, (size_t)k * 8, "multiaxpy coefficients");
    hc::check_range(y, (size_t)n * 8, "multiaxpy y");
  });
}
hipError_t launch_dot_f64(const double* x, const double* y, int64_t n, double* out, double* scratch, hipStream_t) {
  return hc::run([=]() {
    hc::check_range(x, (size_t)n * 8, "dot x");
    hc::check_range(y, (size_t)n * 8, "dot y");
    hc::check_range(out, 8, "dot out");
    hc::check_range(scratch, (size_t)kRedBlocks * 8, "dot scratch");
  });
}
hipError_t launch_dot_f32(const float* x, const float* y, int64_t n, double* out, double* scratch, hipStream_t) {
  return hc::run([=]() {
    hc::check_range(x, (size_t)n * 4, "dot x");
    hc::check_range(y, (size_t)n * 4, "dot y");
    hc::check_range(out, 8, "dot out");
    hc::check_range(scratch, (size_t)kRedBlocks * 8, "dot scratch");
  });
}
hipError_t launch_scale_f64(double* x, int64_t n, double, hipStream_t) {
  return hc::run([=]() { hc::check_range(x, (size_t)n * 8, "scale x"); });
}
hipError_t launch_scale_f32(float* x, int64_t n, float, hipStream_t) {
  return hc::run([=]() { hc::check_range(x, (size_t)n * 4, "scale x"); });
}

}  // namespace heff

// the allocation-free energy's static scratch lives in device code, which
// this host-only build does not compile
hipError_t heff::noalloc_setup(int) { return hipSuccess; }

// summary of what was checked (called by the driver)
extern "C" void hostcheck_report(long* violations, long* launches, long* items, long* tasks, size_t* peak_bytes,
                                 size_t* live_bytes, long* live_allocs) {
  *violations = hc::g_violations;
  *launches = hc::g_launches;
  *items = hc::g_items;
  *tasks = hc::g_tasks;
  *peak_bytes = hc::g_peak;
  *live_bytes = hc::g_live;
  *live_allocs = (long)hc::g_allocs.size();
}
