// Host-side helpers shared by the translation units of the library's host
// code: error type and HIP check, device buffers on the context's memory
// provider, work lists of the matrix-core kernels, the C-ABI exception
// boundary, and the product planning and launch helpers.
#pragma once

#include "heff_internal.h"
#include "../../include/heff.h"

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <set>
#include <unordered_set>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

namespace heff {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HCHECK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess)                                                                  \
      throw Error(HEFF_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));              \
  } while (0)

// C-ABI calls on a context allocate through its provider
struct AllocScope {
  Alloc saved;
  explicit AllocScope(const heff_ctx* c) : saved(tl_alloc) { tl_alloc = c ? c->alloc : Alloc{}; }
  ~AllocScope() { tl_alloc = saved; }
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  Alloc al;  // provider p came from
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void alloc(size_t n) {
    release();
    if (n == 0) n = 256;
    al = tl_alloc;
    p = dev_alloc(n, al);
    if (!p) throw Error(HEFF_ENOMEM, "device allocation of " + std::to_string(n) + " bytes failed");
    bytes = n;
  }
  void release() {
    dev_free(p, al);
    p = nullptr;
    bytes = 0;
  }
  template <typename T>
  T* as() const { return reinterpret_cast<T*>(p); }
};

template <typename T>
inline void upload(DevBuf& d, const std::vector<T>& v, hipStream_t s) {
  d.alloc(v.size() * sizeof(T));
  if (!v.empty()) HCHECK(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

struct DevWorkSet {
  DevBuf buf[kNumVariants];
  WorkSet ws{};
  void upload_lists(std::vector<Work> (&lists)[kNumVariants], hipStream_t s) {
    for (int v = 0; v < kNumVariants; ++v) {
      upload(buf[v], lists[v], s);
      ws.w[v] = buf[v].as<Work>();
      ws.n[v] = (int64_t)lists[v].size();
    }
  }
};

// product planning and launch helpers (heff_host.hip)
int tile_dim(const Tile& t, const std::vector<Task>& tasks);
int64_t split_chains(std::vector<Tile>& tiles, const std::vector<Task>& tasks, int slots, int max_parts,
                     int64_t part_base, std::vector<RedJob>& jobs);
bool split_large(std::vector<Tile>& tiles, std::vector<Task>& tasks, int max_dim, std::vector<int>* parent = nullptr);
double task_flops(const Task& t);
void split_work(const std::vector<Tile>& tiles, const std::vector<Task>& tasks, const std::vector<int>& order,
                std::vector<Work> (&lists)[kNumVariants], const std::vector<int>* key = nullptr);
int64_t elems64(const DevBuf& d);
void set_limits(Bases<double>& b, const DevBuf& l0, const DevBuf& l1, int64_t x, const DevBuf& r0, const DevBuf& r1);
void fork_variants(heff_ctx* c, hipStream_t out[kNumVariants]);
void join_variants(heff_ctx* c);
// one product of a task table on the context's stream: psi and out fill the
// X and out slots of the bases of precision prec (HEFF_FP64: b64; HEFF_FP32
// and HEFF_BF16X3: b32, refused unless prec_mask has the bit); the kernel
// variants run on forked streams, timed when the context times
void run_product(heff_ctx* ctx, const Tile* tl, const Task* tk, const WorkSet& ws, int prec, uint32_t prec_mask,
                 Bases<double> b64, Bases<float> b32, const void* psi, void* out);

}  // namespace heff

#define ABI_BEGIN                    \
  heff::AllocScope alloc_scope_(ctx); \
  try {
#define ABI_END(ctx)                                                \
  }                                                                 \
  catch (const Error& e) {                                          \
    if (ctx) (ctx)->err = e.what();                                 \
    return e.code;                                                  \
  }                                                                 \
  catch (const std::bad_alloc&) {                                   \
    if (ctx) (ctx)->err = "host allocation failed";                 \
    return HEFF_ENOMEM;                                             \
  }                                                                 \
  catch (const std::exception& e) {                                 \
    if (ctx) (ctx)->err = e.what();                                 \
    return HEFF_EINVAL;                                             \
  }                                                                 \
  return HEFF_OK;

