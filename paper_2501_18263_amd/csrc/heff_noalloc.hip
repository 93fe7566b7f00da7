// Allocation-free form of heff_energy for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid it).  heff_energy keeps H psi and the partial sums
// of its dot product in a scratch buffer taken from the context's memory
// provider; here that scratch is one file-scope device array of fixed size,
// resident on every device the library runs on until the process ends.
//
// Host code never passes the array's name to a kernel or copy: its device
// address, different on every device, is taken once per device with
// hipGetSymbolAddress when a context is created on it (noalloc_setup) and
// kept in a per-device table.
#include <mutex>

#include "heff_internal.h"
#include "../../include/heff.h"

namespace heff {
// H psi part of the scratch (the largest psi accepted: 6291456 FP64 or
// 12582912 FP32 elements), then the kRedBlocks + 1 doubles of the dot
// product's partial sums and result
constexpr size_t kNoAllocVecBytes = size_t(48) << 20;
constexpr size_t kNoAllocBytes = kNoAllocVecBytes + (((kRedBlocks + 1) * sizeof(double) + 255) / 256) * 256;
constexpr int kMaxDevices = 64;
}  // namespace heff

static __device__ __align__(256) unsigned char scratch[heff::kNoAllocBytes];

namespace {
std::mutex g_mu;
void* g_scratch[heff::kMaxDevices] = {};  // device address of `scratch` per device
}  // namespace

// Called by heff_create with `device` current: records the device address
// of the scratch array on it (once per device).
hipError_t heff::noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch[device] = p;
  return hipSuccess;
}

static void* scratch_of(int device) {
  if (device < 0 || device >= heff::kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_scratch[device];
}

extern "C" int heff_energy_noalloc(heff_ctx* ctx, const heff_blocks* b, int prec, const void* psi, double* E) {
  using namespace heff;
  if (!ctx) return HEFF_EINVAL;
  if (!b || !psi || !E) {
    ctx->err = "null argument";
    return HEFF_EINVAL;
  }
  if (blocks_sharded(b)) {
    ctx->err = "the product is restricted to one shard's output blocks";
    return HEFF_ESTATE;
  }
  if (prec != HEFF_FP64 && prec != HEFF_FP32) {
    ctx->err = "energy is available in FP64 and FP32";
    return HEFF_ENOTSUP;
  }
  const int64_t n = blocks_n_elem(b);
  const size_t es = prec == HEFF_FP64 ? 8 : 4;
  if ((size_t)n * es > kNoAllocVecBytes) {
    ctx->err = "psi of " + std::to_string(n) + " elements (" + std::to_string((size_t)n * es) +
               " bytes) exceeds the " + std::to_string(kNoAllocVecBytes) + "-byte static scratch of heff_energy_noalloc";
    return HEFF_EINVAL;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) {
    ctx->err = "hipSetDevice failed";
    return HEFF_EHIP;
  }
  char* base = static_cast<char*>(scratch_of(ctx->device));
  if (!base) {
    ctx->err = "static scratch address not recorded for this device";
    return HEFF_ESTATE;
  }
  // the product writes every element of H psi; no timing events are made
  const bool timing = ctx->timing;
  ctx->timing = false;
  int rc = heff_apply(ctx, b, prec, psi, base);
  ctx->timing = timing;
  if (rc != HEFF_OK) return rc;
  double* red = reinterpret_cast<double*>(base + kNoAllocVecBytes);
  hipStream_t s = ctx->stream;
  hipError_t e = prec == HEFF_FP64
                     ? launch_dot_f64(static_cast<const double*>(psi), reinterpret_cast<const double*>(base), n,
                                      red + kRedBlocks, red, s)
                     : launch_dot_f32(static_cast<const float*>(psi), reinterpret_cast<const float*>(base), n,
                                      red + kRedBlocks, red, s);
  if (e == hipSuccess) e = hipMemcpyAsync(E, red + kRedBlocks, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    ctx->err = std::string("heff_energy_noalloc: ") + hipGetErrorString(e);
    return HEFF_EHIP;
  }
  return HEFF_OK;
}
