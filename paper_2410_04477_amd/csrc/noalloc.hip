// vecchia_loglik_noalloc: the value path of vecchia_loglik with its per-call
// buffers in a static device array instead of the plan's workspace, for
// callers that cannot allocate device memory at call time.
//
// The array below is one per GPU the library runs on (the code object is
// loaded per device) and lives until the process ends.  In host code its name
// is only a host-side stand-in: the kernels receive the device address that
// hipGetSymbolAddress returns for the current device, resolved once per
// device and kept in g_addr.
#include <mutex>

#include "internal.hpp"

using namespace bv;

namespace {

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Layout of the array for VECCHIA_NOALLOC_MAX_ITEMS (theta, block) work items:
// per-block terms (FP64), flags, compaction list (int32), class counters.
constexpr size_t kItems = VECCHIA_NOALLOC_MAX_ITEMS;
constexpr size_t kOffPartial = 0;
constexpr size_t kOffFlag = align256(kOffPartial + sizeof(double) * kItems);
constexpr size_t kOffList = align256(kOffFlag + sizeof(int) * kItems);
constexpr size_t kOffCount = align256(kOffList + sizeof(int) * kItems);
constexpr size_t kBytes = align256(kOffCount + sizeof(int) * 64);
static_assert(kBytes == VECCHIA_NOALLOC_SCRATCH_BYTES, "header constant out of date");

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void* g_addr[kMaxDevices];
hipError_t g_err[kMaxDevices];

}  // namespace

static __device__ __align__(256) unsigned char scratch[kBytes];

int bv::noalloc_prepare_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return VECCHIA_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return VECCHIA_EUNSUPPORTED;
  std::call_once(g_once[dev], [dev]() {
    void* p = nullptr;
    g_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_addr[dev] = g_err[dev] == hipSuccess ? p : nullptr;
  });
  return g_err[dev] == hipSuccess && g_addr[dev] ? VECCHIA_OK : VECCHIA_EHIP;
}

extern "C" size_t vecchia_noalloc_scratch_bytes(void) { return kBytes; }

extern "C" int vecchia_loglik_noalloc(const vecchia_plan* plan, const double* locs_perm, const double* y_perm,
                                      int32_t d, const int32_t* block_ptr, const int32_t* nbr_ptr,
                                      const int32_t* nbr_idx, const vecchia_theta* theta, int32_t ntheta,
                                      int32_t precision, double* loglik, int32_t* counters, double* partial,
                                      void* stream) {
  int st = check_loglik_args(plan, locs_perm, y_perm, d, block_ptr, nbr_ptr, nbr_idx, theta, ntheta, precision,
                             loglik, false);
  if (st) return st;
  // blocks above the one-wave limit are factored in the auxiliary workspace
  if (plan->nlarge > 0) return VECCHIA_EUNSUPPORTED;
  if ((size_t)plan->bc * (size_t)ntheta > kItems) return VECCHIA_ENOMEM;
  st = noalloc_prepare_current_device();
  if (st) return st;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return VECCHIA_EHIP;
  char* base = static_cast<char*>(g_addr[dev]);
  CallBuffers cb;
  cb.partial = reinterpret_cast<double*>(base + kOffPartial);
  cb.flag = reinterpret_cast<int*>(base + kOffFlag);
  cb.list = reinterpret_cast<int*>(base + kOffList);
  cb.count = reinterpret_cast<int*>(base + kOffCount);
  return loglik_run(plan, locs_perm, y_perm, d, block_ptr, nbr_ptr, nbr_idx, theta, ntheta, precision, loglik,
                    counters, partial, cb, stream);
}
