// ace_apply_noalloc: the ACE apply with its scratch (the coefficient matrix
// C = dV psi xi^T and the fixed-order split-K partial products) in a static
// device array of the library instead of the caller's workspace, for callers
// that cannot allocate.  Same kernels and launch sequence as ace_apply.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ace.h"
#include "kernels.h"

namespace {

// One copy per device, held until the process ends.
static __device__ __align__(256) unsigned char scratch[ACE_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {nullptr};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Device address of this device's scratch array, looked up once per device
// with that device current.  Host code never uses the array's own name.
int scratch_of_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return acex::apply_hip_fail(e);
  if (dev < 0 || dev >= kMaxDevices) return ACE_ERR_ARG;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return acex::apply_hip_fail(e != hipSuccess ? e : hipErrorUnknown);
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return ACE_OK;
}

}  // namespace

extern "C" int ace_apply_noalloc(const ace_plan* p, void* stream, const double* xi,
                                 const double* psi, int n_vec, double* out) {
  int rc = acex::apply_check(p, xi, psi, n_vec, out);
  if (rc != ACE_OK) return rc;
  // C, then as many split-K partial products as fit (at most ace_apply's own
  // count, at least one)
  const size_t c_bytes = align256((size_t)n_vec * acex::apply_orbitals(p) * sizeof(double));
  const size_t part_bytes = (size_t)n_vec * acex::apply_orbitals(p) * sizeof(double);
  if (c_bytes + part_bytes > (size_t)ACE_NOALLOC_SCRATCH_BYTES) return ACE_ERR_SIZE;
  size_t ns = acex::apply_splits(p, n_vec);
  const size_t fit = ((size_t)ACE_NOALLOC_SCRATCH_BYTES - c_bytes) / part_bytes;
  if (ns > fit) ns = fit;
  if (!acex::apply_device_present()) return ACE_ERR_NODEV;
  void* base = nullptr;
  rc = scratch_of_current_device(&base);
  if (rc != ACE_OK) return rc;
  char* w = static_cast<char*>(base);
  return acex::apply_enqueue(p, static_cast<hipStream_t>(stream), reinterpret_cast<double*>(w),
                             reinterpret_cast<double*>(w + c_bytes), (int)ns, xi, psi, n_vec, out);
}
