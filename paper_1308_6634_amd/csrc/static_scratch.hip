// Device memory of the no-allocation entry point (plsqr_solve_static): a file-scope device
// array that the runtime places on every GPU the library runs on, held until the process
// ends. A request run through that entry point takes its whole workspace (descriptor,
// scalars, records, Krylov vectors, multigrid levels, reduction partials) from it, so the
// call allocates no device or pinned memory.
//
// In host code `scratch` names a host-side stand-in, not the device address: the address is
// looked up once per device with hipGetSymbolAddress (resolve_scratch, called when an engine
// is created on that device) and only that pointer is used afterwards.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "engine.hpp"

namespace plsqr {

namespace {

__device__ __align__(256) unsigned char scratch[PLSQR_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];   // device address of `scratch` per GPU (null: unresolved)

static_assert(sizeof(InstDesc) % 4 == 0, "descriptor copied as 32-bit words");
static_assert(sizeof(InstDesc) <= 3584, "descriptor passed as a kernel argument (4 KB limit)");

// Writes the request's descriptor (passed by value, so a captured launch keeps its own copy),
// the one-entry descriptor pointer array, and clears the per-outer records, which the caller
// reads back: the scratch keeps whatever the previous call on this GPU left there.
__global__ void __launch_bounds__(256) k_static_setup(InstDesc desc, InstDesc *d_desc,
                                                      InstDesc **d_ptrs, double *records,
                                                      int n_records) {
  const unsigned *src = reinterpret_cast<const unsigned *>(&desc);
  unsigned *dst = reinterpret_cast<unsigned *>(d_desc);
  constexpr int words = (int)(sizeof(InstDesc) / 4);
  for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
  for (int i = threadIdx.x; i < n_records; i += blockDim.x) records[i] = 0.0;
  if (threadIdx.x == 0) d_ptrs[0] = d_desc;
}

}  // namespace

int resolve_scratch(int device, std::string *why) {
  if (device < 0 || device >= kMaxDevices) {
    *why = "device index beyond the static scratch table";
    return PLSQR_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return PLSQR_OK;
  void *p = nullptr;
  // the caller has made `device` current
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    *why = std::string("hipGetSymbolAddress of the static scratch failed: ") + hipGetErrorString(e);
    return PLSQR_E_HIP;
  }
  g_scratch_ptr[device] = p;
  return PLSQR_OK;
}

void *scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

void launch_static_setup(hipStream_t st, const InstDesc &desc, InstDesc *d_desc, InstDesc **d_ptrs,
                         double *records, int n_records) {
  hipLaunchKernelGGL(k_static_setup, dim3(1), dim3(256), 0, st, desc, d_desc, d_ptrs, records,
                     n_records);
}

}  // namespace plsqr
