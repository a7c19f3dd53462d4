// Fixed device workspace of stag_apply_m_noalloc: one array per GPU, resident until the process ends.
//
// M = 4 m^2 - D_eo D_oe needs two things beyond its input and output: the parameter block of the
// batched Dslash launch (problem table and per-RHS scalars) and the odd-parity temporary D_oe in.
// stag_apply_m keeps both in lattice workspace that grows with hipMalloc; the no-allocation variant
// places them in the array below and writes the parameter block with a kernel whose arguments carry
// it, so the call issues only kernel launches (nothing a stream capture cannot record, no memset, no
// host-to-device copy from host memory that may change before a replay).
//
// Layout of the array: [0, kParamBytes) parameter block (ProbDev at 0, Scal[nrhs] at kScalOffset),
// then the FP64 odd temporary [nrhs][V/2][3] complex128.
#include <mutex>

#include "noalloc.h"

namespace stag {

namespace {

constexpr size_t kScalOffset = 1024;
static_assert(sizeof(ProbDev) <= kScalOffset, "problem table must fit before the scalars");
static_assert(kScalOffset + sizeof(Scal) * kNoAllocMaxRhs <= kNoAllocParamBytes, "parameter block size");

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};  // device address of `scratch` on each GPU (null until looked up)

struct ParamArgs {
  ProbDev pd;
  double mass4[kNoAllocMaxRhs];
  int nrhs;
};

__global__ __launch_bounds__(kNoAllocMaxRhs) void k_noalloc_params(ParamArgs a, unsigned char* base) {
  const int r = threadIdx.x;
  if (r == 0) *reinterpret_cast<ProbDev*>(base) = a.pd;
  if (r < a.nrhs) {
    Scal z{};
    z.mass4 = a.mass4[r];
    reinterpret_cast<Scal*>(base + kScalOffset)[r] = z;
  }
}

}  // namespace

hipError_t noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_addr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_addr[device] = p;
  return hipSuccess;
}

hipError_t noalloc_address(int device, unsigned char** out) {
  *out = nullptr;
  hipError_t e = noalloc_init(device);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_mu);
  *out = static_cast<unsigned char*>(g_addr[device]);
  return hipSuccess;
}

hipError_t noalloc_write_params(unsigned char* base, const ProbDev& pd, const double* mass, int nrhs,
                                hipStream_t st) {
  if (nrhs < 1 || nrhs > kNoAllocMaxRhs) return hipErrorInvalidValue;
  ParamArgs a{};
  a.pd = pd;
  for (int r = 0; r < nrhs; ++r) a.mass4[r] = 4.0 * mass[r] * mass[r];
  a.nrhs = nrhs;
  k_noalloc_params<<<1, kNoAllocMaxRhs, 0, st>>>(a, base);
  return hipGetLastError();
}

size_t noalloc_scal_offset() { return kScalOffset; }

}  // namespace stag
