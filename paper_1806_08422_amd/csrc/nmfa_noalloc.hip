// Energies of caller-supplied spin vectors without any allocation (nmfa_energies_of_noalloc).
//
// The exact-energy kernels on the int8 matrix cores need two scratch buffers: the zero-padded
// signs [roundup(R, 64)][Np8] and R 64-bit partial sums. nmfa_energies_of allocates them per
// call; this variant takes them from one fixed device array instead, so that callers that cannot
// allocate (code under HIP graph capture, tight serving loops) can evaluate Eq. 1. The kernels
// are the ones nmfa_energies_of launches, so the results are identical.
#include <hip/hip_runtime.h>

#include <mutex>

#include "nmfa_ctx.h"
#include "nmfa_internal.h"

// The scratch array. In host code this name is only a stand-in for the symbol: the device
// address comes from hipGetSymbolAddress, once per device, and only that address is used.
static __device__ __align__(256) unsigned char scratch[NMFA_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Device address of `scratch` on `device`, which must be current. Looked up on the first call on
// that device and kept until the process ends.
hipError_t scratch_ptr(int device, unsigned char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace

extern "C" int nmfa_energies_of_noalloc(nmfa_ctx* c, int32_t R, const int8_t* d_spins, double* d_E,
                                        int64_t* d_E_int, void* hip_stream) {
  if (!c || !d_spins || !d_E || R < 1) return nmfa_fail(NMFA_EINVAL, "nmfa_energies_of_noalloc: invalid argument");
  if (c->device < 0 || c->device >= kMaxDevices)
    return nmfa_fail(NMFA_EINVAL, "nmfa_energies_of_noalloc: device %d out of range", c->device);
  const hipStream_t st = (hipStream_t)hip_stream;
  size_t sp_bytes = 0, need = 0;
  if (c->d_J8) {
    sp_bytes = align256((size_t)((R + 63) / 64) * 64 * (size_t)c->Np8);
    need = sp_bytes + (size_t)R * 8;
    if (need > (size_t)NMFA_NOALLOC_SCRATCH_BYTES)
      return nmfa_fail(NMFA_EINVAL,
                       "nmfa_energies_of_noalloc: R = %d replicas of n = %d spins need %zu bytes of scratch, "
                       "more than the fixed %zu",
                       R, c->n, need, (size_t)NMFA_NOALLOC_SCRATCH_BYTES);
  }
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess && c->d_J8) {
    unsigned char* base = nullptr;
    e = scratch_ptr(c->device, &base);
    // the partial sums start at zero: launch_energy_i8 clears them with a fill kernel
    if (e == hipSuccess)
      e = nmfa::launch_energy_i8(c->d_J8, c->Np8, c->d_h, c->h_integral ? 1 : 0, d_spins, c->n, R,
                                 reinterpret_cast<int8_t*>(base),
                                 reinterpret_cast<unsigned long long*>(base + sp_bytes),
                                 reinterpret_cast<long long*>(d_E_int), d_E, st);
  } else if (e == hipSuccess) {
    e = nmfa::launch_energy(nullptr, c->d_J64, c->d_h, c->exact_int ? 1 : 0, d_spins, c->n, R,
                            reinterpret_cast<long long*>(d_E_int), d_E, st);
  }
  // energies that are not exact integers are reported as 0, as nmfa_energies_of does
  if (e == hipSuccess && d_E_int && !c->exact_int)
    e = nmfa::launch_zero_words(reinterpret_cast<uint32_t*>(d_E_int), 0, 2 * (size_t)R, 0, 0, st);
  if (e != hipSuccess) return nmfa_fail(NMFA_EDEVICE, "nmfa_energies_of_noalloc: %s", hipGetErrorString(e));
  return NMFA_OK;
}
