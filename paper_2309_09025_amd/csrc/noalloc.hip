// Static scratch for the entry point that allocates nothing
// (fs_pbs_lif_noalloc): one file-scope device array per GPU, its address
// looked up once per device at context creation, and the kernel that writes
// the LIF test polynomials into it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

namespace fs {

// Layout: [0, kNoallocTpWords) two test polynomials of up to 2048 words
// (function 0 at word 0, function 1 at word N); then kNoallocExtWords words
// of extracted samples between the blind rotation and the key switch.
static __device__ __align__(256) uint32_t scratch[kNoallocTpWords + kNoallocExtWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint32_t* g_ptr[kMaxDevices] = {};
}  // namespace

// Looks up this device's copy of the array.  The caller has made `device`
// current.  In host code `scratch` names a host-side stand-in, never the
// device memory: every use on the host goes through the looked-up address.
int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return 0;
  uint32_t* p = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return (int)e;
  if (!p) return (int)hipErrorInvalidSymbol;
  g_ptr[device] = p;
  return 0;
}

uint32_t* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

// v[k][i] = Delta * f_k(floor((i p + N) / (2N)) mod p), the test polynomial
// of program function k (the Initialization step after Theorem 2.1); the
// residue tables come by value in the kernel arguments.
__global__ void __launch_bounds__(256)
tpoly_pair_kernel(TpPair a, uint32_t* __restrict__ v) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x, k = blockIdx.y;
  if (i >= a.N) return;
  const uint32_t mask = a.p - 1;
  const uint32_t msg = (uint32_t)(((uint64_t)i * a.p + a.N) / (2ull * a.N)) & mask;
  v[(size_t)k * a.N + i] = (a.f[k][msg] & mask) * a.delta;
}

int launch_tpoly_pair(const TpPair& a, uint32_t* dst, hipStream_t st) {
  if (a.N == 0 || a.N > kNoallocTpWords / 2 || a.p == 0 || a.p > kTpPairMaxP) return -2;
  tpoly_pair_kernel<<<dim3((a.N + 255) / 256, 2), 256, 0, st>>>(a, dst);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

}  // namespace fs
