// The allocation-free variant of the learned-preconditioner apply, for
// callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc).
//
// Its work memory (the scaled residual rh = s r and the apply's partial
// sums) lives in `scratch`, a static device array of kScratchBytes that each
// GPU the library runs on holds until the process ends.  Host code never
// uses the array's name as an address: its device address is looked up once
// per device, with that device current, by hipGetSymbolAddress (at context
// creation), and kept per device.  Every call on a GPU shares that GPU's
// array: calls that overlap in time on one GPU (other streams, threads or
// contexts) race on it.  Nothing in it must start at zero: k_rh writes all
// of rh and every workgroup of the apply writes its own partials.
#include <mutex>

#include "gnn.h"

namespace sfem {

namespace {

constexpr size_t kScratchBytes = size_t(8) << 20;  // 8 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex scratch_mu;
void* scratch_addr[kMaxDevices] = {};

// The device address of this device's scratch, looked up on first use.
// The caller has made `device` current.
void* scratch_ptr(int device) {
  SFEM_REQUIRE(device >= 0 && device < kMaxDevices, SFEM_EINVAL,
               "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_addr[device]) {
    void* p = nullptr;
    SFEM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    SFEM_REQUIRE(p != nullptr, SFEM_EHIP, "no device address for the scratch array");
    scratch_addr[device] = p;
  }
  return scratch_addr[device];
}

// A pointer the caller gave for device memory of the current device.
bool on_device(const void* p, int device) {
  hipPointerAttribute_t a{};
  const hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // a plain host pointer reports an error: clear it
    return false;
  }
  return a.type == hipMemoryTypeDevice && a.device == device;
}

}  // namespace

void scratch_init(int device) { (void)scratch_ptr(device); }

void precond_apply_noalloc(Ctx& c, const double* r, double* z) {
  const int64_t n = c.n_dof();
  const size_t rh_bytes = (size_t(8) * size_t(n) + 255) & ~size_t(255);
  const size_t need = rh_bytes + size_t(8) * size_t(learned_apply_partials(c));
  SFEM_REQUIRE(need <= kScratchBytes, SFEM_EINVAL,
               "mesh too large for the allocation-free apply: it needs " +
                   std::to_string(need) + " bytes of scratch, at most " +
                   std::to_string(kScratchBytes) + " (3 n_nodes + 3 x 4096 doubles)");
  SFEM_REQUIRE(c.have_learned, SFEM_ESTATE, "call sfem_gnn_apply first");
  SFEM_REQUIRE(r && z, SFEM_EINVAL, "null vector");
  SFEM_REQUIRE(on_device(r, c.device) && on_device(z, c.device), SFEM_EINVAL,
               "r and z must be device memory of the context's GPU");
  char* base = static_cast<char*>(scratch_ptr(c.device));
  learned_apply_into(c, r, z, reinterpret_cast<double*>(base),
                     reinterpret_cast<double*>(base + rh_bytes));
}

}  // namespace sfem
