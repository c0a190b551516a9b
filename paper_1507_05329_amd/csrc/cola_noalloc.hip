// cola_density_noalloc: the deterministic CIC density of a displacement field
// (the deposit of cola_density_of) for callers that cannot allocate device
// memory.  The tile sort's buffers (bucket keys, ranks, permutation, bucket
// counts and offsets, scan scratch) live in one file-scope device array of
// fixed size; each device holds its own copy until the process ends.
#include <atomic>

#include "cola_internal.h"

namespace {

// Largest run served from the static array: 64^3 particles, a 256^3 mesh.
constexpr long kMaxParticles = 64L * 64 * 64;
constexpr int kMaxMesh = 256;
constexpr long kAlignWords = 64;  // 256 bytes
constexpr long align_words(long n) { return (n + kAlignWords - 1) / kAlignWords * kAlignWords; }
constexpr long buckets_of(int nm) { return 8L * (nm / 16) * (nm / 16) * (nm / 16); }
constexpr long scratch_words(long np3, int nm) {
  return 3 * align_words(np3) + 2 * align_words(buckets_of(nm) + 1) + align_words((buckets_of(nm) + 1) / 4096 + 2);
}
constexpr long kScratchWords = scratch_words(kMaxParticles, kMaxMesh);

}  // namespace

static __device__ __align__(256) uint32_t scratch[kScratchWords];

namespace {

// Device address of `scratch` on each device, looked up once per device with
// that device current (the array's name is not a device address in host code).
constexpr int kMaxDevices = 64;
std::atomic<uint32_t*> g_scratch[kMaxDevices];

int scratch_address(uint32_t** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return COLA_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return COLA_EUNSUPPORTED;
  uint32_t* p = g_scratch[dev].load(std::memory_order_acquire);
  if (!p) {
    void* q = nullptr;
    if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return COLA_EHIP;
    p = static_cast<uint32_t*>(q);
    g_scratch[dev].store(p, std::memory_order_release);
  }
  *out = p;
  return COLA_OK;
}

}  // namespace

extern "C" int cola_density_noalloc(const float* disp, int32_t np, int32_t nmesh, float* out, void* stream) {
  if (!disp || !out) return COLA_EINVAL;
  if (np < 16 || np % 16 != 0 || nmesh < 32 || nmesh % 16 != 0 || nmesh < np) return COLA_EINVAL;
  const long np3 = (long)np * np * np;
  if (np3 > kMaxParticles || nmesh > kMaxMesh) return COLA_ENOMEM;
  uint32_t* base = nullptr;
  const int r = scratch_address(&base);
  if (r != COLA_OK) return r;
  const long nb = buckets_of(nmesh);
  uint32_t* pkey = base;
  uint32_t* prank = pkey + align_words(np3);
  uint32_t* perm = prank + align_words(np3);
  uint32_t* counts = perm + align_words(np3);
  uint32_t* offsets = counts + align_words(nb + 1);
  uint32_t* scan = offsets + align_words(nb + 1);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // counts start at zero: cleared by a kernel on every call (the array keeps
  // the previous call's contents)
  cola::launch_fill_u32(counts, nb + 1, 0u, s);
  cola::launch_bin_count(disp, np, nmesh, 1.0f, counts, pkey, prank, s);
  cola::launch_exclusive_scan(counts, offsets, nb, scan, s);
  cola::launch_scatter_walk(pkey, prank, offsets, np, perm, s);
  cola::launch_deposit(disp, perm, offsets, np, nmesh, 1.0f, out, nmesh, 1, s);
  return hipGetLastError() == hipSuccess ? COLA_OK : COLA_EHIP;
}
