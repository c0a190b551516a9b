// Tile sort for the deterministic CIC deposit: bucket = (16^3 tile of the home
// cell, face class).  Integer atomics only; the order inside a bucket is left
// to the deposit, which orders particles by id itself.
#include "cola_device.h"
#include "cola_internal.h"

namespace cola {

__global__ void k_fill_u32(uint32_t* __restrict__ p, long n, uint32_t v, long mstride) {
  p = mock_ptr(p, mstride);
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = v;
}

void launch_fill_u32(uint32_t* p, long n, uint32_t v, hipStream_t s, int nmock, long mstride) {
  if (n <= 0) return;
  long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks, 1, (unsigned)nmock), dim3(256), 0, s, p, n, v,
                     mstride);
}

__global__ __launch_bounds__(256) void k_bin_count(const float* __restrict__ disp, int np, int nm,
                                                   float dscale, long np3, uint32_t* __restrict__ counts,
                                                   uint32_t* __restrict__ pkey,
                                                   uint32_t* __restrict__ prank, long mstride) {
  disp = mock_ptr(disp, mstride);
  counts = mock_ptr(counts, mstride);
  pkey = mock_ptr(pkey, mstride);
  prank = mock_ptr(prank, mstride);
  // Sub-cube order: a workgroup's particles share few buckets. Every supported
  // np is a multiple of 16, so np^3 is a multiple of 256 and each thread of
  // the grid has a particle.
  const long i = subcube_particle(xcd_remap(blockIdx.x, gridDim.x), threadIdx.x, np);
  int c[3];
  float f[3];
  home_cell(disp, np3, (uint32_t)i, np, nm, dscale, c, f);
  const uint32_t b = bucket_of(c, nm >> 4);
  pkey[i] = b;
  // Workgroup-aggregated count: an LDS table (open addressing, 512 slots for
  // at most 256 keys) counts the workgroup's particles per bucket, then one
  // global atomic per distinct bucket reserves their places.
  constexpr uint32_t kEmpty = 0xffffffffu, kSlots = 512;
  __shared__ uint32_t hkey[kSlots], hcnt[kSlots], hbase[kSlots];
  for (uint32_t j = threadIdx.x; j < kSlots; j += 256) {
    hkey[j] = kEmpty;
    hcnt[j] = 0u;
  }
  __syncthreads();
  uint32_t h = (b * 2654435761u) >> 23;
  for (;;) {
    const uint32_t prev = atomicCAS(&hkey[h], kEmpty, b);
    if (prev == kEmpty || prev == b) break;
    h = (h + 1) & (kSlots - 1);
  }
  const uint32_t local = atomicAdd(&hcnt[h], 1u);
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < kSlots; j += 256)
    if (hkey[j] != kEmpty) hbase[j] = atomicAdd(&counts[hkey[j]], hcnt[j]);
  __syncthreads();
  prank[i] = hbase[h] + local;
}

void launch_bin_count(const float* disp, int np, int nm, float dscale, uint32_t* counts,
                      uint32_t* pkey, uint32_t* prank, hipStream_t s, int nmock, long mstride) {
  const long np3 = (long)np * np * np;
  hipLaunchKernelGGL(k_bin_count, dim3((unsigned)((np3 + 255) / 256), 1, (unsigned)nmock), dim3(256), 0,
                     s, disp, np, nm, dscale, np3, counts, pkey, prank, mstride);
}

// ---------------------------------------------------------------------------
// Exclusive scan, three passes: block sums, scan of block sums, block scan.
constexpr int kScanT = 256;
constexpr int kScanPer = 16;
constexpr long kScanChunk = (long)kScanT * kScanPer;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  // sh: kScanT entries.  Hillis-Steele in LDS (deterministic for integers anyway).
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanT; off <<= 1) {
    const uint32_t a = t >= off ? sh[t - off] : 0u;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const uint32_t incl = sh[t];
  *total = sh[kScanT - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kScanT) void k_scan_reduce(const uint32_t* __restrict__ in, long n,
                                                        uint32_t* __restrict__ bsum, long mstride) {
  __shared__ uint32_t sh[kScanT];
  in = mock_ptr(in, mstride);
  bsum = mock_ptr(bsum, mstride);
  const long base = blockIdx.x * kScanChunk;
  uint32_t acc = 0;
  for (int j = 0; j < kScanPer; ++j) {
    const long i = base + (long)j * kScanT + threadIdx.x;
    if (i < n) acc += in[i];
  }
  uint32_t tot;
  block_exclusive_scan(acc, sh, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Scans nb <= kScanT*kScanPer*... block sums in place with one workgroup.
__global__ __launch_bounds__(kScanT) void k_scan_blocksums(uint32_t* __restrict__ bsum, long nb,
                                                           long mstride) {
  __shared__ uint32_t sh[kScanT];
  bsum = mock_ptr(bsum, mstride);
  uint32_t carry = 0;
  for (long base = 0; base < nb; base += kScanT * (long)kScanPer) {
    uint32_t v[kScanPer];
    uint32_t loc = 0;
    for (int j = 0; j < kScanPer; ++j) {
      const long i = base + (long)threadIdx.x * kScanPer + j;
      v[j] = i < nb ? bsum[i] : 0u;
      loc += v[j];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(loc, sh, &tot) + carry;
    for (int j = 0; j < kScanPer; ++j) {
      const long i = base + (long)threadIdx.x * kScanPer + j;
      if (i < nb) bsum[i] = ex;
      ex += v[j];
    }
    carry += tot;
  }
}

__global__ __launch_bounds__(kScanT) void k_scan_apply(const uint32_t* __restrict__ in, long n,
                                                       const uint32_t* __restrict__ bsum,
                                                       uint32_t* __restrict__ out, long mstride) {
  __shared__ uint32_t sh[kScanT];
  in = mock_ptr(in, mstride);
  bsum = mock_ptr(bsum, mstride);
  out = mock_ptr(out, mstride);
  const long base = blockIdx.x * kScanChunk + (long)threadIdx.x * kScanPer;
  uint32_t v[kScanPer];
  uint32_t loc = 0;
  for (int j = 0; j < kScanPer; ++j) {
    const long i = base + j;
    v[j] = i < n ? in[i] : 0u;
    loc += v[j];
  }
  uint32_t tot;
  uint32_t ex = block_exclusive_scan(loc, sh, &tot) + bsum[blockIdx.x];
  for (int j = 0; j < kScanPer; ++j) {
    const long i = base + j;
    if (i < n) out[i] = ex;
    ex += v[j];
  }
  // out[n] = total, written by the thread that holds element n-1
  if (base <= n - 1 && n - 1 < base + kScanPer) out[n] = ex;
}

void launch_exclusive_scan(const uint32_t* in, uint32_t* out, long n, uint32_t* scratch,
                           hipStream_t s, int nmock, long mstride) {
  const long nb = (n + kScanChunk - 1) / kScanChunk;
  const unsigned z = (unsigned)nmock;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb, 1, z), dim3(kScanT), 0, s, in, n, scratch, mstride);
  hipLaunchKernelGGL(k_scan_blocksums, dim3(1, 1, z), dim3(kScanT), 0, s, scratch, nb, mstride);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb, 1, z), dim3(kScanT), 0, s, in, n, scratch, out,
                     mstride);
}

__global__ __launch_bounds__(256) void k_scatter(const uint32_t* __restrict__ pkey,
                                                 const uint32_t* __restrict__ prank,
                                                 const uint32_t* __restrict__ off, long np3,
                                                 uint32_t* __restrict__ perm, long mstride) {
  pkey = mock_ptr(pkey, mstride);
  prank = mock_ptr(prank, mstride);
  off = mock_ptr(off, mstride);
  perm = mock_ptr(perm, mstride);
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= np3) return;
  perm[off[pkey[i]] + prank[i]] = (uint32_t)i;
}

void launch_scatter(const uint32_t* pkey, const uint32_t* prank, const uint32_t* off, long np3,
                    uint32_t* perm, hipStream_t s, int nmock, long mstride) {
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)((np3 + 255) / 256), 1, (unsigned)nmock), dim3(256), 0, s,
                     pkey, prank, off, np3, perm, mstride);
}

// The tile sort's scatter, in the bucket count's particle-to-workgroup walk:
// the count reserved one contiguous run per (workgroup, bucket), so each
// workgroup's writes fill a few whole runs instead of single ids scattered
// over many.  The result is the same in any walk (every id has its slot).
__global__ __launch_bounds__(256) void k_scatter_walk(const uint32_t* __restrict__ pkey,
                                                      const uint32_t* __restrict__ prank,
                                                      const uint32_t* __restrict__ off, int np,
                                                      uint32_t* __restrict__ perm, long mstride) {
  pkey = mock_ptr(pkey, mstride);
  prank = mock_ptr(prank, mstride);
  off = mock_ptr(off, mstride);
  perm = mock_ptr(perm, mstride);
  const long i = subcube_particle(xcd_remap(blockIdx.x, gridDim.x), threadIdx.x, np);
  perm[off[pkey[i]] + prank[i]] = (uint32_t)i;
}

void launch_scatter_walk(const uint32_t* pkey, const uint32_t* prank, const uint32_t* off, int np,
                         uint32_t* perm, hipStream_t s, int nmock, long mstride) {
  const long np3 = (long)np * np * np;   // np is a multiple of 16: whole workgroups
  hipLaunchKernelGGL(k_scatter_walk, dim3((unsigned)(np3 / 256), 1, (unsigned)nmock), dim3(256), 0, s,
                     pkey, prank, off, np, perm, mstride);
}

}  // namespace cola
