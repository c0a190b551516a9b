// Deterministic CIC mass assignment as a gather (no float atomics).
//
// CIC (Koda et al. 2015, Sec. 3.3; Hockney & Eastwood): a particle with home
// cell c and fraction f gives weight prod_e w_{s_e}(f_e) to node c + s.
// One workgroup owns an 8^3 tile of nodes.  The cells that feed those nodes
// are the tile's own 8^3 cells plus the one-cell layer below it on each axis
// (a 9^3 region); their particles come from the tile's buckets and from the
// face/edge/corner buckets of the 7 lower neighbour tiles.  Particles are
// keyed (region cell, particle id) and sorted in LDS, so every cell's
// weights are added in ascending particle id; a node then adds its 8 source
// cells in the fixed offset order k = 4 sx + 2 sy + sz.  The result does not
// depend on launch order, atomics or the bucket order inside the sort.
// Tiles whose region holds more particles than fit in LDS are processed in
// x-slabs of the region, then single cells, then by an ordered selection.
#include "cola_device.h"
#include "cola_internal.h"

// Every float operation in this file is a single IEEE rounding (the
// deterministic order is part of the result): no fused multiply-add.
#pragma clang fp contract(off)

namespace cola {

constexpr int kDT = 256;        // threads per workgroup
constexpr int kCap = 2048;      // keys held in LDS at once (power of two)
constexpr int kReg = 9;         // region side (8 + 1 lower layer)
constexpr int kNReg = kReg * kReg * kReg;

struct DepShared {
  uint64_t keys[kCap];
  float P[8 * kNReg];           // per-cell partial sums, offset-major
  uint32_t seg_start[27];
  uint32_t seg_pre[28];
  int nseg;
  uint32_t count;
  uint32_t red[kDT / 64];
  float acc8[8];
};

__device__ __forceinline__ int region_coord(int c, int t8, int nm) {
  int r = c - t8 + 1;
  if (r < 0) r += nm;
  if (r >= nm) r -= nm;
  return r;
}

// Entry j (0 <= j < total) of the workgroup's particle list -> particle id.
__device__ __forceinline__ uint32_t list_id(const DepShared& sh, const uint32_t* __restrict__ perm,
                                            uint32_t j) {
  int s = 0;
  while (s + 1 < sh.nseg && sh.seg_pre[s + 1] <= j) ++s;
  return perm[sh.seg_start[s] + (j - sh.seg_pre[s])];
}

// filter: 0 = all, 1 = region x index == fv, 2 = region cell == fv.
__device__ uint32_t gather_keys(DepShared& sh, const float* __restrict__ disp,
                                const uint32_t* __restrict__ perm, long np3, int np, int nm,
                                float dscale, const int t8[3], uint32_t total, int filter, int fv) {
  if (threadIdx.x == 0) sh.count = 0;
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < total; j += kDT) {
    const uint32_t id = list_id(sh, perm, j);
    int c[3];
    float f[3];
    home_cell(disp, np3, id, np, nm, dscale, c, f);
    const int rx = region_coord(c[0], t8[0], nm), ry = region_coord(c[1], t8[1], nm),
              rz = region_coord(c[2], t8[2], nm);
    const int lc = (rx * kReg + ry) * kReg + rz;
    const bool inside = rx < kReg && ry < kReg && rz < kReg;
    const bool pass = inside && (filter == 0 || (filter == 1 && rx == fv) || (filter == 2 && lc == fv));
    if (pass) {
      const uint32_t slot = atomicAdd(&sh.count, 1u);
      if (slot < (uint32_t)kCap) sh.keys[slot] = ((uint64_t)lc << 32) | id;
    }
  }
  __syncthreads();
  return sh.count;
}

__device__ void sort_keys(DepShared& sh, uint32_t n) {
  uint32_t p2 = 1;
  while (p2 < n) p2 <<= 1;
  for (uint32_t j = n + threadIdx.x; j < p2; j += kDT) sh.keys[j] = ~0ull;
  __syncthreads();
  for (uint32_t k = 2; k <= p2; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < p2; i += kDT) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const uint64_t a = sh.keys[i], b = sh.keys[ixj];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            sh.keys[i] = b;
            sh.keys[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Per-cell partial sums of the n sorted keys (one thread per run of equal cell).
__device__ void cell_partials(DepShared& sh, const float* __restrict__ disp, long np3, int np,
                              int nm, float dscale, uint32_t n) {
  for (uint32_t j = threadIdx.x; j < n; j += kDT) {
    const uint32_t lc = (uint32_t)(sh.keys[j] >> 32);
    if (j > 0 && (uint32_t)(sh.keys[j - 1] >> 32) == lc) continue;
    float acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.0f;
    for (uint32_t m = j; m < n && (uint32_t)(sh.keys[m] >> 32) == lc; ++m) {
      int c[3];
      float f[3];
      home_cell(disp, np3, (uint32_t)sh.keys[m], np, nm, dscale, c, f);
#pragma unroll
      for (int k = 0; k < 8; ++k) acc[k] = __fadd_rn(acc[k], cic_weight(f, k));
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) sh.P[k * kNReg + lc] = acc[k];
  }
  __syncthreads();
}

// A cell with more than kCap particles: add them in ascending id by repeated
// workgroup-wide minimum search (slow; only for extreme clustering).
__device__ void cell_partials_select(DepShared& sh, const float* __restrict__ disp,
                                     const uint32_t* __restrict__ perm, long np3, int np, int nm,
                                     float dscale, const int t8[3], uint32_t total, int lc_target) {
  if (threadIdx.x < 8) sh.acc8[threadIdx.x] = 0.0f;
  uint32_t last = 0;
  bool first = true;
  for (;;) {
    uint32_t best = 0xffffffffu;
    for (uint32_t j = threadIdx.x; j < total; j += kDT) {
      const uint32_t id = list_id(sh, perm, j);
      if (!first && id <= last) continue;
      if (id >= best) continue;
      int c[3];
      float f[3];
      home_cell(disp, np3, id, np, nm, dscale, c, f);
      const int lc = (region_coord(c[0], t8[0], nm) * kReg + region_coord(c[1], t8[1], nm)) * kReg +
                     region_coord(c[2], t8[2], nm);
      if (lc == lc_target) best = id;
    }
    // workgroup min
    for (int o = 32; o > 0; o >>= 1) {
      const uint32_t other = __shfl_xor(best, o, 64);
      best = other < best ? other : best;
    }
    if ((threadIdx.x & 63) == 0) sh.red[threadIdx.x >> 6] = best;
    __syncthreads();
    uint32_t m = sh.red[0];
    for (int w = 1; w < kDT / 64; ++w) m = sh.red[w] < m ? sh.red[w] : m;
    __syncthreads();
    if (m == 0xffffffffu) break;
    if (threadIdx.x == 0) {
      int c[3];
      float f[3];
      home_cell(disp, np3, m, np, nm, dscale, c, f);
      for (int k = 0; k < 8; ++k) sh.acc8[k] = __fadd_rn(sh.acc8[k], cic_weight(f, k));
    }
    last = m;
    first = false;
    __syncthreads();
  }
  if (threadIdx.x < 8) sh.P[threadIdx.x * kNReg + lc_target] = sh.acc8[threadIdx.x];
  __syncthreads();
}

__global__ __launch_bounds__(kDT) void k_deposit(const float* __restrict__ disp,
                                                 const uint32_t* __restrict__ perm,
                                                 const uint32_t* __restrict__ off, int np, int nm,
                                                 float dscale, long np3, float* __restrict__ out,
                                                 long row_stride, int contrast, float cinv) {
  __shared__ DepShared sh;
  const int nt = nm >> 3;
  const uint32_t t = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = t / (nt * nt), ty = (t / nt) % nt, tz = t % nt;
  const int t8[3] = {tx * 8, ty * 8, tz * 8};

  if (threadIdx.x == 0) {
    int ns = 0;
    uint32_t acc = 0;
    for (int nb = 0; nb < 8; ++nb) {
      const int dx = (nb >> 2) & 1, dy = (nb >> 1) & 1, dz = nb & 1;
      int ux = tx - dx, uy = ty - dy, uz = tz - dz;
      if (ux < 0) ux += nt;
      if (uy < 0) uy += nt;
      if (uz < 0) uz += nt;
      const uint32_t tn = ((uint32_t)ux * nt + uy) * nt + uz;
      const int req = nb;
      int cls = 0;
      while (cls < 8) {
        if ((cls & req) != req) { ++cls; continue; }
        int c2 = cls;
        while (c2 + 1 < 8 && ((c2 + 1) & req) == req) ++c2;
        const uint32_t a = off[tn * 8u + cls], b = off[tn * 8u + c2 + 1];
        if (b > a) {
          sh.seg_start[ns] = a;
          sh.seg_pre[ns] = acc;
          acc += b - a;
          ++ns;
        }
        cls = c2 + 1;
      }
    }
    sh.seg_pre[ns] = acc;
    sh.nseg = ns;
  }
  for (int i = threadIdx.x; i < 8 * kNReg; i += kDT) sh.P[i] = 0.0f;
  __syncthreads();
  const uint32_t total = sh.seg_pre[sh.nseg];

  if (total > 0) {
    uint32_t n = gather_keys(sh, disp, perm, np3, np, nm, dscale, t8, total, 0, 0);
    if (n <= (uint32_t)kCap) {
      sort_keys(sh, n);
      cell_partials(sh, disp, np3, np, nm, dscale, n);
    } else {
      for (int slab = 0; slab < kReg; ++slab) {
        n = gather_keys(sh, disp, perm, np3, np, nm, dscale, t8, total, 1, slab);
        if (n == 0) continue;
        if (n <= (uint32_t)kCap) {
          sort_keys(sh, n);
          cell_partials(sh, disp, np3, np, nm, dscale, n);
          continue;
        }
        for (int cc = 0; cc < kReg * kReg; ++cc) {
          const int lc = slab * kReg * kReg + cc;
          n = gather_keys(sh, disp, perm, np3, np, nm, dscale, t8, total, 2, lc);
          if (n == 0) continue;
          if (n <= (uint32_t)kCap) {
            sort_keys(sh, n);
            cell_partials(sh, disp, np3, np, nm, dscale, n);
          } else {
            cell_partials_select(sh, disp, perm, np3, np, nm, dscale, t8, total, lc);
          }
        }
      }
    }
  }

  for (int nn = threadIdx.x; nn < 512; nn += kDT) {
    const int nx = nn >> 6, ny = (nn >> 3) & 7, nz = nn & 7;
    float rho = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int sx = (k >> 2) & 1, sy = (k >> 1) & 1, sz = k & 1;
      const int lc = ((nx - sx + 1) * kReg + (ny - sy + 1)) * kReg + (nz - sz + 1);
      rho = __fadd_rn(rho, sh.P[k * kNReg + lc]);
    }
    const float val = contrast ? __fsub_rn(__fmul_rn(rho, cinv), 1.0f) : rho;
    out[((long)(t8[0] + nx) * nm + (t8[1] + ny)) * row_stride + (t8[2] + nz)] = val;
  }
}

void launch_deposit(const float* disp, const uint32_t* perm, const uint32_t* off, int np, int nm,
                    float dscale, float* out, long row_stride, int contrast, hipStream_t s) {
  const long np3 = (long)np * np * np;
  const int nt = nm >> 3;
  const long ntiles = (long)nt * nt * nt;
  const float cinv = (float)((double)nm * nm * nm / (double)np3);
  hipLaunchKernelGGL(k_deposit, dim3((unsigned)ntiles), dim3(kDT), 0, s, disp, perm, off, np, nm,
                     dscale, np3, out, row_stride, contrast, cinv);
}

}  // namespace cola
