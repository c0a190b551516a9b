// Friends-of-friends groups (Koda et al. 2015: Sec. 2.3 runs a FoF halo finder
// on the fly; Sec. 3.1 links at 0.2 times the mean particle separation, 0.37
// for 2LPT).
//
// Two particles are friends when their nearest-image separation is at most b;
// the groups are the connected components, each labelled by its smallest
// particle id (unique, so the output is deterministic).  The link decision is
// made in float32 from the displacement in mesh units, one correctly rounded
// operation per step:
//   q = float(i nm) / float(np),  x = q + d,  dx = x_a - x_b,
//   dx -= nm rint(dx / nm),       r2 = (dx0^2 + dx1^2) + dx2^2 <= b^2.
//
// Search: particles are counted into cells of the mean separation s = nm/np
// (np^3 cells); b < s/2, so friends sit in the same or adjacent cells even
// where rounding moves a particle across a cell face.  Cell lists come from a
// counting sort (count, exclusive scan, scatter); each particle scans its own
// cell and half of the neighbouring ones.
//
// Union-find over the label array: parent[x] <= x always (a root is only ever
// hooked under a smaller root, by compare-and-swap), so every parent chain
// strictly decreases and each find ends.  Finds halve paths with plain
// coherent stores of a grandparent (a valid ancestor; a non-root never
// becomes a root again, and only roots are hooked, so no hook is undone).
// A failed compare-and-swap means another thread hooked that root first;
// the retry count is bounded and an exceeded bound raises a flag.  The last
// pass writes every particle's root without halving (see fof_root).
#include "cola_device.h"
#include "cola_internal.h"

namespace cola {

namespace {

constexpr int kFofMaxRetry = 1 << 20;

__device__ __forceinline__ uint32_t ld_rel(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void fof_pos(const float* __restrict__ disp, long np3, uint32_t id, int np, int nm,
                                        float x[3]) {
#pragma clang fp contract(off)
  const uint32_t unp = (uint32_t)np;
  const uint32_t li[3] = {id / (unp * unp), (id / unp) % unp, id % unp};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const float q = __fdiv_rn((float)(li[e] * (uint32_t)nm), (float)np);   // i nm < 2^24: exact
    x[e] = __fadd_rn(q, disp[e * np3 + id]);
  }
}

__device__ __forceinline__ int fof_cell1(float x, float s_inv, int np) {
  int c = (int)floorf(x * s_inv) % np;
  return c < 0 ? c + np : c;
}

// Root without writes: the final pass must not halve paths, or a thread that
// read par[x] before another wrote x's root there could overwrite that root
// with an intermediate ancestor.
__device__ __forceinline__ uint32_t fof_root(const uint32_t* par, uint32_t x) {
  for (;;) {
    const uint32_t p = ld_rel(par + x);
    if (p == x) return x;
    x = p;
  }
}

__device__ __forceinline__ uint32_t fof_find(uint32_t* par, uint32_t x) {
  for (;;) {
    const uint32_t p = ld_rel(par + x);
    if (p == x) return x;
    const uint32_t gp = ld_rel(par + p);
    if (gp != p) st_rel(par + x, gp);
    x = gp;
  }
}

}  // namespace

__global__ __launch_bounds__(256) void k_fof_cell(const float* __restrict__ disp, int np, int nm, long np3,
                                                  float s_inv, uint32_t* __restrict__ count,
                                                  uint32_t* __restrict__ key, uint32_t* __restrict__ rank) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= np3) return;
  float x[3];
  fof_pos(disp, np3, (uint32_t)i, np, nm, x);
  const uint32_t c = ((uint32_t)fof_cell1(x[0], s_inv, np) * (uint32_t)np + (uint32_t)fof_cell1(x[1], s_inv, np)) *
                         (uint32_t)np +
                     (uint32_t)fof_cell1(x[2], s_inv, np);
  key[i] = c;
  rank[i] = atomicAdd(&count[c], 1u);
}

__global__ __launch_bounds__(256) void k_fof_init(uint32_t* __restrict__ par, long np3) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < np3) par[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_fof_link(const float* __restrict__ disp, int np, int nm, long np3,
                                                  float b2, const uint32_t* __restrict__ key,
                                                  const uint32_t* __restrict__ start,
                                                  const uint32_t* __restrict__ sorted, uint32_t* par,
                                                  uint32_t* flag) {
#pragma clang fp contract(off)
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= np3) return;
  const uint32_t i = sorted[t];
  float xi[3];
  fof_pos(disp, np3, i, np, nm, xi);
  const uint32_t c = key[i];
  const int unp = np;
  const int c0 = (int)(c / (uint32_t)(unp * unp)), c1 = (int)((c / (uint32_t)unp) % (uint32_t)unp),
            c2 = (int)(c % (uint32_t)unp);
  const float nmf = (float)nm;
  // half shell: the own cell (o = 13, pairs j > i) and the 13 offsets that
  // follow (0, 0, 0) in lexicographic order; every unordered pair of adjacent
  // cells is then visited from exactly one side (np >= 3)
  for (int o = 13; o < 27; ++o) {
    const int a0 = (c0 + o / 9 - 1 + unp) % unp, a1 = (c1 + (o / 3) % 3 - 1 + unp) % unp,
              a2 = (c2 + o % 3 - 1 + unp) % unp;
    const uint32_t nc = ((uint32_t)a0 * (uint32_t)unp + (uint32_t)a1) * (uint32_t)unp + (uint32_t)a2;
    const uint32_t s0 = start[nc], s1 = start[nc + 1];
    for (uint32_t s = s0; s < s1; ++s) {
      const uint32_t j = sorted[s];
      if (o == 13 && j <= i) continue;
      float xj[3];
      fof_pos(disp, np3, j, np, nm, xj);
      float r2 = 0.f;
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        float dx = __fsub_rn(xi[e], xj[e]);
        dx = __fsub_rn(dx, __fmul_rn(nmf, rintf(__fdiv_rn(dx, nmf))));
        r2 = e == 0 ? __fmul_rn(dx, dx) : __fadd_rn(r2, __fmul_rn(dx, dx));
      }
      if (!(r2 <= b2)) continue;
      int tries = 0;
      for (;;) {
        const uint32_t ri = fof_find(par, i), rj = fof_find(par, j);
        if (ri == rj) break;
        const uint32_t hi = ri > rj ? ri : rj, lo = ri > rj ? rj : ri;
        if (atomicCAS(par + hi, hi, lo) == hi) break;
        if (++tries >= kFofMaxRetry) {
          atomicOr(flag, 1u);
          break;
        }
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_fof_compress(uint32_t* par, long np3) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < np3) {
    const uint32_t r = fof_root(par, (uint32_t)i);   // each thread writes only its own entry
    st_rel(par + i, r);
  }
}

void launch_fof(const float* disp, int np, int nm, double b_frac, uint32_t* labels, uint32_t* count,
                uint32_t* start, uint32_t* scan_scratch, uint32_t* key, uint32_t* rank, uint32_t* sorted,
                uint32_t* flag, hipStream_t s) {
  const long np3 = (long)np * np * np;
  const unsigned blocks = (unsigned)((np3 + 255) / 256);
  const double b = b_frac * nm / np;
  const float b2 = (float)(b * b);
  const float s_inv = (float)((double)np / (double)nm);
  launch_fill_u32(count, np3 + 1, 0u, s);
  hipLaunchKernelGGL(k_fof_cell, dim3(blocks), dim3(256), 0, s, disp, np, nm, np3, s_inv, count, key, rank);
  launch_exclusive_scan(count, start, np3, scan_scratch, s);
  launch_scatter(key, rank, start, np3, sorted, s);
  hipLaunchKernelGGL(k_fof_init, dim3(blocks), dim3(256), 0, s, labels, np3);
  hipLaunchKernelGGL(k_fof_link, dim3(blocks), dim3(256), 0, s, disp, np, nm, np3, b2, key, start, sorted,
                     labels, flag);
  hipLaunchKernelGGL(k_fof_compress, dim3(blocks), dim3(256), 0, s, labels, np3);
}

// ---------------------------------------------------------------------------
// Halo catalogue of the groups with at least min_members particles, in
// increasing root id: member count, centre of mass (the root's position plus
// the mean nearest-image offset of the members from it, wrapped into
// [0, nm)) and mean velocity.  Offsets and velocities are summed as 64-bit
// fixed point (2^-20 cells, 2^-16 velocity units): integer sums do not
// depend on the order of the atomics, so the catalogue is reproducible.

constexpr double kPosFix = 1048576.0, kVelFix = 65536.0;

__global__ __launch_bounds__(256) void k_halo_count(const int32_t* __restrict__ lab, long np3,
                                                    uint32_t* __restrict__ count, uint32_t* bad) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= np3) return;
  const int32_t l = lab[i];
  if (l < 0 || (long)l >= np3) {   // not a label of this particle set
    atomicOr(bad, 1u);
    return;
  }
  atomicAdd(&count[l], 1u);
}

__global__ __launch_bounds__(256) void k_halo_flag(const uint32_t* __restrict__ count, long np3, uint32_t minm,
                                                   uint32_t* __restrict__ flg) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < np3) flg[i] = count[i] >= minm ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_halo_roots(const uint32_t* __restrict__ count,
                                                    const uint32_t* __restrict__ flg,
                                                    const uint32_t* __restrict__ hidx, long np3,
                                                    int32_t* __restrict__ root, int32_t* __restrict__ cnt) {
  const long r = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (r < np3 && flg[r]) {
    root[hidx[r]] = (int32_t)r;
    cnt[hidx[r]] = (int32_t)count[r];
  }
}

__global__ __launch_bounds__(256) void k_halo_accum(const float* __restrict__ disp, const float* __restrict__ vel,
                                                    const int32_t* __restrict__ lab,
                                                    const uint32_t* __restrict__ flg,
                                                    const uint32_t* __restrict__ hidx, int np, int nm, long np3,
                                                    unsigned long long* __restrict__ acc) {
#pragma clang fp contract(off)
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= np3) return;
  const int32_t l = lab[i];
  if (l < 0 || (long)l >= np3) return;
  const uint32_t r = (uint32_t)l;
  if (!flg[r]) return;
  const long h = hidx[r];
  float xi[3], xr[3];
  fof_pos(disp, np3, (uint32_t)i, np, nm, xi);
  fof_pos(disp, np3, r, np, nm, xr);
  const float nmf = (float)nm;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    float dx = __fsub_rn(xi[e], xr[e]);
    dx = __fsub_rn(dx, __fmul_rn(nmf, rintf(__fdiv_rn(dx, nmf))));
    atomicAdd(acc + h * 6 + e, (unsigned long long)llrint((double)dx * kPosFix));
    if (vel) atomicAdd(acc + h * 6 + 3 + e, (unsigned long long)llrint((double)vel[e * np3 + i] * kVelFix));
  }
}

__global__ __launch_bounds__(256) void k_halo_final(const float* __restrict__ disp,
                                                    const int32_t* __restrict__ root,
                                                    const int32_t* __restrict__ cnt,
                                                    const unsigned long long* __restrict__ acc, int np, int nm,
                                                    long np3, int nh, int stride, float* __restrict__ pos,
                                                    float* __restrict__ vout) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nh) return;
  float xr[3];
  fof_pos(disp, np3, (uint32_t)root[h], np, nm, xr);
  const double n = (double)cnt[h];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    double c = (double)xr[e] + (double)(long long)acc[(long)h * 6 + e] / kPosFix / n;
    c -= nm * floor(c / nm);
    float fc = (float)c;                 // rounding can reach nm itself
    if (fc >= (float)nm) fc -= (float)nm;
    pos[(long)e * stride + h] = fc;
    if (vout) vout[(long)e * stride + h] = (float)((double)(long long)acc[(long)h * 6 + 3 + e] / kVelFix / n);
  }
}

void launch_halo_count(const int32_t* lab, long np3, int32_t minm, uint32_t* count, uint32_t* flg, uint32_t* hidx,
                       uint32_t* scan_scratch, uint32_t* bad, hipStream_t s) {
  const unsigned blocks = (unsigned)((np3 + 255) / 256);
  launch_fill_u32(count, np3, 0u, s);
  hipLaunchKernelGGL(k_halo_count, dim3(blocks), dim3(256), 0, s, lab, np3, count, bad);
  hipLaunchKernelGGL(k_halo_flag, dim3(blocks), dim3(256), 0, s, count, np3, (uint32_t)minm, flg);
  launch_exclusive_scan(flg, hidx, np3, scan_scratch, s);
}

void launch_halo_fill(const float* disp, const float* vel, const int32_t* lab, const uint32_t* count,
                      const uint32_t* flg, const uint32_t* hidx, int np, int nm, int nh, int stride,
                      unsigned long long* acc, int32_t* root, int32_t* cnt, float* pos, float* vout,
                      hipStream_t s) {
  const long np3 = (long)np * np * np;
  const unsigned blocks = (unsigned)((np3 + 255) / 256);
  if (nh > 0) launch_fill_u32(reinterpret_cast<uint32_t*>(acc), 12L * nh, 0u, s);
  hipLaunchKernelGGL(k_halo_roots, dim3(blocks), dim3(256), 0, s, count, flg, hidx, np3, root, cnt);
  hipLaunchKernelGGL(k_halo_accum, dim3(blocks), dim3(256), 0, s, disp, vel, lab, flg, hidx, np, nm, np3, acc);
  if (nh > 0)
    hipLaunchKernelGGL(k_halo_final, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0, s, disp, root, cnt, acc,
                       np, nm, np3, nh, stride, pos, vout);
}

}  // namespace cola
