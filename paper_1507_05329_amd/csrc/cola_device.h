// Device helpers shared by the libcola kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace cola {

// Division by the lattice side np (1 .. 1024) of values below 2^30 with one
// 32 x 32 -> 64-bit multiply: q = (n m) >> s, s = 30 + ceil(log2 np),
// m = ceil(2^s / np) < 2^32.  Exact: m = 2^s / np + e with 0 <= e < 1, so
// n m / 2^s = n / np + n e / 2^s, and n e / 2^s < 2^-ceil(log2 np) <= 1/np
// cannot carry floor(n / np) to the next integer.
// The offset (2 rem - np) / (2 np) is the double product (2 rem - np) x
// (1 / (2 np)) rounded once to float, which equals the correctly rounded
// float quotient: a quotient of integers below 2^12 is either a float or
// more than 2^-35 (relative) away from every float rounding boundary, while
// the double product is within 2^-52 of it.
struct LatDivTable {
  uint32_t m[1025];
  uint32_t s[1025];
  double inv2[1025];   // 1 / (2 np)
  constexpr LatDivTable() : m(), s(), inv2() {
    for (uint32_t d = 1; d <= 1024; ++d) {
      uint32_t l = 0;
      while ((1u << l) < d) ++l;
      const uint64_t p = 1ull << (30 + l);
      m[d] = (uint32_t)((p + d - 1) / d);
      s[d] = 30 + l;
      inv2[d] = 1.0 / (2.0 * (double)d);
    }
  }
};
static __constant__ LatDivTable kLatDiv;

struct LatGeom {
  uint32_t np, nm, m, s;
  double inv2;
};
__device__ __forceinline__ LatGeom lat_geom(int np, int nm) {
  return {(uint32_t)np, (uint32_t)nm, kLatDiv.m[np], kLatDiv.s[np], kLatDiv.inv2[np]};
}
__device__ __forceinline__ uint32_t lat_div(uint32_t n, const LatGeom& g) {
  return (uint32_t)(((uint64_t)n * g.m) >> g.s);
}

// Home cell and fractional offset of particle `id` (CIC, nodes at cell
// centres).  Lattice point of axis e sits at i_e * nm / np cells; the node
// coordinate is u = i_e nm / np - 1/2 + d_e, computed as
//   qi = (i_e nm) div np,  qf = float(2 rem - np) / float(2 np)   (-1/2 exactly
//   when nm/np is whole),  u = qf + d_e,  cell = qi + floor(u),  f = u - floor(u).
// Every step is a single correctly rounded float32 operation so the deposit
// is reproducible bit for bit.  `nm` is the target grid; displacements are
// stored in cells of the PM mesh and multiplied by dscale = target/PM
// (exactly 1 on the PM mesh, where the product is the identity).
__device__ __forceinline__ void home_cell_of(const float dv[3], uint32_t id, int np, int nm, float dscale,
                                             int c[3], float f[3]) {
#pragma clang fp contract(off)
  const LatGeom g = lat_geom(np, nm);
  const uint32_t q1 = lat_div(id, g);
  const uint32_t q0 = lat_div(q1, g);
  const uint32_t li[3] = {q0, q1 - q0 * g.np, id - q1 * g.np};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const uint32_t t = li[e] * g.nm;                // < 1024 * 2048: below 2^30
    const uint32_t qi = lat_div(t, g);
    const int rem = (int)(t - qi * g.np);
    const float qf = (float)((double)(2 * rem - np) * g.inv2);
    const float u = __fadd_rn(qf, __fmul_rn(dv[e], dscale));
    const float fl = floorf(u);
    f[e] = __fsub_rn(u, fl);
    // the cell, periodic: one conditional add or subtract unless the
    // displacement exceeds the box
    int ci = (int)qi + (int)fl;
    if (ci >= nm) ci -= nm;
    else if (ci < 0) ci += nm;
    if ((uint32_t)ci >= (uint32_t)nm) {
      ci %= nm;
      if (ci < 0) ci += nm;
    }
    c[e] = ci;
  }
}

__device__ __forceinline__ void home_cell(const float* __restrict__ disp, long np3, uint32_t id,
                                          int np, int nm, float dscale, int c[3], float f[3]) {
  const float dv[3] = {disp[id], disp[np3 + id], disp[2 * np3 + id]};
  home_cell_of(dv, id, np, nm, dscale, c, f);
}

// CIC weight of offset k = 4 sx + 2 sy + sz: (w_sx(fx) * w_sy(fy)) * w_sz(fz),
// w_0(f) = 1 - f, w_1(f) = f; two float32 roundings, no fused multiply-add.
__device__ __forceinline__ float cic_weight(const float f[3], int k) {
#pragma clang fp contract(off)
  const float wx = (k & 4) ? f[0] : __fsub_rn(1.0f, f[0]);
  const float wy = (k & 2) ? f[1] : __fsub_rn(1.0f, f[1]);
  const float wz = (k & 1) ? f[2] : __fsub_rn(1.0f, f[2]);
  return __fmul_rn(__fmul_rn(wx, wy), wz);
}

// The PM step's force field, interleaved by node: (g_x, g_y, g_z) of node
// (x, y, z) at g[(x nm + y) row_stride + 3 z + {0, 1, 2}].  Offset of the
// first component of the 8 nodes of home cell c, in the order of k.
struct ForceCorners {
  long rows[4];
  int z0, z1;
  __device__ __forceinline__ ForceCorners(const int c[3], int nm, long row_stride) {
    const int cx1 = c[0] + 1 == nm ? 0 : c[0] + 1;
    const int cy1 = c[1] + 1 == nm ? 0 : c[1] + 1;
    const int cz1 = c[2] + 1 == nm ? 0 : c[2] + 1;
    rows[0] = ((long)c[0] * nm + c[1]) * row_stride;
    rows[1] = ((long)c[0] * nm + cy1) * row_stride;
    rows[2] = ((long)cx1 * nm + c[1]) * row_stride;
    rows[3] = ((long)cx1 * nm + cy1) * row_stride;
    z0 = 3 * c[2];
    z1 = 3 * cz1;
  }
  __device__ __forceinline__ long at(int k) const { return rows[k >> 1] + ((k & 1) ? z1 : z0); }
};

// CIC readout of the three force components at a particle (offsets k = 0 .. 7
// in order, the deposit's weights).
__device__ __forceinline__ void force_readout(const float* __restrict__ g, long row_stride, int nm,
                                              const int c[3], const float f[3], float F[3]) {
  const ForceCorners fc(c, nm, row_stride);
  F[0] = F[1] = F[2] = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float w = cic_weight(f, k);
    const float* q = g + fc.at(k);
    F[0] += w * q[0];
    F[1] += w * q[1];
    F[2] += w * q[2];
  }
}

// Tile (16^3 cells) and class bits of a home cell: class bit 4/2/1 set when
// the cell is on the upper x/y/z face of its tile (it then also feeds nodes
// of the next tile along that axis).  nt = tiles per side.
__device__ __forceinline__ uint32_t bucket_of(const int c[3], int nt) {
  const uint32_t tile = ((uint32_t)(c[0] >> 4) * nt + (uint32_t)(c[1] >> 4)) * nt + (uint32_t)(c[2] >> 4);
  const uint32_t cls = (((c[0] & 15) == 15) << 2) | (((c[1] & 15) == 15) << 1) | ((c[2] & 15) == 15);
  return tile * 8u + cls;
}

// Workgroup order across the 8 XCDs of the chip: consecutive hardware
// workgroup ids go to different XCDs; remap so each XCD walks a contiguous
// range of tiles (shared cache lines stay in one XCD's L2).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nblocks) {
  const uint32_t nx = 8;
  const uint32_t per = (nblocks + nx - 1) / nx;
  const uint32_t xcd = bid % nx, local = bid / nx;
  const uint32_t full = nblocks % nx == 0 ? nx : nblocks % nx;  // XCDs that get `per` blocks
  uint32_t base;
  if (xcd < full) base = xcd * per;
  else base = full * per + (xcd - full) * (per - 1);
  return base + local;
}

// Particle of thread t (0..255) in block b of a particle-parallel launch of
// np^3 / 256 blocks: blocks tile the lattice in sub-cubes of 2 x 4 x 32 ids
// (4 x 4 x 16 when np is not a multiple of 32; every supported np is a
// multiple of 16), k fastest inside a block and across blocks.  Particles of
// one block stay close in space as they cluster, so they share the mesh
// lines they read; rows of 32 (16) consecutive ids keep the state arrays'
// accesses in whole cache lines.
__device__ __forceinline__ long subcube_particle(uint32_t b, int t, int np) {
  const int lk = (np & 31) == 0 ? 5 : 4;           // ids along k per block row: 32 or 16
  const int si = 256 >> (lk + 2);                   // block depth along i: 2 or 4
  const uint32_t nbk = (uint32_t)np >> lk, nbj = (uint32_t)np >> 2;
  const uint32_t bk = b % nbk, bj = (b / nbk) % nbj, bi = b / (nbk * nbj);
  const int k = (int)bk * (1 << lk) + (t & ((1 << lk) - 1));
  const int j = (int)bj * 4 + ((t >> lk) & 3);
  const int i = (int)bi * si + (t >> (lk + 2));
  return ((long)i * np + j) * np + k;
}

// The same for the force readout and its adjoint.  Where the mesh is at
// least 3x the particle grid (particles 3 or more cells apart) and np is a
// multiple of 256: one row of 256 ids along k (1.13 against 1.24 ms for
// 8 x 1 x 32 columns at 256^3 / 768^3).  Otherwise blocks of 4 x 2 x 32 ids
// (i, j, k; 47.0 against 47.7 ms for 8 x 1 x 32 at 1024^3 / 2048^3, where
// rows of 64, 128 and 256 along k take 48.7, 53.3 and 59.5 ms and 16 x 1 x
// 16 56.1 ms), or 16 x 1 x 16 when np is not a multiple of 32.
__device__ __forceinline__ long readout_particle(uint32_t b, int t, int np, int nm) {
  if (nm >= 3 * np && (np & 255) == 0) {
    const uint32_t bj = b % (uint32_t)np, bi = b / (uint32_t)np;
    return ((long)bi * np + (int)bj) * np + t;
  }
  const int lk = (np & 31) == 0 ? 5 : 4;           // ids along k per block row: 32 or 16
  const int lj = lk == 5 ? 1 : 0;                   // block depth along j: 2 or 1
  const uint32_t nbk = (uint32_t)np >> lk, nbj = (uint32_t)np >> lj;
  const uint32_t bk = b % nbk, bj = (b / nbk) % nbj, bi = b / (nbk * nbj);
  const int k = (int)bk * (1 << lk) + (t & ((1 << lk) - 1));
  const int j = (int)bj * (1 << lj) + ((t >> lk) & ((1 << lj) - 1));
  const int i = (int)bi * (256 >> (lk + lj)) + (t >> (lk + lj));
  return ((long)i * np + j) * np + k;
}

// Mock index of a batched launch is blockIdx.z; every per-mock array of a
// batch sits at the same offset inside equal per-mock workspace blocks, so a
// single byte stride locates mock b's copy of any array.
template <class T>
__device__ __forceinline__ T* mock_ptr(T* p, long mstride) {
  using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return reinterpret_cast<T*>(reinterpret_cast<B*>(p) + (long)blockIdx.z * mstride);
}

}  // namespace cola
