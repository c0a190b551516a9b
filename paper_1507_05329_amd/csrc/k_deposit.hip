// Deterministic CIC mass assignment as a gather (no float atomics).
//
// CIC (Koda et al. 2015, Sec. 3.3; Hockney & Eastwood): a particle with home
// cell c and fraction f gives weight prod_e w_{s_e}(f_e) to node c + s.
// One workgroup owns a 16^3 tile of nodes.  The cells that feed those nodes
// are the tile's 16^3 cells plus the one-cell layer below it on each axis
// (a 17^3 region); their particles come from the tile's buckets and from the
// face/edge/corner buckets of the 7 lower neighbour tiles.
//
// Mass (k_deposit_mass): every weight is taken to 64-bit fixed point,
// q = rint(w 2^32), and the tile's nodes add them with integer LDS atomics;
// the integer sum is exact, so the node mass float32(sum) 2^-32 does not
// depend on the order of the particles, the buckets or the workgroups.  The
// particles are streamed, never held, so a region of any size takes one pass.
//
// Weighted deposits (k_deposit, NC = 3: the transpose of the
// three-component readout; weights of either sign and any size): particles
// are keyed (region cell, particle id, LDS slot) and sorted in LDS, so each
// cell's 8 partial sums add its particles' weights in ascending id.  Nodes
// then receive the partial sums of their 8 source cells in ascending
// source-cell order, in 8 phases (offset k = 7 .. 0) that are each
// conflict-free (distinct cells -> distinct nodes).  Regions holding more
// particles than fit in LDS are processed in contiguous ranges of their
// cells (halved until they fit), a single overfull cell by an ordered
// selection, keeping the same order.
#include "cola_device.h"
#include "cola_internal.h"

// Every float operation in this file is a single IEEE rounding (the
// deterministic order is part of the result): no fused multiply-add.
#pragma clang fp contract(off)

namespace cola {

constexpr int kTile = 16;                 // nodes per tile side
constexpr int kReg = kTile + 1;           // region side (tile + lower layer)
constexpr int kNReg = kReg * kReg * kReg;
constexpr int kSlotBits = 11;             // slot field width (capacity <= 2048)
constexpr int kIdBits = 30;
constexpr int kMaxSeg = 32;
static_assert(kNReg < (1 << (64 - kIdBits - kSlotBits)), "cell field");

// NC = 1: unit masses (density).  NC = 3: three weighted deposits at once
// (the transpose of the three-component CIC readout); weights are read by
// particle id from global memory.
// NC deposits, CAP particles held in LDS at once (power of two), DT threads.
template <int NC, int CAP, int DT>
struct DepShared {
  static constexpr int kNC = NC, kCap = CAP, kT = DT;
  uint64_t keys[kCap];                    // cell << 41 | id << 11 | slot
  float fx[kCap], fy[kCap], fz[kCap];
  alignas(16) float rho[NC][kTile * kTile * kTile];
  uint16_t run[kCap + 1];                 // start of each run of equal cell
  uint32_t scan[DT / 64];
  uint32_t seg_start[kMaxSeg], seg_len[kMaxSeg];
  uint32_t seg_pre[kMaxSeg];              // particles in the segments before
  uint32_t seg_total;
  uint32_t offs[8][9];                    // bucket offsets of the 8 source tiles
  int nseg;
  int nrun;
  uint32_t count;
  uint32_t red[DT / 64];
  float acc8[8 * NC];
};

__device__ __forceinline__ int region_coord(int c, int t0, int nm) {
  int r = c - t0 + 1;
  if (r < 0) r += nm;
  if (r >= nm) r -= nm;
  return r;
}

__device__ __forceinline__ uint32_t key_cell(uint64_t k) { return (uint32_t)(k >> (kIdBits + kSlotBits)); }
__device__ __forceinline__ uint32_t key_id(uint64_t k) { return (uint32_t)(k >> kSlotBits) & ((1u << kIdBits) - 1u); }
__device__ __forceinline__ uint32_t key_slot(uint64_t k) { return (uint32_t)k & ((1u << kSlotBits) - 1u); }

// Takes the particles whose region cell lies in [lo, hi).
// Returns the number of matching particles (keys stored only when <= kCap).
// The segments are one index space of seg_total particles; a thread takes
// kG of them per round, issuing all their loads before using any.
constexpr int kG = 2;
template <class S>
__device__ uint32_t gather_keys(S& sh, const float* __restrict__ disp,
                                const uint32_t* __restrict__ perm, long np3, int np, int nm,
                                float dscale, const int t0[3], int lo, int hi) {
  constexpr int kDT = S::kT;
  if (threadIdx.x == 0) sh.count = 0;
  __syncthreads();
  const uint32_t total = sh.seg_total;
  const int nseg = sh.nseg;
  for (uint32_t base = 0; base < total; base += kG * kDT) {
    uint32_t ids[kG];
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      const uint32_t x = base + g * kDT + threadIdx.x;
      ids[g] = 0xffffffffu;
      if (x < total) {
        int sg = 0;  // last segment with seg_pre <= x
#pragma unroll
        for (int step = kMaxSeg / 2; step > 0; step >>= 1)
          if (sg + step < nseg && sh.seg_pre[sg + step] <= x) sg += step;
        ids[g] = perm[sh.seg_start[sg] + (x - sh.seg_pre[sg])];
      }
    }
    int c[kG][3];
    float f[kG][3];
#pragma unroll
    for (int g = 0; g < kG; ++g)
      if (ids[g] != 0xffffffffu) home_cell(disp, np3, ids[g], np, nm, dscale, c[g], f[g]);
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      if (ids[g] == 0xffffffffu) continue;
      const int rx = region_coord(c[g][0], t0[0], nm), ry = region_coord(c[g][1], t0[1], nm),
                rz = region_coord(c[g][2], t0[2], nm);
      const bool inside = rx < kReg && ry < kReg && rz < kReg;
      const int lc = (rx * kReg + ry) * kReg + rz;
      const bool pass = inside && lc >= lo && lc < hi;
      if (pass) {
        const uint32_t slot = atomicAdd(&sh.count, 1u);
        if (slot < (uint32_t)S::kCap) {
          sh.keys[slot] = ((uint64_t)lc << (kIdBits + kSlotBits)) | ((uint64_t)ids[g] << kSlotBits) | slot;
          sh.fx[slot] = f[g][0];
          sh.fy[slot] = f[g][1];
          sh.fz[slot] = f[g][2];
        }
      }
    }
  }
  __syncthreads();
  const uint32_t n = sh.count;
  // every thread has its copy before a later call's thread 0 resets count
  __syncthreads();
  return n;
}

// Bitonic sort of keys[0, n) ascending (padding with ~0).  Each active
// thread holds E = p2/kDT (>= 1) consecutive keys in registers; compare-
// exchange partners closer than 64 E are reached through registers or lane
// shuffles, farther ones through LDS (two barriers per such stage).
template <int E, class S>
__device__ void bitonic_regs(S& sh, uint32_t p2) {
  constexpr int kDT = S::kT;
  const uint32_t tid = threadIdx.x;
  const bool act = tid * E < p2;
  uint64_t v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = act ? sh.keys[tid * E + e] : ~0ull;
  for (uint32_t k = 2; k <= p2; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      if (j >= 64u * E) {
        __syncthreads();
        if (act) {
#pragma unroll
          for (int e = 0; e < E; ++e) sh.keys[tid * E + e] = v[e];
        }
        __syncthreads();
        if (act) {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const uint32_t i = tid * E + e;
            const uint64_t o = sh.keys[i ^ j];
            const bool up = (i & k) == 0;
            const bool lower = (i & j) == 0;
            v[e] = (lower == up) ? (v[e] < o ? v[e] : o) : (v[e] < o ? o : v[e]);
          }
        }
      } else if (j >= (uint32_t)E) {
        const int lanemask = (int)(j / E);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const uint32_t i = tid * E + e;
          const uint64_t o = __shfl_xor(v[e], lanemask, 64);
          const bool up = (i & k) == 0;
          const bool lower = (i & j) == 0;
          v[e] = (lower == up) ? (v[e] < o ? v[e] : o) : (v[e] < o ? o : v[e]);
        }
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if ((e & j) == 0) {
            const uint32_t i = tid * E + e;
            const int e2 = e ^ (int)j;
            const bool up = (i & k) == 0;
            const uint64_t a = v[e], b = v[e2];
            if ((a > b) == up) {
              v[e] = b;
              v[e2] = a;
            }
          }
        }
      }
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int e = 0; e < E; ++e) sh.keys[tid * E + e] = v[e];
  }
  __syncthreads();
}

template <class S>
__device__ void sort_keys(S& sh, uint32_t n) {
  constexpr int kDT = S::kT;
  uint32_t p2 = 64;
  while (p2 < n) p2 <<= 1;
  for (uint32_t j = n + threadIdx.x; j < p2; j += kDT) sh.keys[j] = ~0ull;
  __syncthreads();
  if (p2 <= (uint32_t)kDT) bitonic_regs<1>(sh, p2);
  else if (p2 <= 2u * kDT) bitonic_regs<2>(sh, p2);
  else if constexpr (S::kCap >= 4 * kDT) bitonic_regs<4>(sh, p2);
}

// Ordered list of run starts (runs of equal cell in the sorted keys):
// wave-level scan of start flags, one barrier for the wave totals.
template <class S>
__device__ void find_runs(S& sh, uint32_t n) {
  constexpr int kDT = S::kT;
  constexpr int kPer = S::kCap / kDT;
  uint32_t flags = 0, cnt = 0;
  const uint32_t base = threadIdx.x * kPer;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const uint32_t j = base + q;
    const bool st = j < n && (j == 0 || key_cell(sh.keys[j]) != key_cell(sh.keys[j - 1]));
    flags |= (uint32_t)st << q;
    cnt += st;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = cnt;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t a = __shfl_up(incl, off, 64);
    if (lane >= off) incl += a;
  }
  if (lane == 63) sh.scan[wave] = incl;
  __syncthreads();
  uint32_t before = 0, total = 0;
  for (int w = 0; w < kDT / 64; ++w) {
    const uint32_t t = sh.scan[w];
    if (w < wave) before += t;
    total += t;
  }
  uint32_t pos = before + incl - cnt;
#pragma unroll
  for (int q = 0; q < kPer; ++q)
    if (flags >> q & 1u) sh.run[pos++] = (uint16_t)(base + q);
  if (threadIdx.x == 0) {
    sh.nrun = (int)total;
    sh.run[total] = (uint16_t)n;
  }
  __syncthreads();
}

// Adds the 8 partial sums of region cell lc to its tile nodes for offset k.
template <class S>
__device__ __forceinline__ void add_partial(S& sh, int lc, int k, const float* acc) {
  constexpr int NC = S::kNC;
  const int rx = lc / (kReg * kReg), ry = (lc / kReg) % kReg, rz = lc % kReg;
  const int nx = rx + ((k >> 2) & 1) - 1, ny = ry + ((k >> 1) & 1) - 1, nz = rz + (k & 1) - 1;
  if (nx >= 0 && nx < kTile && ny >= 0 && ny < kTile && nz >= 0 && nz < kTile) {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      float& r = sh.rho[q][(nx * kTile + ny) * kTile + nz];
      r = __fadd_rn(r, acc[q]);
    }
  }
}

// Partial sums of the n sorted keys (runs of equal cell, ascending id), then
// the node accumulation in 8 phases k = 7 .. 0.  In phase k every node gets
// at most one contribution (from cell n - s_k), so the phases fix the order
// (ascending source cell) whatever the assignment of runs to threads.
template <class S>
__device__ void accumulate_sorted(S& sh, uint32_t n, const float* __restrict__ wt,
                                  long np3) {
  constexpr int NC = S::kNC, kDT = S::kT;
  constexpr int kRuns = S::kCap / kDT;  // runs per thread (nrun <= n <= kCap)
  find_runs(sh, n);
  const int nrun = sh.nrun;
  float acc[kRuns][8][NC];
  int lcs[kRuns];
#pragma unroll
  for (int q = 0; q < kRuns; ++q) {
    const int r = (int)threadIdx.x + q * kDT;
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[q][k][c] = 0.0f;
    lcs[q] = -1;
    if (r < nrun) {
      const uint32_t j0 = sh.run[r], j1 = sh.run[r + 1];
      lcs[q] = (int)key_cell(sh.keys[j0]);
      for (uint32_t j = j0; j < j1; ++j) {
        const uint64_t key = sh.keys[j];
        const uint32_t sl = key_slot(key);
        const float f[3] = {sh.fx[sl], sh.fy[sl], sh.fz[sl]};
        float m[NC];
        if constexpr (NC == 1) {
          m[0] = 1.0f;
        } else {
          const uint32_t id = key_id(key);
#pragma unroll
          for (int c = 0; c < NC; ++c) m[c] = wt[c * np3 + id];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const float w = cic_weight(f, k);
#pragma unroll
          for (int c = 0; c < NC; ++c)
            acc[q][k][c] = __fadd_rn(acc[q][k][c], NC == 1 ? w : __fmul_rn(m[c], w));
        }
      }
    }
  }
#pragma unroll
  for (int k = 7; k >= 0; --k) {
#pragma unroll
    for (int q = 0; q < kRuns; ++q)
      if (lcs[q] >= 0) add_partial(sh, lcs[q], k, acc[q][k]);
    __syncthreads();
  }
}

// A cell with more than kCap particles: its weights added in ascending id by
// repeated workgroup-wide minimum search (slow; extreme clustering only).
template <class S>
__device__ void accumulate_select(S& sh, const float* __restrict__ disp,
                                  const uint32_t* __restrict__ perm, long np3, int np, int nm,
                                  float dscale, const int t0[3], int lc_target,
                                  const float* __restrict__ wt) {
  constexpr int NC = S::kNC, kDT = S::kT;
  if (threadIdx.x < 8 * NC) sh.acc8[threadIdx.x] = 0.0f;
  uint32_t last = 0;
  bool first = true;
  for (;;) {
    uint32_t best = 0xffffffffu;
    for (int s = 0; s < sh.nseg; ++s) {
      for (uint32_t j = threadIdx.x; j < sh.seg_len[s]; j += kDT) {
        const uint32_t id = perm[sh.seg_start[s] + j];
        if ((!first && id <= last) || id >= best) continue;
        int c[3];
        float f[3];
        home_cell(disp, np3, id, np, nm, dscale, c, f);
        const int lc = (region_coord(c[0], t0[0], nm) * kReg + region_coord(c[1], t0[1], nm)) * kReg +
                       region_coord(c[2], t0[2], nm);
        if (lc == lc_target) best = id;
      }
    }
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
      for (int k = 0; k < 8; ++k) {
        const float w = cic_weight(f, k);
        for (int q = 0; q < NC; ++q)
          sh.acc8[k * NC + q] = __fadd_rn(sh.acc8[k * NC + q], NC == 1 ? w : __fmul_rn(wt[q * np3 + m], w));
      }
    }
    last = m;
    first = false;
    __syncthreads();
  }
#pragma unroll
  for (int k = 7; k >= 0; --k) {
    if (threadIdx.x == 0) add_partial(sh, lc_target, k, &sh.acc8[k * NC]);
    __syncthreads();
  }
}

// The region's particles as up to kMaxSeg segments of the permutation, in
// a fixed order: thread nb < 8 takes the buckets of source tile
// (tx, ty, tz) - (dx, dy, dz), nb = 4 dx + 2 dy + dz, whose face class covers
// the offset bits; empty segments are dropped and seg_pre holds the
// particles before each (one index space of seg_total particles).  Ends
// with a barrier.
template <class S>
__device__ void setup_segments(S& sh, const uint32_t* __restrict__ off, int tx, int ty, int tz, int nt) {
  // Bucket offsets of the source tiles (tx-dx, ty-dy, tz-dz), one per thread.
  if (threadIdx.x < 72) {
    const int nb = threadIdx.x / 9, q = threadIdx.x - nb * 9;
    const int dx = (nb >> 2) & 1, dy = (nb >> 1) & 1, dz = nb & 1;
    int ux = tx - dx, uy = ty - dy, uz = tz - dz;
    if (ux < 0) ux += nt;
    if (uy < 0) uy += nt;
    if (uz < 0) uz += nt;
    sh.offs[nb][q] = off[(((uint32_t)ux * nt + uy) * nt + uz) * 8u + q];
  }
  __syncthreads();
  // Segments: thread nb < 8 takes the buckets of source tile nb whose face
  // class covers the required offset bits.
  if (threadIdx.x < 8) {
    const int nb = threadIdx.x;
    uint32_t o[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) o[q] = sh.offs[nb][q];
    int slot = nb * 4;
    int cls = 0;
    while (cls < 8) {
      if ((cls & nb) != nb) { ++cls; continue; }
      int c2 = cls;
      while (c2 + 1 < 8 && ((c2 + 1) & nb) == nb) ++c2;
      sh.seg_start[slot] = o[cls];
      sh.seg_len[slot] = o[c2 + 1] - o[cls];
      ++slot;
      cls = c2 + 1;
    }
    for (; slot < nb * 4 + 4; ++slot) sh.seg_len[slot] = 0;
  }
  __syncthreads();
  // Drop the empty segments, keeping their order (one wave: ballot for the
  // positions, a lane scan for the particles before each segment).
  if (threadIdx.x < 64) {
    const int q = threadIdx.x;
    const uint32_t len = q < kMaxSeg ? sh.seg_len[q] : 0u;
    const uint32_t st = q < kMaxSeg ? sh.seg_start[q] : 0u;
    const uint64_t mask = __ballot(len > 0);
    uint32_t incl = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t a = __shfl_up(incl, o, 64);
      if (q >= o) incl += a;
    }
    if (len > 0) {
      const int pos = __popcll(mask & ((1ull << q) - 1ull));
      sh.seg_start[pos] = st;
      sh.seg_len[pos] = len;
      sh.seg_pre[pos] = incl - len;
    }
    if (q == 63) {
      sh.nseg = __popcll(mask);
      sh.seg_total = incl;
    }
  }
  __syncthreads();
}

template <int NC, int CAP, int kDT>
__global__ __launch_bounds__(kDT) void k_deposit(const float* __restrict__ disp,
                                                 const uint32_t* __restrict__ perm,
                                                 const uint32_t* __restrict__ off, int np, int nm,
                                                 float dscale, long np3, float* __restrict__ out,
                                                 long row_stride, long mesh_stride, int contrast,
                                                 float cinv, const float* __restrict__ wt,
                                                 long mstride) {
  __shared__ DepShared<NC, CAP, kDT> sh;
  disp = mock_ptr(disp, mstride);
  perm = mock_ptr(perm, mstride);
  off = mock_ptr(off, mstride);
  out = mock_ptr(out, mstride);
  if (wt) wt = mock_ptr(wt, mstride);
  constexpr uint32_t kCap = CAP;
  const int nt = nm / kTile;
  const uint32_t t = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = t / (nt * nt), ty = (t / nt) % nt, tz = t % nt;
  const int t0[3] = {tx * kTile, ty * kTile, tz * kTile};

  for (int i = threadIdx.x; i < kTile * kTile * kTile; i += kDT)
#pragma unroll
    for (int q = 0; q < NC; ++q) sh.rho[q][i] = 0.0f;
  setup_segments(sh, off, tx, ty, tz, nt);

  // The region's cells in contiguous ranges [lo, hi) of the cell index,
  // taken in increasing order; a range holding more than kCap particles is
  // halved.  A node's contributions then still arrive in ascending source
  // cell, i.e. descending offset k (k = 7 comes from the lowest cell), across
  // ranges as within one.  A single cell above kCap: ordered selection.
  int lo = 0, hi = kNReg;
  uint32_t n = gather_keys(sh, disp, perm, np3, np, nm, dscale, t0, lo, hi);
  for (;;) {
    if (n <= kCap || hi - lo == 1) {
      if (n > kCap) {
        accumulate_select(sh, disp, perm, np3, np, nm, dscale, t0, lo, wt);
      } else if (n > 0) {
        sort_keys(sh, n);
        accumulate_sorted(sh, n, wt, np3);
      }
      if (hi == kNReg) break;
      lo = hi;
      hi = kNReg;
    } else {
      hi = lo + (hi - lo) / 2;
    }
    n = gather_keys(sh, disp, perm, np3, np, nm, dscale, t0, lo, hi);
  }

  // four consecutive z nodes per thread and store (rows of the padded
  // layout and tile origins are 16-byte aligned); measured 1.60 against
  // 1.65 ms on the 768^3 mesh with one node per store
  for (int qd = threadIdx.x; qd < kTile * kTile * kTile / 4; qd += kDT) {
    const int nn = qd * 4;
    const int nx = nn / (kTile * kTile), ny = (nn / kTile) % kTile, nz = nn % kTile;
    const long o = ((long)(t0[0] + nx) * nm + (t0[1] + ny)) * row_stride + (t0[2] + nz);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      float4 r = *reinterpret_cast<const float4*>(&sh.rho[q][nn]);
      if (contrast) {
        r.x = __fsub_rn(__fmul_rn(r.x, cinv), 1.0f);
        r.y = __fsub_rn(__fmul_rn(r.y, cinv), 1.0f);
        r.z = __fsub_rn(__fmul_rn(r.z, cinv), 1.0f);
        r.w = __fsub_rn(__fmul_rn(r.w, cinv), 1.0f);
      }
      *reinterpret_cast<float4*>(out + q * mesh_stride + o) = r;
    }
  }
}

// Fixed-point mass deposit: node masses in units of 2^-32 particle masses.
struct MassShared {
  unsigned long long acc[kTile * kTile * kTile];   // 32 KB
  uint32_t seg_start[kMaxSeg], seg_len[kMaxSeg];
  uint32_t seg_pre[kMaxSeg];
  uint32_t seg_total;
  uint32_t offs[8][9];
  int nseg;
};

constexpr float kFixScale = 4294967296.0f;           // 2^32
constexpr float kFixInv = 2.3283064365386963e-10f;   // 2^-32
constexpr int kMassG = 4;                            // particles in flight per thread

template <int kDT>
__global__ __launch_bounds__(kDT) void k_deposit_mass(const float* __restrict__ disp,
                                                      const uint32_t* __restrict__ perm,
                                                      const uint32_t* __restrict__ off, int np, int nm,
                                                      float dscale, long np3, float* __restrict__ out,
                                                      long row_stride, int contrast, float cinv,
                                                      long mstride) {
  __shared__ MassShared sh;
  disp = mock_ptr(disp, mstride);
  perm = mock_ptr(perm, mstride);
  off = mock_ptr(off, mstride);
  out = mock_ptr(out, mstride);
  const int nt = nm / kTile;
  const uint32_t t = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = t / (nt * nt), ty = (t / nt) % nt, tz = t % nt;
  const int t0[3] = {tx * kTile, ty * kTile, tz * kTile};
  for (int i = threadIdx.x; i < kTile * kTile * kTile; i += kDT) sh.acc[i] = 0ull;
  setup_segments(sh, off, tx, ty, tz, nt);

  const uint32_t total = sh.seg_total;
  const int nseg = sh.nseg;
  for (uint32_t base = 0; base < total; base += kMassG * kDT) {
    uint32_t ids[kMassG];
#pragma unroll
    for (int g = 0; g < kMassG; ++g) {
      const uint32_t x = base + g * kDT + threadIdx.x;
      ids[g] = 0xffffffffu;
      if (x < total) {
        int sg = 0;  // last segment with seg_pre <= x
#pragma unroll
        for (int step = kMaxSeg / 2; step > 0; step >>= 1)
          if (sg + step < nseg && sh.seg_pre[sg + step] <= x) sg += step;
        ids[g] = perm[sh.seg_start[sg] + (x - sh.seg_pre[sg])];
      }
    }
    int c[kMassG][3];
    float f[kMassG][3];
#pragma unroll
    for (int g = 0; g < kMassG; ++g)
      if (ids[g] != 0xffffffffu) home_cell(disp, np3, ids[g], np, nm, dscale, c[g], f[g]);
#pragma unroll
    for (int g = 0; g < kMassG; ++g) {
      if (ids[g] == 0xffffffffu) continue;
      // region coordinates 0..16; the tile's nodes are region 1..16, and a
      // cell at r feeds nodes r and r + 1, i.e. tile nodes r - 1 and r
      const int rx = region_coord(c[g][0], t0[0], nm), ry = region_coord(c[g][1], t0[1], nm),
                rz = region_coord(c[g][2], t0[2], nm);
      if (rx >= kReg || ry >= kReg || rz >= kReg) continue;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int nx = rx + ((k >> 2) & 1) - 1, ny = ry + ((k >> 1) & 1) - 1, nz = rz + (k & 1) - 1;
        if (nx < 0 || nx >= kTile || ny < 0 || ny >= kTile || nz < 0 || nz >= kTile) continue;
        const unsigned long long q = __float2ull_rn(__fmul_rn(cic_weight(f[g], k), kFixScale));
        atomicAdd(&sh.acc[(nx * kTile + ny) * kTile + nz], q);
      }
    }
  }
  __syncthreads();

  // four consecutive z nodes per thread and store (rows of the padded
  // layout and tile origins are 16-byte aligned)
  for (int qd = threadIdx.x; qd < kTile * kTile * kTile / 4; qd += kDT) {
    const int nn = qd * 4;
    const int nx = nn / (kTile * kTile), ny = (nn / kTile) % kTile, nz = nn % kTile;
    const long o = ((long)(t0[0] + nx) * nm + (t0[1] + ny)) * row_stride + (t0[2] + nz);
    float r[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      r[j] = __fmul_rn(__ull2float_rn(sh.acc[nn + j]), kFixInv);
      if (contrast) r[j] = __fsub_rn(__fmul_rn(r[j], cinv), 1.0f);
    }
    *reinterpret_cast<float4*>(out + o) = make_float4(r[0], r[1], r[2], r[3]);
  }
}

// One 256-thread workgroup per tile, 33 KB of LDS (four tiles per compute
// unit).  The result does not depend on the shape.
void launch_deposit(const float* disp, const uint32_t* perm, const uint32_t* off, int np, int nm,
                    float dscale, float* out, long row_stride, int contrast, hipStream_t s,
                    int nmock, long mstride) {
  const long np3 = (long)np * np * np;
  const int nt = nm / kTile;
  const long ntiles = (long)nt * nt * nt;
  const float cinv = (float)((double)nm * nm * nm / (double)np3);
  hipLaunchKernelGGL(k_deposit_mass<256>, dim3((unsigned)ntiles, 1, (unsigned)nmock), dim3(256), 0, s, disp,
                     perm, off, np, nm, dscale, np3, out, row_stride, contrast, cinv, mstride);
}

void launch_deposit3_weighted(const float* disp, const uint32_t* perm, const uint32_t* off, int np,
                              int nm, const float* wt, float* out, long row_stride,
                              long mesh_stride_floats, hipStream_t s) {
  const long np3 = (long)np * np * np;
  const int nt = nm / kTile;
  const long ntiles = (long)nt * nt * nt;
  hipLaunchKernelGGL((k_deposit<3, 1024, 512>), dim3((unsigned)ntiles), dim3(512), 0, s, disp, perm, off,
                     np, nm, 1.0f, np3, out, row_stride, mesh_stride_floats, 0, 1.0f, wt, 0L);
}

}  // namespace cola
