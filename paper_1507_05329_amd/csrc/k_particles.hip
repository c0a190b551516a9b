// CIC force readout fused with the COLA kick and drift (Koda et al. 2015,
// Sec. 2.2, eqs. cola-kick and cola-drift; 2LPT growing mode of Sec. 2.1).
//
// Per particle (one thread each; blocks walk the lattice in columns of
// particles, see readout_particle):
//   F_d   = sum_s w_s g_d[c + s]                      (same CIC weights as the deposit)
//   v_d  += K F_d - c1 Psi1_d - c2 Psi2_d             (c1 = K alpha D1, c2 = K alpha (D2 - D1^2):
//                                                      the residual force F - d^2/dt^2-term of 2LPT)
//   d_d  += I v_d + e1 Psi1_d + e2 Psi2_d             (e1 = dD1, e2 = dD2)
// The force field is interleaved by node (cola_device.h: force_readout), so
// a corner's three components share one cache line; it is read before the
// particle's own position is updated, so the update is in place.
#include "cola_device.h"
#include "cola_internal.h"

namespace cola {

// FORCE_ONLY: write the interpolated force (no kick or drift).  Otherwise
// the particle's state is requested together with its displacement, so its
// loads are in flight during the mesh gathers.
template <bool FORCE_ONLY>
__global__ __launch_bounds__(256) void k_readout_kick_drift(
    const float* __restrict__ g, long row_stride, float* __restrict__ disp, float* __restrict__ vres,
    const float* __restrict__ psi1, const float* __restrict__ psi2, int np, int nm, long np3,
    const StepCoef* __restrict__ coef, float* __restrict__ force_out, long mstride) {
  // neighbouring blocks share mesh lines: keep them on one XCD (L2)
  const long i = readout_particle(xcd_remap(blockIdx.x, gridDim.x), threadIdx.x, np, nm);
  if (i >= np3) return;
  g = mock_ptr(g, mstride);
  disp = mock_ptr(disp, mstride);
  float d0[3], v0[3], p1[3], p2[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) d0[d] = disp[d * np3 + i];
  if constexpr (!FORCE_ONLY) {
    vres = mock_ptr(vres, mstride);
    psi1 = mock_ptr(psi1, mstride);
    psi2 = mock_ptr(psi2, mstride);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      v0[d] = vres[d * np3 + i];
      p1[d] = psi1[d * np3 + i];
      p2[d] = psi2[d * np3 + i];
    }
  }
  // every state load issued before the mesh gathers (the scheduler would
  // otherwise sink some below the first store: one more memory round trip)
  __builtin_amdgcn_sched_barrier(0);
  int c[3];
  float f[3];
  home_cell_of(d0, (uint32_t)i, np, nm, 1.0f, c, f);
  float F[3];
  force_readout(g, row_stride, nm, c, f, F);
  if constexpr (FORCE_ONLY) {
    force_out = mock_ptr(force_out, mstride);
#pragma unroll
    for (int d = 0; d < 3; ++d) force_out[d * np3 + i] = F[d];
  } else {
    const KickDrift kd = mock_ptr(coef, mstride)->kd;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const long j = d * np3 + i;
      const float v = v0[d] + kd.K * F[d] - kd.c1 * p1[d] - kd.c2 * p2[d];
      vres[j] = v;
      disp[j] = d0[d] + kd.I * v + kd.e1 * p1[d] + kd.e2 * p2[d];
    }
  }
}

void launch_readout_kick_drift(const float* g, long row_stride, float* disp, float* vres, const float* psi1,
                               const float* psi2, int np, int nm, const StepCoef* coef, float* force_out,
                               hipStream_t s, int nmock, long mstride) {
  const long np3 = (long)np * np * np;
  const dim3 grid((unsigned)((np3 + 255) / 256), 1, (unsigned)nmock);
  if (force_out)
    hipLaunchKernelGGL(k_readout_kick_drift<true>, grid, dim3(256), 0, s, g, row_stride, disp, vres,
                       psi1, psi2, np, nm, np3, coef, force_out, mstride);
  else
    hipLaunchKernelGGL(k_readout_kick_drift<false>, grid, dim3(256), 0, s, g, row_stride, disp,
                       vres, psi1, psi2, np, nm, np3, coef, force_out, mstride);
}

__global__ void k_set_coef(StepCoef* dst, StepCoef v, long mstride) { *mock_ptr(dst, mstride) = v; }

void launch_set_coef(StepCoef* dst, const StepCoef& v, int nmock, long mstride, hipStream_t s) {
  hipLaunchKernelGGL(k_set_coef, dim3(1, 1, (unsigned)nmock), dim3(1), 0, s, dst, v, mstride);
}

__global__ void k_check_finite(const float* __restrict__ x, long n, uint32_t* flag) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) { atomicOr(flag, 1u); return; }
}

void launch_check_finite(const float* x, long n, uint32_t* flag, hipStream_t s) {
  long blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(256), 0, s, x, n, flag);
}

}  // namespace cola
