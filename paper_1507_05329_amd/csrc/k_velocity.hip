// Particle velocities at the position time and redshift-space displacements
// (Koda et al. 2015: Sec. 2.1, velocity = residual + time derivative of the
// 2LPT trajectory; Sec. 2.2, canonical velocity a^2 dx/dt and the kick
// ansatz that carries the residual velocity between kicks; Sec. 4.4,
// redshift-space position shifted along the line of sight by
// (dx/dt . xhat) / H).
//
// Per particle (one thread each, the readout's column order):
//   F_d  = sum_s w_s g_d[c + s]                 (only when the kick is not zero; the
//                                                force field interleaved by node)
//   v_d  = v_res_d + K F_d + u1 Psi1_d + u2 Psi2_d
//          K  = kick factor from a_v to a_x with the force at a_x,
//          u1 = a^2 adot D1' - K alpha D1,  u2 = a^2 adot D2' - K alpha (D2 - D1^2)
//   s_d  = d_d + (d == axis ? v_d / (a adot) : 0)
// Snapshot at a_s inside the coming step a_x -> a1 (Sec. 2.2, eqs.
// ansatz-drift and cola-drift): the step's kick to the half step a_h, then
// the residual velocity decays as (a/a_h)^n and the position follows its
// drift integral to a_s; the 2LPT part is taken at a_s:
//   v_h  = v_res + K F - c1 Psi1 - c2 Psi2          (the step's kick)
//   d_s  = d + I_s v_h + e1 Psi1 + e2 Psi2          (I_s: drift integral a_x -> a_s,
//                                                    e = D(a_s) - D(a_x))
//   v_s  = sv v_h + w1 Psi1 + w2 Psi2               (sv = (a_s/a_h)^n, w = a_s^2 adot D'(a_s))
// Nothing of the state is written.
#include "cola_device.h"
#include "cola_internal.h"

namespace cola {

template <bool KICK, bool RSD>
__global__ __launch_bounds__(256) void k_velocity(const float* __restrict__ g, long row_stride,
                                                  const float* __restrict__ disp, const float* __restrict__ vres,
                                                  const float* __restrict__ psi1, const float* __restrict__ psi2,
                                                  int np, int nm, long np3, VelCoef k, float* __restrict__ vel,
                                                  float* __restrict__ sdisp, int axis) {
  const long i = readout_particle(xcd_remap(blockIdx.x, gridDim.x), threadIdx.x, np, nm);
  if (i >= np3) return;
  float v[3], p1[3], p2[3], d[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    v[e] = vres[e * np3 + i];
    p1[e] = psi1[e * np3 + i];
    p2[e] = psi2[e * np3 + i];
    if constexpr (RSD) d[e] = disp[e * np3 + i];
  }
  float F[3] = {0.f, 0.f, 0.f};
  if constexpr (KICK) {
    int c[3];
    float f[3];
    home_cell(disp, np3, (uint32_t)i, np, nm, 1.0f, c, f);
    force_readout(g, row_stride, nm, c, f, F);
  }
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const float ve = v[e] + k.K * F[e] + k.u1 * p1[e] + k.u2 * p2[e];
    vel[e * np3 + i] = ve;
    if constexpr (RSD) sdisp[e * np3 + i] = e == axis ? d[e] + k.rsd * ve : d[e];
  }
}

template <bool RSD>
__global__ __launch_bounds__(256) void k_snapshot(const float* __restrict__ g, long row_stride,
                                                  const float* __restrict__ disp, const float* __restrict__ vres,
                                                  const float* __restrict__ psi1, const float* __restrict__ psi2,
                                                  int np, int nm, long np3, SnapCoef k, float* __restrict__ dout,
                                                  float* __restrict__ vout, float* __restrict__ sdisp, int axis) {
  const long i = readout_particle(xcd_remap(blockIdx.x, gridDim.x), threadIdx.x, np, nm);
  if (i >= np3) return;
  float v[3], p1[3], p2[3], d[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    v[e] = vres[e * np3 + i];
    p1[e] = psi1[e * np3 + i];
    p2[e] = psi2[e * np3 + i];
    d[e] = disp[e * np3 + i];
  }
  int c[3];
  float f[3];
  home_cell(disp, np3, (uint32_t)i, np, nm, 1.0f, c, f);
  float F[3];
  force_readout(g, row_stride, nm, c, f, F);
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const float vh = v[e] + k.K * F[e] - k.c1 * p1[e] - k.c2 * p2[e];
    const float ds = d[e] + k.I * vh + k.e1 * p1[e] + k.e2 * p2[e];
    const float vs = k.sv * vh + k.w1 * p1[e] + k.w2 * p2[e];
    dout[e * np3 + i] = ds;
    vout[e * np3 + i] = vs;
    if constexpr (RSD) sdisp[e * np3 + i] = e == axis ? ds + k.rsd * vs : ds;
  }
}

void launch_snapshot(const float* g, long row_stride, const float* disp,
                     const float* vres, const float* psi1, const float* psi2, int np, int nm,
                     const SnapCoef& k, float* dout, float* vout, float* sdisp, int axis, hipStream_t s) {
  const long np3 = (long)np * np * np;
  const dim3 grid((unsigned)((np3 + 255) / 256));
  if (sdisp)
    hipLaunchKernelGGL(k_snapshot<true>, grid, dim3(256), 0, s, g, row_stride, disp, vres, psi1, psi2,
                       np, nm, np3, k, dout, vout, sdisp, axis);
  else
    hipLaunchKernelGGL(k_snapshot<false>, grid, dim3(256), 0, s, g, row_stride, disp, vres, psi1, psi2,
                       np, nm, np3, k, dout, vout, sdisp, axis);
}

// Weights of the density / line-of-sight momentum deposit: wt[0] = w0 (1/nbar),
// wt[1] = scale * v_axis (the velocity of k_velocity, scaled to the shift per
// particle over nbar), wt[2] = 0.
template <bool KICK>
__global__ __launch_bounds__(256) void k_los_weights(const float* __restrict__ g, long row_stride,
                                                     const float* __restrict__ disp, const float* __restrict__ vres,
                                                     const float* __restrict__ psi1, const float* __restrict__ psi2,
                                                     int np, int nm, long np3, VelCoef k, int axis, float w0,
                                                     float scale, float* __restrict__ wt) {
  const long i = readout_particle(xcd_remap(blockIdx.x, gridDim.x), threadIdx.x, np, nm);
  if (i >= np3) return;
  const long j = axis * np3 + i;
  float F = 0.f;
  if constexpr (KICK) {
    int c[3];
    float f[3];
    home_cell(disp, np3, (uint32_t)i, np, nm, 1.0f, c, f);
    const ForceCorners fc(c, nm, row_stride);
#pragma unroll
    for (int s = 0; s < 8; ++s) F += cic_weight(f, s) * g[fc.at(s) + axis];
  }
  const float v = vres[j] + k.K * F + k.u1 * psi1[j] + k.u2 * psi2[j];
  wt[i] = w0;
  wt[np3 + i] = scale * v;
  wt[2 * np3 + i] = 0.f;
}

void launch_los_weights(const float* g, long row_stride, const float* disp,
                        const float* vres, const float* psi1, const float* psi2, int np, int nm,
                        const VelCoef& k, int axis, float w0, float scale, float* wt, hipStream_t s) {
  const long np3 = (long)np * np * np;
  const dim3 grid((unsigned)((np3 + 255) / 256));
  if (g)
    hipLaunchKernelGGL(k_los_weights<true>, grid, dim3(256), 0, s, g, row_stride, disp, vres, psi1, psi2,
                       np, nm, np3, k, axis, w0, scale, wt);
  else
    hipLaunchKernelGGL(k_los_weights<false>, grid, dim3(256), 0, s, g, row_stride, disp, vres, psi1,
                       psi2, np, nm, np3, k, axis, w0, scale, wt);
}

void launch_velocity(const float* g, long row_stride, const float* disp,
                     const float* vres, const float* psi1, const float* psi2, int np, int nm,
                     const VelCoef& k, float* vel, float* sdisp, int axis, hipStream_t s) {
  const long np3 = (long)np * np * np;
  const dim3 grid((unsigned)((np3 + 255) / 256));
  const bool kick = g != nullptr, rsd = sdisp != nullptr;
  if (kick && rsd)
    hipLaunchKernelGGL((k_velocity<true, true>), grid, dim3(256), 0, s, g, row_stride, disp, vres, psi1,
                       psi2, np, nm, np3, k, vel, sdisp, axis);
  else if (kick)
    hipLaunchKernelGGL((k_velocity<true, false>), grid, dim3(256), 0, s, g, row_stride, disp, vres, psi1,
                       psi2, np, nm, np3, k, vel, sdisp, axis);
  else if (rsd)
    hipLaunchKernelGGL((k_velocity<false, true>), grid, dim3(256), 0, s, g, row_stride, disp, vres, psi1,
                       psi2, np, nm, np3, k, vel, sdisp, axis);
  else
    hipLaunchKernelGGL((k_velocity<false, false>), grid, dim3(256), 0, s, g, row_stride, disp, vres,
                       psi1, psi2, np, nm, np3, k, vel, sdisp, axis);
}

}  // namespace cola
