// Reverse-mode kernels of the COLA step (Koda et al. 2015, Sec. 2.2, eqs.
// cola-kick and cola-drift with the PM force), of the density and P(k)
// outputs (Sec. 3.3) and of the 2LPT source term (Sec. 2.1).
//
// Step, per particle (mesh units, x = q + d at the step start):
//   vt = vbar' + I dbar';  Psi1bar += e1 dbar' - c1 vt;  Psi2bar += e2 dbar' - c2 vt
//   vbar = vt;  Fbar = K vt
//   dbar = dbar' + sum_d Fbar_d sum_s grad w_s(x) g_d[c + s]     (readout weights)
// and, after the transpose deposit and the Green transpose, the deposit
// weight gradient dbar += sum_s grad w_s(x) rhobar[c + s].
// CIC weight gradient: d w_s / d u_e = (s_e ? +1 : -1) prod_{e' != e} w_{s_e'}(f_e').
#include "cola_device.h"
#include "cola_internal.h"

namespace cola {

__device__ __forceinline__ void weight_grads(const float f[3], int k, float gw[3]) {
  const float wx = (k & 4) ? f[0] : 1.0f - f[0];
  const float wy = (k & 2) ? f[1] : 1.0f - f[1];
  const float wz = (k & 1) ? f[2] : 1.0f - f[2];
  const float sx = (k & 4) ? 1.0f : -1.0f, sy = (k & 2) ? 1.0f : -1.0f, sz = (k & 1) ? 1.0f : -1.0f;
  gw[0] = sx * wy * wz;
  gw[1] = wx * sy * wz;
  gw[2] = wx * wy * sz;
}

__device__ __forceinline__ long node_index(const int c[3], int k, int nm, long row_stride) {
  int x = c[0] + ((k >> 2) & 1), y = c[1] + ((k >> 1) & 1), z = c[2] + (k & 1);
  if (x == nm) x = 0;
  if (y == nm) y = 0;
  if (z == nm) z = 0;
  return ((long)x * nm + y) * row_stride + z;
}

__global__ __launch_bounds__(256) void k_adj_readout_kick(
    const float* __restrict__ disp, const float* __restrict__ g, long row_stride, int np, int nm, long np3,
    KickDrift kd,
    float* __restrict__ dbar, float* __restrict__ vbar, float* __restrict__ p1bar,
    float* __restrict__ p2bar, float* __restrict__ fbar) {
  // particles of a block share mesh lines; neighbouring blocks stay on one XCD (L2)
  const long i = readout_particle(xcd_remap(blockIdx.x, gridDim.x), threadIdx.x, np, nm);
  if (i >= np3) return;
  float F[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const long j = e * np3 + i;
    const float db = dbar[j];
    const float vt = vbar[j] + kd.I * db;
    p1bar[j] += kd.e1 * db - kd.c1 * vt;
    p2bar[j] += kd.e2 * db - kd.c2 * vt;
    vbar[j] = vt;
    F[e] = kd.K * vt;
    fbar[j] = F[e];
  }
  int c[3];
  float f[3];
  home_cell(disp, np3, (uint32_t)i, np, nm, 1.0f, c, f);
  const ForceCorners fc(c, nm, row_stride);  // the force field interleaved by node
  float xb[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    float gw[3];
    weight_grads(f, k, gw);
    const float* q = g + fc.at(k);
    const float s = F[0] * q[0] + F[1] * q[1] + F[2] * q[2];
#pragma unroll
    for (int e = 0; e < 3; ++e) xb[e] += gw[e] * s;
  }
#pragma unroll
  for (int e = 0; e < 3; ++e) dbar[e * np3 + i] += xb[e];
}

void launch_adj_readout_kick(const float* disp, const float* g, long row_stride, int np, int nm,
                             const KickDrift& kd, float* dbar, float* vbar, float* p1bar, float* p2bar,
                             float* fbar, hipStream_t s) {
  const long np3 = (long)np * np * np;
  hipLaunchKernelGGL(k_adj_readout_kick, dim3((unsigned)((np3 + 255) / 256)), dim3(256), 0, s, disp,
                     g, row_stride, np, nm, np3, kd, dbar, vbar, p1bar, p2bar, fbar);
}

// dbar += coef * dscale * sum_s grad w_s(u) field[c + s]  on an ng^3 grid.
__global__ __launch_bounds__(256) void k_adj_deposit_grad(const float* __restrict__ disp,
                                                          const float* __restrict__ field,
                                                          long row_stride, int np, int ng,
                                                          float dscale, long np3, float coef,
                                                          float* __restrict__ dbar) {
  // particles of a block share mesh lines; neighbouring blocks stay on one XCD (L2)
  const long i = readout_particle(xcd_remap(blockIdx.x, gridDim.x), threadIdx.x, np, ng);
  if (i >= np3) return;
  int c[3];
  float f[3];
  home_cell(disp, np3, (uint32_t)i, np, ng, dscale, c, f);
  float xb[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    float gw[3];
    weight_grads(f, k, gw);
    const float v = field[node_index(c, k, ng, row_stride)];
#pragma unroll
    for (int e = 0; e < 3; ++e) xb[e] += gw[e] * v;
  }
  const float s = coef * dscale;
#pragma unroll
  for (int e = 0; e < 3; ++e) dbar[e * np3 + i] += s * xb[e];
}

void launch_adj_deposit_grad(const float* disp, const float* field, long row_stride, int np, int ng,
                             float dscale, float coef, float* dbar, hipStream_t s) {
  const long np3 = (long)np * np * np;
  hipLaunchKernelGGL(k_adj_deposit_grad, dim3((unsigned)((np3 + 255) / 256)), dim3(256), 0, s, disp,
                     field, row_stride, np, ng, dscale, np3, coef, dbar);
}

// mesh_q = a_q + alpha * b_q for the three components of particle arrays.
__global__ void k_axpy_to_mesh(const float* __restrict__ a, const float* __restrict__ b, float alpha,
                               int n, long n3, float* __restrict__ mesh, long row_stride,
                               long mesh_stride) {
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < n3;
       p += (long)gridDim.x * blockDim.x) {
    const long row = p / n, col = p - row * n;
  #pragma unroll
    for (int q = 0; q < 3; ++q)
      mesh[q * mesh_stride + row * row_stride + col] = a[q * n3 + p] + alpha * (b ? b[q * n3 + p] : 0.f);
  }
}

void launch_axpy_to_mesh(const float* a, const float* b, float alpha, int n, float* mesh,
                         long row_stride, long mesh_stride_floats, hipStream_t s) {
  const long n3 = (long)n * n * n;
  hipLaunchKernelGGL(k_axpy_to_mesh, dim3(grid_1d(n3)), dim3(256), 0, s, a, b, alpha,
                     n, n3, mesh, row_stride, mesh_stride_floats);
}

// 2LPT source adjoint (S = pxx pyy + pyy pzz + pzz pxx - pxy^2 - pyz^2 - pzx^2):
// diagonal: (a, b, c) <- Sbar (b + c, a + c, a + b); off-diagonal: a <- -2 Sbar a.
__global__ void k_phibar_diag(float* __restrict__ a, float* __restrict__ b, float* __restrict__ c,
                              const float* __restrict__ sbar, int n, long n3, long row_stride) {
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < n3;
       p += (long)gridDim.x * blockDim.x) {
    const long row = p / n, col = p - row * n;
    const long j = row * row_stride + col;
    const float x = a[j], y = b[j], z = c[j], sb = sbar[j];
    a[j] = sb * (y + z);
    b[j] = sb * (x + z);
    c[j] = sb * (x + y);
  }
}

__global__ void k_phibar_off(float* __restrict__ a, const float* __restrict__ sbar, int n, long n3,
                             long row_stride, long mesh_stride) {
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < n3;
       p += (long)gridDim.x * blockDim.x) {
    const long row = p / n, col = p - row * n;
    const long j = row * row_stride + col;
    const float sb = sbar[j];
  #pragma unroll
    for (int q = 0; q < 3; ++q) a[q * mesh_stride + j] = -2.0f * sb * a[q * mesh_stride + j];
  }
}

void launch_phibar_diag(float* a, float* b, float* c, const float* sbar, int n, long row_stride,
                        hipStream_t s) {
  const long n3 = (long)n * n * n;
  hipLaunchKernelGGL(k_phibar_diag, dim3(grid_1d(n3)), dim3(256), 0, s, a, b, c, sbar,
                     n, n3, row_stride);
}

void launch_phibar_off(float* a, const float* sbar, int n, long row_stride, long mesh_stride_floats,
                       hipStream_t s) {
  const long n3 = (long)n * n * n;
  hipLaunchKernelGGL(k_phibar_off, dim3(grid_1d(n3)), dim3(256), 0, s, a, sbar, n, n3,
                     row_stride, mesh_stride_floats);
}

// P(k) adjoint: for half-space modes with |k| <= k_Nyq in bin b,
//   u_k = cbar_b / N_b (V/Ng^3)^2 / V / W_CIC(k)^2,
// and the real field  deltabar(x) = sum_modes 2 u_k Re(X_k e^{ikx})  is written
// as a half spectrum Z for the unnormalised complex-to-real inverse:
//   0 < nz < Ng/2: Z_k = u X_k (the inverse doubles it);  nz = 0: Z_k = u X_k and
//   Z_{-k} = conj(u X_k) (Hermitian plane);  nz = Ng/2: Z_k = 2 u X_k.
__device__ __forceinline__ double sinc_pi_d(double x) {
  if (x == 0.0) return 1.0;
  const double a = 3.14159265358979323846 * x;
  return sin(a) / a;
}

__global__ void k_pk_adj_modes(const float2* __restrict__ X, float2* __restrict__ Z, int ng, long cols,
                               double kf, double kmax, double vol_fac,
                               const double* __restrict__ edges, int nbins,
                               const double* __restrict__ cbar, const double* __restrict__ sums) {
  const int h = ng / 2;
  const long nmode = (long)ng * ng * (h + 1);
  for (long m = blockIdx.x * (long)blockDim.x + threadIdx.x; m < nmode; m += (long)gridDim.x * blockDim.x) {
    const int iz = (int)(m % (h + 1));
    const long r = m / (h + 1);
    const int ix = (int)(r / ng), iy = (int)(r % ng);
    const int nx = ix < h ? ix : ix - ng, ny = iy < h ? iy : iy - ng, nz = iz;
    if (nz == 0 && !(ny > 0 || (ny == 0 && nx > 0))) continue;
    const double n2 = (double)nx * nx + (double)ny * ny + (double)nz * nz;
    const double kk = kf * sqrt(n2);
    if (kk > kmax) continue;
    // bin: last edge <= kk
    if (!(kk >= edges[0] && kk < edges[nbins])) continue;
    int lo = 0, hi = nbins;  // edges[0..nbins]
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (edges[mid] <= kk) lo = mid; else hi = mid;
    }
    const double cnt = sums[3 * lo + 2];
    if (cnt <= 0) continue;
    double w = sinc_pi_d((double)nx / ng) * sinc_pi_d((double)ny / ng) * sinc_pi_d((double)nz / ng);
    w = w * w;
    const double u = cbar[lo] / cnt * vol_fac / (w * w);
    const float2 x = X[r * cols + iz];
    const double fac = (nz == h) ? 2.0 * u : u;
    Z[r * cols + iz] = make_float2((float)(fac * x.x), (float)(fac * x.y));
    if (nz == 0) {
      const int jx = (ng - ix) % ng, jy = (ng - iy) % ng;
      Z[((long)jx * ng + jy) * cols] = make_float2((float)(u * x.x), (float)(-u * x.y));
    }
  }
}

void launch_pk_adj_modes(const float2* X, float2* Z, int ng, double box, const double* edges,
                         int nbins, const double* cbar, const double* sums, hipStream_t s) {
  const double pi = 3.14159265358979323846;
  const double kf = 2.0 * pi / box, kmax = pi * ng / box;
  const double v = box * box * box, n3 = (double)ng * ng * ng;
  const double vol_fac = (v / n3) * (v / n3) / v;
  const long nmode = (long)ng * ng * (ng / 2 + 1);
  hipLaunchKernelGGL(k_pk_adj_modes, dim3(grid_1d(nmode)), dim3(256), 0, s, X, Z, ng,
                     padded_cols(ng), kf, kmax, vol_fac, edges, nbins, cbar, sums);
}

}  // namespace cola
