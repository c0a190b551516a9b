// Initial-condition kernels: white noise, copies between particle arrays and
// padded meshes, the 2LPT source term and the initial particle state
// (Koda et al. 2015, Sec. 2.1: x = q + D1 Psi1 + D2 Psi2; Sec. 2.3: Gaussian
// initial random modes).
#include "cola_device.h"
#include "cola_internal.h"

namespace cola {

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw 2011): 10 rounds of the
// multiply-xorshift bijection on a 4x32-bit counter with a 2x32-bit key and
// the Weyl key schedule.  Constants are the published ones.
__device__ __forceinline__ void philox4x32_10(uint32_t ctr[4], uint32_t key[2]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * ctr[0];
    const uint64_t p1 = (uint64_t)M1 * ctr[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ ctr[1] ^ key[0];
    const uint32_t n2 = hi0 ^ ctr[3] ^ key[1];
    ctr[0] = n0;
    ctr[1] = lo1;
    ctr[2] = n2;
    ctr[3] = lo0;
    key[0] += W0;
    key[1] += W1;
  }
}

// Noise for particle id p: counter (p, 0, 0, 0), key (seed lo, seed hi);
// Box-Muller on the first two words: u1 = (x0 + 1) 2^-32 in (0, 1],
// u2 = x1 2^-32, z = sqrt(-2 ln u1) cos(2 pi u2), evaluated in float64.
__global__ void k_philox_noise(uint64_t seed, int np, long np3, float* __restrict__ out,
                               long row_stride) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p >= np3) return;
  uint32_t ctr[4] = {(uint32_t)p, (uint32_t)((uint64_t)p >> 32), 0u, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  philox4x32_10(ctr, key);
  const double u1 = ((double)ctr[0] + 1.0) * 2.3283064365386963e-10;
  const double u2 = (double)ctr[1] * 2.3283064365386963e-10;
  const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  const long row = p / np, col = p - row * np;
  out[row * row_stride + col] = (float)z;
}

void launch_philox_noise(uint64_t seed, int np, float* out, long row_stride, hipStream_t s) {
  const long np3 = (long)np * np * np;
  hipLaunchKernelGGL(k_philox_noise, dim3((unsigned)((np3 + 255) / 256)), dim3(256), 0, s, seed, np,
                     np3, out, row_stride);
}

__global__ void k_copy_to_mesh(const float* __restrict__ src, int n, long n3, float* __restrict__ mesh,
                               long row_stride) {
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < n3;
       p += (long)gridDim.x * blockDim.x) {
    const long row = p / n, col = p - row * n;
    mesh[row * row_stride + col] = src[p];
  }
}

void launch_copy_to_mesh(const float* src, int n, float* mesh, long row_stride, hipStream_t s) {
  const long n3 = (long)n * n * n;
  hipLaunchKernelGGL(k_copy_to_mesh, dim3(grid_1d(n3)), dim3(256), 0, s, src, n, n3,
                     mesh, row_stride);
}

__global__ void k_copy_from_mesh(const float* __restrict__ mesh, int n, long n3, long row_stride,
                                 float* __restrict__ dst, float scale, int elem) {
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < n3;
       p += (long)gridDim.x * blockDim.x) {
    const long row = p / n, col = p - row * n;
    dst[p] = scale * mesh[row * row_stride + col * elem];
  }
}

void launch_copy_from_mesh(const float* mesh, int n, long row_stride, float* dst, float scale,
                           hipStream_t s, int elem) {
  const long n3 = (long)n * n * n;
  hipLaunchKernelGGL(k_copy_from_mesh, dim3(grid_1d(n3)), dim3(256), 0, s, mesh, n,
                     n3, row_stride, dst, scale, elem);
}

// 2LPT source, diagonal part: a <- a b + b c + c a (a, b, c = phi_xx, phi_yy, phi_zz).
__global__ void k_source_diag(float* __restrict__ a, const float* __restrict__ b,
                              const float* __restrict__ c, int n, long n3, long row_stride) {
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < n3;
       p += (long)gridDim.x * blockDim.x) {
    const long row = p / n, col = p - row * n;
    const long j = row * row_stride + col;
    const float x = a[j], y = b[j], z = c[j];
    a[j] = x * y + y * z + z * x;
  }
}

void launch_source_diag(float* a, const float* b, const float* c, int n, long row_stride,
                        hipStream_t s) {
  const long n3 = (long)n * n * n;
  hipLaunchKernelGGL(k_source_diag, dim3(grid_1d(n3)), dim3(256), 0, s, a, b, c, n,
                     n3, row_stride);
}

// 2LPT source, off-diagonal part: a <- a - b^2.
__global__ void k_source_sub_sq(float* __restrict__ a, const float* __restrict__ b, int n, long n3,
                                long row_stride) {
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < n3;
       p += (long)gridDim.x * blockDim.x) {
    const long row = p / n, col = p - row * n;
    const long j = row * row_stride + col;
    const float y = b[j];
    a[j] = a[j] - y * y;
  }
}

void launch_source_sub_sq(float* a, const float* b, int n, long row_stride, hipStream_t s) {
  const long n3 = (long)n * n * n;
  hipLaunchKernelGGL(k_source_sub_sq, dim3(grid_1d(n3)), dim3(256), 0, s, a, b, n,
                     n3, row_stride);
}

// d = D1 Psi1 + D2 Psi2, v_res = 0 (x_res = v_res = 0 at the initial time).
__global__ void k_init_particles(float* __restrict__ disp, float* __restrict__ vres,
                                 const float* __restrict__ psi1, const float* __restrict__ psi2,
                                 long n, float D1, float D2) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    disp[i] = D1 * psi1[i] + D2 * psi2[i];
    vres[i] = 0.0f;
  }
}

void launch_init_particles(float* disp, float* vres, const float* psi1, const float* psi2, long np3,
                           float D1, float D2, hipStream_t s) {
  const long n = 3 * np3;
  hipLaunchKernelGGL(k_init_particles, dim3(grid_1d(n)), dim3(256), 0, s, disp, vres,
                     psi1, psi2, n, D1, D2);
}

__global__ void k_axpby(float* __restrict__ y, const float* __restrict__ x, float a, float b, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    y[i] = a * y[i] + b * x[i];
}

void launch_axpby(float* y, const float* x, float a, float b, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_1d(n)), dim3(256), 0, s, y, x, a, b, n);
}

}  // namespace cola
