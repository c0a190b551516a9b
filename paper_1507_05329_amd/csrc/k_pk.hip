// Binned matter power spectrum (Koda et al. 2015, Sec. 3.3): P = |delta_k|^2 / V
// over the half space {kz > 0} U {kz = 0, ky > 0} U {kz = 0, ky = 0, kx > 0},
// delta_k = (V / Ng^3) DFT[delta] / W_CIC(k), W_CIC = prod sinc^2(pi n_e / Ng),
// averaged per |k| bin with the mean |k|.  Only |k| <= pi Ng / L is used.
//
// Deterministic reduction: workgroup (bin b, chunk c) visits the (kx, ky)
// rows of chunk c; a thread walks one row's kz range that can fall in bin b
// (found analytically, each mode then tested exactly), accumulating in FP64
// in a fixed order; the workgroup sums its threads by a fixed tree, and a
// second kernel sums the chunks in order.
#include "cola_device.h"
#include "cola_internal.h"

namespace cola {

constexpr int kPT = 256;

__device__ __forceinline__ double sinc_pi(double x) {  // sin(pi x) / (pi x)
  if (x == 0.0) return 1.0;
  const double a = 3.14159265358979323846 * x;
  return sin(a) / a;
}

__global__ __launch_bounds__(kPT) void k_pk_bin(const float2* __restrict__ spec, int ng, long cols,
                                                double kf, double kmax, double vol_fac,
                                                const double* __restrict__ edges,
                                                int nbins, double* __restrict__ partial, int nchunk,
                                                int deconvolve) {
  __shared__ double sk[kPT], sp[kPT], sn[kPT];
  const int b = blockIdx.y;
  const int c = blockIdx.x;
  const double e0 = edges[b], e1 = edges[b + 1];
  const double lo2 = (e0 / kf) * (e0 / kf), hi2 = (e1 / kf) * (e1 / kf);
  const long nrows = (long)ng * ng;
  const long per = (nrows + nchunk - 1) / nchunk;
  const long r0 = (long)c * per, r1 = r0 + per < nrows ? r0 + per : nrows;
  double ak = 0.0, ap = 0.0, an = 0.0;
  const int h = ng / 2;
  for (long r = r0 + threadIdx.x; r < r1; r += kPT) {
    const int ix = (int)(r / ng), iy = (int)(r - (long)ix * ng);
    const int nx = ix < h ? ix : ix - ng, ny = iy < h ? iy : iy - ng;  // DFT signed indices
    const double p2 = (double)nx * nx + (double)ny * ny;
    if (p2 >= hi2) continue;
    int zlo = 0;
    if (lo2 > p2) zlo = (int)floor(sqrt(lo2 - p2)) - 1;
    if (zlo < 0) zlo = 0;
    int zhi = (int)ceil(sqrt(hi2 - p2)) + 1;
    if (zhi > h) zhi = h;
    const double wxy = sinc_pi((double)nx / ng) * sinc_pi((double)ny / ng);
    for (int nz = zlo; nz <= zhi; ++nz) {
      if (nz == 0 && !(ny > 0 || (ny == 0 && nx > 0))) continue;
      const double n2 = p2 + (double)nz * nz;
      const double kk = kf * sqrt(n2);
      if (kk > kmax) continue;
      if (!(kk >= e0 && kk < e1)) continue;
      const float2 v = spec[r * cols + nz];
      double w = deconvolve ? wxy * sinc_pi((double)nz / ng) : 1.0;
      w = w * w;
      const double re = (double)v.x, im = (double)v.y;
      ap += (re * re + im * im) * vol_fac / (w * w);
      ak += kk;
      an += 1.0;
    }
  }
  sk[threadIdx.x] = ak;
  sp[threadIdx.x] = ap;
  sn[threadIdx.x] = an;
  __syncthreads();
  for (int o = kPT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sk[threadIdx.x] += sk[threadIdx.x + o];
      sp[threadIdx.x] += sp[threadIdx.x + o];
      sn[threadIdx.x] += sn[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = partial + ((long)b * nchunk + c) * 3;
    o[0] = sk[0];
    o[1] = sp[0];
    o[2] = sn[0];
  }
}

__global__ void k_pk_reduce(const double* __restrict__ partial, int nbins, int nchunk,
                            double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  double s0 = 0, s1 = 0, s2 = 0;
  for (int c = 0; c < nchunk; ++c) {
    const double* p = partial + ((long)b * nchunk + c) * 3;
    s0 += p[0];
    s1 += p[1];
    s2 += p[2];
  }
  out[3 * b + 0] = s0;
  out[3 * b + 1] = s1;
  out[3 * b + 2] = s2;
}

// Density / line-of-sight momentum spectra over the same modes and bins:
// per bin, sums of |k|, |d|^2, sign(n_axis) Im(d p*), |p|^2 (each scaled and
// deconvolved like P(k)) and the count; the same fixed-order reduction.
__global__ __launch_bounds__(kPT) void k_pk_cross(const float2* __restrict__ sd, const float2* __restrict__ sp,
                                                  int ng, long cols, double kf, double kmax, double vol_fac,
                                                  const double* __restrict__ edges, int nbins, int axis,
                                                  double* __restrict__ partial, int nchunk) {
  __shared__ double acc[5][kPT];
  const int b = blockIdx.y;
  const int c = blockIdx.x;
  const double e0 = edges[b], e1 = edges[b + 1];
  const double lo2 = (e0 / kf) * (e0 / kf), hi2 = (e1 / kf) * (e1 / kf);
  const long nrows = (long)ng * ng;
  const long per = (nrows + nchunk - 1) / nchunk;
  const long r0 = (long)c * per, r1 = r0 + per < nrows ? r0 + per : nrows;
  double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int h = ng / 2;
  for (long r = r0 + threadIdx.x; r < r1; r += kPT) {
    const int ix = (int)(r / ng), iy = (int)(r - (long)ix * ng);
    const int nx = ix < h ? ix : ix - ng, ny = iy < h ? iy : iy - ng;
    const double p2 = (double)nx * nx + (double)ny * ny;
    if (p2 >= hi2) continue;
    int zlo = 0;
    if (lo2 > p2) zlo = (int)floor(sqrt(lo2 - p2)) - 1;
    if (zlo < 0) zlo = 0;
    int zhi = (int)ceil(sqrt(hi2 - p2)) + 1;
    if (zhi > h) zhi = h;
    const double wxy = sinc_pi((double)nx / ng) * sinc_pi((double)ny / ng);
    for (int nz = zlo; nz <= zhi; ++nz) {
      if (nz == 0 && !(ny > 0 || (ny == 0 && nx > 0))) continue;
      const double n2 = p2 + (double)nz * nz;
      const double kk = kf * sqrt(n2);
      if (kk > kmax) continue;
      if (!(kk >= e0 && kk < e1)) continue;
      const int na = axis == 0 ? nx : axis == 1 ? ny : nz;
      const double sg = na > 0 ? 1.0 : na < 0 ? -1.0 : 0.0;
      const float2 d = sd[r * cols + nz], p = sp[r * cols + nz];
      double w = wxy * sinc_pi((double)nz / ng);
      w = w * w;
      const double f = vol_fac / (w * w);
      const double dr = d.x, di = d.y, pr = p.x, pi = p.y;
      a[0] += kk;
      a[1] += (dr * dr + di * di) * f;
      a[2] += sg * (di * pr - dr * pi) * f;
      a[3] += (pr * pr + pi * pi) * f;
      a[4] += 1.0;
    }
  }
  for (int q = 0; q < 5; ++q) acc[q][threadIdx.x] = a[q];
  __syncthreads();
  for (int o = kPT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int q = 0; q < 5; ++q) acc[q][threadIdx.x] += acc[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = partial + ((long)b * nchunk + c) * 5;
    for (int q = 0; q < 5; ++q) o[q] = acc[q][0];
  }
}

__global__ void k_pk_cross_reduce(const double* __restrict__ partial, int nbins, int nchunk,
                                  double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int c = 0; c < nchunk; ++c)
    for (int q = 0; q < 5; ++q) s[q] += partial[((long)b * nchunk + c) * 5 + q];
  for (int q = 0; q < 5; ++q) out[5 * b + q] = s[q];
}

void launch_pk_cross(const float2* sd, const float2* sp, int ng, double box, const double* edges, int nbins,
                     int axis, double* partial, int nchunk, double* out, hipStream_t s) {
  const double pi = 3.14159265358979323846;
  const double kf = 2.0 * pi / box;
  const double kmax = pi * ng / box;
  const double v = box * box * box;
  const double n3 = (double)ng * ng * ng;
  const double vol_fac = (v / n3) * (v / n3) / v;
  hipLaunchKernelGGL(k_pk_cross, dim3((unsigned)nchunk, (unsigned)nbins), dim3(kPT), 0, s, sd, sp, ng,
                     padded_cols(ng), kf, kmax, vol_fac, edges, nbins, axis, partial, nchunk);
  hipLaunchKernelGGL(k_pk_cross_reduce, dim3((unsigned)((nbins + 63) / 64)), dim3(64), 0, s, partial, nbins,
                     nchunk, out);
}

void launch_pk_bin(const float2* spec, int ng, double box, const double* edges, int nbins,
                   double* partial, int nchunk, hipStream_t s, int deconvolve) {
  const double pi = 3.14159265358979323846;
  const double kf = 2.0 * pi / box;
  const double kmax = pi * ng / box;
  const double v = box * box * box;
  const double n3 = (double)ng * ng * ng;
  const double vol_fac = (v / n3) * (v / n3) / v;  // |(V/Ng^3) X|^2 / V
  hipLaunchKernelGGL(k_pk_bin, dim3((unsigned)nchunk, (unsigned)nbins), dim3(kPT), 0, s, spec, ng,
                     padded_cols(ng), kf, kmax, vol_fac, edges, nbins, partial, nchunk, deconvolve);
}

// Smoothing + aliasing correction of Jing (2005) (Sec. 3.3): per bin b, the
// sum over its modes of the CIC window's image sum
//   C(k; s_b) = sum_{|m_e| <= kAliasImages} W^2(k + 2 k_N m) (|k + 2 k_N m| / |k|)^s_b,
// W the CIC window sinc^2 per axis continued to the images, s_b = slope[b].
// Per axis the image windows are sinc^4(x + pi m) = sin^4(x) / (x + pi m)^4
// with x = pi n / Ng (1 for m = 0 and 0 otherwise when n = 0).  The terms of
// a mode are summed in FP32 in a fixed order, the modes of a thread and the
// threads of a workgroup in FP64 as in k_pk_bin; partial holds one value per
// (bin, chunk).
constexpr int kAliasImages = 2;

__device__ __forceinline__ void image_windows(int n, int ng, float w[2 * kAliasImages + 1]) {
  if (n == 0) {
#pragma unroll
    for (int m = -kAliasImages; m <= kAliasImages; ++m) w[m + kAliasImages] = m == 0 ? 1.0f : 0.0f;
    return;
  }
  const double x = 3.14159265358979323846 * (double)n / (double)ng;
  const double s = sin(x);
  const double s4 = s * s * s * s;
#pragma unroll
  for (int m = -kAliasImages; m <= kAliasImages; ++m) {
    const double y = x + 3.14159265358979323846 * m;
    const double y2 = y * y;
    w[m + kAliasImages] = (float)(s4 / (y2 * y2));
  }
}

__global__ __launch_bounds__(kPT) void k_pk_alias(int ng, double kf, double kmax,
                                                  const double* __restrict__ edges, int nbins,
                                                  const double* __restrict__ slope,
                                                  double* __restrict__ partial, int nchunk) {
  __shared__ double sc[kPT];
  constexpr int kM = 2 * kAliasImages + 1;
  const int b = blockIdx.y;
  const int c = blockIdx.x;
  const double e0 = edges[b], e1 = edges[b + 1];
  const double lo2 = (e0 / kf) * (e0 / kf), hi2 = (e1 / kf) * (e1 / kf);
  const float hs = (float)(0.5 * slope[b]);
  const long nrows = (long)ng * ng;
  const long per = (nrows + nchunk - 1) / nchunk;
  const long r0 = (long)c * per, r1 = r0 + per < nrows ? r0 + per : nrows;
  double acc = 0.0;
  const int h = ng / 2;
  const float fng = (float)ng;
  for (long r = r0 + threadIdx.x; r < r1; r += kPT) {
    const int ix = (int)(r / ng), iy = (int)(r - (long)ix * ng);
    const int nx = ix < h ? ix : ix - ng, ny = iy < h ? iy : iy - ng;
    const double p2 = (double)nx * nx + (double)ny * ny;
    if (p2 >= hi2) continue;
    int zlo = 0;
    if (lo2 > p2) zlo = (int)floor(sqrt(lo2 - p2)) - 1;
    if (zlo < 0) zlo = 0;
    int zhi = (int)ceil(sqrt(hi2 - p2)) + 1;
    if (zhi > h) zhi = h;
    float wx[kM], wy[kM];
    image_windows(nx, ng, wx);
    image_windows(ny, ng, wy);
    for (int nz = zlo; nz <= zhi; ++nz) {
      if (nz == 0 && !(ny > 0 || (ny == 0 && nx > 0))) continue;
      const double n2 = p2 + (double)nz * nz;
      const double kk = kf * sqrt(n2);
      if (kk > kmax) continue;
      if (!(kk >= e0 && kk < e1)) continue;
      float wz[kM];
      image_windows(nz, ng, wz);
      const float l0 = log2f((float)n2);
      float sum = 0.0f;
#pragma unroll
      for (int mx = 0; mx < kM; ++mx) {
        if (wx[mx] == 0.0f) continue;
        const float kx = (float)nx + fng * (float)(mx - kAliasImages);
#pragma unroll
        for (int my = 0; my < kM; ++my) {
          if (wy[my] == 0.0f) continue;
          const float ky = (float)ny + fng * (float)(my - kAliasImages);
          const float wxy = wx[mx] * wy[my];
#pragma unroll
          for (int mz = 0; mz < kM; ++mz) {
            if (wz[mz] == 0.0f) continue;
            const float kz = (float)nz + fng * (float)(mz - kAliasImages);
            const float k2 = kx * kx + ky * ky + kz * kz;
            sum += wxy * wz[mz] * exp2f(hs * (log2f(k2) - l0));
          }
        }
      }
      acc += (double)sum;
    }
  }
  sc[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kPT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sc[threadIdx.x] += sc[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(long)b * nchunk + c] = sc[0];
}

__global__ void k_pk_alias_reduce(const double* __restrict__ partial, int nbins, int nchunk,
                                  double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += partial[(long)b * nchunk + c];
  out[b] = s;
}

void launch_pk_alias(int ng, double box, const double* edges, int nbins, const double* slope, double* partial,
                     int nchunk, double* out, hipStream_t s) {
  const double pi = 3.14159265358979323846;
  const double kf = 2.0 * pi / box;
  const double kmax = pi * ng / box;
  hipLaunchKernelGGL(k_pk_alias, dim3((unsigned)nchunk, (unsigned)nbins), dim3(kPT), 0, s, ng, kf, kmax, edges,
                     nbins, slope, partial, nchunk);
  hipLaunchKernelGGL(k_pk_alias_reduce, dim3((unsigned)((nbins + 63) / 64)), dim3(64), 0, s, partial, nbins,
                     nchunk, out);
}

void launch_pk_reduce(const double* partial, int nbins, int nchunk, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_pk_reduce, dim3((unsigned)((nbins + 63) / 64)), dim3(64), 0, s, partial, nbins,
                     nchunk, out);
}

}  // namespace cola
