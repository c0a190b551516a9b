// 3D real-to-complex FFT for the PM solver (Koda et al. 2015, Sec. 2.3: FFTs
// dominate the run time), written as a mixed-radix Stockham autosort FFT
// staged through LDS.  A 3D transform is three passes over HBM:
//   z (contiguous rows): real-to-complex by a half-length complex FFT plus
//     the split step, in place in rows of padded_cols(n) complex values;
//   y and x (strided): a workgroup loads W adjacent columns x n elements
//     (W-wide contiguous runs), transforms them in LDS and writes back.
// The x pass also hosts the k-space multipliers: the PM Green's function
// times i k (three outputs from one forward transform), and the 2LPT
// multipliers of the initial conditions.
//
// Stockham stage with radix R on a line of length L after Ns = product of
// earlier radices: butterfly j (0 <= j < L/R) reads x[j + r L/R], applies
// twiddles W_{Ns R}^{r (j mod Ns)}, does a length-R DFT and writes
// y[(j - j mod Ns) R + j mod Ns + r Ns].  Every stage reads all of its
// inputs into registers before any thread writes, so one LDS buffer is
// enough.  Twiddles come from a per-length table exp(-2 pi i k / n).
#include "cola_device.h"
#include "cola_internal.h"

namespace cola {

constexpr int kFT = 256;        // threads per workgroup
constexpr int kMaxE = 32;       // complex elements per thread (lines * length <= kFT * kMaxE)
constexpr int kLdsC = kFT * kMaxE;

bool make_plan(int n, FftPlan* plan) {
  if (n < 2) return false;
  plan->n = n;
  plan->nstage = 0;
  int m = n;
  int threes = 0;
  while (m % 3 == 0) { m /= 3; ++threes; }
  for (int i = 0; i < threes; ++i) plan->radix[plan->nstage++] = 3;
  while (m % 16 == 0) { m /= 16; plan->radix[plan->nstage++] = 16; }
  if (m % 8 == 0) { m /= 8; plan->radix[plan->nstage++] = 8; }
  if (m % 4 == 0) { m /= 4; plan->radix[plan->nstage++] = 4; }
  if (m % 2 == 0) { m /= 2; plan->radix[plan->nstage++] = 2; }
  if (m != 1 || plan->nstage > 12) return false;
  return true;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// i * s * a for s = +-1
__device__ __forceinline__ float2 cmul_is(float2 a, float s) { return make_float2(-s * a.y, s * a.x); }

template <int R> struct Dft;

template <> struct Dft<2> {
  __device__ __forceinline__ static void run(float2* v, float) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};
template <> struct Dft<3> {
  __device__ __forceinline__ static void run(float2* v, float s) {
    const float c = 0.86602540378443864676f;
    const float2 a = v[0], sm = cadd(v[1], v[2]), df = csub(v[1], v[2]);
    const float2 t = make_float2(a.x - 0.5f * sm.x, a.y - 0.5f * sm.y);
    const float2 r = cmul_is(make_float2(c * df.x, c * df.y), s);
    v[0] = cadd(a, sm);
    v[1] = cadd(t, r);
    v[2] = csub(t, r);
  }
};
template <> struct Dft<4> {
  __device__ __forceinline__ static void run(float2* v, float s) {
    const float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    const float2 b0 = cadd(v[1], v[3]), b1 = cmul_is(csub(v[1], v[3]), s);
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd(a1, b1);
    v[3] = csub(a1, b1);
  }
};
template <> struct Dft<8> {
  __device__ __forceinline__ static void run(float2* v, float s) {
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4>::run(e, s);
    Dft<4>::run(o, s);
    const float h = 0.70710678118654752440f;
    const float2 w[4] = {make_float2(1.f, 0.f), make_float2(h, s * h), make_float2(0.f, s),
                         make_float2(-h, s * h)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float2 t = cmul(w[k], o[k]);
      v[k] = cadd(e[k], t);
      v[k + 4] = csub(e[k], t);
    }
  }
};
template <> struct Dft<16> {
  __device__ __forceinline__ static void run(float2* v, float s) {
    float2 e[8], o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) { e[k] = v[2 * k]; o[k] = v[2 * k + 1]; }
    Dft<8>::run(e, s);
    Dft<8>::run(o, s);
    const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;
    const float h = 0.70710678118654752440f;
    const float2 w[8] = {make_float2(1.f, 0.f),   make_float2(c1, s * s1), make_float2(h, s * h),
                         make_float2(s1, s * c1), make_float2(0.f, s),     make_float2(-s1, s * c1),
                         make_float2(-h, s * h),  make_float2(-c1, s * s1)};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float2 t = cmul(w[k], o[k]);
      v[k] = cadd(e[k], t);
      v[k + 8] = csub(e[k], t);
    }
  }
};

template <int R>
__device__ __forceinline__ void stockham_stage(float2* __restrict__ buf, int len, int nl, int ld,
                                               int Ns, const float2* __restrict__ tw, int tw_stride,
                                               float sgn) {
  constexpr int kB = (kMaxE + R - 1) / R;
  const int nbl = len / R;
  const int nbf = nbl * nl;
  const int step = (len / (Ns * R)) * tw_stride;
  float2 v[kB][R];
#pragma unroll
  for (int b = 0; b < kB; ++b) {
    const int t = threadIdx.x + b * kFT;
    if (t < nbf) {
      const int l = t / nbl, j = t - l * nbl;
      const float2* src = buf + l * ld + j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = src[r * nbl];
      const int k = j % Ns;
      if (k != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[r * k * step];  // exp(-2 pi i m / n)
          if (sgn > 0.f) w.y = -w.y;    // inverse: conjugate
          v[b][r] = cmul(v[b][r], w);
        }
      }
      Dft<R>::run(v[b], sgn);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < kB; ++b) {
    const int t = threadIdx.x + b * kFT;
    if (t < nbf) {
      const int l = t / nbl, j = t - l * nbl;
      const int k = j % Ns;
      float2* dst = buf + l * ld + (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * Ns] = v[b][r];
    }
  }
  __syncthreads();
}

// Transforms nl lines of length plan.n stored at buf[l * ld + i].
// sgn = -1 forward (exp(-i...)), +1 inverse (unnormalised).
__device__ void lds_fft(float2* __restrict__ buf, int nl, int ld, const FftPlan& plan,
                        const float2* __restrict__ tw, int tw_stride, float sgn) {
  int Ns = 1;
  for (int s = 0; s < plan.nstage; ++s) {
    const int R = plan.radix[s];
    switch (R) {
      case 16: stockham_stage<16>(buf, plan.n, nl, ld, Ns, tw, tw_stride, sgn); break;
      case 8: stockham_stage<8>(buf, plan.n, nl, ld, Ns, tw, tw_stride, sgn); break;
      case 4: stockham_stage<4>(buf, plan.n, nl, ld, Ns, tw, tw_stride, sgn); break;
      case 3: stockham_stage<3>(buf, plan.n, nl, ld, Ns, tw, tw_stride, sgn); break;
      default: stockham_stage<2>(buf, plan.n, nl, ld, Ns, tw, tw_stride, sgn); break;
    }
    Ns *= R;
  }
}

// ---------------------------------------------------------------------------
// z pass: rows of n reals (row stride `cols` complex).  nl rows per workgroup.
__global__ __launch_bounds__(kFT) void k_r2c_z(float2* __restrict__ mesh, long nrows, int cols,
                                               int nl, long mesh_stride, FftPlan plan,
                                               const float2* __restrict__ tw) {
  extern __shared__ float2 lds[];
  const int h = plan.n;  // half length
  const int n = 2 * h;
  const int ld = h + 1;
  float2* base = mesh + blockIdx.y * mesh_stride;
  const long r0 = (long)blockIdx.x * nl;
  const int nrow = (int)((nrows - r0) < nl ? (nrows - r0) : nl);
  for (int i = threadIdx.x; i < nrow * h; i += kFT) {
    const int l = i / h, j = i - l * h;
    lds[l * ld + j] = base[(r0 + l) * cols + j];
  }
  __syncthreads();
  lds_fft(lds, nrow, ld, plan, tw, 2, -1.f);
  // split step: X_k = E_k + W_n^k O_k, E = (Z_k + conj Z_{h-k})/2, O = -i (Z_k - conj Z_{h-k})/2
  for (int i = threadIdx.x; i < nrow * cols; i += kFT) {
    const int l = i / cols, k = i - l * cols;
    float2 x = make_float2(0.f, 0.f);
    if (k <= h) {
      const float2 a = lds[l * ld + (k == h ? 0 : k)];
      float2 b = lds[l * ld + (k == 0 ? 0 : h - k)];
      b.y = -b.y;
      const float2 e = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y + b.y));
      const float2 o = make_float2(0.5f * (a.y - b.y), -0.5f * (a.x - b.x));
      x = cadd(e, cmul(tw[k], o));
    }
    base[(r0 + l) * cols + k] = x;
  }
}

// Inverse z pass: half spectrum (h+1 values) -> n reals, unnormalised.
__global__ __launch_bounds__(kFT) void k_c2r_z(float2* __restrict__ mesh, long nrows, int cols,
                                               int nl, long mesh_stride, FftPlan plan,
                                               const float2* __restrict__ tw) {
  extern __shared__ float2 lds[];
  const int h = plan.n;
  const int ld = h + 1;
  float2* base = mesh + blockIdx.y * mesh_stride;
  const long r0 = (long)blockIdx.x * nl;
  const int nrow = (int)((nrows - r0) < nl ? (nrows - r0) : nl);
  for (int i = threadIdx.x; i < nrow * (h + 1); i += kFT) {
    const int l = i / (h + 1), j = i - l * (h + 1);
    lds[l * ld + j] = base[(r0 + l) * cols + j];
  }
  __syncthreads();
  // Z'_k = (X_k + conj X_{h-k}) + i (X_k - conj X_{h-k}) exp(+2 pi i k / n), k < h.
  // Pairs (k, h-k) are handled by one thread, in place.
  const int hp = h / 2 + 1;
  for (int i = threadIdx.x; i < nrow * hp; i += kFT) {
    const int l = i / hp, k = i - l * hp;
    const int k2 = h - k;
    const float2 xa = lds[l * ld + k], xb = lds[l * ld + k2];
    float2 za, zb;
    {
      const float2 cb = make_float2(xb.x, -xb.y);
      const float2 e = cadd(xa, cb);
      float2 w = tw[k];
      w.y = -w.y;
      const float2 o = cmul(csub(xa, cb), w);
      za = cadd(e, make_float2(-o.y, o.x));
    }
    {
      const float2 ca = make_float2(xa.x, -xa.y);
      const float2 e = cadd(xb, ca);
      float2 w = tw[k2];
      w.y = -w.y;
      const float2 o = cmul(csub(xb, ca), w);
      zb = cadd(e, make_float2(-o.y, o.x));
    }
    // each pair belongs to exactly one thread: no other thread touches k or k2
    lds[l * ld + k] = za;
    if (k2 != k && k2 != h) lds[l * ld + k2] = zb;
  }
  __syncthreads();
  lds_fft(lds, nrow, ld, plan, tw, 2, 1.f);
  for (int i = threadIdx.x; i < nrow * h; i += kFT) {
    const int l = i / h, j = i - l * h;
    base[(r0 + l) * cols + j] = lds[l * ld + j];
  }
}

// ---------------------------------------------------------------------------
// Strided column passes.  Element e of column c in plane p sits at
// data[p * plane_stride + e * elem_stride + c].
struct ColGeom {
  long elem_stride;
  long plane_stride;
  int cols;       // padded columns (multiple of W)
  int w;          // columns per workgroup
  int nchunk;     // cols / w
  int nplanes;
};

__device__ __forceinline__ int signed_freq(int i, int n) { return i <= n / 2 ? i : i - n; }

// k-space multiplier for mode (nx, ny, nz); rfft axis nz in [0, n/2].
__device__ __forceinline__ float2 multiplier(int kind, int green, int ca, int cb, float scale,
                                             int nx, int ny, int nz, int n,
                                             const float* __restrict__ amp, int is_amp) {
  const int h = n / 2;
  if (nz > h) return make_float2(0.f, 0.f);
  const int ax = nx < 0 ? -nx : nx, ay = ny < 0 ? -ny : ny;
  const int n2 = nx * nx + ny * ny + nz * nz;
  if (n2 == 0) return make_float2(0.f, 0.f);
  const bool nyq = ax == h || ay == h || nz == h;
  const int nv[3] = {nx, ny, nz};
  if (is_amp) {
    if (nyq) return make_float2(0.f, 0.f);
    return make_float2(amp[n2], 0.f);
  }
  if (kind == M_GRAD) {
    const int na = nv[ca];
    const int aa = na < 0 ? -na : na;
    if (green ? (aa == h) : nyq) return make_float2(0.f, 0.f);
    return make_float2(0.f, scale * (float)na / (float)n2);
  }
  if (kind == M_HESS) {
    if (nyq) return make_float2(0.f, 0.f);
    return make_float2(scale * (float)nv[ca] * (float)nv[cb] / (float)n2, 0.f);
  }
  return make_float2(1.f, 0.f);
}

template <int MODE>
__global__ __launch_bounds__(kFT) void k_cols(const float2* __restrict__ in, float2* out0,
                                              float2* out1, float2* out2, long mesh_stride,
                                              ColGeom g, FftPlan plan,
                                              const float2* __restrict__ tw, int mult, int ca,
                                              int cb, float scale, const float* __restrict__ amp,
                                              int y_is_plane_freq) {
  extern __shared__ float2 lds[];
  const int n = plan.n;
  const int ld = n + 1;
  const uint32_t nblk = (uint32_t)g.nchunk * g.nplanes;
  const uint32_t bid = xcd_remap(blockIdx.x, nblk);
  const int p = bid / g.nchunk;
  const int c0 = (bid - p * g.nchunk) * g.w;
  const long mofs = (long)blockIdx.y * mesh_stride;
  const float2* src = in + mofs + p * g.plane_stride + c0;
  // load: consecutive threads take consecutive columns
  for (int i = threadIdx.x; i < n * g.w; i += kFT) {
    const int e = i / g.w, c = i - e * g.w;
    lds[c * ld + e] = src[e * g.elem_stride + c];
  }
  __syncthreads();
  const int pfreq = y_is_plane_freq ? signed_freq(p, n) : 0;

  if (MODE == X_FWD || MODE == X_INV) {
    lds_fft(lds, g.w, ld, plan, tw, 1, MODE == X_FWD ? -1.f : 1.f);
  } else if (MODE == X_FWD_AMP) {
    lds_fft(lds, g.w, ld, plan, tw, 1, -1.f);
    for (int i = threadIdx.x; i < n * g.w; i += kFT) {
      const int c = i / n, e = i - c * n;
      const float2 m = multiplier(0, 0, 0, 0, 0.f, signed_freq(e, n), pfreq, c0 + c, n, amp, 1);
      lds[c * ld + e] = cmul(lds[c * ld + e], m);
    }
    __syncthreads();
  } else if (MODE == X_MULT_INV) {
    for (int i = threadIdx.x; i < n * g.w; i += kFT) {
      const int c = i / n, e = i - c * n;
      const float2 m = multiplier(mult, 0, ca, cb, scale, signed_freq(e, n), pfreq, c0 + c, n, amp, 0);
      lds[c * ld + e] = cmul(lds[c * ld + e], m);
    }
    __syncthreads();
    lds_fft(lds, g.w, ld, plan, tw, 1, 1.f);
  }

  if (MODE != X_FWD_GREEN3) {
    float2* dst = out0 + mofs + p * g.plane_stride + c0;
    for (int i = threadIdx.x; i < n * g.w; i += kFT) {
      const int e = i / g.w, c = i - e * g.w;
      dst[e * g.elem_stride + c] = lds[c * ld + e];
    }
    return;
  }

  // PM: forward along x, then for each axis d: multiply by i k_d alpha / k^2
  // (scaled to mesh units and 1/N^3), inverse along x, store to out_d.
  lds_fft(lds, g.w, ld, plan, tw, 1, -1.f);
  float2 spec[kMaxE];
#pragma unroll
  for (int b = 0; b < kMaxE; ++b) {
    const int i = threadIdx.x + b * kFT;
    if (i < n * g.w) {
      const int c = i / n, e = i - c * n;
      spec[b] = lds[c * ld + e];
    }
  }
  __syncthreads();
  float2* outs[3] = {out0, out1, out2};
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int b = 0; b < kMaxE; ++b) {
      const int i = threadIdx.x + b * kFT;
      if (i < n * g.w) {
        const int c = i / n, e = i - c * n;
        const float2 m = multiplier(M_GRAD, 1, d, 0, scale, signed_freq(e, n), pfreq, c0 + c, n, amp, 0);
        lds[c * ld + e] = cmul(spec[b], m);
      }
    }
    __syncthreads();
    lds_fft(lds, g.w, ld, plan, tw, 1, 1.f);
    float2* dst = outs[d] + p * g.plane_stride + c0;
    for (int i = threadIdx.x; i < n * g.w; i += kFT) {
      const int e = i / g.w, c = i - e * g.w;
      dst[e * g.elem_stride + c] = lds[c * ld + e];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
namespace {

int cols_per_wg(int n) {
  int w = kLdsC / (n + 1);
  if (w > 16) w = 16;
  int p = 1;
  while (p * 2 <= w) p *= 2;
  return p;
}

size_t lds_bytes_cols(int n, int w) { return (size_t)w * (n + 1) * sizeof(float2); }

ColGeom geom(int n, int axis) {
  ColGeom g;
  const long cols = padded_cols(n);
  g.cols = (int)cols;
  g.w = cols_per_wg(n);
  if (g.w > g.cols) g.w = g.cols;
  g.nchunk = (int)(cols / g.w);
  g.nplanes = n;
  if (axis == 1) {  // y: planes are x
    g.elem_stride = cols;
    g.plane_stride = (long)n * cols;
  } else {          // x: planes are y
    g.elem_stride = (long)n * cols;
    g.plane_stride = cols;
  }
  return g;
}

}  // namespace

void fft_r2c_z(float2* mesh, int n, int nbatch, long mesh_stride, const TwiddleSet& tw, hipStream_t s) {
  FftPlan plan;
  make_plan(n / 2, &plan);
  const int h = n / 2;
  int nl = kLdsC / (h + 1);
  if (nl > 16) nl = 16;
  const long nrows = (long)n * n;
  const int cols = (int)padded_cols(n);
  dim3 grid((unsigned)((nrows + nl - 1) / nl), (unsigned)nbatch);
  hipLaunchKernelGGL(k_r2c_z, grid, dim3(kFT), (size_t)nl * (h + 1) * sizeof(float2), s, mesh,
                     nrows, cols, nl, mesh_stride, plan, tw.get(n));
}

void fft_c2r_z(float2* mesh, int n, int nbatch, long mesh_stride, const TwiddleSet& tw, hipStream_t s) {
  FftPlan plan;
  make_plan(n / 2, &plan);
  const int h = n / 2;
  int nl = kLdsC / (h + 1);
  if (nl > 16) nl = 16;
  const long nrows = (long)n * n;
  const int cols = (int)padded_cols(n);
  dim3 grid((unsigned)((nrows + nl - 1) / nl), (unsigned)nbatch);
  hipLaunchKernelGGL(k_c2r_z, grid, dim3(kFT), (size_t)nl * (h + 1) * sizeof(float2), s, mesh,
                     nrows, cols, nl, mesh_stride, plan, tw.get(n));
}

void fft_y(float2* mesh, int n, int nbatch, long mesh_stride, int inverse, const TwiddleSet& tw,
           hipStream_t s) {
  FftPlan plan;
  make_plan(n, &plan);
  const ColGeom g = geom(n, 1);
  dim3 grid((unsigned)(g.nchunk * g.nplanes), (unsigned)nbatch);
  const size_t lds = lds_bytes_cols(n, g.w);
  if (inverse)
    hipLaunchKernelGGL(k_cols<X_INV>, grid, dim3(kFT), lds, s, mesh, mesh, nullptr, nullptr,
                       mesh_stride, g, plan, tw.get(n), 0, 0, 0, 1.f, nullptr, 0);
  else
    hipLaunchKernelGGL(k_cols<X_FWD>, grid, dim3(kFT), lds, s, mesh, mesh, nullptr, nullptr,
                       mesh_stride, g, plan, tw.get(n), 0, 0, 0, 1.f, nullptr, 0);
}

void fft_x(const XPassArgs& a, int n, const TwiddleSet& tw, hipStream_t s) {
  FftPlan plan;
  make_plan(n, &plan);
  const ColGeom g = geom(n, 0);
  dim3 grid((unsigned)(g.nchunk * g.nplanes), 1);
  const size_t lds = lds_bytes_cols(n, g.w);
  const float2* twp = tw.get(n);
  switch (a.mode) {
    case X_FWD:
      hipLaunchKernelGGL(k_cols<X_FWD>, grid, dim3(kFT), lds, s, a.in, a.out[0], nullptr, nullptr, 0L,
                         g, plan, twp, 0, 0, 0, 1.f, nullptr, 1);
      break;
    case X_INV:
      hipLaunchKernelGGL(k_cols<X_INV>, grid, dim3(kFT), lds, s, a.in, a.out[0], nullptr, nullptr, 0L,
                         g, plan, twp, 0, 0, 0, 1.f, nullptr, 1);
      break;
    case X_FWD_AMP:
      hipLaunchKernelGGL(k_cols<X_FWD_AMP>, grid, dim3(kFT), lds, s, a.in, a.out[0], nullptr, nullptr,
                         0L, g, plan, twp, 0, 0, 0, 1.f, a.amp, 1);
      break;
    case X_MULT_INV:
      hipLaunchKernelGGL(k_cols<X_MULT_INV>, grid, dim3(kFT), lds, s, a.in, a.out[0], nullptr, nullptr,
                         0L, g, plan, twp, a.mult, a.comp_a, a.comp_b, a.scale, nullptr, 1);
      break;
    case X_FWD_GREEN3:
      hipLaunchKernelGGL(k_cols<X_FWD_GREEN3>, grid, dim3(kFT), lds, s, a.in, a.out[0], a.out[1],
                         a.out[2], 0L, g, plan, twp, M_GRAD, 0, 0, a.scale, nullptr, 1);
      break;
  }
}

void fft3d_forward(float2* mesh, int n, const TwiddleSet& tw, hipStream_t s) {
  fft_r2c_z(mesh, n, 1, 0, tw, s);
  fft_y(mesh, n, 1, 0, 0, tw, s);
  XPassArgs a;
  a.in = mesh;
  a.out[0] = mesh;
  a.mode = X_FWD;
  fft_x(a, n, tw, s);
}

void fft3d_inverse(float2* mesh, int n, const TwiddleSet& tw, hipStream_t s) {
  XPassArgs a;
  a.in = mesh;
  a.out[0] = mesh;
  a.mode = X_INV;
  fft_x(a, n, tw, s);
  fft_y(mesh, n, 1, 0, 1, tw, s);
  fft_c2r_z(mesh, n, 1, 0, tw, s);
}

}  // namespace cola
