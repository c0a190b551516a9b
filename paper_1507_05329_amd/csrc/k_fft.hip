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

// Compile-time plan: a {2,3}-smooth length factored as 3s first, then 16s,
// then one each of 8, 4, 2 as needed.
constexpr int radix_at(int n, int s) {
  int r[16] = {};
  int ns = 0, m = n;
  while (m % 3 == 0) { m /= 3; r[ns++] = 3; }
  while (m % 16 == 0) { m /= 16; r[ns++] = 16; }
  if (m % 8 == 0) { m /= 8; r[ns++] = 8; }
  if (m % 4 == 0) { m /= 4; r[ns++] = 4; }
  if (m % 2 == 0) { m /= 2; r[ns++] = 2; }
  return (m == 1 && s < ns) ? r[s] : 0;
}
constexpr int nstage(int n) { int s = 0; while (radix_at(n, s)) ++s; return s; }
constexpr int ns_before(int n, int s) { int p = 1; for (int i = 0; i < s; ++i) p *= radix_at(n, i); return p; }

// LDS line layout: element e of a line sits at pe(e) = e + e/32 (one pad
// slot after every 32), so the stride-R writes of a Stockham stage spread
// over the banks; lines are lds_ld(n) apart (odd, for the column loads).
constexpr int lds_ld(int n) { return n + n / 32 + 1; }
__device__ __forceinline__ int pe(int e) { return e + (e >> 5); }

// Launch shapes: at most 80 KB of LDS per workgroup, 256 threads below
// 4096 staged complex values, 512 from 4096 (measured on the 768 mesh: the
// row and column passes run 8-18% faster on 512 threads than on 256).
constexpr int kLdsLimit = 80 * 1024;
constexpr int cols_w(int n) { int w = 16; while (w > 1 && w * lds_ld(n) * 8 + n * 4 > kLdsLimit) w /= 2; return w; }
constexpr int rows_nl(int h) { int nl = 16; while (nl > 1 && nl * lds_ld(h) * 8 + h * 8 > kLdsLimit) nl /= 2; return nl; }
constexpr int threads_for(int elems) { return elems >= 4096 ? 512 : 256; }
// The two gradient passes keep a spectrum in registers across a transform:
// spread it over 512 threads, and cap them at 128 VGPRs (4 waves per SIMD).
constexpr bool holds_regs(int mode) { return mode == X_FWD_GREEN || mode == X_INV_GRAD_YZ; }
constexpr int cols_threads(int n, int mode) {
  return (holds_regs(mode) && cols_w(n) * n >= 4096) ? 512 : threads_for(cols_w(n) * n);
}

bool make_plan(int n, FftPlan* plan) {
  if (n < 2 || nstage(n) == 0) return false;
  plan->n = n;
  plan->nstage = nstage(n);
  for (int s = 0; s < plan->nstage; ++s) plan->radix[s] = radix_at(n, s);
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

// Twiddle exp(-2 pi i m / n) for 0 <= m < n from a half table of n/2 entries
// (the second half is the negated first half).
template <int NT>
__device__ __forceinline__ float2 tw_get(const float2* __restrict__ twl, int m) {
  if (m < NT / 2) return twl[m];
  const float2 w = twl[m - NT / 2];
  return make_float2(-w.x, -w.y);
}

// Stages S.. of a length-N transform of NL lines (line l at buf[l * LD]), T
// threads, twiddle table stride TWS, FWD = 1 forward / 0 inverse.
template <int N, int NL, int LD, int T, int TWS, int FWD, int S>
__device__ __forceinline__ void fft_stages(float2* __restrict__ buf, const float2* __restrict__ tw,
                                           int tid) {
  if constexpr (S < nstage(N)) {
    constexpr int R = radix_at(N, S), NS = ns_before(N, S);
    constexpr int NBL = N / R, NBF = NBL * NL, KB = (NBF + T - 1) / T;
    constexpr int STEP = (N / (NS * R)) * TWS;
    constexpr float sgn = FWD ? -1.f : 1.f;
    float2 v[KB][R];
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      const int t = tid + b * T;
      if (NBF % T == 0 || t < NBF) {
        const int l = t / NBL, j = t - l * NBL;
        const float2* src = buf + l * LD;
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = src[pe(j + r * NBL)];
        if constexpr (NS > 1) {
          const int k = j % NS;
#pragma unroll
          for (int r = 1; r < R; ++r) {
            float2 w = tw_get<N * TWS>(tw, r * k * STEP);  // exp(-2 pi i m / n)
            if (!FWD) w.y = -w.y;         // inverse: conjugate
            v[b][r] = cmul(v[b][r], w);
          }
        }
        Dft<R>::run(v[b], sgn);
      }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      const int t = tid + b * T;
      if (NBF % T == 0 || t < NBF) {
        const int l = t / NBL, j = t - l * NBL;
        const int k = j % NS;
        float2* dst = buf + l * LD;
        const int o = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[pe(o + r * NS)] = v[b][r];
      }
    }
    __syncthreads();
    fft_stages<N, NL, LD, T, TWS, FWD, S + 1>(buf, tw, tid);
  }
}

// threadIdx.x through an empty asm: the compiler cannot prove two such
// values equal, so address arithmetic derived from them is not shared.
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// tid: the thread's index (threadIdx.x; a caller inside a loop passes a
// value the compiler cannot treat as loop-invariant, so that the stages'
// address arithmetic is not hoisted out of the loop and kept live).
template <int N, int NL, int LD, int T, int TWS, int FWD>
__device__ __forceinline__ void lds_fft(float2* __restrict__ buf, const float2* __restrict__ tw,
                                        int tid = threadIdx.x) {
  fft_stages<N, NL, LD, T, TWS, FWD, 0>(buf, tw, tid);
}

// Global -> LDS copies with every load of a thread issued before the first
// LDS store, so each wave keeps all of its loads in flight.
template <int NT, int T>
__device__ __forceinline__ void load_twiddles(float2* __restrict__ twl, const float2* __restrict__ tw) {
  constexpr int K = (NT + T - 1) / T;
  float2 t[K];
#pragma unroll
  for (int b = 0; b < K; ++b) {
    const int i = threadIdx.x + b * T;
    if (NT % T == 0 || i < NT) t[b] = tw[i];
  }
#pragma unroll
  for (int b = 0; b < K; ++b) {
    const int i = threadIdx.x + b * T;
    if (NT % T == 0 || i < NT) twl[i] = t[b];
  }
}

// W adjacent columns of N elements (element stride es) into LDS lines.
template <int N, int W, int LD, int T>
__device__ __forceinline__ void load_cols(float2* __restrict__ lds, const float2* __restrict__ src, long es) {
  constexpr int K = (N * W + T - 1) / T;
  float2 t[K];
#pragma unroll
  for (int b = 0; b < K; ++b) {
    const int i = threadIdx.x + b * T;
    const int e = i / W, c = i - e * W;
    if ((N * W) % T == 0 || i < N * W) t[b] = src[e * es + c];
  }
#pragma unroll
  for (int b = 0; b < K; ++b) {
    const int i = threadIdx.x + b * T;
    const int e = i / W, c = i - e * W;
    if ((N * W) % T == 0 || i < N * W) lds[c * LD + pe(e)] = t[b];
  }
}

// LDS lines -> W adjacent columns, in chunks of kCh values per thread (the
// LDS reads of a chunk before its stores; the empty asm keeps the compiler
// from hoisting later chunks and raising the register count).
constexpr int kCh = 6;
template <int N, int W, int LD, int T>
__device__ __forceinline__ void store_cols(float2* __restrict__ dst, long es, const float2* __restrict__ lds) {
  constexpr int K = (N * W + T - 1) / T;
#pragma unroll
  for (int b0 = 0; b0 < K; b0 += kCh) {
    float2 t[kCh];
#pragma unroll
    for (int q = 0; q < kCh; ++q) {
      const int i = threadIdx.x + (b0 + q) * T;
      const int e = i / W, c = i - e * W;
      if (b0 + q < K && ((N * W) % T == 0 || i < N * W)) t[q] = lds[c * LD + pe(e)];
    }
#pragma unroll
    for (int q = 0; q < kCh; ++q) {
      const int i = threadIdx.x + (b0 + q) * T;
      const int e = i / W, c = i - e * W;
      if (b0 + q < K && ((N * W) % T == 0 || i < N * W)) dst[e * es + c] = t[q];
    }
    asm volatile("" ::: "memory");
  }
}

// Padded complex row length (compile-time copy of padded_cols).
constexpr int pcols(int n) { return ((n / 2 + 1) + 15) / 16 * 16; }

// ---------------------------------------------------------------------------
// z pass: rows of N reals (row stride `cols` complex).  NL rows per workgroup.
template <int N>
__global__ __launch_bounds__(threads_for(rows_nl(N / 2) * (N / 2))) void k_r2c_z(
    float2* __restrict__ mesh, long nrows, int cols, long mesh_stride, const float2* __restrict__ tw,
    long mstride) {
  constexpr int H = N / 2, LD = lds_ld(H), NL = rows_nl(H), T = threads_for(NL * H);
  constexpr int LE = (NL * H + T - 1) / T;
  mesh = mock_ptr(mesh, mstride);
  __shared__ float2 lds[NL * LD];
  __shared__ float2 twl[N / 2];
  float2* base = mesh + blockIdx.y * mesh_stride;
  const long r0 = (long)blockIdx.x * NL;
  load_twiddles<N / 2, T>(twl, tw);
  {
    float2 t[LE];
#pragma unroll
    for (int b = 0; b < LE; ++b) {
      const int i = threadIdx.x + b * T;
      const int l = i / H, j = i - l * H;
      if (((NL * H) % T == 0 || i < NL * H) && r0 + l < nrows) t[b] = base[(r0 + l) * cols + j];
    }
#pragma unroll
    for (int b = 0; b < LE; ++b) {
      const int i = threadIdx.x + b * T;
      const int l = i / H, j = i - l * H;
      if (((NL * H) % T == 0 || i < NL * H) && r0 + l < nrows) lds[l * LD + pe(j)] = t[b];
    }
  }
  __syncthreads();
  lds_fft<H, NL, LD, T, 2, 1>(lds, twl);
  // split step: X_k = E_k + W_n^k O_k, E = (Z_k + conj Z_{h-k})/2, O = -i (Z_k - conj Z_{h-k})/2
  constexpr int COLS = pcols(N), NO = NL * COLS, KO = (NO + T - 1) / T;
  float2 xs[KO];
#pragma unroll
  for (int q = 0; q < KO; ++q) {
    const int i = threadIdx.x + q * T;
    const int l = i / COLS, k = i - l * COLS;
    xs[q] = make_float2(0.f, 0.f);
    if ((NO % T == 0 || i < NO) && k <= H) {
      const float2 a = lds[l * LD + pe(k == H ? 0 : k)];
      float2 b = lds[l * LD + pe(k == 0 ? 0 : H - k)];
      b.y = -b.y;
      const float2 e = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y + b.y));
      const float2 o = make_float2(0.5f * (a.y - b.y), -0.5f * (a.x - b.x));
      xs[q] = cadd(e, cmul(tw_get<N>(twl, k), o));
    }
  }
#pragma unroll
  for (int q = 0; q < KO; ++q) {
    const int i = threadIdx.x + q * T;
    const int l = i / COLS, k = i - l * COLS;
    if ((NO % T == 0 || i < NO) && r0 + l < nrows) base[(r0 + l) * COLS + k] = xs[q];
  }
}

// Inverse z pass: half spectrum (H+1 values) -> N reals, unnormalised.
template <int N>
__global__ __launch_bounds__(threads_for(rows_nl(N / 2) * (N / 2))) void k_c2r_z(
    float2* __restrict__ mesh, long nrows, int cols, long mesh_stride, const float2* __restrict__ tw,
    long mstride) {
  constexpr int H = N / 2, LD = lds_ld(H), NL = rows_nl(H), T = threads_for(NL * H);
  mesh = mock_ptr(mesh, mstride);
  __shared__ float2 lds[NL * LD];
  __shared__ float2 twl[N / 2];
  float2* base = mesh + blockIdx.y * mesh_stride;
  const long r0 = (long)blockIdx.x * NL;
  // Each thread loads whole pairs (k, h-k) of a row and forms
  //   Z'_k = (X_k + conj X_{h-k}) + i (X_k - conj X_{h-k}) exp(+2 pi i k / n)
  // (and Z'_{h-k} likewise) in registers, k = 0 .. h/2.
  constexpr int HP = H / 2 + 1, NPR = NL * HP, KP = (NPR + T - 1) / T;
  float2 xa[KP], xb[KP];
#pragma unroll
  for (int b = 0; b < KP; ++b) {
    const int i = threadIdx.x + b * T;
    const int l = i / HP, k = i - l * HP;
    xa[b] = make_float2(0.f, 0.f);
    xb[b] = make_float2(0.f, 0.f);
    if ((NPR % T == 0 || i < NPR) && r0 + l < nrows) {
      xa[b] = base[(r0 + l) * cols + k];
      xb[b] = base[(r0 + l) * cols + (H - k)];
    }
  }
  load_twiddles<N / 2, T>(twl, tw);
  __syncthreads();
#pragma unroll
  for (int b = 0; b < KP; ++b) {
    const int i = threadIdx.x + b * T;
    if (NPR % T == 0 || i < NPR) {
      const int l = i / HP, k = i - l * HP;
      const int k2 = H - k;
      float2 za, zb;
      {
        const float2 cb = make_float2(xb[b].x, -xb[b].y);
        const float2 e = cadd(xa[b], cb);
        float2 w = tw_get<N>(twl, k);
        w.y = -w.y;
        const float2 o = cmul(csub(xa[b], cb), w);
        za = cadd(e, make_float2(-o.y, o.x));
      }
      {
        const float2 ca = make_float2(xa[b].x, -xa[b].y);
        const float2 e = cadd(xb[b], ca);
        float2 w = tw_get<N>(twl, k2);
        w.y = -w.y;
        const float2 o = cmul(csub(xb[b], ca), w);
        zb = cadd(e, make_float2(-o.y, o.x));
      }
      lds[l * LD + pe(k)] = za;
      if (k2 != k && k2 != H) lds[l * LD + pe(k2)] = zb;
    }
  }
  __syncthreads();
  lds_fft<H, NL, LD, T, 2, 0>(lds, twl);
  {
    constexpr int KO = (NL * H + T - 1) / T;
    float2 t[KO];
#pragma unroll
    for (int q = 0; q < KO; ++q) {
      const int i = threadIdx.x + q * T;
      const int l = i / H, j = i - l * H;
      if ((NL * H) % T == 0 || i < NL * H) t[q] = lds[l * LD + pe(j)];
    }
#pragma unroll
    for (int q = 0; q < KO; ++q) {
      const int i = threadIdx.x + q * T;
      const int l = i / H, j = i - l * H;
      if (((NL * H) % T == 0 || i < NL * H) && r0 + l < nrows) base[(r0 + l) * cols + j] = t[q];
    }
  }
}

// ---------------------------------------------------------------------------
// Strided column passes.  Element e of column c in plane p sits at
// data[p * plane_stride + e * elem_stride + c].
struct ColGeom {
  long elem_stride;
  long plane_stride;
  int cols;       // padded columns (multiple of W)
  int nchunk;     // cols / W
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
  if (is_amp) {
    if (nyq) return make_float2(0.f, 0.f);
    return make_float2(amp[n2], 0.f);
  }
  if (kind == M_GRAD) {
    const int na = ca == 0 ? nx : (ca == 1 ? ny : nz);
    const int aa = na < 0 ? -na : na;
    if (green ? (aa == h) : nyq) return make_float2(0.f, 0.f);
    return make_float2(0.f, scale * (float)na / (float)n2);
  }
  if (kind == M_HESS) {
    if (nyq) return make_float2(0.f, 0.f);
    const int na = ca == 0 ? nx : (ca == 1 ? ny : nz);
    const int nb = cb == 0 ? nx : (cb == 1 ? ny : nz);
    return make_float2(scale * (float)na * (float)nb / (float)n2, 0.f);
  }
  return make_float2(1.f, 0.f);
}

template <int N, int MODE>
__global__ __launch_bounds__(cols_threads(N, MODE), holds_regs(MODE) ? 4 : 1) void k_cols(
    const float2* __restrict__ in, float2* out0, float2* out1, float2* out2, long mesh_stride,
    ColGeom g, const float2* __restrict__ tw, int mult, int ca, int cb, float scale,
    const float* __restrict__ amp, int y_is_plane_freq, const StepCoef* __restrict__ coef,
    long mstride) {
  in = mock_ptr(in, mstride);
  out0 = mock_ptr(out0, mstride);
  if constexpr (MODE == X_FWD_GREEN || MODE == X_INV_GRAD_YZ) out1 = mock_ptr(out1, mstride);
  if constexpr (MODE == X_FWD_GREEN) {
    if (coef) scale = mock_ptr(coef, mstride)->gscale;
  }
  constexpr int W = cols_w(N), LD = lds_ld(N), T = cols_threads(N, MODE);
  constexpr int E = (W * N + T - 1) / T;
  __shared__ float2 lds[W * LD];
  __shared__ float2 twl[N / 2];
  const uint32_t nblk = (uint32_t)g.nchunk * g.nplanes;
  const uint32_t bid = xcd_remap(blockIdx.x, nblk);
  const int p = bid / g.nchunk;
  const int c0 = (bid - p * g.nchunk) * W;
  const long mofs = (long)blockIdx.y * mesh_stride;
  const float2* src = in + mofs + p * g.plane_stride + c0;
  // load: consecutive threads take consecutive columns
  load_twiddles<N / 2, T>(twl, tw);
  load_cols<N, W, LD, T>(lds, src, g.elem_stride);
  __syncthreads();
  const int pfreq = y_is_plane_freq ? signed_freq(p, N) : 0;

  if constexpr (MODE == X_FWD || MODE == X_INV) {
    lds_fft<N, W, LD, T, 1, MODE == X_FWD ? 1 : 0>(lds, twl);
  } else if constexpr (MODE == X_FWD_AMP) {
    lds_fft<N, W, LD, T, 1, 1>(lds, twl);
    for (int i = threadIdx.x; i < N * W; i += T) {
      const int c = i / N, e = i - c * N;
      const float2 m = multiplier(0, 0, 0, 0, 0.f, signed_freq(e, N), pfreq, c0 + c, N, amp, 1);
      lds[c * LD + pe(e)] = cmul(lds[c * LD + pe(e)], m);
    }
    __syncthreads();
  } else if constexpr (MODE == X_MULT_INV) {
    for (int i = threadIdx.x; i < N * W; i += T) {
      const int c = i / N, e = i - c * N;
      const float2 m = multiplier(mult, 0, ca, cb, scale, signed_freq(e, N), pfreq, c0 + c, N, amp, 0);
      lds[c * LD + pe(e)] = cmul(lds[c * LD + pe(e)], m);
    }
    __syncthreads();
    lds_fft<N, W, LD, T, 1, 0>(lds, twl);
  }

  if constexpr (MODE == X_FWD_GREEN) {
    // PM, x pass: forward along x gives S = DFT[delta]; with phi = scale S / |n|^2
    //   out0 = IDFT_x[i n_x phi]  (n_x on its Nyquist index -> 0)  -> g_x,
    //   out1 = IDFT_x[phi]                                         -> g_y, g_z
    // (n_y and n_z are constant along an x line; the y pass applies them).
    lds_fft<N, W, LD, T, 1, 1>(lds, twl);
    float2 phi[E];
#pragma unroll
    for (int b = 0; b < E; ++b) {
      const int i = threadIdx.x + b * T;
      if ((W * N) % T == 0 || i < N * W) {
        const int c = i / N, e = i - c * N;
        const int nx = signed_freq(e, N), nz = c0 + c;
        const int n2 = nx * nx + pfreq * pfreq + nz * nz;
        const float inv = (n2 == 0 || nz > N / 2) ? 0.f : scale / (float)n2;
        const float2 v = lds[c * LD + pe(e)];
        phi[b] = make_float2(inv * v.x, inv * v.y);
        const float kx = (nx == N / 2 || nx == -N / 2) ? 0.f : (float)nx;
        lds[c * LD + pe(e)] = make_float2(-kx * phi[b].y, kx * phi[b].x);  // i n_x phi
      }
    }
    __syncthreads();
    lds_fft<N, W, LD, T, 1, 0>(lds, twl);
    {
      float2* dst = out0 + p * g.plane_stride + c0;
      for (int i = threadIdx.x; i < N * W; i += T) {
        const int e = i / W, c = i - e * W;
        dst[e * g.elem_stride + c] = lds[c * LD + pe(e)];
      }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < E; ++b) {
      const int i = threadIdx.x + b * T;
      if ((W * N) % T == 0 || i < N * W) {
        const int c = i / N, e = i - c * N;
        lds[c * LD + pe(e)] = phi[b];
      }
    }
    __syncthreads();
    lds_fft<N, W, LD, T, 1, 0>(lds, twl);
    {
      float2* dst = out1 + p * g.plane_stride + c0;
      for (int i = threadIdx.x; i < N * W; i += T) {
        const int e = i / W, c = i - e * W;
        dst[e * g.elem_stride + c] = lds[c * LD + pe(e)];
      }
    }
  } else if constexpr (MODE == X_INV_GRAD_YZ) {
    // PM, inverse y pass of B = IDFT_x[phi]: out0 = IDFT_y[i n_y B], out1 =
    // IDFT_y[i n_z B] (each component zeroed on its own Nyquist index).
    float2 bv[E];
#pragma unroll
    for (int b = 0; b < E; ++b) {
      const int i = threadIdx.x + b * T;
      if ((W * N) % T == 0 || i < N * W) {
        const int c = i / N, e = i - c * N;
        const int ny = signed_freq(e, N);
        const float ky = (ny == N / 2 || ny == -N / 2) ? 0.f : (float)ny;
        bv[b] = lds[c * LD + pe(e)];
        lds[c * LD + pe(e)] = make_float2(-ky * bv[b].y, ky * bv[b].x);  // i n_y B
      }
    }
    __syncthreads();
    lds_fft<N, W, LD, T, 1, 0>(lds, twl);
    {
      float2* dst = out0 + p * g.plane_stride + c0;
      for (int i = threadIdx.x; i < N * W; i += T) {
        const int e = i / W, c = i - e * W;
        dst[e * g.elem_stride + c] = lds[c * LD + pe(e)];
      }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < E; ++b) {
      const int i = threadIdx.x + b * T;
      if ((W * N) % T == 0 || i < N * W) {
        const int c = i / N, e = i - c * N;
        const float kz = (c0 + c >= N / 2) ? 0.f : (float)(c0 + c);
        lds[c * LD + pe(e)] = make_float2(-kz * bv[b].y, kz * bv[b].x);  // i n_z B
      }
    }
    __syncthreads();
    lds_fft<N, W, LD, T, 1, 0>(lds, twl);
    {
      float2* dst = out1 + p * g.plane_stride + c0;
      for (int i = threadIdx.x; i < N * W; i += T) {
        const int e = i / W, c = i - e * W;
        dst[e * g.elem_stride + c] = lds[c * LD + pe(e)];
      }
    }
  } else {
    store_cols<N, W, LD, T>(out0 + mofs + p * g.plane_stride + c0, g.elem_stride, lds);
  }
}

// x pass of a spectral combination: out = IDFT_x[ sum_q m_q(k) DFT_x(in_q) ]
// for inputs already transformed along z and y (so m_q sees the full k).
// m_q is the gradient (i n_d scale / |n|^2) or Hessian (n_a n_b scale / |n|^2)
// multiplier, optionally times the amplitude table; accumulate adds the result
// to out instead of overwriting it.  Used by the adjoint (transposed Green's
// function and transposed 2LPT maps).
template <int N>
__global__ __launch_bounds__(cols_threads(N, X_FWD_GREEN)) void k_combine(
    const float2* __restrict__ in0, const float2* __restrict__ in1, const float2* __restrict__ in2,
    float2* out, ColGeom g, const float2* __restrict__ tw, CombineSpec cs,
    const float* __restrict__ amp) {
  // the accumulator lives in registers across the inputs: spread it over
  // as many threads as the Green's-function pass
  constexpr int W = cols_w(N), LD = lds_ld(N), T = cols_threads(N, X_FWD_GREEN);
  constexpr int E = (W * N + T - 1) / T;
  __shared__ float2 lds[W * LD];
  __shared__ float2 twl[N / 2];
  const uint32_t nblk = (uint32_t)g.nchunk * g.nplanes;
  const uint32_t bid = xcd_remap(blockIdx.x, nblk);
  const int p = bid / g.nchunk;
  const int c0 = (bid - p * g.nchunk) * W;
  const int pfreq = signed_freq(p, N);
  load_twiddles<N / 2, T>(twl, tw);
  // per-element scale / |n|^2 (times the amplitude), shared by the inputs
  float2 acc[E];
  float rw[E];
  const int h = N / 2;
#pragma unroll
  for (int b = 0; b < E; ++b) {
    acc[b] = make_float2(0.f, 0.f);
    rw[b] = 0.f;
    const int i = threadIdx.x + b * T;
    if ((W * N) % T == 0 || i < N * W) {
      const int c = i / N, e = i - c * N;
      const int nx = signed_freq(e, N), nz = c0 + c;
      const int n2 = nx * nx + pfreq * pfreq + nz * nz;
      const bool nyq = nx == h || nx == -h || pfreq == h || pfreq == -h || nz == h;
      if (n2 != 0 && nz <= h && !(cs.use_amp && nyq))
        rw[b] = cs.scale / (float)n2 * (cs.use_amp ? amp[n2] : 1.f);
    }
  }
  const float2* ins[3] = {in0, in1, in2};
#pragma unroll 1
  for (int q = 0; q < cs.nin; ++q) {
    const float2* src = ins[q] + p * g.plane_stride + c0;
    load_cols<N, W, LD, T>(lds, src, g.elem_stride);
    __syncthreads();
    lds_fft<N, W, LD, T, 1, 1>(lds, twl, opaque_tid());
    const int kind = cs.kind[q], ca = cs.ca[q], cb = cs.cb[q];
#pragma unroll
    for (int b = 0; b < E; ++b) {
      const int i = threadIdx.x + b * T;
      if ((W * N) % T == 0 || i < N * W) {
        const int c = i / N, e = i - c * N;
        const int nx = signed_freq(e, N), nz = c0 + c;
        const int na = ca == 0 ? nx : (ca == 1 ? pfreq : nz);
        const bool nyq = nx == h || nx == -h || pfreq == h || pfreq == -h || nz == h;
        const float2 x = lds[c * LD + pe(e)];
        if (kind == M_GRAD) {
          // i n_a rw; zero on the axis' own Nyquist plane (Green) or any Nyquist index
          const bool z = cs.green ? (na == h || na == -h) : nyq;
          const float f = z ? 0.f : (float)na * rw[b];
          acc[b] = cadd(acc[b], make_float2(-f * x.y, f * x.x));
        } else {
          const int nb = cb == 0 ? nx : (cb == 1 ? pfreq : nz);
          const float f = nyq ? 0.f : (float)na * (float)nb * rw[b];
          acc[b] = cadd(acc[b], make_float2(f * x.x, f * x.y));
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < E; ++b) {
    const int i = threadIdx.x + b * T;
    if ((W * N) % T == 0 || i < N * W) {
      const int c = i / N, e = i - c * N;
      lds[c * LD + pe(e)] = acc[b];
    }
  }
  __syncthreads();
  lds_fft<N, W, LD, T, 1, 0>(lds, twl);
  float2* dst = out + p * g.plane_stride + c0;
  for (int i = threadIdx.x; i < N * W; i += T) {
    const int e = i / W, c = i - e * W;
    const float2 v = lds[c * LD + pe(e)];
    if (cs.accumulate) {
      const float2 o = dst[e * g.elem_stride + c];
      dst[e * g.elem_stride + c] = cadd(o, v);
    } else {
      dst[e * g.elem_stride + c] = v;
    }
  }
}

// ---------------------------------------------------------------------------
namespace {

ColGeom geom(int n, int w, int axis) {
  ColGeom g;
  const long cols = padded_cols(n);
  g.cols = (int)cols;
  g.nchunk = (int)(cols / w);
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

template <int N>
void r2c_n(float2* mesh, int nbatch, long mesh_stride, const float2* tw, hipStream_t s, int nmock,
           long mstride) {
  constexpr int NL = rows_nl(N / 2), T = threads_for(NL * (N / 2));
  const long nrows = (long)N * N;
  dim3 grid((unsigned)((nrows + NL - 1) / NL), (unsigned)nbatch, (unsigned)nmock);
  hipLaunchKernelGGL(k_r2c_z<N>, grid, dim3(T), 0, s, mesh, nrows, (int)padded_cols(N), mesh_stride, tw,
                     mstride);
}

template <int N>
void c2r_n(float2* mesh, int nbatch, long mesh_stride, const float2* tw, hipStream_t s, int nmock,
           long mstride) {
  constexpr int NL = rows_nl(N / 2), T = threads_for(NL * (N / 2));
  const long nrows = (long)N * N;
  dim3 grid((unsigned)((nrows + NL - 1) / NL), (unsigned)nbatch, (unsigned)nmock);
  hipLaunchKernelGGL(k_c2r_z<N>, grid, dim3(T), 0, s, mesh, nrows, (int)padded_cols(N), mesh_stride, tw,
                     mstride);
}

template <int N>
void cols_n(int mode, int axis, const float2* in, float2* const out[3], int nbatch, long mesh_stride,
            const float2* tw, int mult, int ca, int cb, float scale, const float* amp, hipStream_t s,
            const StepCoef* coef = nullptr, int nmock = 1, long mstride = 0) {
  constexpr int W = cols_w(N);
  const ColGeom g = geom(N, W, axis);
  dim3 grid((unsigned)(g.nchunk * g.nplanes), (unsigned)nbatch, (unsigned)nmock);
  const int yf = axis == 0 ? 1 : 0;
  switch (mode) {
    case X_FWD:
      hipLaunchKernelGGL((k_cols<N, X_FWD>), grid, dim3(cols_threads(N, X_FWD)), 0, s, in, out[0], nullptr, nullptr,
                         mesh_stride, g, tw, 0, 0, 0, 1.f, nullptr, yf, nullptr, mstride);
      break;
    case X_INV:
      hipLaunchKernelGGL((k_cols<N, X_INV>), grid, dim3(cols_threads(N, X_INV)), 0, s, in, out[0], nullptr, nullptr,
                         mesh_stride, g, tw, 0, 0, 0, 1.f, nullptr, yf, nullptr, mstride);
      break;
    case X_FWD_AMP:
      hipLaunchKernelGGL((k_cols<N, X_FWD_AMP>), grid, dim3(cols_threads(N, X_FWD_AMP)), 0, s, in, out[0], nullptr, nullptr,
                         mesh_stride, g, tw, 0, 0, 0, 1.f, amp, yf, nullptr, mstride);
      break;
    case X_MULT_INV:
      hipLaunchKernelGGL((k_cols<N, X_MULT_INV>), grid, dim3(cols_threads(N, X_MULT_INV)), 0, s, in, out[0], nullptr, nullptr,
                         mesh_stride, g, tw, mult, ca, cb, scale, nullptr, yf, nullptr, mstride);
      break;
    case X_FWD_GREEN:
      hipLaunchKernelGGL((k_cols<N, X_FWD_GREEN>), grid, dim3(cols_threads(N, X_FWD_GREEN)), 0, s, in, out[0], out[1], nullptr,
                         mesh_stride, g, tw, M_GRAD, 0, 0, scale, nullptr, yf, coef, mstride);
      break;
    case X_INV_GRAD_YZ:
      hipLaunchKernelGGL((k_cols<N, X_INV_GRAD_YZ>), grid, dim3(cols_threads(N, X_INV_GRAD_YZ)), 0, s, in, out[0], out[1], nullptr,
                         mesh_stride, g, tw, 0, 0, 0, 1.f, nullptr, yf, nullptr, mstride);
      break;
  }
}

#define COLA_FFT_SIZES(X) X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) \
  X(768) X(1024) X(1536) X(2048)

}  // namespace

bool fft_size_supported(int n) {
  switch (n) {
#define X(NN) case NN: return true;
    COLA_FFT_SIZES(X)
#undef X
    default: return false;
  }
}

void fft_r2c_z(float2* mesh, int n, int nbatch, long mesh_stride, const TwiddleSet& tw, hipStream_t s,
               int nmock, long mstride) {
  switch (n) {
#define X(NN) case NN: r2c_n<NN>(mesh, nbatch, mesh_stride, tw.get(NN), s, nmock, mstride); break;
    COLA_FFT_SIZES(X)
#undef X
    default: break;
  }
}

void fft_c2r_z(float2* mesh, int n, int nbatch, long mesh_stride, const TwiddleSet& tw, hipStream_t s,
               int nmock, long mstride) {
  switch (n) {
#define X(NN) case NN: c2r_n<NN>(mesh, nbatch, mesh_stride, tw.get(NN), s, nmock, mstride); break;
    COLA_FFT_SIZES(X)
#undef X
    default: break;
  }
}

void fft_y(float2* mesh, int n, int nbatch, long mesh_stride, int inverse, const TwiddleSet& tw,
           hipStream_t s, int nmock, long mstride) {
  float2* outs[3] = {mesh, nullptr, nullptr};
  const int mode = inverse ? X_INV : X_FWD;
  switch (n) {
#define X(NN) case NN: cols_n<NN>(mode, 1, mesh, outs, nbatch, mesh_stride, tw.get(NN), 0, 0, 0, 1.f, nullptr, s, nullptr, nmock, mstride); break;
    COLA_FFT_SIZES(X)
#undef X
    default: break;
  }
}

void fft_y_grad_yz(float2* b, float2* gz, int n, const TwiddleSet& tw, hipStream_t s, int nmock,
                   long mstride) {
  float2* outs[3] = {b, gz, nullptr};
  switch (n) {
#define X(NN) case NN: cols_n<NN>(X_INV_GRAD_YZ, 1, b, outs, 1, 0, tw.get(NN), 0, 0, 0, 1.f, nullptr, s, nullptr, nmock, mstride); break;
    COLA_FFT_SIZES(X)
#undef X
    default: break;
  }
}

void fft_x(const XPassArgs& a, int n, const TwiddleSet& tw, hipStream_t s) {
  float2* outs[3] = {a.out[0], a.out[1], a.out[2]};
  switch (n) {
#define X(NN) case NN: cols_n<NN>(a.mode, 0, a.in, outs, 1, 0, tw.get(NN), a.mult, a.comp_a, a.comp_b, a.scale, a.amp, s, a.coef, a.nmock, a.mstride); break;
    COLA_FFT_SIZES(X)
#undef X
    default: break;
  }
}

namespace {
template <int N>
void combine_n(const float2* const in[3], float2* out, const CombineSpec& cs, const float* amp,
               const float2* tw, hipStream_t s) {
  constexpr int W = cols_w(N);
  const ColGeom g = geom(N, W, 0);
  dim3 grid((unsigned)(g.nchunk * g.nplanes), 1);
  hipLaunchKernelGGL(k_combine<N>, grid, dim3(cols_threads(N, X_FWD_GREEN)), 0, s, in[0], in[1], in[2], out,
                     g, tw, cs, amp);
}
}  // namespace

void fft_combine_x(const float2* const in[3], float2* out, int n, const CombineSpec& cs,
                   const float* amp, const TwiddleSet& tw, hipStream_t s) {
  switch (n) {
#define X(NN) case NN: combine_n<NN>(in, out, cs, amp, tw.get(NN), s); break;
    COLA_FFT_SIZES(X)
#undef X
    default: break;
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
