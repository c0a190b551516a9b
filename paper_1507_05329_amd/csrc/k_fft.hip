// 3D real-to-complex FFT for the PM solver (Koda et al. 2015, Sec. 2.3: FFTs
// dominate the run time), written as a mixed-radix Stockham autosort FFT.
// A 3D transform is three passes over HBM:
//   z (contiguous rows): real-to-complex by a half-length complex FFT plus
//     the split step, in place in rows of padded_cols(n) complex values;
//   y and x (strided): a workgroup takes W adjacent columns x n elements
//     (W-wide contiguous runs) and transforms them.
// Inside a pass the first stage's inputs come straight from HBM into
// registers and the last stage's outputs go straight back; only the stage
// boundaries in between are exchanged through LDS.  The x pass also hosts
// the k-space multipliers: the PM Green's function times i k (two outputs
// from one forward transform), the 2LPT multipliers of the initial
// conditions and the adjoint's combinations.
//
// Stockham stage with radix R on a line of length L after Ns = product of
// earlier radices: butterfly j (0 <= j < L/R) reads x[j + r L/R], applies
// twiddles W_{Ns R}^{r (j mod Ns)}, does a length-R DFT and writes
// y[(j - j mod Ns) R + j mod Ns + r Ns].  Every stage reads all of its
// inputs into registers before any thread writes, so one LDS buffer is
// enough.  Twiddles come from a per-length table exp(-2 pi i k / n).
#include <atomic>

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

// Launch shapes: at most 80 KB of LDS per workgroup; 256 threads below 4096
// staged complex values, 512 from 4096 (measured on the 768 mesh: the row
// and column passes run 8-18% faster on 512 threads than on 256).
constexpr int kLdsLimit = 80 * 1024;
constexpr int threads_for(int elems) { return elems >= 4096 ? 512 : 256; }

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

// threadIdx.x through an empty asm: the compiler cannot prove two such
// values equal, so address arithmetic derived from them is not shared.
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Twiddle table into LDS, every load of a thread issued before its first
// LDS store.
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

// Padded complex row length (compile-time copy of padded_cols).
constexpr int pcols(int n) { return ((n / 2 + 1) + 15) / 16 * 16; }

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

// ---------------------------------------------------------------------------
// Register-staged transforms.  The first stage of a transform takes its
// inputs from registers (filled straight from HBM), the last one leaves its
// outputs in registers (written straight to HBM), and only the stage
// boundaries in between go through LDS.
//
// Orders: ORD 0 takes the radices as radix_at lists them, ORD 1 in reverse.
// After a transform in one order the last stage of radix R leaves each thread
// with elements j + r n/R; the first stage of the other order has the same
// radix and reads exactly these, so a spectral multiplier between a forward
// and an inverse transform is applied in registers.
constexpr int rad_o(int n, int ord, int s) { return ord ? radix_at(n, nstage(n) - 1 - s) : radix_at(n, s); }
constexpr int ns_o(int n, int ord, int s) {
  int p = 1;
  for (int i = 0; i < s; ++i) p *= rad_o(n, ord, i);
  return p;
}
// LDS layout between stages s and s+1: the line is cut into the R_{s+1}
// segments of n / R_{s+1} elements that one butterfly of stage s+1 reads
// together, each followed by PAD unused slots.  Reads of stage s+1 and
// writes of stage s (whose R outputs lie in one segment) are then a
// per-thread base plus compile-time offsets.  PAD = (NS_s - segment) mod 16
// puts the output blocks of neighbouring stage-s butterflies on different
// LDS banks (segments shorter than 16 are left unpadded).
constexpr int seg_o(int n, int ord, int s) { return n / rad_o(n, ord, s + 1); }
constexpr int pad_o(int n, int ord, int s) {
  return seg_o(n, ord, s) < 16 ? 0 : ((ns_o(n, ord, s) - seg_o(n, ord, s)) % 16 + 16) % 16;
}
// Longest line any layout of either order needs.
constexpr int fspan(int n) {
  int m = n;
  for (int o = 0; o < 2; ++o)
    for (int s = 0; s + 1 < nstage(n); ++s) {
      const int sp = rad_o(n, o, s + 1) * (seg_o(n, o, s) + pad_o(n, o, s));
      if (sp > m) m = sp;
    }
  return m;
}
// Line pitch of the z passes (and the size model of the column passes):
// 2 mod 16 float2.
constexpr int fld(int n) { return (fspan(n) + 13) / 16 * 16 + 2; }
// Column passes: W lines of length n.  Twiddle entries kept in LDS: the
// whole period where it fits, else the first half.  lim: LDS bytes per
// workgroup (kLdsLimit: two workgroups per compute unit).
constexpr int fcols_w(int n, int lim = kLdsLimit) {
  int w = 16;
  while (w > 1 && w * fld(n) * 8 + n * 4 > lim) w /= 2;
  return w;
}
constexpr int ftw_len(int n, int lim = kLdsLimit) { return fcols_w(n, lim) * fld(n) * 8 + n * 8 <= lim ? n : n / 2; }
constexpr int fcols_threads(int n, int lim = kLdsLimit) {
  return lim > kLdsLimit ? 1024 : threads_for(fcols_w(n, lim) * n);
}
// Line pitch of the column passes.  The 16 lanes that share an LDS cycle of
// a 64-bit access cover W lines x 16/W rows (lane -> line t mod W, row t / W);
// a pitch of 16/W mod 16 float2 puts them on 16 distinct bank pairs (a
// model of every stage's reads and writes: 1.0x the conflict-free cycles at
// W = 16 against 2.0x with pitch 2; 1.75x against 2.25x at length 2048).
// Only the LDS addresses change, not the arithmetic.
constexpr int fcols_ld(int n, int lim = kLdsLimit) {
  return (fspan(n) + 15) / 16 * 16 + (fcols_w(n, lim) >= 2 ? 16 / fcols_w(n, lim) : 2);
}
// The Green's function x pass at length 2048 runs one workgroup of 1024
// threads per compute unit on 8 columns (156 KB of LDS) instead of two of
// 512 threads on 4 columns: its three transforms per column leave the
// memory idle for long stretches, and wider runs per row cut its HBM
// transactions (measured at 1024^3/2048^3: 38.9 against 43.9 ms; the
// one-transform passes are faster on 4 columns).
constexpr int kWideLds = 156 * 1024;
constexpr int cols_lim(int n, int mode) { return (mode == X_FWD_GREEN && n == 2048) ? kWideLds : kLdsLimit; }
static_assert(fcols_w(2048) * fcols_ld(2048) * 8 + ftw_len(2048) * 8 <= kLdsLimit, "column-pass LDS");
static_assert(fcols_w(512) * fcols_ld(512) * 8 + ftw_len(512) * 8 <= kLdsLimit, "column-pass LDS");
static_assert(fcols_w(1024) * fcols_ld(1024) * 8 + ftw_len(1024) * 8 <= kLdsLimit, "column-pass LDS");
static_assert(fcols_w(2048, kWideLds) == 8 && fcols_threads(2048, kWideLds) == 1024 &&
                  8 * fcols_ld(2048, kWideLds) * 8 + ftw_len(2048, kWideLds) * 8 <= kWideLds,
              "wide Green pass LDS");

// Waves per SIMD the register budget must allow: two 1024-thread workgroups per CU.
constexpr int min_waves(int t) { return t >= 1024 ? 8 : 4; }
// The order whose first stage has the smaller radix, i.e. the more
// butterflies to spread a pass's HBM loads over.
constexpr int lo_first(int n) { return rad_o(n, 0, 0) <= rad_o(n, 1, 0) ? 0 : 1; }
// z passes: NL rows of n reals, i.e. of h = n/2 complex values; the twiddle
// table has period n (the transform of length h takes every second entry).
constexpr int frows_nl(int n) {
  int nl = 16;
  while (nl > 1 && nl * fld(n / 2) * 8 + n * 4 > kLdsLimit) nl /= 2;
  return nl;
}
constexpr int frows_tw_len(int n) { return frows_nl(n) * fld(n / 2) * 8 + n * 8 <= kLdsLimit ? n : n / 2; }
// 1024 threads where that leaves 6 values per thread (the register budget of
// two such workgroups per CU; measured on the 768 mesh: r2c 0.72 against
// 0.75 ms, c2r 2.25 against 2.28 ms on 512 threads).
constexpr int frows_threads(int n) {
  return frows_nl(n) * (n / 2) == 6144 ? 1024 : threads_for(frows_nl(n) * (n / 2));
}

// exp(-2 pi i m / NT) from an LDS table of TL = NT or NT / 2 entries.
template <int NT, int TL>
__device__ __forceinline__ float2 tw_at(const float2* __restrict__ twl, int m) {
  if constexpr (TL == NT) return twl[m];
  else return tw_get<NT>(twl, m);
}
// a * conj(w)
__device__ __forceinline__ float2 cmulc(float2 a, float2 w) {
  return make_float2(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y);
}

// Stage S of order ORD on W lines of length N with T threads.  Column passes
// (ROWS = false): butterfly t = tid + b T is line c = t mod W, index
// j = t / W, so the lanes of a wave cover W adjacent columns and their HBM
// accesses are W-wide runs.  z passes (ROWS = true): line l = t / NBL,
// j = t mod NBL, lanes run along a row; the twiddle table has period 2N.
template <int N, int ORD, int S, int W, int T, bool ROWS>
struct Stg {
  static constexpr int LEN = N, NST = nstage(N), TWS = ROWS ? 2 : 1;
  static constexpr int R = rad_o(N, ORD, S), NS = ns_o(N, ORD, S), NBL = N / R;
  static constexpr int NB = W * NBL, KB = (NB + T - 1) / T;
  static constexpr int STEP = N / (NS * R) * TWS;
  // element j + r NBL of the layout before this stage sits at j + r RSTR
  static constexpr int RSTR = S > 0 ? NBL + pad_o(N, ORD, S - 1) : NBL;
  // outputs go to the layout after this stage: blocks of QB butterfly
  // groups per segment, WPAD slots after each segment
  static constexpr int WPAD = S + 1 < NST ? pad_o(N, ORD, S) : 0;
  static constexpr int QB = S + 1 < NST ? seg_o(N, ORD, S) / (NS * R) : 1;
  __device__ static bool ok(int t) { return NB % T == 0 || t < NB; }
  __device__ static void map(int t, int& line, int& j) {
    if constexpr (ROWS) {
      line = t / NBL;
      j = t - line * NBL;
    } else {
      line = t % W;
      j = t / W;
    }
  }
};

// Twiddles of the stage (none at NS = 1), then the length-R DFT.
template <class St, int FWD, int TL>
__device__ __forceinline__ void st_bfly(float2* v, const float2* __restrict__ twl, int j) {
  if constexpr (St::NS > 1) {
    const int m1 = (j % St::NS) * St::STEP;
#pragma unroll
    for (int r = 1; r < St::R; ++r) {
      const float2 w = tw_at<St::LEN * St::TWS, TL>(twl, r * m1);
      v[r] = FWD ? cmul(v[r], w) : cmulc(v[r], w);
    }
  }
  Dft<St::R>::run(v, FWD ? -1.f : 1.f);
}

template <class St, int T, int LD, int FWD, int TL>
__device__ __forceinline__ void lds_gather_bfly(float2 (&v)[St::KB][St::R], const float2* __restrict__ lds,
                                                const float2* __restrict__ twl, int tid) {
#pragma unroll
  for (int b = 0; b < St::KB; ++b) {
    const int t = tid + b * T;
    if (St::ok(t)) {
      int c, j;
      St::map(t, c, j);
      const float2* p = lds + c * LD + j;
#pragma unroll
      for (int r = 0; r < St::R; ++r) v[b][r] = p[r * St::RSTR];
      st_bfly<St, FWD, TL>(v[b], twl, j);
    }
  }
}

template <class St, int T, int LD>
__device__ __forceinline__ void lds_scatter(const float2 (&v)[St::KB][St::R], float2* lds, int tid) {
#pragma unroll
  for (int b = 0; b < St::KB; ++b) {
    const int t = tid + b * T;
    if (St::ok(t)) {
      int c, j;
      St::map(t, c, j);
      const int q = j / St::NS, k = j - q * St::NS;
      float2* p = lds + c * LD + q * (St::NS * St::R) + k + St::WPAD * (q / St::QB);
#pragma unroll
      for (int r = 0; r < St::R; ++r) p[r * St::NS] = v[b][r];
    }
  }
}

// Stages S .. NST-2, LDS to LDS.
template <int N, int ORD, int S, int W, int T, bool ROWS, int LD, int FWD, int TL>
__device__ __forceinline__ void mid_stages(float2* lds, const float2* __restrict__ twl, int tid) {
  if constexpr (S + 1 < nstage(N)) {
    using St = Stg<N, ORD, S, W, T, ROWS>;
    float2 v[St::KB][St::R];
    lds_gather_bfly<St, T, LD, FWD, TL>(v, lds, twl, tid);
    __syncthreads();
    lds_scatter<St, T, LD>(v, lds, tid);
    __syncthreads();
    mid_stages<N, ORD, S + 1, W, T, ROWS, LD, FWD, TL>(lds, twl, tid);
  }
}

// One transform of order ORD from the first stage's inputs in registers (v0,
// overwritten) to the last stage's outputs in registers (vl): value r of
// slot b is element j + r N/R of line c (Stg::map).  The caller has the
// twiddle table in LDS and no thread still reading LDS.
template <int N, int ORD, int W, int T, bool ROWS, int LD, int FWD, int TL, class A0, class AL>
__device__ __forceinline__ void reg_fft(A0& v0, AL& vl, float2* lds, const float2* __restrict__ twl, int tid) {
  using S0 = Stg<N, ORD, 0, W, T, ROWS>;
  using SL = Stg<N, ORD, nstage(N) - 1, W, T, ROWS>;
  static_assert(sizeof(A0) == sizeof(float2) * S0::KB * S0::R, "first-stage registers");
  static_assert(sizeof(AL) == sizeof(float2) * SL::KB * SL::R, "last-stage registers");
#pragma unroll
  for (int b = 0; b < S0::KB; ++b) Dft<S0::R>::run(v0[b], FWD ? -1.f : 1.f);
  if constexpr (nstage(N) == 1) {
#pragma unroll
    for (int b = 0; b < S0::KB; ++b)
#pragma unroll
      for (int r = 0; r < S0::R; ++r) vl[b][r] = v0[b][r];
  } else {
    lds_scatter<S0, T, LD>(v0, lds, tid);
    __syncthreads();
    mid_stages<N, ORD, 1, W, T, ROWS, LD, FWD, TL>(lds, twl, tid);
    lds_gather_bfly<SL, T, LD, FWD, TL>(vl, lds, twl, tid);
  }
}

// Element index (returned) and line of value r of slot b in stage St.
template <class St, int T>
__device__ __forceinline__ int st_elem(int tid, int b, int r, int& c) {
  int j;
  St::map(tid + b * T, c, j);
  return j + r * St::NBL;
}

template <class St, int W, int T>
__device__ __forceinline__ void col_load_global(float2 (&v)[St::KB][St::R], const float2* __restrict__ src,
                                                long es, int tid) {
#pragma unroll
  for (int b = 0; b < St::KB; ++b) {
    const int t = tid + b * T;
    int c, j;
    St::map(t, c, j);
    const float2* p = src + (long)j * es + c;
#pragma unroll
    for (int r = 0; r < St::R; ++r)
      v[b][r] = St::ok(t) ? p[(long)r * St::NBL * es] : make_float2(0.f, 0.f);
  }
}

// Last stage: element j + r NS (NS = N / R).
template <class St, int W, int T>
__device__ __forceinline__ void col_store_global(const float2 (&v)[St::KB][St::R], float2* dst, long es,
                                                 int tid) {
#pragma unroll
  for (int b = 0; b < St::KB; ++b) {
    const int t = tid + b * T;
    if (St::ok(t)) {
      int c, j;
      St::map(t, c, j);
      float2* p = dst + (long)j * es + c;
#pragma unroll
      for (int r = 0; r < St::R; ++r) p[(long)r * St::NS * es] = v[b][r];
    }
  }
}

// Radix order of the plain column transforms (measured on the 768 mesh:
// the y passes take 0.78 ms in order 1 (16, 16, 3) against 0.84 in order 0).
constexpr int kPlainOrd = 1;

template <int N, int MODE>
__global__ __launch_bounds__(fcols_threads(N, cols_lim(N, MODE)), 4) void k_cols(
    const float2* __restrict__ in, float2* out0, float2* out1, float2* out2, long mesh_stride,
    ColGeom g, const float2* __restrict__ tw, int mult, int ca, int cb, float scale,
    const float* __restrict__ amp, int y_is_plane_freq, const StepCoef* __restrict__ coef,
    long mstride, int xcd_order) {
  in = mock_ptr(in, mstride);
  out0 = mock_ptr(out0, mstride);
  if constexpr (MODE == X_FWD_GREEN || MODE == X_INV_GRAD_YZ) out1 = mock_ptr(out1, mstride);
  if constexpr (MODE == X_FWD_GREEN) {
    if (coef) scale = mock_ptr(coef, mstride)->gscale;
  }
  constexpr int LIM = cols_lim(N, MODE);
  constexpr int W = fcols_w(N, LIM), LD = fcols_ld(N, LIM), T = fcols_threads(N, LIM), TL = ftw_len(N, LIM);
  constexpr int NST = nstage(N);
  __shared__ float2 lds[W * LD];
  __shared__ float2 twl[TL];
  const uint32_t nblk = (uint32_t)g.nchunk * g.nplanes;
  const uint32_t bid = xcd_order ? xcd_remap(blockIdx.x, nblk) : blockIdx.x;
  const int p = bid / g.nchunk;
  const int c0 = (bid - p * g.nchunk) * W;
  const long es = g.elem_stride;
  const long ofs = (long)blockIdx.y * mesh_stride + (long)p * g.plane_stride + c0;
  const int tid = threadIdx.x;
  const int pfreq = y_is_plane_freq ? signed_freq(p, N) : 0;
  // plain transforms in order kPlainOrd; the others start in the order
  // with the smaller first radix (the Green pass returns in the other one),
  // except at 2048: the gradient y pass (that order spills registers there)
  // and the Green pass (the larger first radix: 38.6 against 39.4 ms)
  constexpr int O0 = (MODE == X_FWD || MODE == X_INV)       ? kPlainOrd
                     : (MODE == X_INV_GRAD_YZ && N >= 2048) ? 0
                     : (MODE == X_FWD_GREEN && N == 2048)   ? 1 - lo_first(N)
                                                            : lo_first(N);
  using S0 = Stg<N, O0, 0, W, T, false>;
  using SL = Stg<N, O0, NST - 1, W, T, false>;
  float2 v[S0::KB][S0::R];
  col_load_global<S0, W, T>(v, in + ofs, es, tid);
  load_twiddles<TL, T>(twl, tw);

  if constexpr (MODE == X_FWD || MODE == X_INV || MODE == X_FWD_AMP || MODE == X_MULT_INV) {
    if constexpr (MODE == X_MULT_INV) {
#pragma unroll
      for (int b = 0; b < S0::KB; ++b)
#pragma unroll
        for (int r = 0; r < S0::R; ++r) {
          int c;
          const int e = st_elem<S0, T>(tid, b, r, c);
          v[b][r] = cmul(v[b][r], multiplier(mult, 0, ca, cb, scale, signed_freq(e, N), pfreq, c0 + c, N,
                                             amp, 0));
        }
    }
    float2 o[SL::KB][SL::R];
    reg_fft<N, O0, W, T, false, LD, (MODE == X_FWD || MODE == X_FWD_AMP) ? 1 : 0, TL>(v, o, lds, twl, tid);
    if constexpr (MODE == X_FWD_AMP) {
#pragma unroll
      for (int b = 0; b < SL::KB; ++b)
#pragma unroll
        for (int r = 0; r < SL::R; ++r) {
          int c;
          const int e = st_elem<SL, T>(tid, b, r, c);
          o[b][r] = cmul(o[b][r], multiplier(0, 0, 0, 0, 0.f, signed_freq(e, N), pfreq, c0 + c, N, amp, 1));
        }
    }
    col_store_global<SL, W, T>(o, out0 + ofs, es, tid);
  } else if constexpr (MODE == X_FWD_GREEN) {
    // PM, x pass: forward along x gives S = DFT[delta]; with phi = scale S / |n|^2
    //   out0 = IDFT_x[i n_x phi]  (n_x on its Nyquist index -> 0)  -> g_x,
    //   out1 = IDFT_x[phi]                                         -> g_y, g_z
    // (n_y and n_z are constant along an x line; the y pass applies them).
    using SI = Stg<N, 1 - O0, NST - 1, W, T, false>;
    float2 f[SL::KB][SL::R];
    reg_fft<N, O0, W, T, false, LD, 1, TL>(v, f, lds, twl, tid);
    float2 u[SL::KB][SL::R];
#pragma unroll
    for (int b = 0; b < SL::KB; ++b)
#pragma unroll
      for (int r = 0; r < SL::R; ++r) {
        int c;
        const int e = st_elem<SL, T>(tid, b, r, c);
        const int nx = signed_freq(e, N), nz = c0 + c;
        const int n2 = nx * nx + pfreq * pfreq + nz * nz;
        // hardware reciprocal (within 1 ulp): one instruction instead of a division
        const float inv = (n2 == 0 || nz > N / 2) ? 0.f : scale * __builtin_amdgcn_rcpf((float)n2);
        f[b][r] = make_float2(inv * f[b][r].x, inv * f[b][r].y);
        const float kx = (nx == N / 2 || nx == -N / 2) ? 0.f : (float)nx;
        u[b][r] = make_float2(-kx * f[b][r].y, kx * f[b][r].x);  // i n_x phi
      }
    float2 o[SI::KB][SI::R];
    __syncthreads();
    reg_fft<N, 1 - O0, W, T, false, LD, 0, TL>(u, o, lds, twl, tid);
    col_store_global<SI, W, T>(o, out0 + ofs, es, tid);
    __syncthreads();
    reg_fft<N, 1 - O0, W, T, false, LD, 0, TL>(f, o, lds, twl, tid);
    col_store_global<SI, W, T>(o, out1 + ofs, es, tid);
  } else if constexpr (MODE == X_INV_GRAD_YZ) {
    // PM, inverse y pass of B = IDFT_x[phi]: out0 = IDFT_y[i n_y B], out1 =
    // IDFT_y[i n_z B] (each component zeroed on its own Nyquist index).
    float2 u[S0::KB][S0::R];
#pragma unroll
    for (int b = 0; b < S0::KB; ++b)
#pragma unroll
      for (int r = 0; r < S0::R; ++r) {
        int c;
        const int ny = signed_freq(st_elem<S0, T>(tid, b, r, c), N);
        const float ky = (ny == N / 2 || ny == -N / 2) ? 0.f : (float)ny;
        u[b][r] = make_float2(-ky * v[b][r].y, ky * v[b][r].x);  // i n_y B
      }
    float2 o[SL::KB][SL::R];
    reg_fft<N, O0, W, T, false, LD, 0, TL>(u, o, lds, twl, tid);
    col_store_global<SL, W, T>(o, out0 + ofs, es, tid);
#pragma unroll
    for (int b = 0; b < S0::KB; ++b)
#pragma unroll
      for (int r = 0; r < S0::R; ++r) {
        int c;
        st_elem<S0, T>(tid, b, r, c);
        const float kz = (c0 + c >= N / 2) ? 0.f : (float)(c0 + c);
        u[b][r] = make_float2(-kz * v[b][r].y, kz * v[b][r].x);  // i n_z B
      }
    __syncthreads();
    reg_fft<N, O0, W, T, false, LD, 0, TL>(u, o, lds, twl, tid);
    col_store_global<SL, W, T>(o, out1 + ofs, es, tid);
  }
}

// ---------------------------------------------------------------------------
// z passes: NL rows of N reals per workgroup (row stride `cols` complex),
// through a length-H = N/2 complex transform of the pairs (x_2m, x_2m+1).

// Forward: Z = DFT_H[x_2m + i x_2m+1], then the split step
//   X_k = E_k + W_N^k O_k,  E = (Z_k + conj Z_{H-k})/2,  O = -i (Z_k - conj Z_{H-k})/2
// for k = 0 .. H (columns beyond H are written as zeros).
// The forward z pass at 2048 runs 2 rows per workgroup on 256 threads
// (14.3 against 15.6 ms for 8 rows on 512 threads); at 768 the most rows
// that fit stay faster (0.78 against 0.80 ms for 4 rows).
constexpr int frows_nl_r2c(int n) { return n == 2048 ? 2 : frows_nl(n); }
constexpr int frows_threads_r2c(int n) {
  return n == 2048 ? threads_for(frows_nl_r2c(n) * (n / 2)) : frows_threads(n);
}

template <int N>
__global__ __launch_bounds__(frows_threads_r2c(N), min_waves(frows_threads_r2c(N))) void k_r2c_z(
    float2* __restrict__ mesh, long nrows, int cols, long mesh_stride, const float2* __restrict__ tw,
    long mstride) {
  constexpr int H = N / 2, LD = fld(H), NL = frows_nl_r2c(N), T = frows_threads_r2c(N), TL = frows_tw_len(N);
  constexpr int OR = lo_first(H);
  using S0 = Stg<H, OR, 0, NL, T, true>;
  using SL = Stg<H, OR, nstage(H) - 1, NL, T, true>;
  mesh = mock_ptr(mesh, mstride);
  __shared__ float2 lds[NL * LD];
  __shared__ float2 twl[TL];
  float2* base = mesh + blockIdx.y * mesh_stride;
  const long r0 = (long)blockIdx.x * NL;
  const int tid = threadIdx.x;
  float2 v[S0::KB][S0::R];
#pragma unroll
  for (int b = 0; b < S0::KB; ++b) {
    const int t = tid + b * T;
    int l, j;
    S0::map(t, l, j);
    const bool in = S0::ok(t) && r0 + l < nrows;
    const float2* p = base + (r0 + l) * cols + j;
#pragma unroll
    for (int r = 0; r < S0::R; ++r) v[b][r] = in ? p[r * S0::NBL] : make_float2(0.f, 0.f);
  }
  load_twiddles<TL, T>(twl, tw);
  float2 z[SL::KB][SL::R];
  reg_fft<H, OR, NL, T, true, LD, 1, TL>(v, z, lds, twl, tid);
  __syncthreads();
  // Z in natural order: element e of row l at lds[l * LD + e]
#pragma unroll
  for (int b = 0; b < SL::KB; ++b) {
    const int t = tid + b * T;
    if (SL::ok(t)) {
      int l, j;
      SL::map(t, l, j);
#pragma unroll
      for (int r = 0; r < SL::R; ++r) lds[l * LD + j + r * SL::NS] = z[b][r];
    }
  }
  __syncthreads();
  constexpr int COLS = pcols(N), NO = NL * COLS, KO = (NO + T - 1) / T;
  float2 xs[KO];
#pragma unroll
  for (int q = 0; q < KO; ++q) {
    const int i = tid + q * T;
    const int l = i / COLS, k = i - l * COLS;
    xs[q] = make_float2(0.f, 0.f);
    if ((NO % T == 0 || i < NO) && k <= H) {
      const float2 a = lds[l * LD + (k == H ? 0 : k)];
      float2 c = lds[l * LD + (k == 0 ? 0 : H - k)];
      c.y = -c.y;
      const float2 e = make_float2(0.5f * (a.x + c.x), 0.5f * (a.y + c.y));
      const float2 o = make_float2(0.5f * (a.y - c.y), -0.5f * (a.x - c.x));
      xs[q] = cadd(e, cmul(tw_at<N, TL>(twl, k), o));
    }
  }
#pragma unroll
  for (int q = 0; q < KO; ++q) {
    const int i = tid + q * T;
    const int l = i / COLS, k = i - l * COLS;
    if ((NO % T == 0 || i < NO) && r0 + l < nrows) base[(r0 + l) * cols + k] = xs[q];
  }
}

// Inverse: half spectrum (H+1 values) -> N reals, unnormalised.  The first
// stage's inputs are formed in registers from X_k and X_{H-k}:
//   Z'_k = (X_k + conj X_{H-k}) + i (X_k - conj X_{H-k}) exp(+2 pi i k / N),
// and z = IDFT_H[Z'] holds the pairs (x_2m, x_2m+1).
template <int N>
__global__ __launch_bounds__(frows_threads(N), min_waves(frows_threads(N))) void k_c2r_z(
    float2* __restrict__ mesh, long nrows, int cols, long mesh_stride, const float2* __restrict__ tw,
    long mstride) {
  constexpr int H = N / 2, LD = fld(H), NL = frows_nl(N), T = frows_threads(N), TL = frows_tw_len(N);
  constexpr int OR = lo_first(H);
  using S0 = Stg<H, OR, 0, NL, T, true>;
  using SL = Stg<H, OR, nstage(H) - 1, NL, T, true>;
  mesh = mock_ptr(mesh, mstride);
  __shared__ float2 lds[NL * LD];
  __shared__ float2 twl[TL];
  float2* base = mesh + blockIdx.y * mesh_stride;
  const long r0 = (long)blockIdx.x * NL;
  const int tid = threadIdx.x;
  float2 xa[S0::KB][S0::R], xb[S0::KB][S0::R];
#pragma unroll
  for (int b = 0; b < S0::KB; ++b) {
    const int t = tid + b * T;
    int l, j;
    S0::map(t, l, j);
    const bool in = S0::ok(t) && r0 + l < nrows;
    const float2* p = base + (r0 + l) * cols;
#pragma unroll
    for (int r = 0; r < S0::R; ++r) {
      const int k = j + r * S0::NBL;
      xa[b][r] = in ? p[k] : make_float2(0.f, 0.f);
      xb[b][r] = in ? p[H - k] : make_float2(0.f, 0.f);
    }
  }
  load_twiddles<TL, T>(twl, tw);
  __syncthreads();
#pragma unroll
  for (int b = 0; b < S0::KB; ++b) {
    int l, j;
    S0::map(tid + b * T, l, j);
#pragma unroll
    for (int r = 0; r < S0::R; ++r) {
      const int k = j + r * S0::NBL;
      const float2 cb = make_float2(xb[b][r].x, -xb[b][r].y);
      const float2 e = cadd(xa[b][r], cb);
      const float2 o = cmulc(csub(xa[b][r], cb), tw_at<N, TL>(twl, k));
      xa[b][r] = cadd(e, make_float2(-o.y, o.x));
    }
  }
  float2 z[SL::KB][SL::R];
  reg_fft<H, OR, NL, T, true, LD, 0, TL>(xa, z, lds, twl, tid);
#pragma unroll
  for (int b = 0; b < SL::KB; ++b) {
    const int t = tid + b * T;
    int l, j;
    SL::map(t, l, j);
    if (SL::ok(t) && r0 + l < nrows) {
      float2* p = base + (r0 + l) * cols + j;
#pragma unroll
      for (int r = 0; r < SL::R; ++r) p[r * SL::NS] = z[b][r];
    }
  }
}

// Inverse z pass of the three force meshes in the row-interleaved layout
// (row r of mesh c is line 3 r + c, lines `cols` complex apart): NL3 lines
// (NL3 / 3 rows, all three meshes) per workgroup, the same transform as
// k_c2r_z, and the real outputs written back interleaved by node, row r
// holding (g_x, g_y, g_z) of its N nodes in its first 3 N floats.  A row's
// output lies inside its own three input lines, and a workgroup reads all
// of its lines before it writes, so the pass runs in place.
// Lines per workgroup: whole row triples, at most about 3072 complex values
// (one triple at 2048, two at 768 and 1024), on 256 threads.  Smaller
// workgroups, several per compute unit, beat the most lines that fit the
// LDS: at 2048 41.6 against 45.1 ms (6 lines) and 52.1 ms (6 lines on 1024
// threads); at 768 2.24 against 2.29 (3 lines), 2.34 (15 lines, 1024
// threads) and 2.74 ms (9 lines).
constexpr int frows_nl3(int n) {
  const int fit = frows_nl(n) / 3 * 3, want = 3 * (3072 / (3 * (n / 2)));
  return fit < want ? fit : (want < 3 ? 3 : want);
}
constexpr int frows_threads3(int n) { return threads_for(frows_nl3(n) * (n / 2)); }
static_assert(frows_nl3(2048) == 3 && frows_nl3(768) == 6 && frows_nl3(1024) == 6 && frows_nl3(1536) == 3 &&
                  frows_nl3(512) == 12 && frows_nl3(256) == frows_nl(256) / 3 * 3,
              "c2r lines per workgroup");

template <int N>
__global__ __launch_bounds__(frows_threads3(N), min_waves(frows_threads3(N))) void k_c2r_z3(
    float2* __restrict__ mesh, long nrows, int cols, const float2* __restrict__ tw, long mstride) {
  constexpr int H = N / 2, LD = fld(H), NL = frows_nl3(N), T = frows_threads3(N), TL = frows_tw_len(N);
  static_assert(NL >= 3, "three lines per workgroup at least");
  constexpr int OR = lo_first(H);
  using S0 = Stg<H, OR, 0, NL, T, true>;
  using SL = Stg<H, OR, nstage(H) - 1, NL, T, true>;
  mesh = mock_ptr(mesh, mstride);
  __shared__ float2 lds[NL * LD];
  __shared__ float2 twl[TL];
  const long l0 = (long)blockIdx.x * NL;          // first line; a multiple of 3
  const long nlines = 3 * nrows;
  const int tid = threadIdx.x;
  float2 xa[S0::KB][S0::R], xb[S0::KB][S0::R];
#pragma unroll
  for (int b = 0; b < S0::KB; ++b) {
    const int t = tid + b * T;
    int l, j;
    S0::map(t, l, j);
    const bool in = S0::ok(t) && l0 + l < nlines;
    const float2* p = mesh + (l0 + l) * cols;
#pragma unroll
    for (int r = 0; r < S0::R; ++r) {
      const int k = j + r * S0::NBL;
      xa[b][r] = in ? p[k] : make_float2(0.f, 0.f);
      xb[b][r] = in ? p[H - k] : make_float2(0.f, 0.f);
    }
  }
  load_twiddles<TL, T>(twl, tw);
  __syncthreads();
#pragma unroll
  for (int b = 0; b < S0::KB; ++b) {
    int l, j;
    S0::map(tid + b * T, l, j);
#pragma unroll
    for (int r = 0; r < S0::R; ++r) {
      const int k = j + r * S0::NBL;
      const float2 cb = make_float2(xb[b][r].x, -xb[b][r].y);
      const float2 e = cadd(xa[b][r], cb);
      const float2 o = cmulc(csub(xa[b][r], cb), tw_at<N, TL>(twl, k));
      xa[b][r] = cadd(e, make_float2(-o.y, o.x));
    }
  }
  float2 z[SL::KB][SL::R];
  reg_fft<H, OR, NL, T, true, LD, 0, TL>(xa, z, lds, twl, tid);
  // pairs (x_2m, x_2m+1) of line l in natural order at lds[l * LD + m]
  __syncthreads();
#pragma unroll
  for (int b = 0; b < SL::KB; ++b) {
    const int t = tid + b * T;
    if (SL::ok(t)) {
      int l, j;
      SL::map(t, l, j);
#pragma unroll
      for (int r = 0; r < SL::R; ++r) lds[l * LD + j + r * SL::NS] = z[b][r];
    }
  }
  __syncthreads();
  // row q of this workgroup: 3 N floats, four per thread per round
  const float* lf = reinterpret_cast<const float*>(lds);
  constexpr int NQ = NL / 3, PER = 3 * N / 4;
  for (int i = tid; i < NQ * PER; i += T) {
    const int q = i / PER, o4 = (i - q * PER) * 4;
    const long row = l0 / 3 + q;
    if (row >= nrows) continue;
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int o = o4 + u, node = o / 3, c = o - node * 3;
      v[u] = lf[2 * ((3 * q + c) * LD) + node];
    }
    float* dst = reinterpret_cast<float*>(mesh + row * 3 * (long)cols) + o4;
    *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
  }
}

// x pass of a spectral combination: out = IDFT_x[ sum_q m_q(k) DFT_x(in_q) ]
// for inputs already transformed along z and y (so m_q sees the full k).
// m_q is the gradient (i n_d scale / |n|^2) or Hessian (n_a n_b scale / |n|^2)
// multiplier, optionally times the amplitude table; accumulate adds the result
// to out instead of overwriting it.  Used by the adjoint (transposed Green's
// function and transposed 2LPT maps).  Each input's forward transform ends
// in registers, where the multiplied spectra are summed; the inverse
// transform starts from that sum (mirrored radix orders).
template <int N>
__global__ __launch_bounds__(fcols_threads(N), 4) void k_combine(
    const float2* __restrict__ in0, const float2* __restrict__ in1, const float2* __restrict__ in2,
    float2* out, ColGeom g, const float2* __restrict__ tw, CombineSpec cs,
    const float* __restrict__ amp) {
  constexpr int W = fcols_w(N), LD = fcols_ld(N), T = fcols_threads(N), TL = ftw_len(N);
  constexpr int NST = nstage(N), OF = lo_first(N);
  using S0 = Stg<N, OF, 0, W, T, false>;
  using SL = Stg<N, OF, NST - 1, W, T, false>;
  using SI = Stg<N, 1 - OF, NST - 1, W, T, false>;
  __shared__ float2 lds[W * LD];
  __shared__ float2 twl[TL];
  const uint32_t nblk = (uint32_t)g.nchunk * g.nplanes;
  const uint32_t bid = xcd_remap(blockIdx.x, nblk);
  const int p = bid / g.nchunk;
  const int c0 = (bid - p * g.nchunk) * W;
  const int pfreq = signed_freq(p, N);
  const long es = g.elem_stride, ofs = (long)p * g.plane_stride + c0;
  const int tid = threadIdx.x;
  const int h = N / 2;
  load_twiddles<TL, T>(twl, tw);
  float2 acc[SL::KB][SL::R];
#pragma unroll
  for (int b = 0; b < SL::KB; ++b)
#pragma unroll
    for (int r = 0; r < SL::R; ++r) acc[b][r] = make_float2(0.f, 0.f);
  const float2* ins[3] = {in0, in1, in2};
#pragma unroll 1
  for (int q = 0; q < cs.nin; ++q) {
    // a thread index the compiler cannot treat as loop-invariant, so the
    // transform's address arithmetic is not hoisted out and kept live
    const int qt = opaque_tid();
    float2 v[S0::KB][S0::R];
    col_load_global<S0, W, T>(v, ins[q] + ofs, es, qt);
    if (q > 0) __syncthreads();  // the previous transform's last LDS reads are done
    float2 f[SL::KB][SL::R];
    reg_fft<N, OF, W, T, false, LD, 1, TL>(v, f, lds, twl, qt);
    const int kind = cs.kind[q], ca = cs.ca[q], cb = cs.cb[q];
#pragma unroll
    for (int b = 0; b < SL::KB; ++b)
#pragma unroll
      for (int r = 0; r < SL::R; ++r) {
        int c;
        const int e = st_elem<SL, T>(qt, b, r, c);
        const int nx = signed_freq(e, N), nz = c0 + c;
        const int na = ca == 0 ? nx : (ca == 1 ? pfreq : nz);
        const bool nyq = nx == h || nx == -h || pfreq == h || pfreq == -h || nz == h;
        // scale / |n|^2 (times the amplitude), recomputed per input rather
        // than held in registers across the inputs (hardware reciprocal)
        const int n2 = nx * nx + pfreq * pfreq + nz * nz;
        const float rw = (n2 != 0 && nz <= h && !(cs.use_amp && nyq))
                             ? cs.scale * __builtin_amdgcn_rcpf((float)n2) * (cs.use_amp ? amp[n2] : 1.f)
                             : 0.f;
        const float2 x = f[b][r];
        if (kind == M_GRAD) {
          // i n_a rw; zero on the axis' own Nyquist plane (Green) or any Nyquist index
          const bool z = cs.green ? (na == h || na == -h) : nyq;
          const float m = z ? 0.f : (float)na * rw;
          acc[b][r] = cadd(acc[b][r], make_float2(-m * x.y, m * x.x));
        } else {
          const int nb = cb == 0 ? nx : (cb == 1 ? pfreq : nz);
          const float m = nyq ? 0.f : (float)na * (float)nb * rw;
          acc[b][r] = cadd(acc[b][r], make_float2(m * x.x, m * x.y));
        }
      }
  }
  __syncthreads();
  float2 o[SI::KB][SI::R];
  reg_fft<N, 1 - OF, W, T, false, LD, 0, TL>(acc, o, lds, twl, tid);
  float2* dst = out + ofs;
#pragma unroll
  for (int b = 0; b < SI::KB; ++b) {
    const int t = tid + b * T;
    if (SI::ok(t)) {
      int c, j;
      SI::map(t, c, j);
      float2* pd = dst + (long)j * es + c;
#pragma unroll
      for (int r = 0; r < SI::R; ++r) {
        float2* e = pd + (long)r * SI::NS * es;
        *e = cs.accumulate ? cadd(*e, o[b][r]) : o[b][r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Schedule table: the block order of the column passes, per transform
// length and pass kind (plain, Green's function x pass, gradient y pass),
// process-wide: 1 hands each XCD a contiguous range of column blocks
// (xcd_remap: neighbouring blocks share the XCD's L2), 0 keeps the
// hardware's round-robin.  The kernels and their arithmetic are the same;
// only the workgroup that transforms a column changes.  Set by the
// autotuner or by the caller.
namespace {
constexpr int kSchedLens[] = {16, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048};
constexpr int kNSched = sizeof(kSchedLens) / sizeof(kSchedLens[0]);
std::atomic<int> g_order[kNSched][3] = {};   // 0: default (1), else value + 1
int sched_slot(int n) {
  for (int i = 0; i < kNSched; ++i)
    if (kSchedLens[i] == n) return i;
  return -1;
}
int pass_kind(int mode) { return mode == X_FWD_GREEN ? 1 : mode == X_INV_GRAD_YZ ? 2 : 0; }
}  // namespace

int fft_block_order(int n, int kind) {
  const int i = sched_slot(n);
  const int v = (i < 0 || kind < 0 || kind > 2) ? 0 : g_order[i][kind].load(std::memory_order_relaxed);
  return v == 0 ? 1 : v - 1;
}

int set_fft_block_order(int n, int kind, int order) {
  const int i = sched_slot(n);
  if (i < 0 || kind < 0 || kind > 2 || (order != 0 && order != 1)) return -1;
  g_order[i][kind].store(order + 1, std::memory_order_relaxed);
  return 0;
}

namespace {

// rowc: complex values from one row (x, y) to the next, padded_cols(n) for a
// plain mesh, 3 padded_cols(n) in the row-interleaved force layout.
ColGeom geom(int n, int w, int axis, long rowc = 0) {
  ColGeom g;
  const long cols = padded_cols(n);
  if (rowc <= 0) rowc = cols;
  g.cols = (int)cols;
  g.nchunk = (int)(cols / w);
  g.nplanes = n;
  if (axis == 1) {  // y: planes are x
    g.elem_stride = rowc;
    g.plane_stride = (long)n * rowc;
  } else {          // x: planes are y
    g.elem_stride = (long)n * rowc;
    g.plane_stride = rowc;
  }
  return g;
}

template <int N>
void r2c_n(float2* mesh, int nbatch, long mesh_stride, const float2* tw, hipStream_t s, int nmock,
           long mstride, long rowc) {
  constexpr int NL = frows_nl_r2c(N), T = frows_threads_r2c(N);
  const long nrows = (long)N * N;
  dim3 grid((unsigned)((nrows + NL - 1) / NL), (unsigned)nbatch, (unsigned)nmock);
  hipLaunchKernelGGL(k_r2c_z<N>, grid, dim3(T), 0, s, mesh, nrows, (int)(rowc > 0 ? rowc : padded_cols(N)),
                     mesh_stride, tw, mstride);
}

template <int N>
void c2r3_n(float2* mesh, const float2* tw, hipStream_t s, int nmock, long mstride) {
  constexpr int NL = frows_nl3(N), T = frows_threads3(N);
  const long nrows = (long)N * N;
  dim3 grid((unsigned)((3 * nrows + NL - 1) / NL), 1, (unsigned)nmock);
  hipLaunchKernelGGL(k_c2r_z3<N>, grid, dim3(T), 0, s, mesh, nrows, (int)padded_cols(N), tw, mstride);
}

template <int N>
void c2r_n(float2* mesh, int nbatch, long mesh_stride, const float2* tw, hipStream_t s, int nmock,
           long mstride) {
  constexpr int NL = frows_nl(N), T = frows_threads(N);
  const long nrows = (long)N * N;
  dim3 grid((unsigned)((nrows + NL - 1) / NL), (unsigned)nbatch, (unsigned)nmock);
  hipLaunchKernelGGL(k_c2r_z<N>, grid, dim3(T), 0, s, mesh, nrows, (int)padded_cols(N), mesh_stride, tw,
                     mstride);
}

template <int N>
void cols_n(int mode, int axis, const float2* in, float2* const out[3], int nbatch, long mesh_stride,
            const float2* tw, int mult, int ca, int cb, float scale, const float* amp, hipStream_t s,
            const StepCoef* coef = nullptr, int nmock = 1, long mstride = 0, long rowc = 0) {
  constexpr int LG = cols_lim(N, X_FWD_GREEN);
  const int W = mode == X_FWD_GREEN ? fcols_w(N, LG) : fcols_w(N);
  const int T = mode == X_FWD_GREEN ? fcols_threads(N, LG) : fcols_threads(N);
  ColGeom g = geom(N, W, axis, rowc);
  // The Green pass takes only the column blocks that hold a frequency
  // 0 .. N/2 (the rest of a padded row is never read; the passes after it
  // transform whatever is there, column by column).  Measured on the 768
  // mesh: 1.71 against 1.77 ms; the same trim slows the other column passes
  // and the c2r pass that follows (rows no longer written in whole lines).
  if (mode == X_FWD_GREEN) g.nchunk = (N / 2 + 1 + W - 1) / W;
  dim3 grid((unsigned)(g.nchunk * g.nplanes), (unsigned)nbatch, (unsigned)nmock);
  const int yf = axis == 0 ? 1 : 0;
  const int xo = fft_block_order(N, pass_kind(mode));
  switch (mode) {
    case X_FWD:
      hipLaunchKernelGGL((k_cols<N, X_FWD>), grid, dim3(T), 0, s, in, out[0], nullptr, nullptr,
                         mesh_stride, g, tw, 0, 0, 0, 1.f, nullptr, yf, nullptr, mstride, xo);
      break;
    case X_INV:
      hipLaunchKernelGGL((k_cols<N, X_INV>), grid, dim3(T), 0, s, in, out[0], nullptr, nullptr,
                         mesh_stride, g, tw, 0, 0, 0, 1.f, nullptr, yf, nullptr, mstride, xo);
      break;
    case X_FWD_AMP:
      hipLaunchKernelGGL((k_cols<N, X_FWD_AMP>), grid, dim3(T), 0, s, in, out[0], nullptr, nullptr,
                         mesh_stride, g, tw, 0, 0, 0, 1.f, amp, yf, nullptr, mstride, xo);
      break;
    case X_MULT_INV:
      hipLaunchKernelGGL((k_cols<N, X_MULT_INV>), grid, dim3(T), 0, s, in, out[0], nullptr, nullptr,
                         mesh_stride, g, tw, mult, ca, cb, scale, nullptr, yf, nullptr, mstride, xo);
      break;
    case X_FWD_GREEN:
      hipLaunchKernelGGL((k_cols<N, X_FWD_GREEN>), grid, dim3(T), 0, s, in, out[0], out[1], nullptr,
                         mesh_stride, g, tw, M_GRAD, 0, 0, scale, nullptr, yf, coef, mstride, xo);
      break;
    case X_INV_GRAD_YZ:
      hipLaunchKernelGGL((k_cols<N, X_INV_GRAD_YZ>), grid, dim3(T), 0, s, in, out[0], out[1], nullptr,
                         mesh_stride, g, tw, 0, 0, 0, 1.f, nullptr, yf, nullptr, mstride, xo);
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
               int nmock, long mstride, long rowc) {
  switch (n) {
#define X(NN) case NN: r2c_n<NN>(mesh, nbatch, mesh_stride, tw.get(NN), s, nmock, mstride, rowc); break;
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

void fft_c2r_z_forces(float2* mesh, int n, const TwiddleSet& tw, hipStream_t s, int nmock, long mstride) {
  switch (n) {
#define X(NN) case NN: c2r3_n<NN>(mesh, tw.get(NN), s, nmock, mstride); break;
    COLA_FFT_SIZES(X)
#undef X
    default: break;
  }
}

void fft_y(float2* mesh, int n, int nbatch, long mesh_stride, int inverse, const TwiddleSet& tw,
           hipStream_t s, int nmock, long mstride, long rowc) {
  float2* outs[3] = {mesh, nullptr, nullptr};
  const int mode = inverse ? X_INV : X_FWD;
  switch (n) {
#define X(NN) case NN: cols_n<NN>(mode, 1, mesh, outs, nbatch, mesh_stride, tw.get(NN), 0, 0, 0, 1.f, nullptr, s, nullptr, nmock, mstride, rowc); break;
    COLA_FFT_SIZES(X)
#undef X
    default: break;
  }
}

void fft_y_grad_yz(float2* b, float2* gz, int n, const TwiddleSet& tw, hipStream_t s, int nmock,
                   long mstride, long rowc) {
  float2* outs[3] = {b, gz, nullptr};
  switch (n) {
#define X(NN) case NN: cols_n<NN>(X_INV_GRAD_YZ, 1, b, outs, 1, 0, tw.get(NN), 0, 0, 0, 1.f, nullptr, s, nullptr, nmock, mstride, rowc); break;
    COLA_FFT_SIZES(X)
#undef X
    default: break;
  }
}

void fft_x(const XPassArgs& a, int n, const TwiddleSet& tw, hipStream_t s) {
  float2* outs[3] = {a.out[0], a.out[1], a.out[2]};
  switch (n) {
#define X(NN) case NN: cols_n<NN>(a.mode, 0, a.in, outs, 1, 0, tw.get(NN), a.mult, a.comp_a, a.comp_b, a.scale, a.amp, s, a.coef, a.nmock, a.mstride, a.rowc); break;
    COLA_FFT_SIZES(X)
#undef X
    default: break;
  }
}

namespace {
template <int N>
void combine_n(const float2* const in[3], float2* out, const CombineSpec& cs, const float* amp,
               const float2* tw, hipStream_t s) {
  constexpr int W = fcols_w(N);
  const ColGeom g = geom(N, W, 0);
  dim3 grid((unsigned)(g.nchunk * g.nplanes), 1);
  hipLaunchKernelGGL(k_combine<N>, grid, dim3(fcols_threads(N)), 0, s, in[0], in[1], in[2], out,
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
