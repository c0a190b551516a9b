// libcola C ABI: context, workspace layout, and the step orchestration.
//
// The PM step (Koda et al. 2015, Sec. 2.2-2.3) on one GPU:
//   tile sort -> deterministic CIC deposit -> r2c FFT (z, y) ->
//   x pass: forward FFT, Green's function, inverse FFTs of i k_x phi and phi ->
//   y pass: inverse of the first, inverses of i k_y and i k_z times the second ->
//   z inverse passes on the 3 force meshes -> CIC readout fused with the
//   COLA kick and drift (eqs. cola-kick, cola-drift; 2LPT terms of Sec. 2.1).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <algorithm>
#include <vector>

#include "cola_internal.h"

using namespace cola;

namespace {

constexpr int kMaxBins = 4096;
constexpr int kPkChunks = 64;
const double kPi = 3.14159265358979323846;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool smooth23(int n) {
  if (n < 2) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

int fail(cola_ctx* c, int code, const char* msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(cola_ctx* c, hipError_t e, const char* where) {
  if (c) {
    c->err = std::string(where) + ": " + hipGetErrorString(e);
  }
  return COLA_EHIP;
}

#define HIP_TRY(ctx, expr)                                   \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr);   \
  } while (0)

#define LAUNCH_CHECK(ctx, where)                             \
  do {                                                       \
    hipError_t e_ = hipGetLastError();                       \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, where);   \
  } while (0)

struct Layout {
  size_t disp, vres, psi1, psi2, pkey, prank, perm, counts, offsets, scan, mesh, tw, amp,
      pk_partial, pk_out, pk_edges, flag, fbar, pk_cbar, coef, total;
  long nbucket, mesh_stride, mesh_region, amp_len;
  int tw_cap;
};

int validate(const cola_params* p) {
  if (!p) return COLA_EINVAL;
  if (p->np < 2 || p->nmesh < 32 || !(p->box > 0) || !(p->omega_m > 0) || p->omega_m > 1.0 ||
      !(p->a_init > 0) || !std::isfinite(p->n_lpt))
    return COLA_EINVAL;
  if (!fft_size_supported(p->np)) return COLA_EUNSUPPORTED;
  if (p->nmesh % 8 != 0 || !fft_size_supported(p->nmesh) || p->nmesh < p->np) return COLA_EUNSUPPORTED;
  // particle ids fill 30 bits of the deposit's sort keys: at most 2^30 particles
  if ((long)p->np * p->np * p->np > (1L << 30)) return COLA_EUNSUPPORTED;
  return COLA_OK;
}

Layout layout(const cola_params* p) {
  Layout L{};
  const long np3 = (long)p->np * p->np * p->np;
  const long nt = p->nmesh / 16;           // 16^3-cell tiles of the deposit
  L.nbucket = 8 * nt * nt * nt;
  L.mesh_stride = mesh_complex_count(p->nmesh);
  const long pm = 3 * L.mesh_stride, ic = 6 * mesh_complex_count(p->np);  // IC adjoint: 6 meshes
  L.mesh_region = pm > ic ? pm : ic;
  L.amp_len = 3L * (p->np / 2) * (p->np / 2) + 1;
  L.tw_cap = p->nmesh > p->np ? p->nmesh : p->np;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
  L.disp = take(3 * np3 * sizeof(float));
  L.vres = take(3 * np3 * sizeof(float));
  L.psi1 = take(3 * np3 * sizeof(float));
  L.psi2 = take(3 * np3 * sizeof(float));
  L.pkey = take(np3 * sizeof(uint32_t));
  L.prank = take(np3 * sizeof(uint32_t));
  L.perm = take(np3 * sizeof(uint32_t));
  L.counts = take((L.nbucket + 1) * sizeof(uint32_t));
  L.offsets = take((L.nbucket + 1) * sizeof(uint32_t));
  L.scan = take(((L.nbucket + 1) / 4096 + 2) * sizeof(uint32_t));
  L.mesh = take(L.mesh_region * sizeof(float2));
  L.tw = take(4 * (size_t)L.tw_cap * sizeof(float2));
  L.amp = take(L.amp_len * sizeof(float));
  L.pk_partial = take((size_t)kMaxBins * kPkChunks * 3 * sizeof(double));
  L.pk_out = take((size_t)kMaxBins * 3 * sizeof(double));
  L.pk_edges = take((size_t)(kMaxBins + 1) * sizeof(double));
  L.flag = take(sizeof(uint32_t) * 64);
  L.fbar = take(3 * np3 * sizeof(float));
  L.pk_cbar = take((size_t)kMaxBins * sizeof(double));
  L.coef = take(sizeof(StepCoef));
  L.total = o;
  return L;
}

// Uploads exp(-2 pi i k / n) for k < n into a free twiddle slot.
int ensure_twiddles(cola_ctx* c, int n) {
  if (c->tw.get(n)) return COLA_OK;
  for (int i = 0; i < 4; ++i) {
    if (c->tw.n[i] == 0) {
      if (n > c->tw_cap) return fail(c, COLA_EINVAL, "transform length exceeds the twiddle capacity");
      std::vector<float2> h(n);
      for (int k = 0; k < n; ++k) {
        const double a = -2.0 * kPi * (double)k / (double)n;
        h[k] = make_float2((float)std::cos(a), (float)std::sin(a));
      }
      float2* dst = c->twbuf + (size_t)i * c->tw_cap;
      HIP_TRY(c, hipMemcpyAsync(dst, h.data(), n * sizeof(float2), hipMemcpyHostToDevice, c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      c->tw.n[i] = n;
      c->tw.tw[i] = dst;
      return COLA_OK;
    }
  }
  // all slots taken: recycle the last slot (never the PM or particle grids, slots 0 and 1)
  c->tw.n[3] = 0;
  return ensure_twiddles(c, n);
}

// Stage timer: records an event pair around a stage when COLA_F_STAGE_TIMERS is set.
struct StageTimer {
  cola_ctx* c;
  hipEvent_t stop = nullptr;
  StageTimer(cola_ctx* ctx, int stage) : c(ctx) {
    if (!(c->p.flags & COLA_F_STAGE_TIMERS)) { c = nullptr; return; }
    if (c->ev_used + 2 > c->ev_pool.size()) {
      if (c->ev_pool.size() >= 1 << 16) { c = nullptr; return; }  // bounded: stop recording
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { c = nullptr; return; }
        c->ev_pool.push_back(e);
      }
    }
    hipEvent_t start = c->ev_pool[c->ev_used];
    stop = c->ev_pool[c->ev_used + 1];
    c->ev_used += 2;
    c->ev_stage.push_back(stage);
    hipEventRecord(start, c->stream);
  }
  ~StageTimer() {
    if (c) hipEventRecord(stop, c->stream);
  }
};

float2* ic_buf(cola_ctx* c, int i) { return c->meshbase + (size_t)i * mesh_complex_count(c->p.np); }

// Tile sort of the current positions on an ng^3 grid.  Batched form: nmock
// contexts with identical layouts, mock b's workspace at byte offset b * mstride.
void tile_sort(cola_ctx* c, int ng, const float* disp, int nmock = 1, long mstride = 0) {
  StageTimer t(c, COLA_STAGE_SORT);
  const float dscale = (float)((double)ng / (double)c->p.nmesh);
  const long nt = ng / 16;
  const long nb = 8 * nt * nt * nt;
  launch_fill_u32(c->counts, nb + 1, 0u, c->stream, nmock, mstride);
  launch_bin_count(disp, c->p.np, ng, dscale, c->counts, c->pkey, c->prank, c->stream, nmock, mstride);
  launch_exclusive_scan(c->counts, c->offsets, nb, c->scan_scratch, c->stream, nmock, mstride);
  launch_scatter_walk(c->pkey, c->prank, c->offsets, c->p.np, c->perm, c->stream, nmock, mstride);
}

void deposit(cola_ctx* c, int ng, float* out, long row_stride, int contrast, const float* disp,
             int nmock = 1, long mstride = 0) {
  const float dscale = (float)((double)ng / (double)c->p.nmesh);
  tile_sort(c, ng, disp, nmock, mstride);
  StageTimer t(c, COLA_STAGE_DEPOSIT);
  launch_deposit(disp, c->perm, c->offsets, c->p.np, ng, dscale, out, row_stride, contrast,
                 c->stream, nmock, mstride);
}

// Green's function scale: g_d = IDFT[i n_d gscale / |n|^2 DFT(delta)] in mesh
// units, gscale = alpha nm / (2 pi nm^3).
double green_scale(int nm, double alpha) { return alpha * nm / (2.0 * kPi) / ((double)nm * nm * nm); }

// Deposit + FFT + Green x ik + inverse FFTs: the three force meshes in
// c->mesh[0..2].  The x pass writes IDFT_x[i k_x phi] and IDFT_x[phi]; the
// y pass turns the second into the y and z components (k_y and k_z are
// constant along x, so phi needs only two inverse x transforms).  The Green
// scale is read from the device coefficients c->coef (set by set_coef).
// The PM force pipeline keeps its three meshes row-interleaved: row (x, y)
// of mesh c starts at complex value (3 (x nm + y) + c) padded_cols, so the
// last (c2r) pass can write the force field interleaved by node in place:
// (g_x, g_y, g_z) of node (x, y, z) at floats (x nm + y) 6 padded_cols + 3 z.
long pm_rowc(int nm) { return 3 * padded_cols(nm); }        // complex values per row
long force_row_stride(int nm) { return 6 * padded_cols(nm); }  // floats per row of the force field
const float* force_field(cola_ctx* c) { return reinterpret_cast<const float*>(c->mesh[0]); }

// The spectral part alone: delta on entry in the rows of mesh 0 (row stride
// pm_rowc), the force field interleaved by node on exit.
void fft_forces(cola_ctx* c, int nmock = 1, long mstride = 0) {
  const int nm = c->p.nmesh;
  const long P = padded_cols(nm), rowc = pm_rowc(nm);
  float2* m0 = c->mesh[0];
  {
    StageTimer t(c, COLA_STAGE_FFT_Z);
    fft_r2c_z(m0, nm, 1, 0, c->tw, c->stream, nmock, mstride, rowc);
  }
  {
    StageTimer t(c, COLA_STAGE_FFT_Y);
    fft_y(m0, nm, 1, 0, 0, c->tw, c->stream, nmock, mstride, rowc);
  }
  XPassArgs a;
  a.in = m0;
  a.out[0] = m0;
  a.out[1] = m0 + P;
  a.mode = X_FWD_GREEN;
  a.coef = c->coef;
  a.nmock = nmock;
  a.mstride = mstride;
  a.rowc = rowc;
  {
    StageTimer t(c, COLA_STAGE_FFT_X);
    fft_x(a, nm, c->tw, c->stream);
  }
  {
    StageTimer t(c, COLA_STAGE_IFFT_Y);
    fft_y(m0, nm, 1, 0, 1, c->tw, c->stream, nmock, mstride, rowc);
  }
  {
    StageTimer t(c, COLA_STAGE_IFFT_Y_GRAD);
    fft_y_grad_yz(m0 + P, m0 + 2 * P, nm, c->tw, c->stream, nmock, mstride, rowc);
  }
  {
    StageTimer t(c, COLA_STAGE_IFFT_Z);
    fft_c2r_z_forces(m0, nm, c->tw, c->stream, nmock, mstride);
  }
}

void force_meshes(cola_ctx* c, const float* disp, int nmock = 1, long mstride = 0) {
  const int nm = c->p.nmesh;
  deposit(c, nm, reinterpret_cast<float*>(c->mesh[0]), 2 * pm_rowc(nm), 1, disp, nmock, mstride);
  fft_forces(c, nmock, mstride);
}

// The whole PM step on the device (no host decisions, no host reads): the
// sequence a batch captures into one graph.  Uses the coefficients in c->coef.
void step_launches(cola_ctx* c, int nmock, long mstride) {
  force_meshes(c, c->disp, nmock, mstride);
  StageTimer t(c, COLA_STAGE_KICKDRIFT);
  launch_readout_kick_drift(force_field(c), force_row_stride(c->p.nmesh), c->disp, c->vres, c->psi1, c->psi2,
                            c->p.np, c->p.nmesh, c->coef, nullptr, c->stream, nmock, mstride);
}

bool same_a(double a, double b) { return std::fabs(a - b) <= 1e-12 * (std::fabs(a) > 1 ? std::fabs(a) : 1.0); }

void step_scalars(const cola_params* p, double a_x, double a_v, double a1, double* o) {
  const double om = p->omega_m, n = p->n_lpt;
  const double ah = 0.5 * (a_x + a1);
  const double d1a = growth_D1(a_x, om), d1b = growth_D1(a1, om);
  const double d2a = D2_of(p, a_x), d2b = D2_of(p, a1);
  o[0] = 1.5 * om / a_x;
  o[1] = d1a;
  o[2] = d2a;
  o[3] = d1b - d1a;
  o[4] = d2b - d2a;
  o[5] = kick_factor(a_v, a_x, ah, om, n);
  o[6] = drift_factor(a_x, a1, ah, om, n);
  o[7] = ah;
  o[8] = d1b;
  o[9] = d2b;
}

// Device coefficients of the step a_x -> a1 (velocity at a_v); s[10] as step_scalars.
StepCoef make_coef(const cola_params* p, double a_x, double a_v, double a1, double* s) {
  step_scalars(p, a_x, a_v, a1, s);
  const double alpha = s[0], D1 = s[1], D2 = s[2], K = s[5], I = s[6];
  StepCoef v{};
  v.kd.K = (float)K;
  v.kd.c1 = (float)(K * alpha * D1);
  v.kd.c2 = (float)(K * alpha * (D2 - D1 * D1));
  v.kd.I = (float)I;
  v.kd.e1 = (float)s[3];
  v.kd.e2 = (float)s[4];
  v.gscale = (float)green_scale(p->nmesh, alpha);
  return v;
}

int check_finite(cola_ctx* c) {
  if (!(c->p.flags & COLA_F_CHECK_FINITE)) return COLA_OK;
  launch_fill_u32(c->flag, 1, 0u, c->stream);
  launch_check_finite(c->disp, 3 * c->np3, c->flag, c->stream);
  launch_check_finite(c->vres, 3 * c->np3, c->flag, c->stream);
  LAUNCH_CHECK(c, "check_finite");
  uint32_t h = 0;
  HIP_TRY(c, hipMemcpyAsync(&h, c->flag, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (h) return fail(c, COLA_ENONFINITE, "non-finite value in the particle state");
  return COLA_OK;
}

int ic_from_mesh_noise(cola_ctx* c, const double* k, const double* pk, int nk) {
  const int np = c->p.np, nm = c->p.nmesh;
  const long rs = 2 * padded_cols(np);
  const double box = c->p.box;
  // amplitude table sqrt(P(|k|) / dq^3) by integer |n|^2
  std::vector<float> amp(c->amp_len);
  const double kf = 2.0 * kPi / box, dq3 = std::pow(box / np, 3);
  for (long n2 = 0; n2 < c->amp_len; ++n2)
    amp[n2] = n2 == 0 ? 0.f : (float)std::sqrt(interp_pk(kf * std::sqrt((double)n2), k, pk, nk) / dq3);
  HIP_TRY(c, hipMemcpyAsync(c->amp, amp.data(), amp.size() * sizeof(float), hipMemcpyHostToDevice,
                            c->stream));
  float2* A = ic_buf(c, 0);
  float2* B[3] = {ic_buf(c, 1), ic_buf(c, 2), ic_buf(c, 3)};
  // delta_L(k) = DFT[w] sqrt(P / dq^3), k = 0 and Nyquist-index modes zeroed
  fft_r2c_z(A, np, 1, 0, c->tw, c->stream);
  fft_y(A, np, 1, 0, 0, c->tw, c->stream);
  XPassArgs xa;
  xa.in = A;
  xa.out[0] = A;
  xa.mode = X_FWD_AMP;
  xa.amp = c->amp;
  fft_x(xa, np, c->tw, c->stream);
  const double inv3 = 1.0 / ((double)np * np * np);
  const float sgrad = (float)(nm / (2.0 * kPi) * inv3);  // mesh units of the PM grid
  auto inverse_into = [&](const float2* in, float2* out, int kind, int ca, int cb, float scale) {
    XPassArgs m;
    m.in = in;
    m.out[0] = out;
    m.mode = X_MULT_INV;
    m.mult = kind;
    m.comp_a = ca;
    m.comp_b = cb;
    m.scale = scale;
    fft_x(m, np, c->tw, c->stream);
    fft_y(out, np, 1, 0, 1, c->tw, c->stream);
    fft_c2r_z(out, np, 1, 0, c->tw, c->stream);
  };
  // Psi1_d = IDFT[i k_d delta_L / k^2]
  for (int d = 0; d < 3; ++d) {
    inverse_into(A, B[0], M_GRAD, d, 0, sgrad);
    launch_copy_from_mesh(reinterpret_cast<float*>(B[0]), np, rs, c->psi1 + d * c->np3, 1.0f, c->stream);
  }
  // S = phi_xx phi_yy + phi_yy phi_zz + phi_zz phi_xx - phi_xy^2 - phi_yz^2 - phi_zx^2
  for (int d = 0; d < 3; ++d) inverse_into(A, B[d], M_HESS, d, d, (float)inv3);
  float* S = reinterpret_cast<float*>(B[0]);
  launch_source_diag(S, reinterpret_cast<float*>(B[1]), reinterpret_cast<float*>(B[2]), np, rs, c->stream);
  const int off[3][2] = {{0, 1}, {1, 2}, {2, 0}};
  for (int q = 0; q < 3; ++q) {
    inverse_into(A, B[1], M_HESS, off[q][0], off[q][1], (float)inv3);
    launch_source_sub_sq(S, reinterpret_cast<float*>(B[1]), np, rs, c->stream);
  }
  // Psi2_d = IDFT[-i k_d S(k) / k^2]
  fft_r2c_z(B[0], np, 1, 0, c->tw, c->stream);
  fft_y(B[0], np, 1, 0, 0, c->tw, c->stream);
  XPassArgs fx;
  fx.in = B[0];
  fx.out[0] = B[0];
  fx.mode = X_FWD;
  fft_x(fx, np, c->tw, c->stream);
  for (int d = 0; d < 3; ++d) {
    inverse_into(B[0], B[1], M_GRAD, d, 0, -sgrad);
    launch_copy_from_mesh(reinterpret_cast<float*>(B[1]), np, rs, c->psi2 + d * c->np3, 1.0f, c->stream);
  }
  const double a0 = c->p.a_init;
  launch_init_particles(c->disp, c->vres, c->psi1, c->psi2, c->np3,
                        (float)growth_D1(a0, c->p.omega_m), (float)D2_of(&c->p, a0),
                        c->stream);
  LAUNCH_CHECK(c, "init_2lpt");
  HIP_TRY(c, hipStreamSynchronize(c->stream));  // the amplitude table's host copy is released here
  c->a_x = c->a_v = a0;
  c->have_state = true;
  return COLA_OK;
}

int check_table(const double* k, const double* pk, int nk) {
  if (!k || !pk || nk < 2) return COLA_EINVAL;
  for (int i = 0; i < nk; ++i) {
    if (!(k[i] > 0) || !(pk[i] > 0) || !std::isfinite(k[i]) || !std::isfinite(pk[i])) return COLA_EINVAL;
    if (i > 0 && !(k[i] > k[i - 1])) return COLA_EINVAL;
  }
  return COLA_OK;
}

}  // namespace

extern "C" {

void cola_params_default(cola_params* p, int32_t np, int32_t nmesh, double box) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->np = np;
  p->nmesh = nmesh;
  p->box = box;
  p->omega_m = 0.27;
  p->n_lpt = -2.5;
  p->a_init = 0.02;
  p->flags = 0;
}

int cola_workspace_query(const cola_params* p, size_t* bytes) {
  if (!bytes) return COLA_EINVAL;
  const int v = validate(p);
  if (v != COLA_OK) return v;
  *bytes = layout(p).total;
  return COLA_OK;
}

int cola_create(const cola_params* p, void* ws, size_t bytes, void* stream, cola_ctx** out) {
  if (!out) return COLA_EINVAL;
  *out = nullptr;
  const int v = validate(p);
  if (v != COLA_OK) return v;
  if (!ws || ((uintptr_t)ws & 255)) return COLA_EINVAL;
  const Layout L = layout(p);
  if (bytes < L.total) return COLA_ENOMEM;
  cola_ctx* c = new (std::nothrow) cola_ctx();
  if (!c) return COLA_ENOMEM;
  c->p = *p;
  c->stream = (hipStream_t)stream;
  c->ws = (char*)ws;
  c->ws_bytes = bytes;
  c->np3 = (long)p->np * p->np * p->np;
  c->disp = (float*)(c->ws + L.disp);
  c->vres = (float*)(c->ws + L.vres);
  c->psi1 = (float*)(c->ws + L.psi1);
  c->psi2 = (float*)(c->ws + L.psi2);
  c->pkey = (uint32_t*)(c->ws + L.pkey);
  c->prank = (uint32_t*)(c->ws + L.prank);
  c->perm = (uint32_t*)(c->ws + L.perm);
  c->counts = (uint32_t*)(c->ws + L.counts);
  c->offsets = (uint32_t*)(c->ws + L.offsets);
  c->scan_scratch = (uint32_t*)(c->ws + L.scan);
  c->nbucket = L.nbucket;
  c->meshbase = (float2*)(c->ws + L.mesh);
  c->mesh_stride = L.mesh_stride;
  c->mesh_region = L.mesh_region;
  for (int i = 0; i < 3; ++i) c->mesh[i] = c->meshbase + (size_t)i * L.mesh_stride;
  c->twbuf = (float2*)(c->ws + L.tw);
  c->tw_cap = L.tw_cap;
  c->amp = (float*)(c->ws + L.amp);
  c->amp_len = L.amp_len;
  c->pk_partial = (double*)(c->ws + L.pk_partial);
  c->pk_out = (double*)(c->ws + L.pk_out);
  c->pk_edges = (double*)(c->ws + L.pk_edges);
  c->flag = (uint32_t*)(c->ws + L.flag);
  c->fbar = (float*)(c->ws + L.fbar);
  c->pk_cbar = (double*)(c->ws + L.pk_cbar);
  c->coef = (StepCoef*)(c->ws + L.coef);
  int r = ensure_twiddles(c, p->nmesh);
  if (r == COLA_OK) r = ensure_twiddles(c, p->np);
  if (r != COLA_OK) {
    delete c;
    return r;
  }
  // second slot is always the particle grid's; keep slots 0/1 fixed
  *out = c;
  return COLA_OK;
}

int cola_destroy(cola_ctx* c) {
  if (!c) return COLA_EINVAL;
  for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
  delete c;
  return COLA_OK;
}

int cola_init_2lpt_from_noise(cola_ctx* c, const float* noise, const double* k, const double* pk,
                              int32_t nk) {
  if (!c || !noise) return fail(c, COLA_EINVAL, "null argument");
  if (check_table(k, pk, nk) != COLA_OK) return fail(c, COLA_EINVAL, "bad P(k) table");
  const long rs = 2 * padded_cols(c->p.np);
  launch_copy_to_mesh(noise, c->p.np, reinterpret_cast<float*>(ic_buf(c, 0)), rs, c->stream);
  LAUNCH_CHECK(c, "copy noise");
  return ic_from_mesh_noise(c, k, pk, nk);
}

int cola_init_2lpt(cola_ctx* c, uint64_t seed, const double* k, const double* pk, int32_t nk,
                   double box, int32_t np) {
  if (!c) return COLA_EINVAL;
  if (np != c->p.np || !(std::fabs(box - c->p.box) <= 1e-12 * c->p.box))
    return fail(c, COLA_EINVAL, "box/np differ from the context parameters");
  if (check_table(k, pk, nk) != COLA_OK) return fail(c, COLA_EINVAL, "bad P(k) table");
  const long rs = 2 * padded_cols(c->p.np);
  launch_philox_noise(seed, c->p.np, reinterpret_cast<float*>(ic_buf(c, 0)), rs, c->stream);
  LAUNCH_CHECK(c, "philox noise");
  return ic_from_mesh_noise(c, k, pk, nk);
}

int cola_noise(cola_ctx* c, uint64_t seed, float* out) {
  if (!c || !out) return fail(c, COLA_EINVAL, "null argument");
  launch_philox_noise(seed, c->p.np, out, c->p.np, c->stream);
  LAUNCH_CHECK(c, "philox noise");
  return COLA_OK;
}

int cola_step(cola_ctx* c, double a0, double a1) {
  if (!c) return COLA_EINVAL;
  if (!c->have_state) return fail(c, COLA_ESTATE, "no initial conditions");
  if (!same_a(a0, c->a_x)) return fail(c, COLA_ESTATE, "a0 differs from the current position time");
  if (!(a1 > a0) || !std::isfinite(a1)) return fail(c, COLA_EINVAL, "a1 must exceed a0");
  double s[10];
  launch_set_coef(c->coef, make_coef(&c->p, c->a_x, c->a_v, a1, s), 1, 0, c->stream);
  step_launches(c, 1, 0);
  LAUNCH_CHECK(c, "cola_step");
  c->a_v = s[7];
  c->a_x = a1;
  return check_finite(c);
}

int cola_force(cola_ctx* c, float* out) {
  if (!c || !out) return fail(c, COLA_EINVAL, "null argument");
  if (!c->have_state) return fail(c, COLA_ESTATE, "no particle state");
  StepCoef v{};
  v.gscale = (float)green_scale(c->p.nmesh, 1.5 * c->p.omega_m / c->a_x);
  launch_set_coef(c->coef, v, 1, 0, c->stream);
  force_meshes(c, c->disp);
  launch_readout_kick_drift(force_field(c), force_row_stride(c->p.nmesh), c->disp, c->vres, c->psi1, c->psi2,
                            c->p.np, c->p.nmesh, c->coef, out, c->stream);
  LAUNCH_CHECK(c, "cola_force");
  return COLA_OK;
}

int cola_pm_gradient(cola_ctx* c, double a, const float* delta, float* g0, float* g1, float* g2) {
  if (!c || !delta) return fail(c, COLA_EINVAL, "null argument");
  if (!(a > 0) || !std::isfinite(a)) return fail(c, COLA_EINVAL, "a must be positive and finite");
  const int nm = c->p.nmesh;
  StepCoef v{};
  v.gscale = (float)green_scale(nm, 1.5 * c->p.omega_m / a);
  launch_set_coef(c->coef, v, 1, 0, c->stream);
  launch_copy_to_mesh(delta, nm, reinterpret_cast<float*>(c->mesh[0]), 2 * pm_rowc(nm), c->stream);
  fft_forces(c);
  float* g[3] = {g0, g1, g2};
  for (int d = 0; d < 3; ++d)
    if (g[d]) launch_copy_from_mesh(force_field(c) + d, nm, force_row_stride(nm), g[d], 1.0f, c->stream, 3);
  LAUNCH_CHECK(c, "cola_pm_gradient");
  return COLA_OK;
}

namespace {

// Coefficients of the velocity at the position time; runs the force pipeline
// into the force meshes (g) when the kick from a_v to a_x is not zero.
VelCoef velocity_coef_and_forces(cola_ctx* c, const float** g) {
  const double om = c->p.omega_m, n = c->p.n_lpt, a = c->a_x;
  const double adot = a * hubble_E(a, om), alpha = 1.5 * om / a;
  const double D1 = growth_D1(a, om), D2 = D2_of(&c->p, a);
  // the kick from a_v to a_x (zero at the initial state, where a_v = a_x)
  const double K = c->a_v == a ? 0.0 : kick_factor(c->a_v, a, a, om, n);
  VelCoef k{};
  k.K = (float)K;
  k.u1 = (float)(a * a * adot * growth_D1_prime(a, om) - K * alpha * D1);
  k.u2 = (float)(a * a * adot * D2_prime_of(&c->p, a) - K * alpha * (D2 - D1 * D1));
  k.rsd = (float)(1.0 / (a * adot));
  *g = nullptr;
  if (K != 0.0) {
    StepCoef v{};
    v.gscale = (float)green_scale(c->p.nmesh, alpha);
    launch_set_coef(c->coef, v, 1, 0, c->stream);
    force_meshes(c, c->disp);
    *g = force_field(c);
  }
  return k;
}

}  // namespace

int cola_velocity(cola_ctx* c, float* vel, float* sdisp, int32_t axis) {
  if (!c || !vel) return fail(c, COLA_EINVAL, "null argument");
  if (!c->have_state) return fail(c, COLA_ESTATE, "no particle state");
  if (sdisp && (axis < 0 || axis > 2)) return fail(c, COLA_EINVAL, "rsd_axis must be 0, 1 or 2");
  if (sdisp == vel) return fail(c, COLA_EINVAL, "dev_vel and dev_sdisp must differ");
  const float* g;
  const VelCoef k = velocity_coef_and_forces(c, &g);
  {
    StageTimer t(c, COLA_STAGE_VELOCITY);
    launch_velocity(g, force_row_stride(c->p.nmesh), c->disp, c->vres, c->psi1, c->psi2, c->p.np,
                    c->p.nmesh, k, vel, sdisp, axis, c->stream);
  }
  LAUNCH_CHECK(c, "cola_velocity");
  return COLA_OK;
}

int cola_density(cola_ctx* c, float* out) {
  if (!c || !out) return fail(c, COLA_EINVAL, "null argument");
  if (!c->have_state) return fail(c, COLA_ESTATE, "no particle state");
  deposit(c, c->p.nmesh, out, c->p.nmesh, 1, c->disp);
  LAUNCH_CHECK(c, "cola_density");
  return COLA_OK;
}

int cola_snapshot(cola_ctx* c, double a1, double a_s, float* dout, float* vout, float* sdisp, int32_t axis) {
  if (!c || !dout || !vout) return fail(c, COLA_EINVAL, "null argument");
  if (!c->have_state) return fail(c, COLA_ESTATE, "no particle state");
  const double a0 = c->a_x;
  if (!(a1 > a0) || !std::isfinite(a1)) return fail(c, COLA_EINVAL, "a1 must exceed the position time");
  if (!(a_s >= a0 && a_s <= a1)) return fail(c, COLA_EINVAL, "a_s must lie in [a_x, a1]");
  if (sdisp && (axis < 0 || axis > 2)) return fail(c, COLA_EINVAL, "rsd_axis must be 0, 1 or 2");
  if (dout == vout || (sdisp && (sdisp == dout || sdisp == vout)))
    return fail(c, COLA_EINVAL, "output arrays must differ");
  const double om = c->p.omega_m, n = c->p.n_lpt;
  double s[10];
  step_scalars(&c->p, a0, c->a_v, a1, s);
  const double alpha = s[0], D1 = s[1], D2 = s[2], K = s[5], a_h = s[7];
  const double adot_s = a_s * hubble_E(a_s, om), u = a_s * a_s * adot_s;
  SnapCoef k{};
  k.K = (float)K;
  k.c1 = (float)(K * alpha * D1);
  k.c2 = (float)(K * alpha * (D2 - D1 * D1));
  k.I = (float)drift_factor(a0, a_s, a_h, om, n);
  k.e1 = (float)(growth_D1(a_s, om) - D1);
  k.e2 = (float)(D2_of(&c->p, a_s) - D2);
  k.sv = (float)std::pow(a_s / a_h, n);
  k.w1 = (float)(u * growth_D1_prime(a_s, om));
  k.w2 = (float)(u * D2_prime_of(&c->p, a_s));
  k.rsd = (float)(1.0 / (a_s * adot_s));
  StepCoef v{};
  v.gscale = (float)green_scale(c->p.nmesh, alpha);
  launch_set_coef(c->coef, v, 1, 0, c->stream);
  force_meshes(c, c->disp);
  {
    StageTimer t(c, COLA_STAGE_VELOCITY);
    launch_snapshot(force_field(c), force_row_stride(c->p.nmesh), c->disp, c->vres,
                    c->psi1, c->psi2, c->p.np, c->p.nmesh, k, dout, vout, sdisp, axis, c->stream);
  }
  LAUNCH_CHECK(c, "cola_snapshot");
  return COLA_OK;
}

int cola_density_of(cola_ctx* c, const float* disp, float* out) {
  if (!c || !disp || !out) return fail(c, COLA_EINVAL, "null argument");
  deposit(c, c->p.nmesh, out, c->p.nmesh, 1, disp);
  LAUNCH_CHECK(c, "cola_density_of");
  return COLA_OK;
}

namespace {

int pk_of(cola_ctx* c, const float* disp, int32_t ng, const double* edges, int32_t nbins, double* kmean,
          double* pk, int64_t* nmodes) {
  if (nbins < 1 || nbins > kMaxBins) return fail(c, COLA_EINVAL, "nbins out of range");
  if (ng < 32 || ng > c->p.nmesh || !fft_size_supported(ng))
    return fail(c, COLA_EUNSUPPORTED, "ngrid must be a supported size in [32, nmesh]");
  for (int i = 0; i < nbins; ++i)
    if (!(edges[i + 1] > edges[i])) return fail(c, COLA_EINVAL, "edges must increase");
  int r = ensure_twiddles(c, ng);
  if (r != COLA_OK) return r;
  HIP_TRY(c, hipMemcpyAsync(c->pk_edges, edges, (nbins + 1) * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
  float2* m = c->mesh[0];
  deposit(c, ng, reinterpret_cast<float*>(m), 2 * padded_cols(ng), 1, disp);
  fft3d_forward(m, ng, c->tw, c->stream);
  launch_pk_bin(m, ng, c->p.box, c->pk_edges, nbins, c->pk_partial, kPkChunks, c->stream);
  launch_pk_reduce(c->pk_partial, nbins, kPkChunks, c->pk_out, c->stream);
  LAUNCH_CHECK(c, "cola_pk");
  std::vector<double> h(3 * (size_t)nbins);
  HIP_TRY(c, hipMemcpyAsync(h.data(), c->pk_out, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int b = 0; b < nbins; ++b) {
    const double n = h[3 * b + 2];
    nmodes[b] = (int64_t)llround(n);
    kmean[b] = n > 0 ? h[3 * b] / n : NAN;
    pk[b] = n > 0 ? h[3 * b + 1] / n : NAN;
  }
  return COLA_OK;
}

// Jing (2005) correction (Sec. 3.3): raw bin power over the bin average of
// the CIC window's image sum at the local slope of the corrected spectrum,
// iterated from slope 0.  The slope of a bin is the log-log slope between
// its non-empty neighbours (one-sided at the ends, 0 alone), limited to
// [kJingSlopeMin, kJingSlopeMax]; kJingIterations passes.
constexpr int kJingIterations = 8;
constexpr double kJingSlopeMin = -3.0, kJingSlopeMax = 1.0;

void jing_slopes(const std::vector<double>& km, const std::vector<double>& p, const std::vector<double>& cnt,
                 std::vector<double>* s) {
  const int nb = (int)p.size();
  std::vector<int> idx;
  for (int b = 0; b < nb; ++b)
    if (cnt[b] > 0) idx.push_back(b);
  s->assign(nb, 0.0);
  for (size_t j = 0; j < idx.size(); ++j) {
    const int b = idx[j];
    const int lo = j > 0 ? idx[j - 1] : b, hi = j + 1 < idx.size() ? idx[j + 1] : b;
    double v = 0.0;
    if (lo != hi && p[lo] > 0 && p[hi] > 0) v = std::log(p[hi] / p[lo]) / std::log(km[hi] / km[lo]);
    (*s)[b] = std::min(kJingSlopeMax, std::max(kJingSlopeMin, v));
  }
}

int pk_jing_of(cola_ctx* c, const float* disp, int32_t ng, const double* edges, int32_t nbins, double* kmean,
               double* pk, int64_t* nmodes) {
  if (nbins < 1 || nbins > kMaxBins) return fail(c, COLA_EINVAL, "nbins out of range");
  if (ng < 32 || ng > c->p.nmesh || !fft_size_supported(ng))
    return fail(c, COLA_EUNSUPPORTED, "ngrid must be a supported size in [32, nmesh]");
  for (int i = 0; i < nbins; ++i)
    if (!(edges[i + 1] > edges[i])) return fail(c, COLA_EINVAL, "edges must increase");
  int r = ensure_twiddles(c, ng);
  if (r != COLA_OK) return r;
  HIP_TRY(c, hipMemcpyAsync(c->pk_edges, edges, (nbins + 1) * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
  float2* m = c->mesh[0];
  deposit(c, ng, reinterpret_cast<float*>(m), 2 * padded_cols(ng), 1, disp);
  fft3d_forward(m, ng, c->tw, c->stream);
  launch_pk_bin(m, ng, c->p.box, c->pk_edges, nbins, c->pk_partial, kPkChunks, c->stream, 0);
  launch_pk_reduce(c->pk_partial, nbins, kPkChunks, c->pk_out, c->stream);
  LAUNCH_CHECK(c, "cola_pk_jing");
  std::vector<double> h(3 * (size_t)nbins);
  HIP_TRY(c, hipMemcpyAsync(h.data(), c->pk_out, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::vector<double> km(nbins), raw(nbins), cnt(nbins), p(nbins), s(nbins, 0.0), csum(nbins);
  for (int b = 0; b < nbins; ++b) {
    cnt[b] = h[3 * b + 2];
    km[b] = cnt[b] > 0 ? h[3 * b] / cnt[b] : NAN;
    raw[b] = cnt[b] > 0 ? h[3 * b + 1] / cnt[b] : NAN;
  }
  for (int it = 0; it < kJingIterations; ++it) {
    // slopes go to the P(k) cotangent buffer (free outside cola_pk_adjoint)
    HIP_TRY(c, hipMemcpyAsync(c->pk_cbar, s.data(), nbins * sizeof(double), hipMemcpyHostToDevice, c->stream));
    launch_pk_alias(ng, c->p.box, c->pk_edges, nbins, c->pk_cbar, c->pk_partial, kPkChunks, c->pk_out, c->stream);
    LAUNCH_CHECK(c, "cola_pk_jing");
    HIP_TRY(c, hipMemcpyAsync(csum.data(), c->pk_out, nbins * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < nbins; ++b) p[b] = cnt[b] > 0 ? raw[b] / (csum[b] / cnt[b]) : NAN;
    jing_slopes(km, p, cnt, &s);
  }
  for (int b = 0; b < nbins; ++b) {
    nmodes[b] = (int64_t)llround(cnt[b]);
    kmean[b] = km[b];
    pk[b] = p[b];
  }
  return COLA_OK;
}

}  // namespace

int cola_pk_jing(cola_ctx* c, int32_t ng, const double* edges, int32_t nbins, double* kmean, double* pk,
                 int64_t* nmodes) {
  if (!c || !edges || !kmean || !pk || !nmodes) return fail(c, COLA_EINVAL, "null argument");
  if (!c->have_state) return fail(c, COLA_ESTATE, "no particle state");
  return pk_jing_of(c, c->disp, ng, edges, nbins, kmean, pk, nmodes);
}

int cola_pk(cola_ctx* c, int32_t ng, const double* edges, int32_t nbins, double* kmean, double* pk,
            int64_t* nmodes) {
  if (!c || !edges || !kmean || !pk || !nmodes) return fail(c, COLA_EINVAL, "null argument");
  if (!c->have_state) return fail(c, COLA_ESTATE, "no particle state");
  return pk_of(c, c->disp, ng, edges, nbins, kmean, pk, nmodes);
}

int cola_pk_velocity(cola_ctx* c, int32_t axis, const double* edges, int32_t nbins, double* kmean,
                     double* pdd, double* pdu, double* puu, int64_t* nmodes) {
  if (!c || !edges || !kmean || !pdd || !pdu || !puu || !nmodes) return fail(c, COLA_EINVAL, "null argument");
  if (!c->have_state) return fail(c, COLA_ESTATE, "no particle state");
  if (axis < 0 || axis > 2) return fail(c, COLA_EINVAL, "axis must be 0, 1 or 2");
  if (nbins < 1 || nbins > kMaxBins / 2) return fail(c, COLA_EINVAL, "nbins out of range");
  for (int i = 0; i < nbins; ++i)
    if (!(edges[i + 1] > edges[i])) return fail(c, COLA_EINVAL, "edges must increase");
  const int nm = c->p.nmesh;
  int r = ensure_twiddles(c, nm);
  if (r != COLA_OK) return r;
  HIP_TRY(c, hipMemcpyAsync(c->pk_edges, edges, (nbins + 1) * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
  const float* g;
  const VelCoef k = velocity_coef_and_forces(c, &g);
  const double a = c->a_x, adot = a * hubble_E(a, c->p.omega_m);
  const double nbar = (double)c->np3 / ((double)nm * nm * nm);
  const long rs = 2 * padded_cols(nm);
  // weights: 1/nbar (density 1 + delta) and the line-of-sight shift v / (a adot) in
  // Mpc/h over nbar (momentum)
  launch_los_weights(g, force_row_stride(nm), c->disp, c->vres, c->psi1, c->psi2, c->p.np, nm, k, axis,
                     (float)(1.0 / nbar), (float)(c->p.box / nm / (a * adot) / nbar), c->fbar, c->stream);
  tile_sort(c, nm, c->disp);
  launch_deposit3_weighted(c->disp, c->perm, c->offsets, c->p.np, nm, c->fbar,
                           reinterpret_cast<float*>(c->mesh[0]), rs, 2 * c->mesh_stride, c->stream);
  fft3d_forward(c->mesh[0], nm, c->tw, c->stream);
  fft3d_forward(c->mesh[1], nm, c->tw, c->stream);
  launch_pk_cross(c->mesh[0], c->mesh[1], nm, c->p.box, c->pk_edges, nbins, axis, c->pk_partial, kPkChunks,
                  c->pk_out, c->stream);
  LAUNCH_CHECK(c, "cola_pk_velocity");
  std::vector<double> h(5 * (size_t)nbins);
  HIP_TRY(c, hipMemcpyAsync(h.data(), c->pk_out, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int b = 0; b < nbins; ++b) {
    const double n = h[5 * b + 4];
    nmodes[b] = (int64_t)llround(n);
    kmean[b] = n > 0 ? h[5 * b] / n : NAN;
    pdd[b] = n > 0 ? h[5 * b + 1] / n : NAN;
    pdu[b] = n > 0 ? h[5 * b + 2] / n : NAN;
    puu[b] = n > 0 ? h[5 * b + 3] / n : NAN;
  }
  return COLA_OK;
}

namespace {

size_t fof_part(long np3, int i) {  // byte offsets of count, start, scan scratch; i = 3: total
  const size_t n1 = align256((size_t)(np3 + 1) * sizeof(uint32_t));
  const size_t n2 = align256((size_t)((np3 + 1) / 4096 + 2) * sizeof(uint32_t));
  const size_t off[4] = {0, n1, 2 * n1, 2 * n1 + n2};
  return off[i];
}

}  // namespace

int cola_fof_workspace_bytes(const cola_ctx* c, size_t* bytes) {
  if (!c || !bytes) return COLA_EINVAL;
  *bytes = fof_part(c->np3, 3);
  return COLA_OK;
}

int cola_fof(cola_ctx* c, double b_frac, int32_t* labels, void* work, size_t work_bytes) {
  if (!c || !labels || !work) return fail(c, COLA_EINVAL, "null argument");
  if (!c->have_state) return fail(c, COLA_ESTATE, "no particle state");
  if (!(b_frac > 0.0 && b_frac < 0.5)) return fail(c, COLA_EINVAL, "b_frac must lie in (0, 0.5)");
  if (((uintptr_t)work & 255) != 0) return fail(c, COLA_EINVAL, "dev_work must be 256-byte aligned");
  if (work_bytes < fof_part(c->np3, 3)) return fail(c, COLA_ENOMEM, "dev_work smaller than cola_fof_workspace_bytes");
  char* w = static_cast<char*>(work);
  launch_fill_u32(c->flag, 1, 0u, c->stream);
  launch_fof(c->disp, c->p.np, c->p.nmesh, b_frac, reinterpret_cast<uint32_t*>(labels),
             reinterpret_cast<uint32_t*>(w + fof_part(c->np3, 0)), reinterpret_cast<uint32_t*>(w + fof_part(c->np3, 1)),
             reinterpret_cast<uint32_t*>(w + fof_part(c->np3, 2)), c->pkey, c->prank, c->perm, c->flag, c->stream);
  LAUNCH_CHECK(c, "cola_fof");
  uint32_t h = 0;
  HIP_TRY(c, hipMemcpyAsync(&h, c->flag, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (h) return fail(c, COLA_ESTATE, "friends-of-friends: a union exceeded its retry bound");
  return COLA_OK;
}

namespace {

size_t halo_part(long np3, int32_t minm, int i) {  // count, flg, hidx, scan scratch, acc; i = 5: total
  const size_t a = align256((size_t)np3 * sizeof(uint32_t));
  const size_t b = align256((size_t)(np3 + 1) * sizeof(uint32_t));
  const size_t sc = align256((size_t)((np3 + 1) / 4096 + 2) * sizeof(uint32_t));
  const size_t ac = align256((size_t)(np3 / minm + 1) * 6 * sizeof(unsigned long long));
  const size_t off[6] = {0, a, 2 * a, 2 * a + b, 2 * a + b + sc, 2 * a + b + sc + ac};
  return off[i];
}

}  // namespace

int cola_fof_halos_workspace_bytes(const cola_ctx* c, int32_t min_members, size_t* bytes) {
  if (!c || !bytes || min_members < 1) return COLA_EINVAL;
  *bytes = halo_part(c->np3, min_members, 5);
  return COLA_OK;
}

int cola_fof_halos(cola_ctx* c, const int32_t* labels, const float* vel, int32_t min_members, int32_t max_halos,
                   int32_t* n_halos, int32_t* root, int32_t* count, float* pos, float* vout, void* work,
                   size_t work_bytes) {
  if (!c || !labels || !n_halos || !root || !count || !pos || !work) return fail(c, COLA_EINVAL, "null argument");
  if (!c->have_state) return fail(c, COLA_ESTATE, "no particle state");
  if (min_members < 1 || max_halos < 0) return fail(c, COLA_EINVAL, "min_members >= 1, max_halos >= 0");
  if ((vel == nullptr) != (vout == nullptr)) return fail(c, COLA_EINVAL, "dev_vel and dev_halo_vel go together");
  if (((uintptr_t)work & 255) != 0) return fail(c, COLA_EINVAL, "dev_work must be 256-byte aligned");
  if (work_bytes < halo_part(c->np3, min_members, 5))
    return fail(c, COLA_ENOMEM, "dev_work smaller than cola_fof_halos_workspace_bytes");
  char* w = static_cast<char*>(work);
  auto u32 = [&](int i) { return reinterpret_cast<uint32_t*>(w + halo_part(c->np3, min_members, i)); };
  launch_fill_u32(c->flag, 1, 0u, c->stream);
  launch_halo_count(labels, c->np3, min_members, u32(0), u32(1), u32(2), u32(3), c->flag, c->stream);
  LAUNCH_CHECK(c, "cola_fof_halos");
  uint32_t h[2] = {0, 0};
  HIP_TRY(c, hipMemcpyAsync(&h[0], c->flag, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(&h[1], u32(2) + c->np3, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (h[0]) return fail(c, COLA_EINVAL, "a label lies outside [0, np^3)");
  *n_halos = (int32_t)h[1];
  if ((long)h[1] > (long)max_halos) return fail(c, COLA_ENOMEM, "more halos than max_halos (count in n_halos)");
  launch_halo_fill(c->disp, vel, labels, u32(0), u32(1), u32(2), c->p.np, c->p.nmesh, (int)h[1], max_halos,
                   reinterpret_cast<unsigned long long*>(u32(4)), root, count, pos, vout, c->stream);
  LAUNCH_CHECK(c, "cola_fof_halos");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return COLA_OK;
}

int cola_pk_of(cola_ctx* c, const float* disp, int32_t ng, const double* edges, int32_t nbins, double* kmean,
               double* pk, int64_t* nmodes) {
  if (!c || !disp || !edges || !kmean || !pk || !nmodes) return fail(c, COLA_EINVAL, "null argument");
  return pk_of(c, disp, ng, edges, nbins, kmean, pk, nmodes);
}

int cola_get_state(cola_ctx* c, float* d, float* v, float* p1, float* p2, double* ax, double* av) {
  if (!c) return COLA_EINVAL;
  const size_t b = 3 * c->np3 * sizeof(float);
  if (d) HIP_TRY(c, hipMemcpyAsync(d, c->disp, b, hipMemcpyDeviceToDevice, c->stream));
  if (v) HIP_TRY(c, hipMemcpyAsync(v, c->vres, b, hipMemcpyDeviceToDevice, c->stream));
  if (p1) HIP_TRY(c, hipMemcpyAsync(p1, c->psi1, b, hipMemcpyDeviceToDevice, c->stream));
  if (p2) HIP_TRY(c, hipMemcpyAsync(p2, c->psi2, b, hipMemcpyDeviceToDevice, c->stream));
  if (ax) *ax = c->a_x;
  if (av) *av = c->a_v;
  return COLA_OK;
}

int cola_set_state(cola_ctx* c, const float* d, const float* v, const float* p1, const float* p2,
                   double ax, double av) {
  if (!c) return COLA_EINVAL;
  if (!(ax > 0) || !(av > 0)) return fail(c, COLA_EINVAL, "scale factors must be positive");
  if (!c->have_state && (!d || !v || !p1 || !p2))
    return fail(c, COLA_ESTATE, "first set_state must provide every array");
  const size_t b = 3 * c->np3 * sizeof(float);
  if (d) HIP_TRY(c, hipMemcpyAsync(c->disp, d, b, hipMemcpyDeviceToDevice, c->stream));
  if (v) HIP_TRY(c, hipMemcpyAsync(c->vres, v, b, hipMemcpyDeviceToDevice, c->stream));
  if (p1) HIP_TRY(c, hipMemcpyAsync(c->psi1, p1, b, hipMemcpyDeviceToDevice, c->stream));
  if (p2) HIP_TRY(c, hipMemcpyAsync(c->psi2, p2, b, hipMemcpyDeviceToDevice, c->stream));
  c->a_x = ax;
  c->a_v = av;
  c->have_state = true;
  return COLA_OK;
}

int cola_fft3d(cola_ctx* c, int32_t n, float* mesh, int32_t inverse) {
  if (!c || !mesh) return fail(c, COLA_EINVAL, "null argument");
  if (n != c->p.np && n != c->p.nmesh) return fail(c, COLA_EINVAL, "n must be np or nmesh");
  if (inverse) fft3d_inverse(reinterpret_cast<float2*>(mesh), n, c->tw, c->stream);
  else fft3d_forward(reinterpret_cast<float2*>(mesh), n, c->tw, c->stream);
  LAUNCH_CHECK(c, "cola_fft3d");
  return COLA_OK;
}

// ---------------------------------------------------------------------------
// Adjoint.

namespace {
// Adjoint of one step.  kept: the step's force meshes left by
// cola_step_keep (three meshes mesh_stride apart), or null to recompute them.
int step_adjoint(cola_ctx* c, double a0, double a1, double a_v0, const float* disp0, const float2* kept,
                 float* dbar, float* vbar, float* p1bar, float* p2bar) {
  if (!c || !disp0 || !dbar || !vbar || !p1bar || !p2bar) return fail(c, COLA_EINVAL, "null argument");
  if (!c->have_state) return fail(c, COLA_ESTATE, "no 2LPT fields (run an initial condition first)");
  if (!(a0 > 0) || !(a1 > a0) || !(a_v0 > 0) || !std::isfinite(a1))
    return fail(c, COLA_EINVAL, "scale factors must satisfy 0 < a0 < a1, a_v0 > 0");
  double s[10];
  const StepCoef coef = make_coef(&c->p, a0, a_v0, a1, s);
  const KickDrift kd = coef.kd;
  const double alpha = s[0];
  const int np = c->p.np, nm = c->p.nmesh;
  const long rs = 2 * padded_cols(nm);
  launch_set_coef(c->coef, coef, 1, 0, c->stream);
  const float* g;
  if (kept) {
    // the forward step's force field; sort the checkpointed positions for
    // the transposed readout below
    tile_sort(c, nm, disp0);
    g = reinterpret_cast<const float*>(kept);
  } else {
    // forward force field at the checkpointed positions (also sorts them)
    force_meshes(c, disp0);
    g = force_field(c);
  }
  float* gbar = reinterpret_cast<float*>(c->mesh[0]);
  // reverse kick/drift and the readout weight gradient; Fbar -> c->fbar
  // (then the meshes are free for the transposed chain, in the plain layout)
  launch_adj_readout_kick(disp0, g, force_row_stride(nm), np, nm, kd, dbar, vbar, p1bar, p2bar, c->fbar,
                          c->stream);
  // gbar_d = R^T Fbar_d (deterministic weighted deposit over the same sort)
  launch_deposit3_weighted(disp0, c->perm, c->offsets, np, nm, c->fbar, gbar, rs, 2 * c->mesh_stride,
                           c->stream);
  // rhobar = (Nm^3/Np) deltabar,  deltabar = -sum_d G_d gbar_d
  fft_r2c_z(c->mesh[0], nm, 3, c->mesh_stride, c->tw, c->stream);
  fft_y(c->mesh[0], nm, 3, c->mesh_stride, 0, c->tw, c->stream);
  CombineSpec cs;
  cs.nin = 3;
  cs.green = 1;
  const double gscale = green_scale(nm, alpha);
  const double cratio = (double)nm * nm * nm / (double)c->np3;
  cs.scale = (float)(-gscale * cratio);
  const float2* ins[3] = {c->mesh[0], c->mesh[1], c->mesh[2]};
  fft_combine_x(ins, c->mesh[0], nm, cs, nullptr, c->tw, c->stream);
  fft_y(c->mesh[0], nm, 1, 0, 1, c->tw, c->stream);
  fft_c2r_z(c->mesh[0], nm, 1, 0, c->tw, c->stream);
  launch_adj_deposit_grad(disp0, gbar, rs, np, nm, 1.0f, 1.0f, dbar, c->stream);
  LAUNCH_CHECK(c, "cola_step_adjoint");
  return COLA_OK;
}
}  // namespace

int cola_step_adjoint(cola_ctx* c, double a0, double a1, double a_v0, const float* disp0,
                      float* dbar, float* vbar, float* p1bar, float* p2bar) {
  return step_adjoint(c, a0, a1, a_v0, disp0, nullptr, dbar, vbar, p1bar, p2bar);
}

int cola_force_slot_bytes(const cola_ctx* c, size_t* bytes) {
  if (!c || !bytes) return COLA_EINVAL;
  *bytes = 3 * (size_t)c->mesh_stride * sizeof(float2);
  return COLA_OK;
}

int cola_step_keep(cola_ctx* c, double a0, double a1, void* slot) {
  if (!c || !slot) return fail(c, COLA_EINVAL, "null argument");
  if (reinterpret_cast<uintptr_t>(slot) % 256 != 0) return fail(c, COLA_EINVAL, "slot must be 256-byte aligned");
  // the step's force pipeline runs in the slot instead of the context's meshes
  float2* own[3] = {c->mesh[0], c->mesh[1], c->mesh[2]};
  for (int d = 0; d < 3; ++d) c->mesh[d] = static_cast<float2*>(slot) + (size_t)d * c->mesh_stride;
  const int r = cola_step(c, a0, a1);
  for (int d = 0; d < 3; ++d) c->mesh[d] = own[d];
  return r;
}

int cola_step_adjoint_kept(cola_ctx* c, double a0, double a1, double a_v0, const float* disp0,
                           const void* slot, float* dbar, float* vbar, float* p1bar, float* p2bar) {
  if (!slot) return fail(c, COLA_EINVAL, "null argument");
  return step_adjoint(c, a0, a1, a_v0, disp0, static_cast<const float2*>(slot), dbar, vbar, p1bar, p2bar);
}

int cola_density_adjoint(cola_ctx* c, const float* disp, const float* delta_bar, float* dbar) {
  if (!c || !disp || !delta_bar || !dbar) return fail(c, COLA_EINVAL, "null argument");
  const int nm = c->p.nmesh;
  const long rs = 2 * padded_cols(nm);
  float* m = reinterpret_cast<float*>(c->mesh[0]);
  launch_copy_to_mesh(delta_bar, nm, m, rs, c->stream);
  const double cratio = (double)nm * nm * nm / (double)c->np3;
  launch_adj_deposit_grad(disp, m, rs, c->p.np, nm, 1.0f, (float)cratio, dbar, c->stream);
  LAUNCH_CHECK(c, "cola_density_adjoint");
  return COLA_OK;
}

int cola_pk_adjoint(cola_ctx* c, const float* disp, int32_t ng, const double* edges, int32_t nbins,
                    const double* cbar, float* dbar) {
  if (!c || !disp || !edges || !cbar || !dbar) return fail(c, COLA_EINVAL, "null argument");
  if (nbins < 1 || nbins > kMaxBins) return fail(c, COLA_EINVAL, "nbins out of range");
  if (ng < 32 || ng > c->p.nmesh || !fft_size_supported(ng))
    return fail(c, COLA_EUNSUPPORTED, "ngrid must be a supported size in [32, nmesh]");
  for (int i = 0; i < nbins; ++i)
    if (!(edges[i + 1] > edges[i])) return fail(c, COLA_EINVAL, "edges must increase");
  int r = ensure_twiddles(c, ng);
  if (r != COLA_OK) return r;
  HIP_TRY(c, hipMemcpyAsync(c->pk_edges, edges, (nbins + 1) * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->pk_cbar, cbar, nbins * sizeof(double), hipMemcpyHostToDevice, c->stream));
  const long rs = 2 * padded_cols(ng);
  float2* X = c->mesh[0];
  float2* Z = c->mesh[1];
  deposit(c, ng, reinterpret_cast<float*>(X), rs, 1, disp);
  fft3d_forward(X, ng, c->tw, c->stream);
  launch_pk_bin(X, ng, c->p.box, c->pk_edges, nbins, c->pk_partial, kPkChunks, c->stream);
  launch_pk_reduce(c->pk_partial, nbins, kPkChunks, c->pk_out, c->stream);
  launch_fill_u32(reinterpret_cast<uint32_t*>(Z), 2 * mesh_complex_count(ng), 0u, c->stream);
  launch_pk_adj_modes(X, Z, ng, c->p.box, c->pk_edges, nbins, c->pk_cbar, c->pk_out, c->stream);
  fft3d_inverse(Z, ng, c->tw, c->stream);
  const float dscale = (float)((double)ng / (double)c->p.nmesh);
  const double cratio = (double)ng * ng * ng / (double)c->np3;
  launch_adj_deposit_grad(disp, reinterpret_cast<float*>(Z), rs, c->p.np, ng, dscale, (float)cratio,
                          dbar, c->stream);
  LAUNCH_CHECK(c, "cola_pk_adjoint");
  HIP_TRY(c, hipStreamSynchronize(c->stream));  // host edges / cbar released
  return COLA_OK;
}

int cola_init_2lpt_adjoint(cola_ctx* c, const float* noise, const float* dbar0, const float* p1bar,
                           const float* p2bar, float* noise_bar) {
  if (!c || !noise || !dbar0 || !p1bar || !p2bar || !noise_bar)
    return fail(c, COLA_EINVAL, "null argument");
  if (!c->have_state) return fail(c, COLA_ESTATE, "no initial conditions (amplitude table)");
  const int np = c->p.np, nm = c->p.nmesh;
  const long rs = 2 * padded_cols(np);
  const long ms = mesh_complex_count(np);
  const double om = c->p.omega_m, a0 = c->p.a_init;
  const float D1 = (float)growth_D1(a0, om), D2 = (float)D2_of(&c->p, a0);
  const double inv3 = 1.0 / ((double)np * np * np);
  const float sgrad = (float)(nm / (2.0 * kPi) * inv3);
  float2* C0 = ic_buf(c, 0);
  float2* S = ic_buf(c, 1);
  float2* B = ic_buf(c, 2);   // B, B + ms, B + 2 ms
  float2* Wb = ic_buf(c, 5);
  auto fwd_zy3 = [&](float2* m) {
    fft_r2c_z(m, np, 3, ms, c->tw, c->stream);
    fft_y(m, np, 3, ms, 0, c->tw, c->stream);
  };
  auto inv_zy = [&](float2* m) {
    fft_y(m, np, 1, 0, 1, c->tw, c->stream);
    fft_c2r_z(m, np, 1, 0, c->tw, c->stream);
  };
  const float2* Bs[3] = {B, B + ms, B + 2 * ms};
  // Sbar = IDFT[sum_d conj(M2_d) DFT(Psi2bar_d)], conj(M2_d) = +i n_d sg / |n|^2
  launch_axpy_to_mesh(p2bar, dbar0, D2, np, reinterpret_cast<float*>(B), rs, 2 * ms, c->stream);
  fwd_zy3(B);
  CombineSpec cs;
  cs.nin = 3;
  cs.scale = sgrad;
  fft_combine_x(Bs, S, np, cs, nullptr, c->tw, c->stream);
  inv_zy(S);
  // delta_L spectrum from the noise
  launch_copy_to_mesh(noise, np, reinterpret_cast<float*>(C0), rs, c->stream);
  fft_r2c_z(C0, np, 1, 0, c->tw, c->stream);
  fft_y(C0, np, 1, 0, 0, c->tw, c->stream);
  XPassArgs xa;
  xa.in = C0;
  xa.out[0] = C0;
  xa.mode = X_FWD_AMP;
  xa.amp = c->amp;
  fft_x(xa, np, c->tw, c->stream);
  auto phi_into = [&](float2* out, int i, int j) {
    XPassArgs m;
    m.in = C0;
    m.out[0] = out;
    m.mode = X_MULT_INV;
    m.mult = M_HESS;
    m.comp_a = i;
    m.comp_b = j;
    m.scale = (float)inv3;
    fft_x(m, np, c->tw, c->stream);
    inv_zy(out);
  };
  // diagonal phi_ii -> phibar_ii, then wbar += IDFT[A n_i n_i / n^2 / np^3 DFT(phibar_ii)]
  for (int d = 0; d < 3; ++d) phi_into(B + d * ms, d, d);
  launch_phibar_diag(reinterpret_cast<float*>(B), reinterpret_cast<float*>(B + ms),
                     reinterpret_cast<float*>(B + 2 * ms), reinterpret_cast<float*>(S), np, rs, c->stream);
  fwd_zy3(B);
  CombineSpec hs;
  hs.nin = 3;
  hs.kind[0] = hs.kind[1] = hs.kind[2] = M_HESS;
  hs.ca[0] = 0; hs.cb[0] = 0;
  hs.ca[1] = 1; hs.cb[1] = 1;
  hs.ca[2] = 2; hs.cb[2] = 2;
  hs.scale = (float)inv3;
  hs.use_amp = 1;
  fft_combine_x(Bs, Wb, np, hs, c->amp, c->tw, c->stream);
  // off-diagonal
  const int od[3][2] = {{0, 1}, {1, 2}, {2, 0}};
  for (int q = 0; q < 3; ++q) phi_into(B + q * ms, od[q][0], od[q][1]);
  launch_phibar_off(reinterpret_cast<float*>(B), reinterpret_cast<float*>(S), np, rs, 2 * ms, c->stream);
  fwd_zy3(B);
  for (int q = 0; q < 3; ++q) {
    hs.ca[q] = od[q][0];
    hs.cb[q] = od[q][1];
  }
  hs.accumulate = 1;
  fft_combine_x(Bs, Wb, np, hs, c->amp, c->tw, c->stream);
  // Psi1: wbar += IDFT[A conj(M1_d) DFT(Psi1bar_d)], conj(M1_d) = -i n_d sg / |n|^2
  launch_axpy_to_mesh(p1bar, dbar0, D1, np, reinterpret_cast<float*>(B), rs, 2 * ms, c->stream);
  fwd_zy3(B);
  CombineSpec gs;
  gs.nin = 3;
  gs.scale = -sgrad;
  gs.use_amp = 1;
  gs.accumulate = 1;
  fft_combine_x(Bs, Wb, np, gs, c->amp, c->tw, c->stream);
  inv_zy(Wb);
  launch_copy_from_mesh(reinterpret_cast<float*>(Wb), np, rs, noise_bar, 1.0f, c->stream);
  LAUNCH_CHECK(c, "cola_init_2lpt_adjoint");
  return COLA_OK;
}

int cola_fft_set_schedule(int32_t n, int32_t pass, int32_t order) {
  return set_fft_block_order(n, pass, order) == 0 ? COLA_OK : COLA_EINVAL;
}

int cola_fft_get_schedule(int32_t n, int32_t pass, int32_t* order) {
  if (!order || !fft_size_supported(n) || pass < 0 || pass > 2) return COLA_EINVAL;
  *order = fft_block_order(n, pass);
  return COLA_OK;
}

int cola_autotune(cola_ctx* c, int32_t reps, int32_t* best, double* ms) {
  if (!c) return COLA_EINVAL;
  if (reps < 1) reps = 3;
  const int nm = c->p.nmesh;
  const long P = padded_cols(nm), rowc = pm_rowc(nm);
  float2* m0 = c->meshbase;
  // the meshes are scratch between calls: zeros in, the step's column passes
  launch_fill_u32(reinterpret_cast<uint32_t*>(m0), 2 * c->mesh_region, 0u, c->stream);
  StepCoef v{};
  v.gscale = 1.0f;
  launch_set_coef(c->coef, v, 1, 0, c->stream);
  XPassArgs green;
  green.in = m0;
  green.out[0] = m0;
  green.out[1] = m0 + P;
  green.mode = X_FWD_GREEN;
  green.coef = c->coef;
  green.rowc = rowc;
  auto run = [&](int kind) {
    if (kind == 0) fft_y(m0, nm, 1, 0, 0, c->tw, c->stream, 1, 0, rowc);
    else if (kind == 1) fft_x(green, nm, c->tw, c->stream);
    else fft_y_grad_yz(m0 + P, m0 + 2 * P, nm, c->tw, c->stream, 1, 0, rowc);
  };
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return fail(c, COLA_EHIP, "hipEventCreate");
  }
  int code = COLA_OK;
  for (int kind = 0; kind < 3 && code == COLA_OK; ++kind) {
    const int before = fft_block_order(nm, kind);
    double tbest = 0.0;
    int pick = before;
    for (int cand = 0; cand < 2 && code == COLA_OK; ++cand) {
      const int order = 1 - cand;                      // the default first
      set_fft_block_order(nm, kind, order);
      run(kind);                                         // warm-up
      hipEventRecord(e0, c->stream);
      for (int r = 0; r < reps; ++r) run(kind);
      hipEventRecord(e1, c->stream);
      hipError_t e = hipEventSynchronize(e1);
      float t = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      if (e != hipSuccess) {
        code = hip_fail(c, e, "cola_autotune");
        break;
      }
      const double per = (double)t / reps;
      if (ms) ms[2 * kind + order] = per;
      // the default order unless the other one is faster by more than 2%
      // (timing noise would otherwise flip near-ties from run to run)
      if (cand == 0 || per < 0.98 * tbest) {
        tbest = per;
        pick = order;
      }
    }
    set_fft_block_order(nm, kind, code == COLA_OK ? pick : before);
    if (code == COLA_OK && best) best[kind] = pick;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return code;
}

int cola_step_scalars(const cola_params* p, double a_x, double a_v, double a1, double* out) {
  if (!p || !out || !(a_x > 0) || !(a_v > 0) || !(a1 > 0)) return COLA_EINVAL;
  step_scalars(p, a_x, a_v, a1, out);
  return COLA_OK;
}

int cola_stage_times(cola_ctx* c, double* ms, int64_t* count) {
  if (!c) return COLA_EINVAL;
  if (!(c->p.flags & COLA_F_STAGE_TIMERS)) return fail(c, COLA_ESTATE, "stage timers not enabled");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  double acc[COLA_NSTAGE] = {};
  int64_t cnt[COLA_NSTAGE] = {};
  for (size_t i = 0; i < c->ev_stage.size(); ++i) {
    float t = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&t, c->ev_pool[2 * i], c->ev_pool[2 * i + 1]));
    acc[c->ev_stage[i]] += t;
    cnt[c->ev_stage[i]] += 1;
  }
  for (int s = 0; s < COLA_NSTAGE; ++s) {
    if (ms) ms[s] = acc[s];
    if (count) count[s] = cnt[s];
  }
  c->ev_stage.clear();
  c->ev_used = 0;
  return COLA_OK;
}

int cola_synchronize(cola_ctx* c) {
  if (!c) return COLA_EINVAL;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return COLA_OK;
}

const char* cola_strerror(int code) {
  switch (code) {
    case COLA_OK: return "ok";
    case COLA_EINVAL: return "invalid argument";
    case COLA_ENOMEM: return "workspace too small";
    case COLA_ESTATE: return "invalid state for this call";
    case COLA_EUNSUPPORTED: return "unsupported size";
    case COLA_EHIP: return "HIP runtime error";
    case COLA_ENONFINITE: return "non-finite value in the state";
    default: return "unknown error";
  }
}

const char* cola_last_error(const cola_ctx* c) { return c ? c->err.c_str() : ""; }

// ---------------------------------------------------------------------------
// Batches of independent realisations.
//
// Mocks with equal (np, nmesh, omega_m, n_lpt, a_init) form a group; the
// contexts of a group sit at a fixed byte stride in the workspace, so each
// launch of the step covers the whole group (grid z = mock) and a group costs
// the same kernel launches as one mock.  The launches of all groups are
// captured once into a HIP graph, one parallel branch per group (independent
// data), that reads the per-step scalars from device memory, so a step is
// one small coefficient write per group plus one graph launch.

}  // extern "C"

struct cola_batch {
  struct Group {
    std::vector<int> idx;   // caller's mock indices, workspace order
    long mstride = 0;
    cola_ctx* first = nullptr;
    int chunk = 0;          // mocks per launch (0: the whole group)
  };
  hipStream_t stream = nullptr;     // caller's stream
  hipStream_t cap = nullptr;        // capture stream
  std::vector<hipStream_t> branch;  // one more capture stream per further group
  std::vector<hipEvent_t> ev;       // fork event, then one join event per branch
  std::vector<cola_ctx*> mocks;     // caller's order
  std::vector<Group> groups;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int use_graph = 1;
  std::string err;
};

namespace {

bool same_group(const cola_params& a, const cola_params& b) {
  return a.np == b.np && a.nmesh == b.nmesh && a.omega_m == b.omega_m && a.n_lpt == b.n_lpt &&
         a.a_init == b.a_init && (a.flags & COLA_F_D2_ODE) == (b.flags & COLA_F_D2_ODE);
}

// Groups in first-appearance order; returns the workspace layout.
size_t batch_plan(const cola_params* p, int n, std::vector<cola_batch::Group>* groups,
                  std::vector<size_t>* offset) {
  groups->clear();
  offset->assign(n, 0);
  std::vector<int> gid(n, -1);
  std::vector<cola_params> key;
  for (int i = 0; i < n; ++i) {
    for (size_t g = 0; g < key.size(); ++g)
      if (same_group(key[g], p[i])) { gid[i] = (int)g; break; }
    if (gid[i] < 0) {
      gid[i] = (int)key.size();
      key.push_back(p[i]);
      groups->emplace_back();
    }
    (*groups)[gid[i]].idx.push_back(i);
  }
  size_t o = 0;
  for (size_t g = 0; g < groups->size(); ++g) {
    cola_batch::Group& G = (*groups)[g];
    G.mstride = (long)align256(layout(&p[G.idx[0]]).total);
    for (int i : G.idx) {
      (*offset)[i] = o;
      o += (size_t)G.mstride;
    }
  }
  return o;
}

int batch_fail(cola_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg;
  return code;
}

void batch_free(cola_batch* b) {
  if (b->exec) {
    hipStreamSynchronize(b->stream);
    hipGraphExecDestroy(b->exec);
  }
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->cap) hipStreamDestroy(b->cap);
  for (hipStream_t t : b->branch) hipStreamDestroy(t);
  for (hipEvent_t e : b->ev) hipEventDestroy(e);
  for (cola_ctx* c : b->mocks)
    if (c) cola_destroy(c);
  delete b;
}

void enqueue_group(cola_batch* b, cola_batch::Group& G, hipStream_t s) {
  const int n = (int)G.idx.size();
  const int per = G.chunk > 0 ? G.chunk : n;
  for (int i0 = 0; i0 < n; i0 += per) {
    cola_ctx* c = b->mocks[G.idx[i0]];
    const hipStream_t keep = c->stream;
    c->stream = s;
    step_launches(c, per < n - i0 ? per : n - i0, G.mstride);
    c->stream = keep;
  }
}

// The groups one after the other on s, or (parallel) group 0 on s and group
// g on branch stream g-1, forked from and joined back into s by events.
void enqueue_batch_step(cola_batch* b, hipStream_t s, bool parallel) {
  const size_t ng = b->groups.size();
  if (!parallel || ng < 2 || b->branch.size() + 1 < ng) {
    for (cola_batch::Group& G : b->groups) enqueue_group(b, G, s);
    return;
  }
  // groups by decreasing work (particles x mocks), the heaviest branch
  // enqueued first: it is the step's critical path
  std::vector<size_t> ord(ng);
  for (size_t g = 0; g < ng; ++g) ord[g] = g;
  auto work = [&](size_t g) { return (double)b->groups[g].first->np3 * (double)b->groups[g].idx.size(); };
  std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return work(x) > work(y); });
  hipEventRecord(b->ev[0], s);
  for (size_t k = 0; k + 1 < ng; ++k) {
    hipStreamWaitEvent(b->branch[k], b->ev[0], 0);
    enqueue_group(b, b->groups[ord[k]], b->branch[k]);
    hipEventRecord(b->ev[k + 1], b->branch[k]);
  }
  enqueue_group(b, b->groups[ord[ng - 1]], s);
  for (size_t k = 1; k < ng; ++k) hipStreamWaitEvent(s, b->ev[k], 0);
}

void drop_graph(cola_batch* b) {
  if (b->exec) {
    hipStreamSynchronize(b->stream);  // no launch of the old graph still pending
    hipGraphExecDestroy(b->exec);
  }
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Captures the step launches of every group into one graph on the capture stream.
int build_graph(cola_batch* b) {
  hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return batch_fail(b, COLA_EHIP, std::string("begin capture: ") + hipGetErrorString(e));
  enqueue_batch_step(b, b->cap, true);
  const hipError_t el = hipGetLastError();
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->cap, &g);
  if (el != hipSuccess || e != hipSuccess) {
    if (g) hipGraphDestroy(g);
    return batch_fail(b, COLA_EHIP, std::string("capture: ") + hipGetErrorString(el != hipSuccess ? el : e));
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    return batch_fail(b, COLA_EHIP, std::string("instantiate: ") + hipGetErrorString(e));
  }
  b->graph = g;
  b->exec = x;
  return COLA_OK;
}

}  // namespace

extern "C" {

int cola_batch_workspace_query(const cola_params* params, int32_t nmock, size_t* bytes) {
  if (!params || nmock < 1 || !bytes) return COLA_EINVAL;
  for (int i = 0; i < nmock; ++i) {
    const int v = validate(&params[i]);
    if (v != COLA_OK) return v;
  }
  std::vector<cola_batch::Group> groups;
  std::vector<size_t> off;
  *bytes = batch_plan(params, nmock, &groups, &off);
  return COLA_OK;
}

int cola_batch_create(const cola_params* params, int32_t nmock, void* ws, size_t bytes, void* stream,
                      cola_batch** out) {
  if (!out) return COLA_EINVAL;
  *out = nullptr;
  if (!params || nmock < 1) return COLA_EINVAL;
  for (int i = 0; i < nmock; ++i) {
    const int v = validate(&params[i]);
    if (v != COLA_OK) return v;
    if (params[i].flags & COLA_F_STAGE_TIMERS) return COLA_EINVAL;  // events do not go into graphs
  }
  if (!ws || ((uintptr_t)ws & 255)) return COLA_EINVAL;
  cola_batch* b = new (std::nothrow) cola_batch();
  if (!b) return COLA_ENOMEM;
  std::vector<size_t> off;
  const size_t need = batch_plan(params, nmock, &b->groups, &off);
  if (bytes < need) {
    delete b;
    return COLA_ENOMEM;
  }
  b->stream = (hipStream_t)stream;
  b->mocks.assign(nmock, nullptr);
  for (int i = 0; i < nmock; ++i) {
    const size_t sz = layout(&params[i]).total;
    const int r = cola_create(&params[i], (char*)ws + off[i], sz, stream, &b->mocks[i]);
    if (r != COLA_OK) {
      batch_free(b);
      return r;
    }
  }
  for (cola_batch::Group& G : b->groups) G.first = b->mocks[G.idx[0]];
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    b->cap = nullptr;
    b->use_graph = 0;
  }
  // branch streams and events for the groups' parallel branches in the graph
  // (default priority); without them the graph runs the groups in sequence
  bool ok = true;
  for (size_t g = 0; ok && g < b->groups.size(); ++g) {
    hipEvent_t e;
    ok = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    if (ok) b->ev.push_back(e);
    if (ok && g > 0) {
      hipStream_t t;
      ok = hipStreamCreateWithFlags(&t, hipStreamNonBlocking) == hipSuccess;
      if (ok) b->branch.push_back(t);
    }
  }
  if (!ok) {
    for (hipStream_t t : b->branch) hipStreamDestroy(t);
    b->branch.clear();
  }
  *out = b;
  return COLA_OK;
}

int cola_batch_destroy(cola_batch* b) {
  if (!b) return COLA_EINVAL;
  batch_free(b);
  return COLA_OK;
}

int32_t cola_batch_size(const cola_batch* b) { return b ? (int32_t)b->mocks.size() : 0; }

int32_t cola_batch_ngroups(const cola_batch* b) { return b ? (int32_t)b->groups.size() : 0; }

cola_ctx* cola_batch_mock(cola_batch* b, int32_t i) {
  if (!b || i < 0 || i >= (int32_t)b->mocks.size()) return nullptr;
  return b->mocks[i];
}

int cola_batch_set_graph(cola_batch* b, int32_t enable) {
  if (!b) return COLA_EINVAL;
  if (enable && !b->cap) return batch_fail(b, COLA_EHIP, "no capture stream");
  b->use_graph = enable ? 1 : 0;
  return COLA_OK;
}

int cola_batch_set_chunk_bytes(cola_batch* b, size_t bytes) {
  if (!b) return COLA_EINVAL;
  for (cola_batch::Group& G : b->groups) {
    const size_t per = bytes / (size_t)G.mstride;
    G.chunk = bytes == 0 ? 0 : (int)(per < 1 ? 1 : (per > G.idx.size() ? G.idx.size() : per));
  }
  drop_graph(b);
  return COLA_OK;
}

int cola_batch_step(cola_batch* b, double a0, double a1) {
  if (!b) return COLA_EINVAL;
  if (!(a1 > a0) || !std::isfinite(a1)) return batch_fail(b, COLA_EINVAL, "a1 must exceed a0");
  for (cola_ctx* c : b->mocks) {
    if (!c->have_state) return batch_fail(b, COLA_ESTATE, "a mock has no initial conditions");
    if (!same_a(a0, c->a_x)) return batch_fail(b, COLA_ESTATE, "a0 differs from a mock's position time");
  }
  for (cola_batch::Group& G : b->groups) {
    const cola_ctx* c0 = G.first;
    for (int i : G.idx)
      if (!same_a(b->mocks[i]->a_v, c0->a_v))
        return batch_fail(b, COLA_ESTATE, "mocks of a group must share the velocity time");
  }
  double s[10];
  for (cola_batch::Group& G : b->groups) {
    cola_ctx* c = G.first;
    launch_set_coef(c->coef, make_coef(&c->p, c->a_x, c->a_v, a1, s), (int)G.idx.size(), G.mstride,
                    b->stream);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return batch_fail(b, COLA_EHIP, std::string("coefficients: ") + hipGetErrorString(e));
  if (b->use_graph) {
    if (!b->exec) {
      const int r = build_graph(b);
      if (r != COLA_OK) return r;
    }
    e = hipGraphLaunch(b->exec, b->stream);
    if (e != hipSuccess) return batch_fail(b, COLA_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
  } else {
    enqueue_batch_step(b, b->stream, false);
    e = hipGetLastError();
    if (e != hipSuccess) return batch_fail(b, COLA_EHIP, std::string("batch step: ") + hipGetErrorString(e));
  }
  for (cola_ctx* c : b->mocks) {
    step_scalars(&c->p, c->a_x, c->a_v, a1, s);
    c->a_v = s[7];
    c->a_x = a1;
  }
  for (cola_ctx* c : b->mocks) {
    const int r = check_finite(c);
    if (r != COLA_OK) return batch_fail(b, r, c->err);
  }
  return COLA_OK;
}

int cola_batch_synchronize(cola_batch* b) {
  if (!b) return COLA_EINVAL;
  const hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return batch_fail(b, COLA_EHIP, hipGetErrorString(e));
  return COLA_OK;
}

const char* cola_batch_last_error(const cola_batch* b) { return b ? b->err.c_str() : ""; }


}  // extern "C"
