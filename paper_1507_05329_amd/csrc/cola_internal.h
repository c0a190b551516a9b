// Internal declarations of libcola: context layout, host scalars, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <string>
#include <vector>

#include "../../include/cola.h"

namespace cola {

// ---------------------------------------------------------------------------
// FFT plan: a {2,3}-smooth length factored into radices {16, 8, 4, 3, 2}.
struct FftPlan {
  int n = 0;          // transform length
  int nstage = 0;
  int radix[12] = {};
};
bool make_plan(int n, FftPlan* plan);
bool fft_size_supported(int n);   // transform sizes with compiled kernels
// Block order (1: contiguous block ranges per XCD, 0: hardware round-robin)
// of the column passes of length n, per pass kind (0 plain, 1 Green's
// function x pass, 2 gradient y pass); process-wide, results do not depend
// on it.  set returns 0, or -1 for an unsupported length, kind or value.
int fft_block_order(int n, int kind);
int set_fft_block_order(int n, int kind, int order);

// Padded complex row length of an n^3 real mesh in the r2c layout: the
// (n/2+1) half-spectrum rounded up to 16 complex values (128-byte rows).
inline long padded_cols(int n) { return ((long)(n / 2 + 1) + 15) / 16 * 16; }
inline long mesh_complex_count(int n) { return (long)n * n * padded_cols(n); }

// Workgroups of 256 for a grid-stride loop over n items: a dispatch holds at
// most 2^32 - 1 work-items, so the grid is capped and each thread loops.
inline unsigned grid_1d(long n) {
  const long b = (n + 255) / 256;
  return (unsigned)(b < (1L << 22) ? (b > 0 ? b : 1) : (1L << 22));
}

// Twiddle tables: one per distinct length, tw[k] = exp(-2 pi i k / n).
struct TwiddleSet {
  int n[4] = {0, 0, 0, 0};
  const float2* tw[4] = {nullptr, nullptr, nullptr, nullptr};
  const float2* get(int len) const {
    for (int i = 0; i < 4; ++i) if (n[i] == len) return tw[i];
    return nullptr;
  }
};

// ---------------------------------------------------------------------------
// Host FP64 scalars of the method (cosmo.cpp).
double hubble_E(double a, double om);
double growth_D1(double a, double om);
double growth_D2(double a, double om);
double kick_factor(double a_v, double a_x, double a_h, double om, double n);
double drift_factor(double a0, double a1, double a_h, double om, double n);
// dD1/da and dD2/da (velocity of the 2LPT trajectory).
double growth_D1_prime(double a, double om);
double growth_D2_prime(double a, double om);
// D2 from its growth equation instead of the fit, and dD2/da.
double growth_D2_ode(double a, double om);
double growth_D2_ode_prime(double a, double om);
// The D2 (and dD2/da) the run uses: the fit, or the ODE under COLA_F_D2_ODE.
double D2_of(const cola_params* p, double a);
double D2_prime_of(const cola_params* p, double a);
// ln-ln interpolation of a P(k) table, end segments extended.
double interp_pk(double k, const double* kt, const double* pt, int nk);

// ---------------------------------------------------------------------------
// Kernel launchers (all asynchronous on `s`).
// Tile sort of particles by the 8^3 tile of their home cell (k_sort.hip).
// Batched launches: nmock mocks, arrays of mock b at byte offset b * mstride.
void launch_fill_u32(uint32_t* p, long n, uint32_t v, hipStream_t s, int nmock = 1, long mstride = 0);
void launch_bin_count(const float* disp, int np, int nm, float dscale, uint32_t* counts,
                      uint32_t* pkey, uint32_t* prank, hipStream_t s, int nmock = 1, long mstride = 0);
void launch_exclusive_scan(const uint32_t* in, uint32_t* out, long n,
                           uint32_t* scratch, hipStream_t s, int nmock = 1, long mstride = 0);
void launch_scatter(const uint32_t* pkey, const uint32_t* prank, const uint32_t* off,
                    long np3, uint32_t* perm, hipStream_t s, int nmock = 1, long mstride = 0);
// The same scatter for the tile sort of np^3 lattice particles, walking them
// as the bucket count does (np a multiple of 16).
void launch_scatter_walk(const uint32_t* pkey, const uint32_t* prank, const uint32_t* off, int np,
                         uint32_t* perm, hipStream_t s, int nmock = 1, long mstride = 0);
// Deterministic CIC gather (k_deposit.hip).
void launch_deposit(const float* disp, const uint32_t* perm, const uint32_t* off,
                    int np, int nm, float dscale, float* out, long row_stride, int contrast,
                    hipStream_t s, int nmock = 1, long mstride = 0);
// Three weighted deposits at once (readout transpose): out[q] += sum_p wt[q][p] w_s(p).
void launch_deposit3_weighted(const float* disp, const uint32_t* perm, const uint32_t* off, int np,
                              int nm, const float* wt, float* out, long row_stride,
                              long mesh_stride_floats, hipStream_t s);
// Per-step scalars of the kick/drift and the Green pass.
struct KickDrift {
  float K, c1, c2;     // v += K F - c1 Psi1 - c2 Psi2
  float I, e1, e2;     // d += I v + e1 Psi1 + e2 Psi2
};
// Per-step scalars read by the step kernels from device memory (so a
// captured graph of the step stays valid from step to step).
struct StepCoef {
  KickDrift kd;
  float gscale;        // Green's function scale alpha nm / (2 pi nm^3)
  float pad;
};
// FFT passes (k_fft.hip).
// X_FWD_GREEN (x pass): forward, phi = Green's function x spectrum,
// out[0] = IDFT_x[i n_x phi], out[1] = IDFT_x[phi].  X_INV_GRAD_YZ (y pass,
// inverse) on that B: out[0] = IDFT_y[i n_y B], out[1] = IDFT_y[i n_z B].
enum XMode { X_FWD = 0, X_FWD_GREEN = 1, X_FWD_AMP = 2, X_MULT_INV = 3, X_INV = 4, X_INV_GRAD_YZ = 5 };
enum MultKind { M_NONE = 0, M_GRAD = 1, M_HESS = 2 };
struct XPassArgs {
  const float2* in = nullptr;
  float2* out[3] = {nullptr, nullptr, nullptr};
  int mode = X_FWD;
  int mult = M_NONE;
  int comp_a = 0, comp_b = 0;   // gradient axis / Hessian axes
  float scale = 1.f;            // multiplier scale
  const float* amp = nullptr;   // amplitude by integer |n|^2 (X_FWD_AMP)
  const StepCoef* coef = nullptr;  // X_FWD_GREEN: scale read from coef->gscale
  int nmock = 1;                // batched mocks (blockIdx.z) ...
  long mstride = 0;             // ... at this byte stride
  long rowc = 0;                // row stride in complex values (0: padded_cols(n))
};
// Spectral combination pass (adjoint): out = IDFT_x[sum_q m_q DFT_x(in_q)].
struct CombineSpec {
  int nin = 0;
  int kind[3] = {M_GRAD, M_GRAD, M_GRAD};
  int ca[3] = {0, 1, 2}, cb[3] = {0, 0, 0};
  float scale = 1.f;
  int green = 0;        // 1: a gradient is zeroed only on its own axis' Nyquist plane
  int use_amp = 0;      // multiply by the amplitude table (all Nyquist modes zeroed)
  int accumulate = 0;   // out += result
};
void fft_combine_x(const float2* const in[3], float2* out, int n, const CombineSpec& cs,
                   const float* amp, const TwiddleSet& tw, hipStream_t s);
void fft3d_forward(float2* mesh, int n, const TwiddleSet& tw, hipStream_t s);
void fft3d_inverse(float2* mesh, int n, const TwiddleSet& tw, hipStream_t s);
// rowc: row stride in complex values (0: padded_cols(n)); the PM force
// pipeline keeps its three meshes row-interleaved (rowc = 3 padded_cols,
// mesh c at offset c padded_cols).
void fft_r2c_z(float2* mesh, int n, int nplanes_mesh, long mesh_stride, const TwiddleSet& tw,
               hipStream_t s, int nmock = 1, long mstride = 0, long rowc = 0);
void fft_c2r_z(float2* mesh, int n, int nmesh_batch, long mesh_stride, const TwiddleSet& tw,
               hipStream_t s, int nmock = 1, long mstride = 0);
// Inverse z pass of the three row-interleaved force meshes, the real
// outputs interleaved by node: (g_x, g_y, g_z) of node (x, y, z) at floats
// (x n + y) 6 padded_cols(n) + 3 z + {0, 1, 2}.
void fft_c2r_z_forces(float2* mesh, int n, const TwiddleSet& tw, hipStream_t s, int nmock = 1, long mstride = 0);
void fft_y(float2* mesh, int n, int nmesh_batch, long mesh_stride, int inverse,
           const TwiddleSet& tw, hipStream_t s, int nmock = 1, long mstride = 0, long rowc = 0);
void fft_x(const XPassArgs& a, int n, const TwiddleSet& tw, hipStream_t s);
// Inverse y pass of the PM gradients: b -> IDFT_y[i n_y b] in place, IDFT_y[i n_z b] -> gz.
void fft_y_grad_yz(float2* b, float2* gz, int n, const TwiddleSet& tw, hipStream_t s, int nmock = 1,
                   long mstride = 0, long rowc = 0);
// Velocity at the position time (k_velocity.hip): v = v_res + K F + u1 Psi1 + u2 Psi2,
// redshift-space shift rsd * v along one axis.
struct VelCoef {
  float K;       // kick factor from a_v to a_x (0: no force read)
  float u1, u2;  // Psi1, Psi2 coefficients (2LPT velocity minus the kick's 2LPT force terms)
  float rsd;     // 1 / (a adot)
};
// g0 == nullptr: no force gather (K must be 0); sdisp == nullptr: no redshift-space output.
// g: the force field interleaved by node (fft_c2r_z_forces), row_stride floats per (x, y) row.
void launch_velocity(const float* g, long row_stride, const float* disp,
                     const float* vres, const float* psi1, const float* psi2, int np, int nm,
                     const VelCoef& k, float* vel, float* sdisp, int axis, hipStream_t s);
// Snapshot inside the coming step (k_velocity.hip): the step's kick to a_h,
// then the drift ansatz to a_s.
struct SnapCoef {
  float K, c1, c2;  // kick to a_h: v_h = v_res + K F - c1 Psi1 - c2 Psi2
  float I, e1, e2;  // d_s = d + I v_h + e1 Psi1 + e2 Psi2
  float sv, w1, w2; // v_s = sv v_h + w1 Psi1 + w2 Psi2
  float rsd;        // 1 / (a_s adot(a_s))
};
void launch_snapshot(const float* g, long row_stride, const float* disp,
                     const float* vres, const float* psi1, const float* psi2, int np, int nm,
                     const SnapCoef& k, float* dout, float* vout, float* sdisp, int axis, hipStream_t s);
// Force readout + kick/drift (k_particles.hip).
void launch_set_coef(StepCoef* dst, const StepCoef& v, int nmock, long mstride, hipStream_t s);
void launch_readout_kick_drift(const float* g, long row_stride, float* disp, float* vres,
                               const float* psi1, const float* psi2, int np, int nm,
                               const StepCoef* coef, float* force_out, hipStream_t s,
                               int nmock = 1, long mstride = 0);
// Initial conditions (k_ic.hip).
void launch_philox_noise(uint64_t seed, int np, float* out, long row_stride, hipStream_t s);
void launch_copy_to_mesh(const float* src, int n, float* mesh, long row_stride, hipStream_t s);
// elem: floats between consecutive nodes of a row (3 for one component of the force field).
void launch_copy_from_mesh(const float* mesh, int n, long row_stride, float* dst, float scale,
                           hipStream_t s, int elem = 1);
void launch_source_diag(float* a, const float* b, const float* c, int n, long row_stride,
                        hipStream_t s);
void launch_source_sub_sq(float* a, const float* b, int n, long row_stride, hipStream_t s);
void launch_init_particles(float* disp, float* vres, const float* psi1, const float* psi2,
                           long np3, float D1, float D2, hipStream_t s);
void launch_axpby(float* y, const float* x, float a, float b, long n, hipStream_t s);
// Power spectrum binning (k_pk.hip).
void launch_pk_bin(const float2* spec, int ng, double box, const double* edges, int nbins,
                   double* partial, int nchunk, hipStream_t s, int deconvolve = 1);
// Jing (2005) image sums of the CIC window per bin at the per-bin slopes (out: nbins sums).
void launch_pk_alias(int ng, double box, const double* edges, int nbins, const double* slope, double* partial,
                     int nchunk, double* out, hipStream_t s);
void launch_pk_reduce(const double* partial, int nbins, int nchunk, double* out, hipStream_t s);
// Density / line-of-sight momentum spectra: partial holds 5 doubles per (bin, chunk),
// out 5 per bin (sum |k|, P_dd, P_du, P_uu, count).
void launch_pk_cross(const float2* sd, const float2* sp, int ng, double box, const double* edges, int nbins,
                     int axis, double* partial, int nchunk, double* out, hipStream_t s);
// Friends-of-friends labels (k_fof.hip): labels[i] = smallest id of i's group.
// count and start hold np^3 + 1 entries, scan_scratch (np^3 + 1) / 4096 + 2;
// key, rank, sorted np^3 each; flag is set if a union exceeded its retry bound.
void launch_fof(const float* disp, int np, int nm, double b_frac, uint32_t* labels, uint32_t* count,
                uint32_t* start, uint32_t* scan_scratch, uint32_t* key, uint32_t* rank, uint32_t* sorted,
                uint32_t* flag, hipStream_t s);
// Halo catalogue of FoF labels (k_fof.hip): count per label, flags of groups with
// >= minm members, their exclusive scan (hidx[np3] = number of halos); then roots,
// counts, centres and mean velocities (SoA with the given stride) from 64-bit
// fixed-point sums (acc: 6 per halo).  bad is set for a label outside [0, np3).
void launch_halo_count(const int32_t* lab, long np3, int32_t minm, uint32_t* count, uint32_t* flg, uint32_t* hidx,
                       uint32_t* scan_scratch, uint32_t* bad, hipStream_t s);
void launch_halo_fill(const float* disp, const float* vel, const int32_t* lab, const uint32_t* count,
                      const uint32_t* flg, const uint32_t* hidx, int np, int nm, int nh, int stride,
                      unsigned long long* acc, int32_t* root, int32_t* cnt, float* pos, float* vout,
                      hipStream_t s);
// Weights of that deposit (k_velocity.hip): 1/nbar, the scaled velocity along axis, 0.
void launch_los_weights(const float* g, long row_stride, const float* disp,
                        const float* vres, const float* psi1, const float* psi2, int np, int nm,
                        const VelCoef& k, int axis, float w0, float scale, float* wt, hipStream_t s);
// Adjoint kernels (k_adjoint.hip).
void launch_adj_readout_kick(const float* disp, const float* g, long row_stride, int np, int nm,
                             const KickDrift& kd, float* dbar, float* vbar, float* p1bar, float* p2bar,
                             float* fbar, hipStream_t s);
void launch_adj_deposit_grad(const float* disp, const float* field, long row_stride, int np, int ng,
                             float dscale, float coef, float* dbar, hipStream_t s);
void launch_axpy_to_mesh(const float* a, const float* b, float alpha, int n, float* mesh,
                         long row_stride, long mesh_stride_floats, hipStream_t s);
void launch_phibar_diag(float* a, float* b, float* c, const float* sbar, int n, long row_stride,
                        hipStream_t s);
void launch_phibar_off(float* a, const float* sbar, int n, long row_stride, long mesh_stride_floats,
                       hipStream_t s);
void launch_pk_adj_modes(const float2* X, float2* Z, int ng, double box, const double* edges,
                         int nbins, const double* cbar, const double* sums, hipStream_t s);
// Non-finite check.
void launch_check_finite(const float* x, long n, uint32_t* flag, hipStream_t s);

}  // namespace cola

// ---------------------------------------------------------------------------
struct cola_ctx {
  cola_params p;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  long np3 = 0;
  // particle state, SoA 3 * np3 each
  float* disp = nullptr;
  float* vres = nullptr;
  float* psi1 = nullptr;
  float* psi2 = nullptr;
  // tile sort
  uint32_t* pkey = nullptr;
  uint32_t* prank = nullptr;
  uint32_t* perm = nullptr;
  uint32_t* counts = nullptr;   // nbucket + 1
  uint32_t* offsets = nullptr;  // nbucket + 1
  uint32_t* scan_scratch = nullptr;
  long nbucket = 0;
  // mesh region: 3 padded complex half meshes of nmesh (PM step), also
  // carved into 4 meshes of np for the initial conditions
  float2* meshbase = nullptr;
  float2* mesh[3] = {nullptr, nullptr, nullptr};
  long mesh_stride = 0;         // complex values per PM mesh
  long mesh_region = 0;         // complex values in the region
  // small buffers
  float2* twbuf = nullptr;
  cola::TwiddleSet tw;
  int tw_cap = 0;               // complex values per twiddle slot
  float* amp = nullptr;         // amplitude table by |n|^2 on the particle grid
  long amp_len = 0;
  double* pk_partial = nullptr;
  double* pk_out = nullptr;
  double* pk_edges = nullptr;
  uint32_t* flag = nullptr;
  float* fbar = nullptr;        // adjoint scratch, 3 * np3
  cola::StepCoef* coef = nullptr;  // per-step scalars (device)
  double* pk_cbar = nullptr;    // P(k) loss cotangents (adjoint)
  // stage timers (COLA_F_STAGE_TIMERS): pairs of events per recorded stage
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_stage;       // stage of each recorded pair
  size_t ev_used = 0;              // events handed out (2 per pair)
  // time state
  double a_x = 0, a_v = 0;
  bool have_state = false;
  std::string err;
};
