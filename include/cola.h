/*
 * libcola -- the COLA particle-mesh step on AMD Instinct MI355X (gfx950).
 *
 * Method: Koda, Blake, Beutler, Kazin & Marin (2015), "Fast and accurate mock
 * catalogue generation for low-mass galaxies", Sec. 2: COmoving Lagrangian
 * Acceleration (COLA).  Particles move in the frame of their 2LPT
 * trajectory x_2LPT = q + D1 Psi1(q) + D2 Psi2(q); only the residual is
 * integrated, with the kick/drift ansatz of eqs. cola-kick and cola-drift,
 * driven by a particle-mesh (PM) force.
 *
 * Conventions used by every call
 *   - Units: lengths Mpc/h at the boundary of cola_init_2lpt / cola_pk;
 *     particle state (displacement, residual velocity, Psi1, Psi2) is held in
 *     units of the PM mesh spacing dx = box / nmesh; time in 1/H0.
 *   - Particle id p = (i * np + j) * np + k for lattice indices (i, j, k) on
 *     axes (x, y, z); Lagrangian point q = (i, j, k) * box / np.
 *   - Particle arrays are structure-of-arrays float32, 3 * np^3 values:
 *     component c of particle p at [c * np^3 + p].
 *   - Meshes are C order [x][y][z], z fastest.  Mesh nodes sit at cell
 *     centres, (n + 1/2) dx.
 *   - Device pointers are HIP device memory owned by the caller.  The library
 *     never allocates device memory: all of its device state lives in the
 *     caller's workspace (cola_workspace_query gives the size).
 *   - Every call is enqueued on the context's HIP stream and returns without
 *     waiting, except where a call returns host data (stated per call).
 *   - Return value: COLA_OK (0) or a negative COLA_E* code.  No call aborts
 *     or throws; cola_last_error() gives a message.  A call that fails with
 *     anything but COLA_EHIP leaves the context state unchanged.
 */
#ifndef COLA_H
#define COLA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define COLA_OK            0
#define COLA_EINVAL       -1   /* bad argument (null pointer, size, range)         */
#define COLA_ENOMEM       -2   /* workspace smaller than cola_workspace_query      */
#define COLA_ESTATE       -3   /* call not valid in the current state (a0 != a_x)  */
#define COLA_EUNSUPPORTED -4   /* size without compiled FFT kernels                */
#define COLA_EHIP         -5   /* HIP runtime error (message in cola_last_error)   */
#define COLA_ENONFINITE   -6   /* non-finite value found (COLA_F_CHECK_FINITE)     */

#define COLA_F_CHECK_FINITE 1  /* after each step, check the state for NaN/Inf */
#define COLA_F_STAGE_TIMERS 2  /* record HIP events around every stage of cola_step */
#define COLA_F_D2_ODE       4  /* second-order growth D2 from its growth equation,
                                  d/dt(a^2 dD2/dt) = alpha (D2 - D1^2), instead of the
                                  fit -(3/7) D1^2 Omega(a)^(-1/143) of Sec. 2.1 (they
                                  differ by 2e-4 at a = 1 for Omega_m = 0.27)      */

/* Stages timed under COLA_F_STAGE_TIMERS (index into cola_stage_times). */
#define COLA_STAGE_SORT      0  /* tile sort: bucket counts, scan, scatter          */
#define COLA_STAGE_DEPOSIT   1  /* deterministic CIC gather                          */
#define COLA_STAGE_FFT_Z     2  /* forward real-to-complex pass along z              */
#define COLA_STAGE_FFT_Y     3  /* forward pass along y                              */
#define COLA_STAGE_FFT_X     4  /* x pass: forward, Green's function, 2 inverses     */
#define COLA_STAGE_IFFT_Y    5  /* inverse y pass of the x force component           */
#define COLA_STAGE_IFFT_Z    6  /* inverse complex-to-real pass along z, 3 meshes    */
#define COLA_STAGE_KICKDRIFT 7  /* CIC readout fused with kick and drift             */
#define COLA_STAGE_IFFT_Y_GRAD 8  /* inverse y pass giving the y and z components    */
#define COLA_STAGE_VELOCITY  9  /* cola_velocity / cola_snapshot particle kernel      */
#define COLA_NSTAGE          10

typedef struct cola_ctx cola_ctx;

/* Run parameters.  Cosmology is flat LCDM, Omega_Lambda = 1 - omega_m
 * (Sec. 1).  np and nmesh must be one of the compiled FFT sizes
 * {16, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048}
 * (COLA_EUNSUPPORTED otherwise), with nmesh >= 32 and nmesh >= np, and at
 * most 2^30 particles (np <= 1024; COLA_EUNSUPPORTED otherwise). */
typedef struct cola_params {
  int32_t np;              /* particles per side                                   */
  int32_t nmesh;           /* PM mesh per side                                     */
  double  box;             /* periodic box side [Mpc/h]                            */
  double  omega_m;         /* matter density parameter                             */
  double  n_lpt;           /* kick/drift ansatz exponent, Sec. 2.1 (paper: -2.5);
                              0: constant v_res in the drift, A + B ln a in the kick */
  double  a_init;          /* scale factor of the initial conditions               */
  int32_t flags;           /* COLA_F_* bits                                        */
  int32_t reserved;
} cola_params;

/* Fills p with defaults: omega_m 0.27, n_lpt -2.5, a_init 0.02, flags 0. */
void cola_params_default(cola_params* p, int32_t np, int32_t nmesh, double box);

/* Workspace the context needs, in bytes (alignment 256).  Sizes scale as
 * 4 meshes of nmesh^2 (nmesh + 2) floats plus 12 + 4 floats of particle
 * state and sort data per particle. */
int cola_workspace_query(const cola_params* p, size_t* bytes);

/* Creates a context that uses dev_workspace (>= cola_workspace_query bytes,
 * 256-byte aligned device memory, owned by the caller and kept alive until
 * cola_destroy) and enqueues all work on hip_stream (a hipStream_t; NULL =
 * the default stream).  Uploads FFT twiddle tables into the workspace. */
int cola_create(const cola_params* p, void* dev_workspace, size_t bytes,
                void* hip_stream, cola_ctx** out);
int cola_destroy(cola_ctx* ctx);

/* Initial conditions (Sec. 2.1 2LPT growing mode; Sec. 2.3 Gaussian initial
 * random modes).  dev_noise: np^3 float32 N(0,1) white noise, C order, device.
 * k[nk], pk[nk]: host tables of the z=0 linear P(k) [h/Mpc, (Mpc/h)^3], k
 * strictly increasing, pk > 0, nk >= 2; interpolated linearly in (ln k, ln P),
 * end segments extended.  Builds Psi1, Psi2 and sets displacement
 * d = D1(a_init) Psi1 + D2(a_init) Psi2, residual velocity 0, a_x = a_v =
 * a_init.  Reads dev_noise only during the call's stream work. */
int cola_init_2lpt_from_noise(cola_ctx* ctx, const float* dev_noise,
                              const double* k, const double* pk, int32_t nk);

/* Same, drawing the white noise on the GPU from a Philox4x32-10 stream
 * (Salmon et al. 2011; key = seed, counter = particle id) with the
 * Box-Muller transform.  box and np must equal the context's (COLA_EINVAL
 * otherwise); they are repeated to follow the method's problem statement. */
int cola_init_2lpt(cola_ctx* ctx, uint64_t seed, const double* k, const double* pk,
                   int32_t nk, double box, int32_t np);

/* Writes the np^3 white noise cola_init_2lpt(seed) would draw. */
int cola_noise(cola_ctx* ctx, uint64_t seed, float* dev_noise);

/* One COLA step a0 -> a1 (eqs. cola-kick and cola-drift): PM force at the
 * positions at a0; residual kick from a_v to (a0+a1)/2; drift of the
 * residual plus the 2LPT increment to a1.  Requires a0 == current a_x
 * (COLA_ESTATE otherwise) and a1 > a0. */
int cola_step(cola_ctx* ctx, double a0, double a1);

/* Density contrast delta = rho/rho_bar - 1 of the current positions on the
 * nmesh^3 mesh by the deterministic CIC deposit (Sec. 3.3 CIC), written to
 * dev_out (nmesh^3 float32, C order).  Bitwise reproducible: per cell the
 * weights are summed in ascending particle id, nodes add their 8 source
 * cells in a fixed order. */
int cola_density(cola_ctx* ctx, float* dev_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * density contrast of cola_density_of, computed without a context.  The
 * tile sort's buffers live in a static device array of 3.4 MB that each
 * device holds until the process ends; the call makes no allocation
 * (no hipMalloc, hipFree or host allocator) and enqueues the tile sort and
 * deposit kernels on hip_stream (a hipStream_t of the current device;
 * NULL = the default stream).  dev_disp: 3 * np^3 float32
 * displacements in mesh cells, the layout of cola_get_state; dev_out:
 * nmesh^3 float32, C order.  np a multiple of 16, nmesh a multiple of 16
 * with 32 <= nmesh and np <= nmesh (COLA_EINVAL otherwise); at most 64^3
 * particles and a 256^3 mesh (COLA_ENOMEM beyond).  Bitwise equal to
 * cola_density_of of a context with the same np and nmesh.  Every call on a
 * device shares that device's array: calls that overlap on one device (two
 * streams, or two host threads) race and must be serialised by the caller. */
int cola_density_noalloc(const float* dev_disp, int32_t np, int32_t nmesh, float* dev_out, void* hip_stream);

/* Matter power spectrum (Sec. 3.3): CIC onto ngrid^3 (a supported size,
 * 32 <= ngrid <= nmesh), FFT, divide by the CIC window, P = |delta_k|^2
 * / V over the half space {kz>0} U {kz=0,ky>0} U {kz=0,ky=0,kx>0} with
 * |k| <= pi ngrid / box, binned by k_edges[nbins+1] (h/Mpc, increasing; bin b
 * holds edges[b] <= |k| < edges[b+1]).  Host outputs: mean |k|, mean P and
 * mode count per bin; a bin without modes reports count 0 and NaN for its
 * mean |k| and P.  Synchronises the stream.  nbins <= 4096. */
int cola_pk(cola_ctx* ctx, int32_t ngrid, const double* k_edges, int32_t nbins,
            double* host_kmean, double* host_pk, int64_t* host_nmodes);

/* The same spectrum corrected for the CIC smoothing and aliasing together
 * by the procedure of Jing (2005, ApJ 620, 559), which Sec. 3.3 applies:
 * per bin, the mean raw |delta_k|^2 / V (no window division) over the mean,
 * over the bin's modes, of the window's image sum
 *   C(k; s) = sum_m W^2(k + 2 k_N m) (|k + 2 k_N m| / |k|)^s,
 * W = prod sinc^2 (CIC), k_N = pi ngrid / box, |m_e| <= 2 images per axis,
 * s the local log-log slope of the corrected spectrum between the bin's
 * non-empty neighbours (one-sided at the ends, 0 for a lone bin) limited to
 * [-3, 1], starting from 0 and iterated 8 times.  Same arguments, outputs,
 * empty-bin NaNs and synchronisation as cola_pk. */
int cola_pk_jing(cola_ctx* ctx, int32_t ngrid, const double* k_edges, int32_t nbins,
                 double* host_kmean, double* host_pk, int64_t* host_nmodes);

/* Snapshot at a_s inside the coming step a_x -> a1 (a_x <= a_s <= a1),
 * without changing the state (Sec. 2.2, eqs. ansatz-drift and cola-drift;
 * the paper interpolates its snapshots this way): the step's kick takes
 * v_res to a_h = (a_x + a1)/2 with the force at the current positions, the
 * residual velocity then decays as (a/a_h)^n_LPT and the position follows
 * its drift integral to a_s; the 2LPT part is taken at a_s.  Writes the
 * displacement to dev_disp and the canonical velocity to dev_vel (3 * np^3
 * float32 each, the layout and units of cola_get_state) and, if dev_sdisp
 * is not NULL, the redshift-space displacement along rsd_axis as
 * cola_velocity does.  At a_s = a1 the displacement is the one cola_step
 * would produce (to rounding); at a_s = a_x it is the current one.  The
 * velocity at a_x differs from cola_velocity's (the drift ansatz against
 * the kick ansatz, two interpolants of the paper).  Runs the force
 * pipeline (the force meshes are overwritten).  Outputs must differ and not
 * overlap the workspace.  Errors: COLA_EINVAL for NULL outputs, equal
 * outputs, a1 <= a_x, a_s outside [a_x, a1] or a bad axis; COLA_ESTATE
 * without a particle state. */
int cola_snapshot(cola_ctx* ctx, double a1, double a_s, float* dev_disp, float* dev_vel, float* dev_sdisp,
                  int32_t rsd_axis);

/* cola_density and cola_pk of another displacement field on the same
 * particle lattice: dev_disp holds 3 * np^3 float32 displacements in mesh
 * units, the layout of cola_get_state (for example the redshift-space
 * displacement of cola_velocity, Sec. 4.4).  Positions wrap periodically;
 * the particle state is not read or changed (the force meshes are
 * overwritten).  Same outputs, bounds and errors as cola_density / cola_pk,
 * COLA_EINVAL for a NULL dev_disp. */
int cola_density_of(cola_ctx* ctx, const float* dev_disp, float* dev_out);
int cola_pk_of(cola_ctx* ctx, const float* dev_disp, int32_t ngrid, const double* k_edges, int32_t nbins,
               double* host_kmean, double* host_pk, int64_t* host_nmodes);

/* Density and line-of-sight momentum spectra on the nmesh^3 mesh (the
 * paper's P_gu and P_uu of Sec. 5, for the matter).  The velocity is
 * cola_velocity's at the position time, expressed as the redshift-space
 * shift u = v_axis / (a adot) in Mpc/h; the fields are delta and the momentum
 * p = sum_p W u_p / nbar (nbar particles per cell on average), both by CIC
 * through the deterministic deposit and deconvolved like cola_pk.  Per bin
 * of k_edges (as cola_pk, same half space and |k| <= pi nmesh / box):
 * mean |k|, P_dd = <|delta|^2>/V, P_du = <sign(k_axis) Im(delta p*)>/V (the
 * line-of-sight cross term is odd in mu; folded onto mu >= 0, negative for
 * infall), P_uu = <|p|^2>/V, and the mode count; a bin without modes
 * reports count 0 and NaN.  axis in {0, 1, 2}; nbins <= 2048.  Runs the
 * force pipeline when a_v != a_x; overwrites the force meshes; synchronises
 * the stream. */
int cola_pk_velocity(cola_ctx* ctx, int32_t axis, const double* k_edges, int32_t nbins, double* host_kmean,
                     double* host_p_dd, double* host_p_du, double* host_p_uu, int64_t* host_nmodes);

/* Friends-of-friends groups of the current positions (Sec. 2.3: the halo
 * finder run on the fly; Sec. 3.1: linking length 0.2 times the mean
 * particle separation, 0.37 for 2LPT).  Two
 * particles are friends when their nearest-image separation is at most
 * b = b_frac * nmesh / np mesh cells (0 < b_frac < 0.5; the paper's 0.2);
 * groups are the connected components.  dev_labels (np^3 int32, device)
 * receives for every particle the smallest particle id of its group, so the
 * output is unique and reproducible.  The decision "separation <= b" is made
 * in float32: q = float(i nmesh)/float(np), x = q + d, dx = x_a - x_b,
 * dx -= nmesh rint(dx/nmesh), r2 = (dx0^2 + dx1^2) + dx2^2 <= float(b^2),
 * one rounding per operation.  dev_work: cola_fof_workspace_bytes bytes of
 * 256-byte aligned device memory, owned by the caller.  Overwrites the tile
 * sort's scratch (rebuilt by every deposit); synchronises the stream.
 * Errors: COLA_EINVAL (NULL pointers, b_frac out of range, misaligned
 * work), COLA_ENOMEM (work too small), COLA_ESTATE (no particle state, or a
 * union that exceeded its retry bound). */
int cola_fof_workspace_bytes(const cola_ctx* ctx, size_t* bytes);
int cola_fof(cola_ctx* ctx, double b_frac, int32_t* dev_labels, void* dev_work, size_t work_bytes);

/* Halo catalogue of cola_fof labels of the current positions (Sec. 2.3: halo
 * catalogues generated on the fly): the groups with at least min_members
 * particles, in increasing root id (the root is the group's smallest id).
 * host_n_halos receives their number; the device arrays (capacity max_halos,
 * caller-owned) receive the root, the member count, the centre of mass
 * dev_halo_pos[3 * max_halos] (component e of halo h at e * max_halos + h,
 * mesh units in [0, nmesh): the root's position plus the mean nearest-image
 * offset of the members from the root) and, if dev_vel (3 * np^3, e.g.
 * cola_velocity's output) is given, the mean velocity dev_halo_vel (same
 * layout; both or neither may be NULL).  Sums are 64-bit fixed point
 * (2^-20 cells, 2^-16 velocity units), so the result does not depend on the
 * order of the atomics.  dev_work: cola_fof_halos_workspace_bytes(min_members)
 * bytes, 256-byte aligned.  Synchronises the stream.  Errors: COLA_EINVAL
 * (NULL pointers, min_members < 1, a label outside [0, np^3)), COLA_ENOMEM
 * (work too small, or more halos than max_halos: host_n_halos then holds the
 * number needed), COLA_ESTATE (no particle state). */
int cola_fof_halos_workspace_bytes(const cola_ctx* ctx, int32_t min_members, size_t* bytes);
int cola_fof_halos(cola_ctx* ctx, const int32_t* dev_labels, const float* dev_vel, int32_t min_members,
                   int32_t max_halos, int32_t* host_n_halos, int32_t* dev_halo_root, int32_t* dev_halo_count,
                   float* dev_halo_pos, float* dev_halo_vel, void* dev_work, size_t work_bytes);

/* PM force F (mesh units) at the current positions, 3 * np^3 float32 into
 * dev_force; no state change (the force of Sec. 2.2 as used by cola_step). */
int cola_force(cola_ctx* ctx, float* dev_force);

/* The PM force meshes of a given density contrast (Sec. 2.2: F = -grad phi,
 * laplacian phi = (3/2) Omega_m a^-1 delta; the Green's function and
 * gradient readings of cola_step): g_d = IDFT[i k_d alpha DFT[delta] / k^2],
 * k = 0 -> 0, k_d zeroed on the Nyquist plane of axis d, in mesh units (the
 * meshes cola_step reads the force from).  dev_delta: nmesh^3 float32, C
 * order.  dev_g0, dev_g1, dev_g2: nmesh^3 float32 each, C order, for the
 * x, y, z components; any may be NULL (not written).  Uses the context's
 * meshes as scratch (no state change). */
int cola_pm_gradient(cola_ctx* ctx, double a, const float* dev_delta, float* dev_g0, float* dev_g1,
                     float* dev_g2);

/* Canonical particle velocity v = a^2 dx/dt at the position time a_x (Koda
 * et al. 2015, Sec. 2.1: residual velocity plus the time derivative of the
 * 2LPT trajectory, a^2 adot (D1' Psi1 + D2' Psi2); Sec. 2.2: the residual
 * velocity, held at the last half step a_v, is carried to a_x by the kick
 * ansatz with the force at the current positions) into dev_vel (3 * np^3
 * float32, the layout and mesh units of cola_get_state; time unit 1/H0).
 * If dev_sdisp is not NULL it also receives the redshift-space displacement
 * (Sec. 4.4, distant observer along box axis rsd_axis in {0, 1, 2}): the
 * displacement with v[rsd_axis] / (a adot) added to that component, the
 * other two copied; positions wrap periodically as everywhere.  When
 * a_v != a_x the force pipeline runs first (the force meshes are overwritten;
 * the particle state is not changed); at the initial state (a_v = a_x) no
 * force is needed.  dev_vel and dev_sdisp must not overlap each other or the
 * workspace.  Errors: COLA_EINVAL for a NULL dev_vel, equal output pointers
 * or a bad axis with dev_sdisp given; COLA_ESTATE without a particle state. */
int cola_velocity(cola_ctx* ctx, float* dev_vel, float* dev_sdisp, int32_t rsd_axis);

/* Copies the particle state out / in (device, 3 * np^3 float32 each, mesh
 * units).  Any pointer may be NULL to skip that array.  set_state also sets
 * a_x, a_v. */
int cola_get_state(cola_ctx* ctx, float* dev_disp, float* dev_vres,
                   float* dev_psi1, float* dev_psi2, double* a_x, double* a_v);
int cola_set_state(cola_ctx* ctx, const float* dev_disp, const float* dev_vres,
                   const float* dev_psi1, const float* dev_psi2, double a_x, double a_v);

/* In-place 3D real FFT on the context's FFT engine: dev_mesh holds an
 * n^3 real field in padded rows of 2 c floats, c = n/2 + 1 rounded up to a
 * multiple of 16 (n one of np, nmesh); forward (inverse = 0) leaves the
 * unnormalised half spectrum [x][y][0..n/2] as interleaved complex (the
 * columns beyond n/2 of a row are zero); inverse (1) maps it back without
 * the 1/n^3 factor; the real result depends only on columns 0 .. n/2. */
int cola_fft3d(cola_ctx* ctx, int32_t n, float* dev_mesh, int32_t inverse);

/* ---- Reverse mode (adjoint).  Cotangents are float32 device arrays in the
 * particle layout (3 * np^3, mesh units); the same conventions as above. */

/* Adjoint of one cola_step a0 -> a1 whose velocity was at a_v0 and whose
 * start positions (displacements) were dev_disp0.  On entry dev_dbar,
 * dev_vbar hold the cotangents of (displacement, residual velocity) at a1;
 * on return those at a0 (overwritten in place).  dev_psi1bar, dev_psi2bar
 * accumulate (+=) the cotangents of Psi1, Psi2.  Recomputes the PM force at
 * dev_disp0 (tile sort, deposit, FFTs), then: reverse kick/drift, readout
 * weight gradient, transposed readout as a deterministic weighted deposit,
 * transposed Green's function (-i k alpha / k^2; 3 forward, 1 inverse FFT)
 * and the deposit weight gradient.  Uses the context's Psi1, Psi2 (from the
 * last initial condition); does not change the particle state. */
int cola_step_adjoint(cola_ctx* ctx, double a0, double a1, double a_v0, const float* dev_disp0,
                      float* dev_dbar, float* dev_vbar, float* dev_psi1bar, float* dev_psi2bar);

/* Storing instead of recomputing the forces of the adjoint (a memory-for-
 * time trade of the reverse pass; the method's forces are those of the PM
 * step, Sec. 2.2 and 2.3).  A force slot holds the three real force-mesh
 * components of one step in the context's padded mesh layout;
 * cola_force_slot_bytes gives its size (3 nmesh^2 c complex float32, c as
 * for cola_fft3d: 5.7 GB at nmesh = 768).  The caller allocates and owns
 * slots (device memory, 256-byte aligned); the library keeps no pointer to
 * them between calls.
 *
 * cola_step_keep is cola_step (same result, bit for bit) with the step's
 * force pipeline run in dev_slot instead of the context's mesh region, so
 * the slot ends up holding the forces at the step's start positions; it
 * overwrites the whole slot.  cola_step_adjoint_kept is cola_step_adjoint
 * (same result, bit for bit) reading those forces from dev_slot instead of
 * recomputing them; dev_disp0 and a0 must be the start positions and time
 * of the step that filled the slot (not checked: other positions give the
 * adjoint of a different force).  The slot is only read.  Errors: EINVAL
 * for a null or misaligned slot, otherwise as cola_step / cola_step_adjoint. */
int cola_force_slot_bytes(const cola_ctx* ctx, size_t* bytes);
int cola_step_keep(cola_ctx* ctx, double a0, double a1, void* dev_slot);
int cola_step_adjoint_kept(cola_ctx* ctx, double a0, double a1, double a_v0, const float* dev_disp0,
                           const void* dev_slot, float* dev_dbar, float* dev_vbar,
                           float* dev_psi1bar, float* dev_psi2bar);

/* dev_dbar += d <delta_bar, delta(disp)> / d disp, where delta is the density
 * contrast cola_density computes at displacements dev_disp and dev_delta_bar
 * is an nmesh^3 float32 C-order mesh. */
int cola_density_adjoint(cola_ctx* ctx, const float* dev_disp, const float* dev_delta_bar,
                         float* dev_dbar);

/* dev_dbar += d (sum_b cbar_b P_b) / d disp for the estimator of cola_pk at
 * displacements dev_disp (ngrid, k_edges, nbins as for cola_pk; host_cbar has
 * nbins entries; bins with no modes contribute nothing).  Synchronises. */
int cola_pk_adjoint(cola_ctx* ctx, const float* dev_disp, int32_t ngrid, const double* k_edges,
                    int32_t nbins, const double* host_cbar, float* dev_dbar);

/* Adjoint of the 2LPT initial condition built from dev_noise (with the P(k)
 * table of the last cola_init_2lpt* call): given the cotangent dev_dbar0 of
 * the initial displacement and the accumulated dev_psi1bar, dev_psi2bar,
 * writes the cotangent of the white noise to dev_noise_bar (np^3).  The
 * initial residual velocity is zero and carries no dependence. */
int cola_init_2lpt_adjoint(cola_ctx* ctx, const float* dev_noise, const float* dev_dbar0,
                           const float* dev_psi1bar, const float* dev_psi2bar,
                           float* dev_noise_bar);

/* Host scalars of the step a_x -> a1 with velocity at a_v (FP64):
 * out[0..9] = alpha, D1(a_x), D2(a_x), D1(a1)-D1(a_x), D2(a1)-D2(a_x),
 * K (kick factor), I (drift factor), a_h, D1(a1), D2(a1). */
int cola_step_scalars(const cola_params* p, double a_x, double a_v, double a1, double* out);

/* FFT schedules.  A column pass (the y and x passes: transforms along
 * strided axes) launches one workgroup per block of W adjacent columns of a
 * plane.  Block order 1 hands each XCD (eight per device, each with its own
 * L2) a contiguous range of blocks, so neighbouring columns share an L2;
 * block order 0 keeps the hardware's round-robin assignment of workgroups
 * to XCDs.  The setting is process-wide per transform length n (a compiled
 * size) and pass kind: COLA_PASS_PLAIN (plain forward and inverse column
 * passes), COLA_PASS_GREEN (the x pass of the PM step: forward transform,
 * Green's function x ik, two inverse transforms), COLA_PASS_GRAD (the
 * inverse y pass giving the y and z force components).  It never changes a
 * result: each column is transformed by the same code on the same data,
 * only the workgroup that does it differs.  Default 1.  COLA_EINVAL for an
 * unknown length, kind or order. */
#define COLA_PASS_PLAIN 0
#define COLA_PASS_GREEN 1
#define COLA_PASS_GRAD  2
int cola_fft_set_schedule(int32_t n, int32_t pass, int32_t order);   /* order 0 or 1 */
int cola_fft_get_schedule(int32_t n, int32_t pass, int32_t* order);

/* Autotuner: times the three column-pass kinds of the PM step at the
 * context's mesh length (in the step's mesh layout) with block order 1 and
 * 0, reps launches each after one warm-up (HIP events on the context's
 * stream), and keeps the faster of each in the schedule table (block
 * order 1 unless order 0 is more than 2% faster).  Uses the
 * context's meshes as scratch (the particle state is not touched).
 * Synchronises.  best (may be NULL, 3 entries, by pass kind) receives the
 * choices, ms (may be NULL, 6 entries: kind-major, order 0 then 1) the time
 * per launch of each candidate. */
int cola_autotune(cola_ctx* ctx, int32_t reps, int32_t* best, double* ms);

/* Under COLA_F_STAGE_TIMERS: synchronises, then writes per-stage totals
 * (milliseconds, summed over the steps since the last call) to
 * ms[COLA_NSTAGE] and the launch count per stage to count[COLA_NSTAGE]
 * (either may be NULL), and resets the totals.  COLA_ESTATE without the flag. */
int cola_stage_times(cola_ctx* ctx, double* ms, int64_t* count);

int cola_synchronize(cola_ctx* ctx);
const char* cola_strerror(int code);
const char* cola_last_error(const cola_ctx* ctx);

/* ---- Batches of independent realisations (many mocks, e.g. the ensembles
 * behind the covariance matrices of Sec. 3; the batching itself is this
 * library's, not the paper's).
 *
 * A batch holds nmock contexts, one per entry of params[] (np and nmesh may
 * differ between mocks).  Mocks that share (np, nmesh, omega_m, n_lpt,
 * a_init) form a group whose workspaces sit at one fixed stride, so that
 * every kernel of the step covers the whole group in one launch; box may
 * differ within a group (the step works in mesh units).  The step launches
 * of all groups are captured once, at the first cola_batch_step, into one
 * HIP graph that reads the per-step scalars from device memory; every later
 * step writes those scalars (one small kernel per group) and launches the
 * graph, in which the groups are parallel branches.  A batched step runs
 * the same kernels in the same order on the same data as cola_step on each
 * mock alone, so its results are bitwise equal. */
typedef struct cola_batch cola_batch;

/* Workspace bytes for the batch (sum of the mocks' workspaces, 256-byte
 * aligned each).  Errors as cola_workspace_query for any entry. */
int cola_batch_workspace_query(const cola_params* params, int32_t nmock, size_t* bytes);

/* Creates the batch in the caller's device workspace (256-byte aligned,
 * >= the query; COLA_ENOMEM if smaller) on hip_stream.  The mocks'
 * contexts are owned by the batch: use them through cola_batch_mock for
 * initial conditions, outputs and single steps, never cola_destroy them.
 * COLA_F_STAGE_TIMERS is refused (COLA_EINVAL): events are not captured. */
int cola_batch_create(const cola_params* params, int32_t nmock, void* dev_workspace, size_t bytes,
                      void* hip_stream, cola_batch** out);
int cola_batch_destroy(cola_batch* batch);
int32_t cola_batch_size(const cola_batch* batch);     /* number of mocks           */
int32_t cola_batch_ngroups(const cola_batch* batch);  /* number of equal-size groups */
/* Context of mock i (caller's order), or NULL when i is out of range. */
cola_ctx* cola_batch_mock(cola_batch* batch, int32_t i);
/* enable = 0: enqueue the step's launches directly instead of the graph
 * (same kernels, same results; used to check graph replays). */
int cola_batch_set_graph(cola_batch* batch, int32_t enable);
/* Mocks per launch: 0 (default) steps each group in one launch per kernel;
 * bytes > 0 splits every group into consecutive chunks of
 * max(1, bytes / per-mock workspace) mocks, launched one after the other in
 * the same graph, so that a chunk's working set can stay in the GPU's
 * last-level cache from kernel to kernel.  Results do not depend on it. */
int cola_batch_set_chunk_bytes(cola_batch* batch, size_t bytes);
/* One COLA step a0 -> a1 of every mock.  Every mock must hold a state at
 * a_x = a0 (COLA_ESTATE otherwise) and the mocks of a group must share
 * their velocity time a_v.  Asynchronous unless COLA_F_CHECK_FINITE is set
 * for a mock. */
int cola_batch_step(cola_batch* batch, double a0, double a1);
int cola_batch_synchronize(cola_batch* batch);
const char* cola_batch_last_error(const cola_batch* batch);

#ifdef __cplusplus
}
#endif
#endif /* COLA_H */
