/*
 * fsd.h -- fast Stokesian dynamics of rigid bead aggregates on one MI355X GPU.
 *
 * The library solves, per time step, the aggregate saddle-point system of
 * Section 2.3.3 (Eq. `spm_agg`) at force-torque level:
 *
 *   [ M      Sigma^T ] [ F ]   [ (E r_i + u_B, w_B)_i                       ]
 *   [ Sigma  -R_agg  ] [ V ] = [ -(F_P + Sigma F_B,nf + R_FE : E_inf)_j     ]
 *
 * with M the periodic force-torque RPY mobility of the beads (positively split
 * Ewald: real-space pair sum + Gaussian spreading / 3D FFT / Green's scaling /
 * interpolation), R_nf the near-field lubrication between beads of different
 * bodies, Sigma the geometric constraint of Eq. `sigma`, R_agg = Sigma R_nf
 * Sigma^T, and V = U - U_inf the aggregate velocity relative to the imposed
 * flow.  R_FE : E_inf (Eq. `FH_agg`) is the near-field force on the bodies when each
 * moves with the imposed flow at its centroid: every inter-body bead pair resists the
 * relative velocity of its bead centres less the imposed rotation's share, so the
 * lab-frame rate at which a near-contact gap closes is what lubrication acts on.  GMRES (Algorithm 1, step 4) with the block-triangular preconditioner
 * of Section 2.3.3 (per-aggregate LU of the block-diagonal Schur
 * approximation, Algorithm 1 step 1) solves it; Eqs. `EM1`-`EM3` advance the
 * bodies (Algorithm 1, step 5).
 *
 * Conventions
 *  - Units are any consistent set; lengths, viscosity and forces as given.
 *  - Every function returns an fsd_status: 0 on success, negative on error.
 *    No function aborts or throws.  fsd_last_error() describes the last error
 *    of a system.
 *  - Host arrays passed in are borrowed for the duration of the call and
 *    copied; outputs are written to caller buffers.  Pointers documented as
 *    "device" must be device memory of the system's GPU; they are used on the
 *    system's HIP stream.
 *  - The primary periodic box is [-L/2, L/2)^3.  Aggregate centroids are kept
 *    wrapped into it; U_inf at a centroid X is grad_u . X.
 *  - Vectors of bead (force, torque) or (velocity, angular velocity) are 6
 *    doubles per bead, force/velocity first.  Aggregate vectors likewise, 6
 *    per aggregate.  Quaternions are (w, x, y, z).
 *  - One fsd_system must not be used from two threads at once; distinct
 *    systems may run concurrently on distinct streams.
 */
#ifndef FSD_H
#define FSD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsd_system fsd_system;

typedef enum {
  FSD_OK = 0,
  FSD_EINVAL = -1,    /* invalid argument; outputs untouched                       */
  FSD_ENOMEM = -2,    /* device allocation failed                                  */
  FSD_ENOCONV = -3,   /* GMRES hit gmres_maxit; outputs hold the last iterate      */
  FSD_EDEVICE = -4,   /* a HIP call failed                                         */
  FSD_ESTATE = -5,    /* call out of order (e.g. solve before init_aggregates)     */
  FSD_EOVERLAP = -6,  /* two beads of different bodies overlap by more than a/2    */
  FSD_EBUSY = -7      /* resource exhausted (batch slots or memory budget)         */
} fsd_status;

typedef enum { FSD_FP64 = 0, FSD_MIXED = 1 } fsd_precision;

/* Solver and physics parameters.  fsd_default_params() fills every field. */
typedef struct {
  double eta;            /* fluid viscosity                                            */
  double radius;         /* bead radius a                                              */
  double kT;             /* thermal energy (0: deterministic)                          */
  double xi;             /* Ewald splitting parameter; <= 0: the cheapest of [25/L, 0.5/a]
                            under the Section 3.2 error rules (cost model of the pair
                            sum against the grid passes)                              */
  double ewald_tol;      /* truncation tolerance x_err of the cutoff rules (Sec. 3.2)  */
  int grid;              /* spectral grid points per side (2^a 3^b 5^c, at most 256); 0: from
                            the k_c rule                                              */
  int support;           /* Gaussian support P (points per side); 0: from ewald_tol    */
  double r_lub;          /* lubrication cutoff (3a); 0 disables lubrication            */
  double r_precond;      /* cutoff of the preconditioner's sparse lubrication (2.1a)   */
  double lub_eps_min;    /* smallest gap/a used in the lubrication functions (1e-3)   */
  double gmres_tol;      /* relative residual ||b - A x|| / ||b||                      */
  int gmres_restart;     /* Krylov dimension m of GMRES(m)                             */
  int gmres_maxit;       /* total inner iterations allowed per solve                   */
  int precision;         /* fsd_precision                                              */
  double lanczos_tol;    /* relative stopping tolerance of the Lanczos square roots of
                            the Brownian terms (1e-4)                                 */
  uint64_t seed;         /* key of the counter-based noise generator                   */
  int lanczos_maxit;     /* most Lanczos steps per square root (100, at most 2000); the
                            basis takes (lanczos_maxit + 1) 6 n_bead doubles           */
} fsd_params;

typedef struct {
  int status;                 /* fsd_status of the solve                              */
  int iterations;             /* GMRES iterations (inner iterations summed in MIXED)  */
  int restarts;               /* GMRES restarts                                       */
  int refinements;            /* FP64 residual replacements (MIXED restarts), 1 in FP64 */
  double rel_residual_fp64;   /* ||b - A x|| / ||b|| recomputed with the FP64 matvec  */
} fsd_solve_info;

/* Geometry and split actually used (after the parameter rules). */
typedef struct {
  double L, xi, r_cut, h, eta_tilde, self_t, self_r;
  int grid, support, n_bead, n_agg;
  long long nnz_real, n_lub_pairs;
} fsd_info;

void fsd_default_params(fsd_params* p);

/* Create a system on the current HIP device: the state of one simulation of
 * Algorithm 1 (a periodic suspension of rigid aggregates, Section 2.3) and the
 * solver settings p (copied).  hip_stream: a hipStream_t to run on (e.g.
 * torch.cuda.current_stream().cuda_stream) or NULL for a private stream.  The
 * system owns all of its device memory.  FSD_EINVAL for a NULL out or
 * parameters outside their ranges, FSD_EDEVICE if no stream can be made. */
fsd_status fsd_create(const fsd_params* p, void* hip_stream, fsd_system** out);

/* Periodic box of sides Lx, Ly, Lz (Section 2.3.1 works in a periodic box; the
 * rules of Section 3.2 size the grid per side).  This library takes cubes only:
 * FSD_EINVAL unless Lx == Ly == Lz > 0.  Call before fsd_init_aggregates. */
fsd_status fsd_init_box(fsd_system* s, double Lx, double Ly, double Lz);

/* Aggregates (Section 2.3.1): n_agg bodies; bead range of body j is
 * [bead_offsets[j], bead_offsets[j+1]); x_body (3 per bead) are body-frame
 * bead centres, re-centred by the callee to zero mean per body (the centroid is
 * the centre of mass); com (3 per body) is wrapped into the primary box; quat
 * (4 per body, (w,x,y,z)) is normalised by the callee.  Empty bodies and
 * zero-norm quaternions give FSD_EINVAL.  Allocates the system's device
 * memory (the only allocation besides neighbour-list growth). */
fsd_status fsd_init_aggregates(fsd_system* s, int32_t n_agg, const int32_t* bead_offsets,
                               const double* x_body, const double* com, const double* quat);

/* Applied force and torque per aggregate, 6 per body (F_P of Eq. `spm_agg`). */
fsd_status fsd_set_forces(fsd_system* s, const double* ft_agg);

/* Bead-level conservative forces, 3 per bead, projected as Sigma F_P
 * (Section 2.3.2; Algorithm 1, step 2).  Replaces the aggregate forces. */
fsd_status fsd_set_bead_forces(fsd_system* s, const double* f_bead);

/* Imposed linear flow u_inf(x) = grad_u . x, grad_u row-major with
 * grad_u[3*a+b] = d u_a / d x_b, traceless.  E_inf = sym(grad_u),
 * W_inf = curl(u)/2 (Eq. `gc`). */
fsd_status fsd_set_shear(fsd_system* s, const double grad_u[9]);

/* One saddle solve at the current configuration.  U_agg (6 per body, host) gets
 * U = V + U_inf; lambda_bead (6 per bead, host, may be NULL) gets the bead
 * force moments F.  info may be NULL.  FSD_ENOCONV leaves the last iterate. */
fsd_status fsd_solve(fsd_system* s, double* U_agg, double* lambda_bead, fsd_solve_info* info);

/* As fsd_solve with device output buffers, stream-ordered on the system stream. */
fsd_status fsd_solve_dev(fsd_system* s, double* d_U_agg, double* d_lambda, fsd_solve_info* info);

/* n_steps x (solve, explicit Euler update of Eqs. `EM1`-`EM3`).  last gets the
 * info of the final solve. */
fsd_status fsd_step(fsd_system* s, double dt, int n_steps, fsd_solve_info* last);

/* Current state, the variables Eqs. `EM1`-`EM3` advance: com (3 per body, the
 * centroids X_j, wrapped into the primary box), quat (4 per body, q_j), x_bead (3 per
 * bead, lab frame, unwrapped X_j + R(q_j) x_body, Eq. `EM3`; may be NULL).  Host
 * buffers; com and quat may be NULL too.  FSD_ESTATE before fsd_init_aggregates. */
fsd_status fsd_get_state(const fsd_system* s, double* com, double* quat, double* x_bead);

/* Aggregate velocities U = V + U_inf (6 per body, translation then rotation; the
 * unknowns of Eq. `spm_agg` plus the imposed flow) of the last completed solve of s,
 * whichever call made it (fsd_solve, fsd_step, fsd_batch_solve, fsd_batch_step).  Host
 * buffer.  FSD_ESTATE before any solve. */
fsd_status fsd_get_velocities(const fsd_system* s, double* U_agg);

fsd_status fsd_get_info(const fsd_system* s, fsd_info* info);

/* Constraint stresslets of the last solve (Section 3.1.4, Eq. `stress_comp`).  At the
 * force-torque level the beads carry no stresslet of their own, so an aggregate's particle
 * stress is its constraint stress S^C_j = sum_{i in j} sym(r_i f_i), r_i = x_i - X_j and f_i
 * the total force on bead i: the far-field hydrodynamic force (the force moments of the
 * solve), the lubrication force at the solved velocities (with its R_FE : E_inf part), the
 * conservative pair forces and, with kT > 0, the near-field Brownian force.  S_agg (9 per
 * body, row-major, may be NULL) gets S^C_j; S_mean (9, may be NULL) gets the suspension's
 * particle stress (1/V) sum_j S^C_j.  The FTS terms of Eq. `stress_comp` (the far-field
 * stresslets, R_SU and R_SE, the Brownian divergence) need the stresslet level, which this
 * library does not build.  Needs a completed solve at the current configuration
 * (fsd_solve or fsd_solve_dev; FSD_ESTATE after a step moved the bodies).  Allocates
 * 15 doubles per bead on first use. */
fsd_status fsd_get_stresslets(fsd_system* s, double* S_agg, double* S_mean);

/* Device bytes fsd_init_aggregates will allocate for a system of n_bead beads in
 * n_agg bodies in a cube of side L with parameters p: the spectral grid of the
 * Section 3.2 rules (or p->grid), the Krylov basis of GMRES(m) (Algorithm 1), the
 * per-body factors and the initial neighbour-list capacity.  For admission
 * decisions (the serving form); 0 for invalid arguments. */
size_t fsd_estimate_bytes(const fsd_params* p, int32_t n_bead, int32_t n_agg, double L);

/* Text of the last error of s; with s == NULL, of the calling thread's last failed
 * call that takes no system (fsd_fft3d).  Owned by the library. */
const char* fsd_last_error(const fsd_system* s);
void fsd_destroy(fsd_system* s);

/* Measured choice of the splitting parameter.  Section 3.2 runs two fixed policies (xi =
 * 0.5/a and 25/L) and notes that the better one depends on the system; any xi between
 * them meets the same error rules.  For each candidate in [xi_lo, xi_hi] (xi_lo itself and,
 * for every grid size the cutoff rule gives there, the largest xi that still gives it) a
 * scratch system with s's geometry, forcing and parameters is built and one saddle-operator
 * apply (Eq. `spm_agg`, in s's precision) is timed over reps back-to-back launches.  xi_out
 * gets the fastest candidate, ms_out (may be NULL) its time per apply; s is left unchanged
 * (create the system again with that xi to use it).  Allocates the scratch systems.
 * FSD_EINVAL unless 0 < xi_lo <= xi_hi and reps >= 1. */
fsd_status fsd_autotune_xi(fsd_system* s, double xi_lo, double xi_hi, int reps, double* xi_out, double* ms_out);

/* Measured tile shapes of the transform passes: the lines per workgroup of the z and y
 * passes (B, a divisor of the grid side) and the row pairs per workgroup of the x+Green pass
 * (G) are timed over reps back-to-back launches each (fsd_time_kernel) in the system's
 * precision, and the fastest are kept for every later launch of s (captured graphs are
 * rebuilt).  Both stay within 64 KB of LDS per workgroup.  lines_b and green_g (may be
 * NULL) get the choice.  The grid is left undefined, as by fsd_time_kernel. */
fsd_status fsd_autotune_tiles(fsd_system* s, int reps, int* lines_b, int* green_g);

/* ---- conservative bead-pair forces (Section 4.2, Eqs. `dlvo_potential` and the Hertz
 * contact force) ------------------------------------------------------------------------
 * Between beads of different bodies closer than r_cut (2a <= r_cut <= fsd_info.r_cut), with
 * r the centre distance, h = r - 2a and n the unit vector from the other bead:
 *   Hertz contact  f = k_n (2a - r)^1.5 n                                  for r < 2a;
 *   van der Waals  f = -dV/ds n, V(s) = -(A/6) [2a^2/(s^2 - 4a^2) + 2a^2/s^2
 *                                              + ln((s^2 - 4a^2)/s^2)],  s = max(r, 2a) + h_c
 *                  (separation regularised by h_c > 0; for r < 2a the force keeps its
 *                  contact value);
 *   double layer   f = -dV/dr n, V(r) = (a^2/r) Z exp(-kappa (r - 2a)).
 * The bead forces are summed into each body's force and torque (Sigma) and added to the
 * forces of fsd_set_forces at every solve, from the positions of that solve.  All three
 * coefficients zero switches the forces off (the default).  FSD_EINVAL for negative k_n
 * or A, A > 0 with h_c <= 0, Z != 0 with kappa <= 0, or r_cut outside the range. */
fsd_status fsd_set_pair_forces(fsd_system* s, double k_n, double hamaker, double Z, double kappa, double h_c,
                               double r_cut);

/* The conservative bead forces at the current positions (3 per bead, host array). */
fsd_status fsd_get_pair_forces(fsd_system* s, double* f_bead);

/* Sheared periodic lattice (Lees-Edwards), the boundary of long steady-shear runs
 * (Section 4.3).  At strain gamma the lattice vectors are (L, 0, 0), (gamma L, L, 0),
 * (0, 0, L): the image of a point across the +y face sits gamma L further along x.  Every
 * step advances gamma by G_xy dt (flow u_x = G_xy y) and keeps it in [-1/2, 1/2), the lattice
 * repeating with period 1; centroids crossing a y face move by -+gamma L along x.  The
 * mobility's Ewald sums run on this lattice (real-space images, and wave vectors
 * (2 pi / L)(m_x, m_y - gamma m_x, m_z) on a grid of sheared coordinates, sized
 * sqrt(5)/2 finer than the cube's so that its spectral cutoff holds at any strain), and
 * lubrication, pair forces and overlap checks take the nearest image on it; the Brownian
 * terms come from the same operators (grid noise through the sheared wave vectors, Lanczos
 * roots of the sheared real-space and near-field parts).  Switch it on after fsd_init_box
 * and before fsd_init_aggregates (FSD_ESTATE after); the strain may be reset at any time
 * while on.  Requires a velocity gradient with G_xy as its only non-zero entry (FSD_EINVAL
 * otherwise, also from a later fsd_set_shear).  Captured graphs read the strain from device
 * memory, so they follow it from step to step; a batch holding such a system runs every
 * system on its own stream (not the multi-system
 * launches).  enable 0 returns to the cube. */
fsd_status fsd_set_lees_edwards(fsd_system* s, int enable, double strain);

/* Warm starts (Algorithm 1 step 2): the initial guess of every GMRES solve of a full
 * right-hand side.  mode 0: zero (default).  mode 1: the last converged solution of such a
 * solve (lambda and V).  mode 2: the linear extrapolation 2 x_n - x_(n-1) of the last two.
 * mode 3: the quadratic one, 3 x_n - 3 x_(n-1) + x_(n-2).  Until enough solutions are held
 * the highest available order is used; the extrapolations assume steps of equal length.  The
 * first cycle forms the true residual b - A x0 as usual and the stopping test
 * ||b - A x|| <= gmres_tol ||b|| is unchanged, so only the iteration count differs.  Solves
 * of the drift right-hand sides start from zero.  Changing the mode forgets the stored
 * solutions; FSD_EINVAL for modes outside 0-3. */
fsd_status fsd_set_warm_start(fsd_system* s, int mode);

/* The current strain gamma in [-1/2, 1/2) (0 on the cube). */
fsd_status fsd_get_strain(const fsd_system* s, double* strain);

/* Surface roughness of lubrication (Section 4.2, Eq. `tan_fric`): for inter-body pairs with
 * gap h = r - 2a below the asperity height h0, the tangential (sliding) resistance function Y
 * gains alpha (a/h0)(h0/h - 3h/h0 + 2h^2/h0^2), which diverges as alpha a / h at contact and
 * switches on with zero value and slope at h0; h is floored at lub_eps_min * a like the other
 * functions.  The squeeze function is unchanged; the stresslet strengths (FE, SE) belong to
 * the FTS level, which this library does not build.  The correction enters the solves, the
 * preconditioner copy and the near-field Brownian force.  alpha = 0 switches it off (h0 is
 * then ignored); otherwise FSD_EINVAL unless lubrication is on (r_lub > 0), alpha > 0 and
 * 0 < h0 <= r_lub - 2a.  Default off. */
fsd_status fsd_set_roughness(fsd_system* s, double alpha, double h0);

/* ---- Brownian motion (kT > 0) --------------------------------------------------------
 * Eq. `SP2` and Algorithm 1 step 3: with kT > 0 every solve adds the Brownian slip
 * velocity u_B = sqrt(2 kT/dt) (M_r^{1/2} psi_r + M_w^{1/2} psi_w) to the bead rows of the
 * right-hand side and the near-field Brownian force F_B = sqrt(2 kT/dt) R_nf^{1/2} psi_nf,
 * projected by Sigma, to the aggregate rows (b2 = -(F_P + Sigma F_B + R_FE : E_inf)).
 * The wave-space part uses the exact square root of the positively split wave-space
 * operator applied to white noise on the grid; the real-space and near-field parts use
 * Lanczos square roots (params.lanczos_tol, at most params.lanczos_maxit steps).  The noise is drawn from
 * Philox4x64-10 keyed by (params.seed, stream) with counters (e/4 + 1, purpose, step, 0),
 * purpose 0 = grid, 1 = real space, 2 = near field; fsd_step advances step by one per
 * time step and sets dt. */

/* Brownian drift (Appendix A).  mode 1, random finite differences (Eq. `rfd`): every
 * fsd_step with kT > 0 first draws dq (6 per aggregate, Philox purpose 3 of the step),
 * solves the saddle system at the configurations displaced by +-(eps/2) dq (centroids
 * moved by (eps/2) dq_t, bodies turned by the exact rotation with rotation vector
 * (eps/2) dq_r) with right-hand side (0, -dq) and no other forcing, and adds
 * kT (U+ - U-) / eps to the aggregate velocities before the update; eps <= 0 selects
 * gmres_tol^(1/3) * radius.  mode 2, Fixman's midpoint scheme: after the step's solve at x,
 * U0 solves with that step's Brownian terms alone (u_B, -Sigma F_B; no ambient flow or other
 * forcing) at x and U' with the same terms at x + (dt/m) U0 (an Euler move), and
 * (m/2) (U' - U0) is added; the second argument is then m (<= 0: 100).  mode 0: off
 * (default).  fsd_batch_step applies it too, per system, around the batched solve (the
 * drift's own solves run on the system's stream). */
fsd_status fsd_set_drift(fsd_system* s, int mode, double eps);

/* The drift kT (U+ - U-) / eps at the current configuration (6 per aggregate, host), for
 * the given dq (6 per aggregate, host) or, with dq == NULL, for the dq of the next step.
 * Three solves' worth of work; leaves the configuration unchanged. */
fsd_status fsd_rfd_drift(fsd_system* s, const double* dq, double* u_drift);

/* Time step used by the Brownian amplitude, noise step index and noise stream id. */
fsd_status fsd_set_brownian(fsd_system* s, double dt, uint64_t step, uint64_t stream);

/* Caller-supplied noise for every following solve (NULL: draw that part from the
 * generator): psi_w 3 N^3 (component-major [c][z][y][x], N = fsd_info.grid),
 * psi_r 6 per bead, psi_nf 3 per bead.  Host buffers, copied. */
fsd_status fsd_set_noise(fsd_system* s, const double* psi_w, const double* psi_r, const double* psi_nf);

/* The Brownian terms of the next solve: u_B (6 per bead) and F_B (3 per bead, the
 * translational near-field force); lanczos_steps (2 ints, may be NULL) gets the
 * Lanczos steps of the real-space and near-field roots. */
fsd_status fsd_brownian_terms(fsd_system* s, double* u_B, double* f_B, int* lanczos_steps);

/* Raw Philox4x64-10 output of the device generator: block b (b < n_blocks) enciphers
 * the counter (counter[0] + b, counter[1], counter[2], counter[3]) under key (k0, k1);
 * out gets 4 words per block. */
fsd_status fsd_philox4x64(uint64_t k0, uint64_t k1, const uint64_t counter[4], int n_blocks, uint64_t* out);

/* n standard normals of stream (k0, k1, purpose, step): Box-Muller on pairs of open
 * (0, 1) uniforms made from the top 53 bits of each word. */
fsd_status fsd_normals(uint64_t k0, uint64_t k1, uint64_t purpose, uint64_t step, size_t n, double* out);

/* ---- operator access (host buffers), for verification and profiling ---------------- */

/* u = M lambda (6 per bead each).  parts: 1 real-space sum only, 2 wave-space
 * (spread/FFT/scale/IFFT/interpolate) only, 3 both.  precision: fsd_precision
 * (MIXED evaluates in FP32).  Section 2.2 far-field mobility. */
fsd_status fsd_apply_mobility(fsd_system* s, const double* lambda, double* u, int parts, int precision);

/* y = A x for the saddle matrix of Eq. `spm_agg`; x, y of length 6 (Nb + N),
 * beads first.  precision as above. */
fsd_status fsd_apply_saddle(fsd_system* s, const double* x, double* y, int precision);

/* z = P^-1 r, the block-triangular preconditioner (Section 2.3.3). */
fsd_status fsd_apply_precond(fsd_system* s, const double* r, double* z);

/* Right-hand side b of Eq. `spm_agg` (length 6 (Nb + N)). */
fsd_status fsd_get_rhs(fsd_system* s, double* b);

/* Real-space pair functions used by the sum at distances r (n values):
 * out[5*k + {0..4}] = (tt_I, tt_rr, rr_I, rr_rr, rt) as in M_real = tt_I I + tt_rr r^r^ ... */
fsd_status fsd_real_functions(fsd_system* s, int n, const double* r, double* out);

/* In-place 3D complex FFT of an n^3 grid (interleaved re/im doubles, x fastest),
 * forward (sign -1) or inverse (sign +1, unnormalised), with the library's
 * transform.  Host buffer; for verification of the FFT stages. */
fsd_status fsd_fft3d(int n, int sign, double* data);

/* The transform of fsd_fft3d on a device buffer, allocating nothing: for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  d_data: n^3 complex values (interleaved re/im
 * doubles, x fastest) in device memory of the current GPU, transformed in place, stream-
 * ordered on hip_stream (NULL: the null stream); the caller owns it.  The twiddle table
 * lives in a fixed device array of 2 x 512 doubles per GPU, held until the process ends, so
 * n is at most 512 (FSD_EINVAL beyond, or for n not a product of 2, 3 and 5; the text is in
 * fsd_last_error(NULL)).  Calls that overlap on one GPU race on that array: order them on
 * one stream.  FSD_EDEVICE if a launch fails. */
fsd_status fsd_fft3d_noalloc(int n, int sign, double* d_data, void* hip_stream);

/* ---- batches of independent systems (many small suspensions sharing the GPU) -------- */

/* A batch holds up to max_slots systems whose device memory counts against
 * mem_budget_bytes (fsd_estimate_bytes of each).  Systems stay owned by the caller
 * and keep their state, neighbour lists and factors resident between steps; give
 * each its own stream (fsd_create with NULL) so their work overlaps on the GPU. */
typedef struct fsd_batch fsd_batch;

/* hip_stream: the stream of the multi-system launches (NULL: a private stream owned
 * by the batch).  FSD_EINVAL for max_slots outside 1..4096. */
fsd_status fsd_batch_create(size_t mem_budget_bytes, int max_slots, void* hip_stream, fsd_batch** out);

/* Admit an initialised system into a free slot.  FSD_EBUSY if no slot is free or
 * the memory budget would be exceeded; slot receives the slot index. */
fsd_status fsd_batch_admit(fsd_batch* b, fsd_system* s, int* slot);

/* Free a slot (the system itself is not destroyed). */
fsd_status fsd_batch_retire(fsd_batch* b, int slot);

/* One saddle solve for every admitted system.  In the fused mode (the default, used
 * when all systems share precision and restart length <= 31 and have grids that are
 * multiples of 8) the Arnoldi steps of all systems run in lock step, one launch per
 * kernel over every system; otherwise each system runs on its own stream and the
 * host interleaves them.  A failing system records its status in its slot info and
 * does not stop the others; the return value is the first failure (or FSD_OK). */
fsd_status fsd_batch_solve(fsd_batch* b);

/* As fsd_batch_solve followed by the Euler update (Eqs. `EM1`-`EM3`) of every
 * system whose solve succeeded. */
fsd_status fsd_batch_step(fsd_batch* b, double dt);

/* As fsd_batch_step with a number of time steps per slot: n_steps has one entry per slot
 * (max_slots of fsd_batch_create; empty slots ignored, 0 leaves a system where it is), so a
 * small system can take several steps while a large one takes one.  The systems still
 * stepping run together, round by round; a slot whose solve fails stops there and keeps
 * its status.  FSD_EINVAL for a negative count. */
fsd_status fsd_batch_step_counts(fsd_batch* b, double dt, const int* n_steps);

/* Info of the last solve in a slot. */
fsd_status fsd_batch_slot_info(const fsd_batch* b, int slot, fsd_solve_info* info);

/* Bytes of the admitted systems (sum of their estimates). */
size_t fsd_batch_used_bytes(const fsd_batch* b);

/* Select multi-system launches (enable != 0, the default) or one stream per system. */
fsd_status fsd_batch_set_fused(fsd_batch* b, int enable);

/* Captured graphs for the multi-system launches (Section 2.5; enable != 0, the default):
 * each lock-step segment of Arnoldi steps (one launch per kernel over every system) is
 * captured on first use and replayed while the batch's tables stay the same (the same
 * systems iterating, the same tiles and LDS caps), so the first GMRES cycle of every time
 * step replays the same graphs; other systems sets are captured anew.  The timing pass
 * (fsd_batch_set_timing) launches eagerly.  enable == 0 launches every segment eagerly
 * and frees the captured graphs.  The results are the same either way. */
fsd_status fsd_batch_set_graphs(fsd_batch* b, int enable);

/* Event timing of the multi-system launches (fsd_timer classes; the Arnoldi steps of the
 * lock-step solve): while on, each launch is bracketed by HIP events on the batch stream,
 * the host checks the stop flags after every Arnoldi step, and each launch is credited
 * with the algorithmic bytes of the systems still iterating in it (the single-system
 * counts of that class).  Turning it on or off resets the accumulators. */
fsd_status fsd_batch_set_timing(fsd_batch* b, int enable);

/* Milliseconds, launches and algorithmic bytes per fsd_timer class accumulated since the
 * last fsd_batch_set_timing (FSD_TIMER_COUNT entries each; bytes may be NULL).
 * Synchronises the batch stream. */
fsd_status fsd_batch_get_timers(fsd_batch* b, double* total_ms, long long* launches, double* bytes);

/* Average duration (ms) of one multi-system launch of class timer (FSD_TIMER_REAL ..
 * FSD_TIMER_PRECOND) over every admitted system, replayed reps times back to back on the
 * batch stream between one pair of HIP events; bytes_per_launch (may be NULL) gets the
 * algorithmic bytes of that launch.  Needs systems that share multi-system launches
 * (FSD_ESTATE otherwise).  Builds lists and factors for moved positions first; leaves the
 * grids and scratch vectors undefined and the systems ready for their next solve. */
fsd_status fsd_batch_time_kernel(fsd_batch* b, int timer, int reps, double* avg_ms, double* bytes_per_launch);

/* Measured LDS caps of the multi-system transform launches (Section 2.5: the wave-space
 * passes of every admitted system in one launch).  Such a launch reserves its largest
 * system's LDS for every workgroup, so one system's wide tile lowers the occupancy of all.
 * For the z/y line passes and then the x+Green pass this times the launch
 * (fsd_batch_time_kernel, reps replays) with each system's tile narrowed to fit caps of
 * 16, 24, 32, 40 and 48 KB and with no cap, and keeps the fastest; later launches of the
 * batch use the caps.  lines_lds and green_lds (may be NULL) get them in bytes (0: no
 * cap).  Needs systems that share multi-system launches (FSD_ESTATE otherwise); leaves the
 * grids and scratch vectors undefined, as fsd_batch_time_kernel does. */
fsd_status fsd_batch_autotune_tiles(fsd_batch* b, int reps, size_t* lines_lds, size_t* green_lds);

/* Sets those caps directly (bytes; 0: no cap).  A system's tile is narrowed (halving the
 * lines per workgroup, or one row pair fewer) until its LDS fits, down to one line or one
 * pair whatever the cap.  The transforms compute the same values at any tile. */
fsd_status fsd_batch_set_lds_caps(fsd_batch* b, size_t lines_lds, size_t green_lds);

void fsd_batch_destroy(fsd_batch* b);

/* ---- kernel timing on the system stream (HIP events carried by each launch) -------- */

typedef enum {
  FSD_TIMER_REAL = 0,        /* real-space pair sum (its own launch outside the saddle
                                operator, or without a spreading plan)                    */
  FSD_TIMER_SPREAD = 1,      /* Gaussian spreading to the grid; in the saddle operator
                                with a spreading plan one launch (fsd::k_spread_fused)
                                also carries the real-space sum and the Sigma/lubrication
                                reduction, all timed here                                 */
  FSD_TIMER_FFT_FIRST = 2,   /* first transform pass (z lines)                            */
  FSD_TIMER_FFT_Y = 3,       /* y transform passes (2 per apply)                          */
  FSD_TIMER_GREEN = 4,       /* the pass with the Green's-function multiplier: x
                                transforms around it                                      */
  FSD_TIMER_FFT_LAST = 5,    /* last transform pass (inverse of the first)                */
  FSD_TIMER_INTERP = 6,      /* interpolation back to the beads, plus Sigma^T V           */
  FSD_TIMER_RIGID = 7,       /* Sigma reductions with the lubrication product (see REAL)  */
  FSD_TIMER_PRECOND = 8,     /* preconditioner apply (forms the next basis vector)        */
  FSD_TIMER_CGS_DOT = 9,     /* first Gram-Schmidt pass, h = V^T w                        */
  FSD_TIMER_CGS_UPDATE = 10, /* second pass: w -= V h with the new inner products         */
  FSD_TIMER_CGS_NORM = 11,   /* last update with ||w||^2 and the Arnoldi (Givens) update  */
  FSD_TIMER_COUNT = 12
} fsd_timer;

/* GMRES launch mode: enable = 1 replays cached HIP graphs (cycle start, batches of
 * `batch` Arnoldi steps, cycle end; default), 0 launches every kernel eagerly.
 * batch = 0 keeps the current batch size (default 8).  Graphs are rebuilt when
 * the neighbour-list storage or launch shapes change. */
fsd_status fsd_set_graphs(fsd_system* s, int enable, int batch);

/* Enable (1) or disable (0) per-kernel event timing and reset the accumulators.  While
 * timing is on, solves launch eagerly (no graphs), the real-space and wave-space parts of
 * the mobility run one after the other on the system stream, GMRES checks its stop flag
 * after every Arnoldi step (so no timed launch is one that returns at once), and each
 * timed kernel is launched with hipExtLaunchKernel carrying its start/stop events; those
 * intervals include the dispatch of the launch (a few microseconds).  Each change of the
 * setting launches one empty kernel (fsd::k_timing_mark), so a profiler trace shows which
 * launches were timed. */
fsd_status fsd_set_timing(fsd_system* s, int enable);

/* Accumulated milliseconds, launch counts and algorithmic HBM bytes (the minimum
 * traffic of each launch's inputs and outputs) per fsd_timer class since the last
 * fsd_set_timing; each array holds FSD_TIMER_COUNT entries, bytes may be NULL.
 * Synchronises. */
fsd_status fsd_get_timers(fsd_system* s, double* total_ms, long long* launches, double* bytes);

/* Average duration (ms) of one launch of the kernel behind timer class `timer`, in the
 * system's Arnoldi precision and launch configuration: the kernel is launched `reps`
 * times back to back on the system stream between one pair of HIP events, so the
 * dispatch of each launch overlaps the previous one.  Inputs are the system's current
 * scratch vectors; classes FSD_TIMER_REAL .. FSD_TIMER_PRECOND (the Gram-Schmidt classes
 * give FSD_EINVAL).  The spectral grid and the scratch vectors are left undefined (every
 * solve rewrites them); positions, lists and solution are untouched.  An empty kernel
 * (fsd::k_timing_mark) is launched before and after the replays.  Neighbour lists, the
 * spreading plan and the preconditioner factors are built first when the positions have
 * moved since they were.  Synchronises the system stream. */
fsd_status fsd_time_kernel(fsd_system* s, int timer, int reps, double* avg_ms);

#ifdef __cplusplus
}
#endif

#endif /* FSD_H */
