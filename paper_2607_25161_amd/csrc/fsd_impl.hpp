// Internal interfaces between the host orchestration (host.cpp) and the HIP
// kernels (k_*.hip).  Each .hip file defines its kernels and exports plain C++
// launch wrappers declared here; host.cpp never launches a kernel directly.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstddef>
#include <cstdint>
#include <tuple>
#include <utility>

namespace fsd {

// ---- timed launches ---------------------------------------------------------------------
// A timed call site arms a start/stop event pair; the next kernel launched through
// launch_k takes it, and hipExtLaunchKernel stamps the pair at that kernel's own start
// and end (events recorded around a launch would also count their marker packets).
struct LaunchEvents {
  hipEvent_t a = nullptr, b = nullptr;
  bool used = false;
  hipError_t status = hipSuccess;
};
extern thread_local LaunchEvents g_launch_events;

template <typename F, typename T, size_t... I>
hipError_t launch_ext(F k, dim3 grid, dim3 block, uint32_t shm, hipStream_t st, const LaunchEvents& e, T& args,
                      std::index_sequence<I...>) {
  void* ptrs[] = {static_cast<void*>(&std::get<I>(args))...};
  return hipExtLaunchKernel(reinterpret_cast<const void*>(k), grid, block, ptrs, shm, st, e.a, e.b, 0);
}

template <typename... P, typename... A>
inline void launch_k(void (*k)(P...), dim3 grid, dim3 block, uint32_t shm, hipStream_t st, A... a) {
  LaunchEvents& e = g_launch_events;
  if (e.a && !e.used) {
    e.used = true;
    std::tuple<P...> args{static_cast<P>(a)...};
    e.status = launch_ext(k, grid, block, shm, st, e, args, std::index_sequence_for<P...>{});
  } else {
    k<<<grid, block, shm, st>>>(static_cast<P>(a)...);
  }
}

constexpr int kMaxStages = 12;

// Mixed-radix plan of one 1D FFT length: n = prod(radix[0..nstage)).
struct FftPlan {
  int n;
  int nstage;
  int radix[kMaxStages];
  unsigned long long rcode;  // the radices again, 4 bits per stage (stage 0 lowest)
};

// LDS distance, in elements of elem_bytes, between the B lines that one workgroup of a z
// or y pass transforms.  Loading B consecutive x of a grid row puts neighbouring lanes on
// different lines, so with a stride of N (a multiple of the 64 banks' width for every even
// N) they would all hit one bank.  A stride S with S / t odd, t = max(1, E / B) and E the
// elements per bank row, sends the lanes of one LDS cycle to distinct banks.
__host__ __device__ inline int fft_line_stride(int N, int B, int elem_bytes) {
  if (B <= 1) return N;
  const int E = 256 / elem_bytes, t = E / B > 1 ? E / B : 1;
  int S = N;
  while (S % (2 * t) != t) ++S;
  return S;
}

// Constants of the wave-space (spectral Ewald) part of the mobility.
struct WaveParams {
  int n;            // grid points per side
  int support;      // Gaussian support P (points per side)
  double L, h;      // box side, grid spacing
  double alpha;     // spreading weight exp(-alpha |x - x_m|^2)
  double xi, eta_t; // splitting parameter and Gaussian split fraction eta~
  double a, eta;    // bead radius and viscosity
  double scale;     // h^6 / V * (normalisation of the two Gaussians)^2
  int brownian;     // 1: the z pass applies the square-root multiplier to grid noise
  const double* gam;  // device scalar: strain of the sheared lattice (nullptr: the cube); read
                      // at run time so captured graphs follow the strain; see launch_bead_positions
  // Green's multipliers by |m|^2 = m_x^2 + m_y^2 + m_z^2 on the cube (5 per entry: sinc(ka),
  // jv(ka), the solve's and the Brownian root's scalar factors, 1/|k|), or nullptr
  const double* gtab;
  // the same multipliers rounded to FP32, 8 per entry: sinc, jv, the solve's and the
  // Brownian root's factors, 1/|k|, then 3 unused (16-byte aligned rows), or nullptr
  const float* gtab32;
  // transform tiles (0: the default rules fft_lines_b / fft_green_rows): lines per workgroup
  // of the z and y passes, row pairs per workgroup of the x+Green pass
  int tile_b, tile_g;
};

// Constants of the real-space part.
struct RealParams {
  double L, a, eta;
  double r_cut;
  double inv_ht;    // 1 / table spacing
  int ntab;         // table nodes covering [0, r_cut] (plus 3 guard nodes)
  double self_t, self_r;
  const double* gam;  // device scalar: strain of the sheared lattice (nullptr: the cube)
};

// ---- geometry (k_geometry.hip) ----------------------------------------------------------
// Sheared lattice (Lees-Edwards) of strain gam: lattice vectors (L, 0, 0), (gam L, L, 0),
// (0, 0, L).  Bead positions pos4 are kept in sheared coordinates s = (x - gam y, y, z),
// each folded into [0, L); a pair's Cartesian separation is then
// (ds_x + gam ds_y, ds_y, ds_z) with ds the sheared difference plus the image shift n L.
// gam = 0 is the cube.
void launch_bead_positions(int nb, int na, const int* body, const double* xbody, const double* com,
                           const double* quat, double L, double gam, double* r4, double* pos4, hipStream_t st);
// centroids folded into [-L/2, L/2)^3 of the lattice of strain gam (crossing a y face moves x
// by -+gam L)
void launch_integrate(int na, const double* U, double dt, double L, double gam, double* com, double* quat,
                      hipStream_t st);
// com = wrap(com0 + h dq_t), quat = r(h dq_r) (x) quat0 (exact rotation), 6 dq per aggregate
void launch_displace(int na, const double* com0, const double* quat0, const double* dq, double h, double L,
                     double gam, double* com, double* quat, hipStream_t st);

// Neighbour lists in CSR form.  Column entries pack the bead index (22 bits)
// and the periodic image shift (3 x 3 bits, offset by 3).
struct NeighborWork;
NeighborWork* neighbor_work_create(int nb);
void neighbor_work_destroy(NeighborWork* w);
// Two phases: neighbors_count launches per-row counts and the scan into rowptr
// and copies the total to pinned memory (read it with neighbors_total once the
// stream has drained); neighbors_fill then writes the columns.
hipError_t neighbors_count(NeighborWork* w, int nb, const double* pos4, const int* body, double L, double gam,
                           double cutoff, bool exclude_same_body, int* rowptr, hipStream_t st);
long long neighbors_total(const NeighborWork* w);
hipError_t neighbors_fill(NeighborWork* w, int nb, const double* pos4, const int* body, double L, double gam,
                          double cutoff, bool exclude_same_body, const int* rowptr, uint32_t* col,
                          hipStream_t st);

void launch_lub_setup(int nb, const double* pos4, double L, double gam, const int* rowptr, const uint32_t* col,
                      double a, double eta, double eps_min, double r_pre, double rough_alpha,
                      double rough_h0, double* coef, double* rdiag, int* overlap_flag, hipStream_t st);
void launch_lub_strain(int nb, const double* pos4, const double* r4, double L, double gam, const int* rowptr,
                       const uint32_t* col, const double* coef, const double* E, double* f, hipStream_t st);
void launch_precond_factor(int na, const int* offsets, const double* r4, const double* rdiag,
                           double drag_t, double drag_r, double* lu, int* piv, int* singular,
                           hipStream_t st);

// ---- mobility (k_mobility.hip) ------------------------------------------------------------
template <typename R>
void launch_real_sum(int nb, const double* pos4, const double* lam, const int* rowptr,
                     const uint32_t* col, const R* table, const RealParams& rp, double* out,
                     bool accumulate, int lanes_per_row, hipStream_t st,
                     const int* skip = nullptr, const int* order = nullptr);
template <typename R>
void launch_spread(int nb, const double* pos4, const double* lam, const WaveParams& wp, R* grid,
                   hipStream_t st, const int* skip = nullptr);
// Spreading and interpolation on the grid of a sheared lattice (wp.gam): grid point
// (i, j, k) sits at sheared coordinates (i, j, k) h, and each grid row j takes the P x-points
// around its own centre p_x - gam (j h - p_y).  Spreading scatters with atomic adds into a
// zeroed grid; interpolation adds into out as launch_interp does (with V: + Sigma^T V).
template <typename R>
void launch_spread_sheared(int nb, const double* pos4, const double* lam, const WaveParams& wp, R* grid,
                           hipStream_t st, const int* skip = nullptr);
template <typename R>
void launch_interp_sheared(int nb, const double* pos4, const R* grid, const WaveParams& wp, double* out,
                           hipStream_t st, const int* skip, const int* body, const double* r4, const double* V);
// pass: 0, 1, 2 = transforms along x, y, z; -1 = all three
// the allocation-free in-place transform of an n^3 complex grid (n <= kNoAllocFftMax) on the
// caller's device buffer, its twiddles in a fixed device array of this GPU
constexpr int kNoAllocFftMax = 512;
constexpr int kMaxDevices = 64;
hipError_t launch_fft3d_noalloc(int n, int sign, double* data, const FftPlan& plan, hipStream_t st);
template <typename R>
void launch_fft3d(R* grid, int ncomp, size_t comp_stride, const FftPlan& plan, const R* twiddle,
                  int sign, hipStream_t st, int pass = -1, const int* skip = nullptr);
// Wave-space transforms, in place on the three packed complex grids (n <= 256):
// stage 0 z forward, 1 y forward, 2 x forward + Green's scaling + x inverse,
// 3 y inverse, 4 z inverse.
constexpr int kMaxGrid = 256;
template <typename R>
void launch_wave_fft(R* grid, const FftPlan& plan, const R* twiddle, const WaveParams& wp, int stage,
                     hipStream_t st, const int* skip = nullptr);
// Gaussian spreading as a gather over beads binned by grid block (no atomics).
struct SpreadPlan;
SpreadPlan* spread_plan_create(int nb, int n_grid, int support);  // nullptr if n_grid % 4 != 0
void spread_plan_destroy(SpreadPlan* sp);
hipError_t spread_plan_update(SpreadPlan* sp, const double* pos4, const WaveParams& wp, hipStream_t st);
template <typename R>
void launch_spread_gather(const SpreadPlan* sp, const double* lam, const WaveParams& wp, R* grid,
                          hipStream_t st, const int* skip = nullptr);
// The first pass of the saddle operator in one launch: the Sigma/lubrication reduction
// y2, the real-space sum out = M_r lam (overwritten) and the gather spreading of lam,
// which all read only the input.  Needs a plan with 8^3 blocks (spread_fuses).
struct RealArgs {
  int nb;
  const double4* pos;
  const int* rowptr;
  const uint32_t* col;
  RealParams rp;
  double* out;
  const int* order;
};
struct RigidArgs {
  int na;
  const int* offsets;
  const int* body;
  const double4* r4;
  const double* V;
  const int* lrow;  // nullptr: no lubrication
  const uint32_t* lcol;
  const double* coef;
  double* y2;
};
bool spread_fuses(const SpreadPlan* sp);
template <typename R>
void launch_spread_fused(const SpreadPlan* sp, const double* lam, const WaveParams& wp, R* grid, const R* table,
                         int lanes_per_row, const RealArgs& ra, const RigidArgs& ga, hipStream_t st,
                         const int* skip = nullptr);
// out += interpolated grid velocities; with V != nullptr also += Sigma^T V (rigid velocities)
// (sp != nullptr: beads in the plan's spatial order with its weights)
template <typename R>
void launch_interp(int nb, const double* pos4, const R* grid, const WaveParams& wp, double* out,
                   hipStream_t st, const int* skip = nullptr, const int* body = nullptr,
                   const double* r4 = nullptr, const double* V = nullptr, const SpreadPlan* sp = nullptr);
// the plan's sorted bead order (sorted index -> bead), nullptr without a plan
const int* spread_plan_order(const SpreadPlan* sp);

// ---- constraint, lubrication, preconditioner, Krylov vectors (k_solver.hip) ---------------
// Conservative bead-pair forces between beads of different bodies (Section 4.2): Hertz
// normal contact k_n delta^1.5 n, van der Waals (Hamaker sphere-sphere, separation
// regularised h -> h + h_c, the force held at its contact value for h < 0) and the
// screened double layer, for pairs closer than r_cut, over the real-space list.
struct PairForceParams {
  double kn, hamaker, Z, kappa, hc, r_cut, a, L;
  double gam;  // strain of the sheared lattice
};
// fe[3 i] = (accumulate ? fe[3 i] : 0) - f_i  (the right-hand side takes -F_P through Sigma)
void launch_pair_forces(int nb, const double* pos4, const int* body, const int* rowptr, const uint32_t* col,
                        const PairForceParams& pf, double* fe, int accumulate, hipStream_t st);
// *flag |= 1 when beads of different bodies in the real-space list are closer than 1.5 a
void launch_overlap_check(int nb, const double* pos4, const int* body, const int* rowptr, const uint32_t* col,
                          double L, double gam, double a, int* flag, hipStream_t st);
void launch_lub_apply(int nb, const int* rowptr, const uint32_t* col, const double* coef,
                      const double* wt, double* f, hipStream_t st, const int* skip = nullptr);
// fused: y2 = Sigma (lambda - R_nf Sigma^T V) with lubrication evaluated on the fly
// (lrow == nullptr: no lubrication)
void launch_agg_lub(int na, const int* offsets, const int* body, const double* r4, const double* lam,
                    const double* V, const int* lrow, const uint32_t* lcol, const double* coef, double* y2,
                    hipStream_t st, const int* skip = nullptr);
// z = P^-1 r; with scal != nullptr, r = scal[0] * src is formed on the fly and stored to vout
void launch_precond_fused(int nb, int na, const int* offsets, const double* r4, const double* lu, const int* piv,
                          double drag_t, double drag_r, const double* src, const double* scal, double* vout,
                          double* z, hipStream_t st, const int* skip = nullptr);
void launch_rhs(int nb, int na, const int* offsets, const int* body, const double* r4,
                const double* E, const double* force, const double* fnf, double* b1, double* e3,
                hipStream_t st);
void launch_rhs_agg(int na, const int* offsets, const double* r4, const double* force,
                    const double* flub_e, double* b2, hipStream_t st);
void launch_add_ambient(int na, const double* V, const double* com, const double* G,
                        const double* W, double* U, hipStream_t st);

// GMRES cycle state kept on the device so the host synchronises once per batch
// of iterations, not once per iteration.
struct GmresCtl {
  int stop;       // 1: no further Arnoldi steps in this cycle (kernels of later steps return early)
  int k_used;     // Arnoldi steps completed in this cycle
  int its;        // iterations in this solve
  int breakdown;  // Krylov space exhausted (happy breakdown)
  int maxit, m;
  double bn;      // ||b||
  double beta;    // ||r|| at the start of the cycle
  double resid;   // Givens estimate |g_k| / ||b|| (true residual at a cycle start)
  double tol;
};
void launch_gmres_begin(GmresCtl* ctl, const double* rr, double* g, double* scal, hipStream_t st);
// fresh solve: ctl->bn = sqrt(bb), its = 0, tolerance, budget, restart length
void launch_gmres_init(GmresCtl* ctl, const double* bb, double tol, int maxit, int m, hipStream_t st);
// Arnoldi step j of the cycle: Hessenberg column from the two Gram-Schmidt passes and the
// new norm, Givens rotations, residual estimate, stop flag, scal = 1 / H[j+1, j]
struct ArnoldiArgs {
  int j;
  GmresCtl* ctl;
  const double* h1;
  const double* h2;
  double *H, *cs, *sn, *g, *scal;
};
void launch_arnoldi_step(const ArnoldiArgs& a, const double* hn2, hipStream_t st);
void launch_gmres_solve(const GmresCtl* ctl, const double* H, const double* g, double* y, hipStream_t st);
void launch_basis_combine(size_t n, int m, const double* V, size_t ldv, const double* y, const GmresCtl* ctl,
                          double* out, hipStream_t st);

// one-launch CGS kernels for any restart length (counters: zeroed device tickets, one per chunk of 8 vectors)
void launch_dots(size_t n, int nq, const double* V, size_t ldv, const double* w, double* partial, double* out,
                 unsigned* counters, hipStream_t st, const int* skip = nullptr);
// w -= V h; then mode 0: out[q] = V_q . w (q < nq), mode 1: out[0] = w . w
void launch_axpy_dots(size_t n, int nq, const double* V, size_t ldv, const double* h, double* w, int mode,
                      double* partial, double* out, unsigned* counters, hipStream_t st,
                      const int* skip = nullptr);
// CGS2 passes with the basis held in registers work for nq <= 32 basis vectors (cgs_fits),
// on cgs_blocks(n) workgroups
bool cgs_fits(int nq);
int cgs_blocks(size_t n);
// The same passes as a chain without fences or tickets (one system): each pass writes only
// its workgroup partial sums pout[q * cgs_blocks(n) + block]; the next launch's workgroups
// each add the previous pass's partials pin in a fixed order (mode 1: h1, mode 2: h2, the
// inner products of this step's column; workgroup 0 stores them to hout), and
// launch_arnoldi_reduce adds the mode-2 partials (w.w) and runs the Arnoldi update.  The
// three partial arrays must not overlap (nq * cgs_blocks(n) doubles each).
void launch_cgs_chain(int mode, size_t n, int nq, const double* V, size_t ldv, const double* pin, double* w,
                      double* pout, double* hout, hipStream_t st, const int* skip);
void launch_arnoldi_reduce(const ArnoldiArgs& a, const double* pin, int nblk, double* hn2, hipStream_t st);
// the preconditioner of step j+1 (z = P^-1 v, v_(j+1) = w / ||w|| stored to vout) with step
// j's Arnoldi update (a.j = j; ||w||^2 partials pin of nblk workgroups) folded in
void launch_precond_arnoldi(int nb, int na, const int* offsets, const double* r4, const double* lu, const int* piv,
                            double drag_t, double drag_r, const double* src, double* vout, double* z,
                            const ArnoldiArgs& a, const double* pin, int nblk, double* hn2, hipStream_t st,
                            const int* skip);
// *p = v (a one-thread kernel, so it is ordered on the stream like the kernels around it)
void launch_set_value(double* p, double v, hipStream_t st);
void launch_axpby(size_t n, double a, const double* x, double b, double* y, hipStream_t st);
// translational rigid-body bead velocities U + Omega x r from the aggregate vector V
void launch_bead_rigid_vel(int nb, const int* body, const double* r4, const double* V, double* w, hipStream_t st);
// S_j = sum_i sym(r_i (F_i + f_i)) per aggregate (9 each); f may be null
void launch_stresslets(int na, const int* offsets, const double* r4, const double* F, const double* f, double* S,
                       hipStream_t st);
// Lanczos step k: alpha[k] = h1[k] + h2[k], beta[k] = sqrt(nrm2[0]), scal[0] = 1 / beta[k]
void launch_lanczos_coef(int k, const double* h1, const double* h2, const double* nrm2, double* alpha, double* beta,
                         double* scal, hipStream_t st);
void launch_scale_dev(size_t n, const double* a, const double* x, double* y, hipStream_t st);  // y = a[0] x

// ---- Brownian terms (k_brownian.hip) ------------------------------------------------------
// Noise stream: Philox4x64-10 under key (k0, k1); normal e of the stream comes from the
// counter (e / 4 + 1, purpose, step, 0).
struct NoiseKey {
  uint64_t k0, k1, purpose, step;
};
void launch_philox_raw(uint64_t k0, uint64_t k1, const uint64_t ctr[4], int nblk, uint64_t* out, hipStream_t st);
void launch_normals(size_t n, const NoiseKey& nk, double* out, hipStream_t st);
// real white noise (3 components per grid point) into the real parts of the three
// complex grids, from the stream or from src (3 N^3 values, component-major)
void launch_noise_grid(int N, const NoiseKey& nk, const double* src, double* grid, hipStream_t st);
void launch_scale(size_t n, double a, const double* x, double* y, hipStream_t st);       // y = a x
void launch_combine(size_t n, int k, const double* V, size_t ldv, const double* c, double* out,
                    hipStream_t st);                                                       // out = V c
void launch_take_trans(int nb, const double* v6, double* t3, hipStream_t st);
void launch_sub(size_t n, const double* b, const double* ax, double* r, hipStream_t st);
void launch_zero(void* p, size_t bytes, hipStream_t st);  // bytes a multiple of 4
void launch_timing_mark(hipStream_t st);  // empty kernel bracketing timed launches

// ---- multi-system launches --------------------------------------------------------------
// Many independent systems advance their Arnoldi steps in lock step; each kernel of the
// step is one launch over all of them.  Block b of a launch belongs to the system s with
// off[s] <= b < off[s+1] (prefix sums of the per-system block counts); the block runs the
// single-system kernel body with that system's pointers and parameters.  Systems whose
// GMRES cycle has stopped return at once (their stop flag), as in the single-system path.
struct BatchDesc {
  int nb, na;
  size_t n;
  const double* pos4;
  const double* r4;
  const int* body;
  const int* offsets;
  // real-space pair sum
  const int* nrow;
  const uint32_t* ncol;
  const double* tab64;
  const float* tab32;
  RealParams rp;
  // wave space
  WaveParams wp;
  FftPlan plan;
  const double* tw64;
  const float* tw32;
  void* grid;
  int bl;  // lines per workgroup of the z and y passes
  int bg;  // row slots per workgroup of the x+Green pass
  // gather spreading (8^3 blocks): per-block candidate lists
  const int* blk_start;
  const int* blk_end;
  const int* cand;
  const int* bin_start;
  const int* bin_end;
  const int* perm;
  const int4* starts;
  const double* w64;
  const float* w32;
  int nbin, K, C;
  // lubrication and preconditioner
  const int* lrow;
  const uint32_t* lcol;
  const double* lcoef;
  const double* lu;
  const int* piv;
  double drag_t, drag_r;
  // Krylov state: the step maps z -> w; V = basis
  double *basis, *z, *w, *r, *scal, *part, *h1, *h2, *hn2, *H, *gcs, *gsn, *g;
  unsigned* counters;
  GmresCtl* ctl;
  int ncgs;  // CGS workgroups (cgs_blocks(n))
};

enum BatchKind {
  BK_PRECOND = 0,
  BK_REAL,
  BK_SPREAD,
  BK_FFT_OUTER,  // first and last transform passes (z)
  BK_FFT_MID,    // y passes
  BK_FFT_GREEN,  // x transforms with the Green's-function scaling
  BK_INTERP,
  BK_AGG,
  BK_CGS,
  BK_COUNT,
  // launch kinds with the block table of another kind: the folded preconditioner and
  // Arnoldi update (BK_PRECOND's table), the segment's last Arnoldi update (one per system)
  BK_PRECOND_ARNOLDI = BK_COUNT,
  BK_ARNOLDI
};

// FFT blocking used by both the single-system and the multi-system launches
int fft_lines_b(int N, int rbytes);  // lines per workgroup of the z/y passes (rbytes: 8 FP64, 4 FP32)
int fft_green_rows(int N);           // row slots per workgroup of the x+Green pass
// the tiles a system's transforms run with (its overrides, else the rules), and whether a
// tile fits: B divides N, and the LDS of either pass stays within 64 KB
int lines_b_of(const WaveParams& wp, int rbytes);
int green_g_of(const WaveParams& wp);
bool tile_b_fits(int N, int B, int rbytes);
bool tile_g_fits(int N, int G, int rbytes);
// fill the spreading fields of d from a gather plan (d.wp must be set first)
void spread_plan_desc(const SpreadPlan* sp, int prec, BatchDesc& d);
// per-system block counts of each kind and the dynamic LDS the kinds need (prec: 0 FP64, 1 FP32)
int batch_blocks(const BatchDesc& d, int kind);
size_t batch_shm(const BatchDesc& d, int kind, int prec);
// one multi-system launch; stage: FFT stage 0..4 for the FFT kinds, j: Arnoldi step for
// the preconditioner and CGS kinds (mode 0..2 in cgs_mode)
void launch_batch_mobility(int kind, int prec, int stage, const BatchDesc* D, const int* off, int nsys, int total,
                           size_t shm, hipStream_t st);
void launch_batch_gather_stop(const BatchDesc* D, int nsys, int* out, hipStream_t st);
void launch_batch_solver(int kind, int j, int cgs_mode, const BatchDesc* D, const int* off, int nsys, int total,
                         hipStream_t st);

}  // namespace fsd
