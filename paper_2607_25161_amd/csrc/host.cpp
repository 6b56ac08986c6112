// Host side of libfsd: parameter rules, the real-space function table, the
// saddle operator, the preconditioned GMRES solve, time stepping and the C ABI
// declared in include/fsd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <map>
#include <tuple>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "fsd.h"
#include "fsd_impl.hpp"
#include "tridiag.hpp"

using namespace fsd;

namespace {

struct HipError : std::runtime_error {
  explicit HipError(const std::string& m) : std::runtime_error(m) {}
};
struct ApiError : std::runtime_error {
  fsd_status code;
  ApiError(fsd_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

inline void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipError(std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPCHK(x) hip_check((x), #x)

template <typename T>
T* dalloc(std::vector<void*>& owned, size_t count) {
  if (count == 0) count = 1;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, sizeof(T) * count);
  if (e != hipSuccess) throw ApiError(FSD_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  owned.push_back(p);
  return static_cast<T*>(p);
}

// ---- spherical Bessel functions, stable near 0 ------------------------------------------
// j0(x), j1(x)/x, j1(x), j2(x): power series for x < 1, trigonometric forms above.
void sph_bessel(double x, double& j0, double& j1x, double& j1, double& j2) {
  if (x < 1.0) {
    const double y = -0.5 * x * x;
    // j_n(x) = x^n sum_k y^k / (k! (2n+2k+1)!!)
    double t0 = 1.0, t1 = 1.0 / 3.0, t2 = 1.0 / 15.0;
    double s0 = t0, s1 = t1, s2 = t2;
    for (int k = 1; k < 12; ++k) {
      t0 *= y / (k * (2.0 * k + 1.0));
      t1 *= y / (k * (2.0 * k + 3.0));
      t2 *= y / (k * (2.0 * k + 5.0));
      s0 += t0;
      s1 += t1;
      s2 += t2;
    }
    j0 = s0;
    j1x = s1;
    j1 = x * s1;
    j2 = x * x * s2;
  } else {
    const double s = std::sin(x), c = std::cos(x);
    j0 = s / x;
    j1 = s / (x * x) - c / x;
    j1x = j1 / x;
    j2 = (3.0 / (x * x) - 1.0) * s / x - 3.0 * c / (x * x);
  }
}

void sinc_jv_host(double x, double& s, double& j) {
  double j0, j1x, j1, j2;
  sph_bessel(x, j0, j1x, j1, j2);
  s = j0;
  j = 3.0 * j1x;  // jv(x) = 3 j1(x) / x
}

// ---- real-space smooth part ----------------------------------------------------------------
// S(r): inverse transform of the Hasimoto-damped FT-RPY multipliers
//   tt: sinc^2(ka) H(k) (I - kk)/k^2,  rr: jv^2(ka) H(k) (I - kk)/4,  rt: (i/2) sinc jv H [k]x / k^2,
//   H(k) = (1 + k^2/(4 xi^2)) exp(-k^2/(4 xi^2)).
// Angular integration leaves radial integrals of j0 - j1/x (I part), j2 (rr part) and
// k j1 (rt part).  The integrands are even, entire in k and Gaussian-decaying, so the
// trapezoid rule on a step below 2 pi / (band of the integrand) is spectrally accurate.
struct SmoothPart {
  std::vector<double> k, wtt, wrr, wrt;  // nodes and multiplier-times-weight
  double eta;
  SmoothPart(double a, double eta_, double xi, double rmax) : eta(eta_) {
    const double kmax = 2.0 * xi * std::sqrt(46.0);
    const double band = rmax + 2.0 * a + 7.0 / xi;
    const double hk = 2.0 * M_PI / band / 2.0;
    const int nk = int(std::ceil(kmax / hk)) + 1;
    for (int m = 0; m < nk; ++m) {
      const double kk = m * hk;
      const double q = kk * kk / (4.0 * xi * xi);
      const double H = (1.0 + q) * std::exp(-q);
      double s, j;
      sinc_jv_host(kk * a, s, j);
      const double w = (m == 0 ? 0.5 : 1.0) * hk;
      k.push_back(kk);
      wtt.push_back(w * s * s * H);
      wrr.push_back(w * 0.25 * kk * kk * j * j * H);
      wrt.push_back(w * kk * s * j * H);
    }
  }
  // out: (tI, tR, rI, rR, c) of S at distance r (r may be negative or zero)
  void eval(double r, double* out) const {
    double tI = 0, tR = 0, rI = 0, rR = 0, c = 0;
    const double ar = std::fabs(r);
    for (size_t m = 0; m < k.size(); ++m) {
      double j0, j1x, j1, j2;
      sph_bessel(k[m] * ar, j0, j1x, j1, j2);
      const double fI = j0 - j1x;
      tI += wtt[m] * fI;
      tR += wtt[m] * j2;
      rI += wrr[m] * fI;
      rR += wrr[m] * j2;
      c += wrt[m] * j1;
    }
    const double p = 1.0 / (2.0 * M_PI * M_PI * eta);
    out[0] = p * tI;
    out[1] = p * tR;
    out[2] = p * rI;
    out[3] = p * rR;
    out[4] = -(r < 0 ? -1.0 : 1.0) * c / (4.0 * M_PI * M_PI * eta);
  }
};

void rpy_free(double r, double a, double eta, double* o) {
  const double c8 = 1.0 / (8.0 * M_PI * eta);
  const double mt = 1.0 / (6.0 * M_PI * eta * a), mr = 1.0 / (8.0 * M_PI * eta * a * a * a);
  if (r >= 2.0 * a) {
    const double ir = 1.0 / r, ir2 = ir * ir;
    o[0] = c8 * ir * (1.0 + 2.0 / 3.0 * a * a * ir2);
    o[1] = c8 * ir * (1.0 - 2.0 * a * a * ir2);
    o[2] = -0.5 * c8 * ir * ir2;
    o[3] = 1.5 * c8 * ir * ir2;
    o[4] = -c8 * ir2;
  } else {
    const double s = r / a;
    o[0] = mt * (1.0 - 9.0 / 32.0 * s);
    o[1] = mt * 3.0 / 32.0 * s;
    o[2] = mr * (1.0 - 27.0 / 32.0 * s + 5.0 / 64.0 * s * s * s);
    o[3] = mr * (9.0 / 32.0 * s - 3.0 / 64.0 * s * s * s);
    o[4] = -0.5 * c8 / (a * a) * s * (1.0 - 3.0 / 8.0 * s);
  }
}

// ---- FFT plan ---------------------------------------------------------------------------------
bool make_plan(int n, FftPlan& p) {
  p.n = n;
  p.nstage = 0;
  p.rcode = 0;
  int m = n;
  for (int r : {8, 4, 2, 3, 5})
    while (m % r == 0 && p.nstage < kMaxStages) {
      p.rcode |= (unsigned long long)r << (4 * p.nstage);
      p.radix[p.nstage++] = r;
      m /= r;
    }
  return m == 1 && n >= 2;
}

// smallest 2^a 3^b 5^c >= n with a >= 3 (a multiple of 8, for the gather spreading blocks)
int next_smooth(int n) {
  for (int m = std::max(n, 8);; ++m) {
    if (m % 8) continue;
    int k = m;
    for (int r : {2, 3, 5})
      while (k % r == 0) k /= r;
    if (k == 1) return m;
  }
}

// Splitting parameter when the caller leaves it to the library: the Ewald error rule of
// Section 3.2 fixes R_c and k_c for a given xi, so the cost of one mobility apply is
// traded between the real-space pair sum (pairs ~ N (4 pi/3) R_c^3 n) and the grid
// passes (~ N_g^3 points).  The per-pair and per-point weights are the measured costs
// of the two FP64 paths on gfx950 (about 2 ps per pair term, 60 ps per grid point);
// candidates run over [25/L, 0.5/a], the two fixed policies of Section 3.2.
double pick_xi(const fsd_params& p, int nb, double L) {
  if (p.xi > 0) return p.xi;
  const double a = p.radius;
  const double hi = 0.5 / a;
  const double lo = std::min(hi, 25.0 / L);
  if (nb <= 0 || !(L > 0) || p.grid > 0) return hi;
  const double lnt = std::sqrt(-std::log(p.ewald_tol));
  const double dens = nb / (L * L * L);
  double best = hi, best_cost = 1e300;
  for (int k = 0; k <= 48; ++k) {
    const double xi = lo * std::pow(hi / lo, k / 48.0);
    const double rc = 1.15 * lnt / xi;  // the grown cutoff sits ~15% above the rule
    const int N = next_smooth(int(std::ceil((2.0 * lnt * xi + 1.0 / a) * L / M_PI)));
    if (N > kMaxGrid) continue;
    const double pairs = nb * (4.0 * M_PI / 3.0) * rc * rc * rc * dens;
    const double cost = 2e-12 * pairs + 6e-11 * double(N) * N * N;
    if (cost < best_cost) best_cost = cost, best = xi;
  }
  return best;
}

}  // namespace

// ==========================================================================================
// system
// ==========================================================================================

struct fsd_system {
  fsd_params p{};
  hipStream_t st = nullptr;
  bool solved = false;  // d_U holds the velocities of a completed solve of the full right-hand side
  double *d_fst = nullptr, *d_wst = nullptr, *d_sst = nullptr;  // stresslet scratch (allocated on first use)
  bool own_stream = false;
  hipStream_t st2 = nullptr;           // side stream: the real-space sum overlaps the wave space
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  unsigned* d_counters = nullptr;      // tickets of the one-launch reductions
  int device = 0;
  std::string err;

  double L = 0;
  int nb = 0, na = 0;
  bool have_box = false, have_agg = false, prepared = false;
  double G[9] = {0}, E[9] = {0}, W[3] = {0};

  RealParams rp{};
  WaveParams wp{};
  FftPlan plan{};
  int lpr = 4;
  double drag_t = 0, drag_r = 0;
  size_t n = 0;
  int m = 30;

  std::vector<int> h_offsets;
  std::vector<void*> owned;
  int *d_offsets = nullptr, *d_body = nullptr;
  double *d_xbody = nullptr, *d_com = nullptr, *d_quat = nullptr, *d_r4 = nullptr, *d_pos4 = nullptr;
  double *d_force = nullptr, *d_G = nullptr, *d_E = nullptr, *d_W = nullptr;
  double* d_tab64 = nullptr;
  float* d_tab32 = nullptr;
  int* d_nrow = nullptr;
  uint32_t* d_ncol = nullptr;
  long long ncap = 0, nnz = 0;
  int* d_lrow = nullptr;
  uint32_t* d_lcol = nullptr;
  double* d_lcoef = nullptr;
  long long lcap = 0, nlub = 0, lcoef_cap = 0;
  double *d_rdiag = nullptr, *d_lu = nullptr;
  int *d_piv = nullptr, *d_flags = nullptr;
  void* d_grid = nullptr;
  double* d_tw64 = nullptr;
  float* d_tw32 = nullptr;
  double *d_b = nullptr, *d_x = nullptr, *d_basis = nullptr, *d_z = nullptr, *d_w = nullptr, *d_t = nullptr;
  double *d_r = nullptr, *d_wt = nullptr, *d_fl = nullptr, *d_h = nullptr, *d_part = nullptr, *d_U = nullptr;
  double* h_small = nullptr;  // pinned
  GmresCtl* d_ctl = nullptr;   // device GMRES cycle state
  GmresCtl* h_ctl = nullptr;   // pinned mirror
  double *d_H = nullptr, *d_cs = nullptr, *d_sn = nullptr, *d_g = nullptr, *d_y = nullptr, *d_scal = nullptr;
  NeighborWork* nw = nullptr;   // real-space list workspace
  NeighborWork* nwl = nullptr;  // lubrication list workspace
  int* h_flags = nullptr;       // pinned: overlap, singular block (checked at the next sync)
  double* h_scal = nullptr;     // pinned: small reductions read by the host (outer residual)

  // resumable solve (state machine advanced after each stream synchronisation)
  struct SolveState {
    enum Phase { IDLE, PREP, START, BATCH, DONE } phase = IDLE;
    const double* b = nullptr;  // right-hand side of the GMRES in progress
    double* x = nullptr;        // its iterate
    bool fp32 = false;
    double tol = 0;
    int maxit = 0, j0 = 0;
    int its = 0, restarts = 0, outer = 0;
    double rel = 0;
    bool converged = false;
    // right-hand side: 0 the full one; 1 (0, -dq) of the random finite differences; 2 the
    // stored Brownian terms alone (Fixman).  Kinds 1 and 2 return V without ambient flow.
    int rhs_kind = 0;
    fsd_status status = FSD_OK;
  } sv;
  // Brownian terms (kT > 0): time step and noise stream of the next solve, optional
  // caller-supplied noise, the two right-hand-side vectors and the Lanczos workspace
  double bdt = 1e-3;
  uint64_t bstep = 0, bstream = 0;
  int lan_max = 100;
  int lan_its[2] = {0, 0};
  bool psi_w_set = false, psi_r_set = false, psi_nf_set = false;
  double *d_psi_w = nullptr, *d_psi_r = nullptr, *d_psi_nf = nullptr;
  double *d_ub = nullptr, *d_fb = nullptr, *d_lan = nullptr, *d_lc = nullptr, *d_u6 = nullptr;
  double *d_lh = nullptr, *d_lpart = nullptr;  // Lanczos reorthogonalisation coefficients and partials
  SpreadPlan* spread = nullptr;  // gather spreading (nullptr: atomic scatter)
  std::vector<double> h_tab;  // host copy of the smooth-part table (5 per node, 8 stride)

  // per-kernel-class event timing (fsd_set_timing)
  struct Pending {
    int cls;
    double bytes;
    hipEvent_t a, b;
  };
  bool timing = false;
  bool pair_forces = false;  // conservative bead-pair forces in the right-hand side
  // Brownian drift by random finite differences (fsd_set_drift)
  int drift_mode = 0;
  double drift_eps = 0;  // <= 0: gmres_tol^(1/3) a
  double *d_dq = nullptr, *d_udrift = nullptr, *d_vplus = nullptr, *d_umain = nullptr, *d_com0 = nullptr,
         *d_quat0 = nullptr;
  PairForceParams pf{};
  double rough_alpha = 0.0, rough_h0 = 0.0;  // tangential roughness of lubrication (h0 = 0: off)
  int warm = 0;     // GMRES initial guess: 0 zero, else the polynomial extrapolation through
                    // the last `warm` converged solutions (1: the previous one)
  int nprev = 0;    // converged solutions held, newest first in d_xp
  double* d_xp[3] = {nullptr, nullptr, nullptr};
  bool le = false;      // sheared periodic lattice (Lees-Edwards)
  double strain = 0.0;  // its strain gamma, kept in [-1/2, 1/2)
  double gam() const { return le ? strain : 0.0; }
  double* d_gam = nullptr;  // the strain where graphed kernels read it
  std::vector<hipEvent_t> ev_pool;
  size_t ev_next = 0;
  std::vector<Pending> pending;
  double t_ms[FSD_TIMER_COUNT] = {0};
  long long t_n[FSD_TIMER_COUNT] = {0};
  double t_bytes[FSD_TIMER_COUNT] = {0};

  // captured GMRES graphs
  struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    struct Pair {
      int cls, iter;
      hipEvent_t a, b;
    };
    std::vector<Pair> pairs;  // timing events recorded as graph nodes
  };
  using GraphKey = std::tuple<int, int, int, int, const void*, const void*>;
  std::map<GraphKey, GraphEntry*> graphs;
  GraphEntry* capturing = nullptr;
  int cap_iter = -1;
  bool use_graphs = true;
  int batch = 8;  // Arnoldi steps per graph segment (8 edges out 4 at 256x8; 16 gains nothing)
  std::tuple<const void*, const void*, const void*, int, int, const void*> graph_sig{};
  void drop_graphs() {
    for (auto& kv : graphs) {
      for (auto& p : kv.second->pairs) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
      }
      if (kv.second->exec) (void)hipGraphExecDestroy(kv.second->exec);
      delete kv.second;
    }
    graphs.clear();
  }

  ~fsd_system() { release(); }
  void release() {
    drop_graphs();
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (st2) (void)hipStreamDestroy(st2);
    ev_fork = ev_join = nullptr;
    st2 = nullptr;
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    ev_pool.clear();
    if (nw) neighbor_work_destroy(nw);
    nw = nullptr;
    if (nwl) neighbor_work_destroy(nwl);
    nwl = nullptr;
    if (h_flags) (void)hipHostFree(h_flags);
    h_flags = nullptr;
    if (h_scal) (void)hipHostFree(h_scal);
    h_scal = nullptr;
    if (spread) spread_plan_destroy(spread);
    spread = nullptr;
    for (void* q : owned) (void)hipFree(q);
    owned.clear();
    if (h_small) (void)hipHostFree(h_small);
    h_small = nullptr;
    if (h_ctl) (void)hipHostFree(h_ctl);
    h_ctl = nullptr;
  }
};

namespace {
// last error of a call that has no system (fsd_fft3d, batch calls)
thread_local std::string g_last_error;
}  // namespace

namespace {

fsd_status fail(fsd_system* s, fsd_status c, const std::string& m) {
  if (s) s->err = m;
  return c;
}

template <typename F>
fsd_status guarded(fsd_system* s, F&& f) {
  try {
    return f();
  } catch (const ApiError& e) {
    return fail(s, e.code, e.what());
  } catch (const HipError& e) {
    return fail(s, FSD_EDEVICE, e.what());
  } catch (const std::bad_alloc&) {
    return fail(s, FSD_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(s, FSD_EDEVICE, e.what());
  }
}

// ---- event timing -------------------------------------------------------------------------
void harvest_timers(fsd_system* s) {
  if (s->pending.empty()) return;
  HIPCHK(hipStreamSynchronize(s->st));
  for (auto& p : s->pending) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
    s->t_ms[p.cls] += ms;
    s->t_n[p.cls] += 1;
    s->t_bytes[p.cls] += p.bytes;
  }
  s->pending.clear();
  s->ev_next = 0;
}

hipEvent_t next_event(fsd_system* s) {
  if (s->ev_next == s->ev_pool.size()) {
    if (s->ev_pool.size() < 4096) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      s->ev_pool.push_back(e);
    } else {
      harvest_timers(s);
    }
  }
  return s->ev_pool[s->ev_next++];
}

// Start/stop events of one eager kernel launch when timing is on (stamped by the launch
// itself, see launch_k), with the launch's algorithmic HBM bytes (the minimum traffic of
// its inputs and outputs).  Launches that take no events (none made, or made inside a
// capture) record nothing.  (This runtime cannot time kernels inside captured graphs,
// so timed runs launch eagerly; see run_body.)
struct Timed {
  fsd_system* s;
  int cls;
  double bytes;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(fsd_system* s_, int c, double by) : s(s_), cls(c), bytes(by) {
    if (!s->timing || s->capturing) return;
    a = next_event(s);
    b = next_event(s);
    g_launch_events = LaunchEvents{a, b, false, hipSuccess};
  }
  ~Timed() noexcept(false) {
    if (!a) return;
    const LaunchEvents e = g_launch_events;
    g_launch_events = LaunchEvents{};
    HIPCHK(e.status);
    if (e.used) s->pending.push_back({cls, bytes, a, b});
  }
};

// ---- graphs ----------------------------------------------------------------------------------
using GraphEntry = fsd_system::GraphEntry;

GraphEntry* graph_for(fsd_system* s, const fsd_system::GraphKey& key, const std::function<void()>& body) {
  auto it = s->graphs.find(key);
  if (it != s->graphs.end()) return it->second;
  auto* e = new GraphEntry;
  s->capturing = e;
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal));
  try {
    body();
  } catch (...) {
    (void)hipStreamEndCapture(s->st, &g);
    if (g) (void)hipGraphDestroy(g);
    s->capturing = nullptr;
    delete e;
    throw;
  }
  s->capturing = nullptr;
  HIPCHK(hipStreamEndCapture(s->st, &g));
  const hipError_t ie = hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    delete e;
    throw HipError(std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
  }
  s->graphs[key] = e;
  return e;
}

// run body captured (cached) or eagerly
GraphEntry* run_body(fsd_system* s, const fsd_system::GraphKey& key, const std::function<void()>& body) {
  if (!s->use_graphs || s->timing) {
    body();
    return nullptr;
  }
  GraphEntry* e = graph_for(s, key, body);
  HIPCHK(hipGraphLaunch(e->exec, s->st));
  return e;
}

// after the stream has drained: add the timings of iterations that did work
void harvest_graph(fsd_system* s, GraphEntry* e, int active) {
  (void)s;
  (void)e;
  (void)active;  // captured graphs carry no timing nodes
}

// ---- parameter rules (Section 3.2: R_c = sqrt(-ln x_err)/xi, k_c = 2 sqrt(-ln x_err) xi + 1) --
void choose_parameters(fsd_system* s) {
  const fsd_params& p = s->p;
  const double a = p.radius, L = s->L;
  const double xi = pick_xi(p, s->nb, L);
  const double tol = p.ewald_tol;
  const double lnt = std::sqrt(-std::log(tol));
  const double rc = lnt / xi;
  const double kc = 2.0 * lnt * xi + 1.0 / a;
  // on a sheared lattice the grid's modes reach |k| >= (N pi / L) / sqrt(1 + gamma^2) in every
  // direction, so the grid grows by sqrt(5)/2 (|gamma| <= 1/2) to keep the cutoff k_c
  const double le_margin = s->le ? std::sqrt(1.25) : 1.0;
  int N = p.grid > 0 ? p.grid : next_smooth(int(std::ceil(kc * L / M_PI * le_margin)));
  if (N > kMaxGrid) throw ApiError(FSD_EINVAL, "spectral grid above 256^3; raise xi or lower the tolerance");
  if (!make_plan(N, s->plan))
    throw ApiError(FSD_EINVAL, "grid size must be a product of powers of 2, 3 and 5");
  int P = p.support > 0 ? p.support : int(std::ceil(2.0 / M_PI * std::log(1.0 / tol))) + 2;
  P = std::max(4, std::min(P, 21));
  if (P > N) throw ApiError(FSD_EINVAL, "Gaussian support exceeds the grid");
  const double h = L / N;
  const double mshape = 0.976 * std::sqrt(M_PI * P);
  const double eta_t = std::pow(P * h * xi / mshape, 2.0);
  if (eta_t >= 1.0) throw ApiError(FSD_EINVAL, "grid too coarse for the splitting parameter and support");
  if (p.r_lub > 0 && p.r_lub >= 0.5 * L) throw ApiError(FSD_EINVAL, "lubrication cutoff must be below L/2");
  WaveParams& w = s->wp;
  w.n = N;
  w.support = P;
  w.L = L;
  w.h = h;
  w.xi = xi;
  w.eta_t = eta_t;
  w.alpha = 2.0 * xi * xi / eta_t;
  w.a = a;
  w.eta = p.eta;
  const double gnorm = std::pow(2.0 * xi * xi / (M_PI * eta_t), 1.5);
  w.scale = std::pow(h, 6) / (L * L * L) * gnorm * gnorm;
  w.brownian = 0;
  w.tile_b = w.tile_g = 0;
  RealParams& r = s->rp;
  r.L = L;
  r.a = a;
  r.eta = p.eta;
  // Real-space cutoff: the rule sqrt(-ln tol)/xi is the floor; the polynomial
  // prefactors of the split leave the pair functions above tol there, so the
  // cutoff grows until every function is below tol times the self-mobility.
  const double mt = 1.0 / (6.0 * M_PI * p.eta * a), mr = 1.0 / (8.0 * M_PI * p.eta * a * a * a);
  double rcut = rc;
  {
    SmoothPart probe(a, p.eta, xi, 3.0 * rc);
    const double scale[5] = {mt, mt, mr, mr, mt};
    for (int it = 0; it < 400; ++it, rcut *= 1.005) {
      double f[5], sm[5];
      rpy_free(rcut, a, p.eta, f);
      probe.eval(rcut, sm);
      double worst = 0;
      for (int k = 0; k < 5; ++k) worst = std::max(worst, std::fabs(f[k] - sm[k]) / scale[k]);
      if (worst <= tol) break;
    }
  }
  // the pair search reaches rcut sqrt(1 + gamma^2) <= rcut sqrt(5)/2 on a sheared lattice; the
  // neighbour-list entries hold image shifts of at most 3 box lengths
  const double reach = rcut * (s->le ? std::sqrt(1.25) : 1.0);
  if (reach >= 3.0 * L) throw ApiError(FSD_EINVAL, "real-space cutoff exceeds three box lengths; raise xi");
  r.r_cut = rcut;
  const int ntab = 4096;
  const double ht = rcut / ntab;
  r.inv_ht = 1.0 / ht;
  r.ntab = ntab;
  SmoothPart sp(a, p.eta, xi, rcut + 4 * ht);
  s->h_tab.assign(size_t(ntab + 4) * 8, 0.0);
  for (int t = 0; t < ntab + 4; ++t) sp.eval((t - 1) * ht, &s->h_tab[8 * size_t(t)]);
  double s0[5];
  sp.eval(0.0, s0);
  r.self_t = mt - s0[0];
  r.self_r = mr - s0[2];
  s->drag_t = 6.0 * M_PI * p.eta * a;
  s->drag_r = 8.0 * M_PI * p.eta * a * a * a;
}

void upload_tables(fsd_system* s) {
  const size_t nt = s->h_tab.size();
  s->d_tab64 = dalloc<double>(s->owned, nt);
  s->d_tab32 = dalloc<float>(s->owned, nt);
  std::vector<float> f(nt);
  for (size_t i = 0; i < nt; ++i) f[i] = float(s->h_tab[i]);
  HIPCHK(hipMemcpy(s->d_tab64, s->h_tab.data(), nt * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s->d_tab32, f.data(), nt * sizeof(float), hipMemcpyHostToDevice));
  const int N = s->wp.n;
  std::vector<double> tw(2 * N);
  std::vector<float> twf(2 * N);
  for (int t = 0; t < N; ++t) {
    // e^{-2 pi i t / N}
    tw[2 * t] = std::cos(2.0 * M_PI * t / N);
    tw[2 * t + 1] = -std::sin(2.0 * M_PI * t / N);
    twf[2 * t] = float(tw[2 * t]);
    twf[2 * t + 1] = float(tw[2 * t + 1]);
  }
  s->d_tw64 = dalloc<double>(s->owned, 2 * N);
  s->d_tw32 = dalloc<float>(s->owned, 2 * N);
  HIPCHK(hipMemcpy(s->d_tw64, tw.data(), 2 * N * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s->d_tw32, twf.data(), 2 * N * sizeof(float), hipMemcpyHostToDevice));
  // Green's multipliers on the cube by q = |m|^2 (k = 2 pi m / L): sinc(ka), jv(ka) =
  // 3 (sin x - x cos x) / x^3, the solve's factor scale H~(k) / k^2 and the Brownian root's
  // sqrt(scale H~(k) / N^3) / k, with H~ = (1 + q~) e^{-(1 - eta~) q~} / eta, q~ = k^2 / 4 xi^2
  const WaveParams& w = s->wp;
  const int Q = 3 * (N / 2) * (N / 2);
  std::vector<double> gt(5 * size_t(Q + 1), 0.0);
  const double tp = 2.0 * M_PI / w.L;
  for (int q = 1; q <= Q; ++q) {
    const double k2 = tp * tp * q, kn = std::sqrt(k2), x = kn * w.a;
    double sk, jk;
    if (x < 0.5) {  // the same series the device uses below 0.5
      const double x2 = x * x;
      sk = 1.0 - x2 / 6.0 * (1.0 - x2 / 20.0 * (1.0 - x2 / 42.0 * (1.0 - x2 / 72.0 * (1.0 - x2 / 110.0))));
      jk = 1.0 - x2 / 10.0 * (1.0 - x2 / 28.0 * (1.0 - x2 / 54.0 * (1.0 - x2 / 88.0 * (1.0 - x2 / 130.0))));
    } else {
      sk = std::sin(x) / x;
      jk = 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
    }
    const double qq = k2 / (4.0 * w.xi * w.xi);
    const double damp = (1.0 + qq) * std::exp(-(1.0 - w.eta_t) * qq) / w.eta;
    double* g = &gt[5 * size_t(q)];
    g[0] = sk;
    g[1] = jk;
    g[2] = w.scale * damp / k2;
    g[3] = std::sqrt(w.scale / (double(N) * N * N) * damp) / kn;
    g[4] = 1.0 / kn;
  }
  double* d_gt = dalloc<double>(s->owned, gt.size());
  HIPCHK(hipMemcpy(d_gt, gt.data(), gt.size() * sizeof(double), hipMemcpyHostToDevice));
  s->wp.gtab = d_gt;
  std::vector<float> gf(8 * size_t(Q + 1), 0.0f);
  for (size_t q = 0; q <= size_t(Q); ++q)
    for (int c = 0; c < 5; ++c) gf[8 * q + c] = float(gt[5 * q + c]);
  float* d_gf = dalloc<float>(s->owned, gf.size());
  HIPCHK(hipMemcpy(d_gf, gf.data(), gf.size() * sizeof(float), hipMemcpyHostToDevice));
  s->wp.gtab32 = d_gf;
}

// grow a column buffer (the only allocation after set-up)
void ensure_cols(fsd_system* s, uint32_t*& col, long long& cap, long long need) {
  if (need <= cap) return;
  auto it = std::find(s->owned.begin(), s->owned.end(), (void*)col);
  if (it != s->owned.end()) {
    (void)hipFree(*it);
    s->owned.erase(it);
  }
  cap = need + need / 4 + 64;
  col = dalloc<uint32_t>(s->owned, size_t(cap));
}

// Algorithm 1 step 1 plus the geometry it needs, in two halves around one stream
// synchronisation: prepare_begin launches bead positions and the neighbour-list counts;
// prepare_end (after the stream drained) fills the lists, lubrication coefficients,
// preconditioner factors and the spreading plan.
void prepare_begin(fsd_system* s) {
  const double g = s->gam();
  s->pf.gam = g;
  // graphed kernels read the strain from device memory (set here, outside any graph)
  if (s->le) {
    if (!s->d_gam) s->d_gam = dalloc<double>(s->owned, 1);
    launch_set_value(s->d_gam, g, s->st);
  }
  s->rp.gam = s->wp.gam = s->le ? s->d_gam : nullptr;
  launch_bead_positions(s->nb, s->na, s->d_body, s->d_xbody, s->d_com, s->d_quat, s->L, g, s->d_r4, s->d_pos4,
                        s->st);
  HIPCHK(neighbors_count(s->nw, s->nb, s->d_pos4, s->d_body, s->L, g, s->rp.r_cut, false, s->d_nrow, s->st));
  if (s->p.r_lub > 0)
    HIPCHK(neighbors_count(s->nwl, s->nb, s->d_pos4, s->d_body, s->L, g, s->p.r_lub, true, s->d_lrow, s->st));
}

void prepare_end(fsd_system* s) {
  s->nnz = neighbors_total(s->nw);
  ensure_cols(s, s->d_ncol, s->ncap, s->nnz);
  HIPCHK(
      neighbors_fill(s->nw, s->nb, s->d_pos4, s->d_body, s->L, s->gam(), s->rp.r_cut, false, s->d_nrow, s->d_ncol, s->st));
  launch_zero(s->d_flags, 2 * sizeof(int), s->st);
  if (s->p.r_lub > 0) {
    s->nlub = neighbors_total(s->nwl);
    ensure_cols(s, s->d_lcol, s->lcap, s->nlub);
    if (s->lcoef_cap < s->lcap) {
      auto it = std::find(s->owned.begin(), s->owned.end(), (void*)s->d_lcoef);
      if (it != s->owned.end()) {
        (void)hipFree(*it);
        s->owned.erase(it);
      }
      s->d_lcoef = dalloc<double>(s->owned, size_t(5 * s->lcap));
      s->lcoef_cap = s->lcap;
    }
    HIPCHK(neighbors_fill(s->nwl, s->nb, s->d_pos4, s->d_body, s->L, s->gam(), s->p.r_lub, true, s->d_lrow, s->d_lcol,
                          s->st));
    launch_lub_setup(s->nb, s->d_pos4, s->L, s->gam(), s->d_lrow, s->d_lcol, s->p.radius, s->p.eta, s->p.lub_eps_min,
                     s->p.r_precond, s->rough_alpha, s->rough_h0, s->d_lcoef, s->d_rdiag, s->d_flags, s->st);
  } else {
    launch_zero(s->d_rdiag, sizeof(double) * 6 * s->nb, s->st);
    s->nlub = 0;
    launch_overlap_check(s->nb, s->d_pos4, s->d_body, s->d_nrow, s->d_ncol, s->L, s->gam(), s->p.radius, s->d_flags,
                         s->st);
  }
  launch_precond_factor(s->na, s->d_offsets, s->d_r4, s->d_rdiag, s->drag_t, s->drag_r, s->d_lu, s->d_piv,
                        s->d_flags + 1, s->st);
  if (s->spread) HIPCHK(spread_plan_update(s->spread, s->d_pos4, s->wp, s->st));
  HIPCHK(hipMemcpyAsync(s->h_flags, s->d_flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s->st));
  const double avg = s->nb ? double(s->nnz) / s->nb : 0.0;
  int l = 1;
  while (l < 64 && l * 6 < avg) l *= 2;
  s->lpr = l;
  // captured graphs hold buffer pointers and launch shapes: drop them when those change
  auto sig = std::make_tuple((const void*)s->d_ncol, (const void*)s->d_lcol, (const void*)s->d_lcoef, s->lpr,
                             int(s->p.r_lub > 0 && s->nlub > 0) | (s->le ? 2 : 0), (const void*)s->spread);
  if (sig != s->graph_sig) {
    s->drop_graphs();
    s->graph_sig = sig;
  }
  s->prepared = true;
}

// flags written by prepare_end, read after a later synchronisation
void check_flags(fsd_system* s) {
  if (s->h_flags[0]) throw ApiError(FSD_EOVERLAP, "beads of different bodies overlap by more than a/2");
  if (s->h_flags[1]) throw ApiError(FSD_EDEVICE, "singular aggregate block in the preconditioner");
}

// synchronous form for the operator-access calls
void prepare(fsd_system* s) {
  if (s->prepared) return;
  prepare_begin(s);
  HIPCHK(hipStreamSynchronize(s->st));
  prepare_end(s);
  HIPCHK(hipStreamSynchronize(s->st));
  check_flags(s);
}

}  // namespace

// ==========================================================================================
// operators
// ==========================================================================================

namespace {

template <typename R>
const R* table_of(fsd_system* s);
template <>
const double* table_of<double>(fsd_system* s) {
  return s->d_tab64;
}
template <>
const float* table_of<float>(fsd_system* s) {
  return s->d_tab32;
}
template <typename R>
const R* twiddle_of(fsd_system* s);
template <>
const double* twiddle_of<double>(fsd_system* s) {
  return s->d_tw64;
}
template <>
const float* twiddle_of<float>(fsd_system* s) {
  return s->d_tw32;
}

// out = M lam (parts: 1 real space, 2 wave space); with Vr != nullptr the rigid
// velocities Sigma^T Vr are added in the interpolation kernel.  Untimed, the
// real-space sum runs on the side stream, overlapping spreading and the transforms.
// One launch of each mobility kernel class (the wave-space ones work on the system grid).
template <typename R>
void mob_real(fsd_system* s, const double* lam, double* out, hipStream_t rs, const int* skip) {
  launch_real_sum<R>(s->nb, s->d_pos4, lam, s->d_nrow, s->d_ncol, table_of<R>(s), s->rp, out, false, s->lpr, rs, skip,
                     spread_plan_order(s->spread));
}

template <typename R>
void mob_spread(fsd_system* s, const double* lam, const int* skip) {
  R* grid = static_cast<R*>(s->d_grid);
  if (s->le) {
    const size_t N = s->wp.n;
    launch_zero(grid, sizeof(R) * 6 * N * N * N, s->st);
    launch_spread_sheared<R>(s->nb, s->d_pos4, lam, s->wp, grid, s->st, skip);
  } else if (s->spread) {
    launch_spread_gather<R>(s->spread, lam, s->wp, grid, s->st, skip);
  } else {
    const size_t N = s->wp.n;
    launch_zero(grid, sizeof(R) * 6 * N * N * N, s->st);
    launch_spread<R>(s->nb, s->d_pos4, lam, s->wp, grid, s->st, skip);
  }
}

template <typename R>
void mob_fft(fsd_system* s, int stage, const int* skip) {
  launch_wave_fft<R>(static_cast<R*>(s->d_grid), s->plan, twiddle_of<R>(s), s->wp, stage, s->st, skip);
}

template <typename R>
void mob_interp(fsd_system* s, double* out, const int* skip, const double* Vr) {
  if (s->le) {
    launch_interp_sheared<R>(s->nb, s->d_pos4, static_cast<const R*>(s->d_grid), s->wp, out, s->st, skip, s->d_body,
                             s->d_r4, Vr);
    return;
  }
  launch_interp<R>(s->nb, s->d_pos4, static_cast<const R*>(s->d_grid), s->wp, out, s->st, skip, s->d_body, s->d_r4, Vr,
                   s->spread);
}

// algorithmic bytes of the mobility launches: the real-space sum reads the row pointers,
// column indices and 128 bytes per bead (position, input, output); every wave-space pass
// moves the three packed complex grids, spreading and interpolation once plus the bead data
double real_bytes(const fsd_system* s) { return 4.0 * (s->nb + 1) + 4.0 * s->nnz + 128.0 * s->nb; }
template <typename R>
double grid_bytes(const fsd_system* s) {
  const double N = s->wp.n;
  return 3.0 * 2.0 * N * N * N * sizeof(R);
}

// `side`, when given, is further work independent of the wave-space chain: it follows the
// real-space sum on the side stream (on the system stream when nothing is forked).
template <typename R>
void apply_mobility(fsd_system* s, const double* lam, double* out, int parts, const int* skip = nullptr,
                    const double* Vr = nullptr, const std::function<void(hipStream_t)>* side = nullptr) {
  const bool fork = (parts & 1) && (parts & 2) && !s->timing;
  if (parts & 1) {
    hipStream_t rs = s->st;
    if (fork) {
      HIPCHK(hipEventRecord(s->ev_fork, s->st));
      HIPCHK(hipStreamWaitEvent(s->st2, s->ev_fork, 0));
      rs = s->st2;
    }
    {
      Timed t(s, FSD_TIMER_REAL, real_bytes(s));
      mob_real<R>(s, lam, out, rs, skip);
    }
    if (side) (*side)(rs);
    if (fork) HIPCHK(hipEventRecord(s->ev_join, s->st2));
  } else {
    launch_zero(out, sizeof(double) * 6 * s->nb, s->st);
  }
  if (parts & 2) {
    const double full = grid_bytes<R>(s), beads = 80.0 * s->nb;
    {
      Timed t(s, FSD_TIMER_SPREAD, full + beads);
      mob_spread<R>(s, lam, skip);
    }
    for (int stage = 0; stage < 5; ++stage) {
      static const int cls_of[5] = {FSD_TIMER_FFT_FIRST, FSD_TIMER_FFT_Y, FSD_TIMER_GREEN, FSD_TIMER_FFT_Y,
                                    FSD_TIMER_FFT_LAST};
      Timed t(s, cls_of[stage], 2.0 * full);  // every pass reads and writes the three packed grids
      mob_fft<R>(s, stage, skip);
    }
    if (fork) HIPCHK(hipStreamWaitEvent(s->st, s->ev_join, 0));
    Timed t(s, FSD_TIMER_INTERP, full + beads + 80.0 * s->nb + (Vr ? 48.0 * s->na : 0.0));
    mob_interp<R>(s, out, skip, Vr);
  }
}

// y = A x for the saddle matrix [[M, Sigma^T], [Sigma, -Sigma R_nf Sigma^T]]:
// y1 = M lambda + Sigma^T V (rigid part added during interpolation),
// y2 = Sigma (lambda - R_nf Sigma^T V) (lubrication evaluated inside the reduction)
double rigid_bytes(const fsd_system* s) {
  const bool lub = s->p.r_lub > 0 && s->nlub > 0;
  return 80.0 * s->nb + 96.0 * s->na + (lub ? 4.0 * (s->nb + 1) + 44.0 * s->nlub : 0.0);
}

// the fused first pass (Sigma/lubrication reduction, real-space sum, spreading) of y = A x
template <typename R>
void mob_first(fsd_system* s, const double* x, double* y, const int* skip) {
  const size_t nb6 = 6 * size_t(s->nb);
  const bool lub = s->p.r_lub > 0 && s->nlub > 0;
  const RealArgs ra{s->nb, reinterpret_cast<const double4*>(s->d_pos4), s->d_nrow, s->d_ncol, s->rp, y,
                    spread_plan_order(s->spread)};
  const RigidArgs ga{s->na, s->d_offsets, s->d_body, reinterpret_cast<const double4*>(s->d_r4), x + nb6,
                     lub ? s->d_lrow : nullptr, s->d_lcol, s->d_lcoef, y + nb6};
  launch_spread_fused<R>(s->spread, x, s->wp, static_cast<R*>(s->d_grid), table_of<R>(s), s->lpr, ra, ga, s->st, skip);
}

// y1 = M lambda + Sigma^T V, y2 = Sigma (lambda - R_nf Sigma^T V).  With a spreading plan
// the reduction, the real-space sum and the spreading share one launch (they read only
// x), timed as the spreading class; otherwise the reduction follows the real-space sum.
template <typename R>
void apply_saddle(fsd_system* s, const double* x, double* y, const int* skip = nullptr) {
  const size_t nb6 = 6 * size_t(s->nb);
  if (spread_fuses(s->spread) && !s->le) {
    const double full = grid_bytes<R>(s), beads = 80.0 * s->nb;
    {
      Timed t(s, FSD_TIMER_SPREAD, full + beads + real_bytes(s) + rigid_bytes(s));
      mob_first<R>(s, x, y, skip);
    }
    for (int stage = 0; stage < 5; ++stage) {
      static const int cls_of[5] = {FSD_TIMER_FFT_FIRST, FSD_TIMER_FFT_Y, FSD_TIMER_GREEN, FSD_TIMER_FFT_Y,
                                    FSD_TIMER_FFT_LAST};
      Timed t(s, cls_of[stage], 2.0 * full);
      mob_fft<R>(s, stage, skip);
    }
    Timed t(s, FSD_TIMER_INTERP, full + beads + 80.0 * s->nb + 48.0 * s->na);
    mob_interp<R>(s, y, skip, x + nb6);
    return;
  }
  const bool lub = s->p.r_lub > 0 && s->nlub > 0;
  const std::function<void(hipStream_t)> rigid = [&](hipStream_t st) {
    Timed t(s, FSD_TIMER_RIGID, rigid_bytes(s));
    launch_agg_lub(s->na, s->d_offsets, s->d_body, s->d_r4, x, x + nb6, lub ? s->d_lrow : nullptr, s->d_lcol,
                   s->d_lcoef, y + nb6, st, skip);
  };
  apply_mobility<R>(s, x, y, 3, skip, x + nb6, &rigid);
}

void apply_saddle_p(fsd_system* s, const double* x, double* y, bool fp32, const int* skip = nullptr) {
  if (fp32)
    apply_saddle<float>(s, x, y, skip);
  else
    apply_saddle<double>(s, x, y, skip);
}

// z = P^-1 r.  With scal != nullptr, r = scal[0] * src is formed on the fly and stored to
// vout (the Krylov basis vector of this step).
void apply_precond(fsd_system* s, const double* src, double* z, const int* skip = nullptr,
                   const double* scal = nullptr, double* vout = nullptr) {
  Timed t(s, FSD_TIMER_PRECOND, 8.0 * s->n * (vout ? 3 : 2) + 32.0 * s->nb + 312.0 * s->na);
  // M~^-1 = diag(6 pi eta a, 8 pi eta a^3): the bead drag (inverse self-mobility)
  launch_precond_fused(s->nb, s->na, s->d_offsets, s->d_r4, s->d_lu, s->d_piv, s->drag_t, s->drag_r, src, scal, vout,
                       z, s->st, skip);
}

// Euler update of the centroids and orientations by the velocities in d_U (Eqs. `EM1`,
// `EM2`); on the sheared lattice the strain first advances with the flow u_x = G_xy y, and
// the centroids are folded into the new lattice
void integrate_step(fsd_system* s, double dt) {
  if (s->le) {
    const double g = s->strain + s->G[1] * dt;
    s->strain = g - std::floor(g + 0.5);
  }
  launch_integrate(s->na, s->d_U, dt, s->L, s->gam(), s->d_com, s->d_quat, s->st);
}

// ---- Brownian terms (Eq. `SP2`, Algorithm 1 step 3) ------------------------------------------

void ensure_brownian(fsd_system* s) {
  if (s->d_ub) return;
  auto& o = s->owned;
  const size_t nb = s->nb;
  s->d_ub = dalloc<double>(o, 6 * nb);
  s->d_fb = dalloc<double>(o, 3 * nb);
  s->d_u6 = dalloc<double>(o, 6 * nb);
  s->d_psi_r = dalloc<double>(o, 6 * nb);
  s->d_psi_nf = dalloc<double>(o, 3 * nb);
  s->d_lan = dalloc<double>(o, size_t(s->lan_max + 1) * 6 * nb);
  s->d_lc = dalloc<double>(o, s->lan_max + 1);
  s->d_lh = dalloc<double>(o, 5 * size_t(s->lan_max + 2));  // h1, h2, ||w||^2, alpha, beta (and 1/beta)
  s->d_lpart = dalloc<double>(o, size_t(s->lan_max + 2) * 1024);  // launch_dots partials: <= 1024 blocks
}

double dev_dot(fsd_system* s, size_t n, const double* x, const double* y) {
  launch_dots(n, 1, x, n, y, s->d_part, s->d_h, s->d_counters, s->st);
  HIPCHK(hipMemcpyAsync(s->h_small, s->d_h, sizeof(double), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  return s->h_small[0];
}

// out = A^{1/2} z for a symmetric positive semi-definite operator by the Lanczos
// method (Chow and Saad's square-root approximation): out = |z| V_k T_k^{1/2} e1.  Each step
// orthogonalises A v_k against the whole basis twice (classical Gram-Schmidt; it keeps the
// vectors orthogonal when the operator is ill-conditioned, as the lubrication matrix is) and
// keeps alpha_k, beta_k and the next vector on the device; the host reads the coefficients
// every kCheck steps and stops once T^{1/2} e1 changes by less than tol (relative) between
// two reads, or at a breakdown.  Returns the number of Lanczos steps.
template <typename Apply>
int lanczos_sqrt(fsd_system* s, size_t n, Apply&& apply, const double* z, double* out, double tol) {
  constexpr int kCheck = 4;
  const double b0 = std::sqrt(std::max(dev_dot(s, n, z, z), 0.0));
  if (b0 == 0.0) {
    launch_zero(out, sizeof(double) * n, s->st);
    return 0;
  }
  const int L = s->lan_max + 2;
  double *h1 = s->d_lh, *h2 = s->d_lh + L, *nrm2 = s->d_lh + 2 * L, *alpha = s->d_lh + 3 * L,
         *beta = s->d_lh + 4 * L;
  double* scal = nrm2 + 1;
  double* V = s->d_lan;
  double* w = s->d_t;
  launch_scale(n, 1.0 / b0, z, V, s->st);
  std::vector<double> al(s->lan_max), be(s->lan_max), prev;
  int k = 0;
  for (int j = 0; j < s->lan_max; ++j) {
    double* vj = V + size_t(j) * n;
    apply(vj, w);
    launch_dots(n, j + 1, V, n, w, s->d_lpart, h1, s->d_counters, s->st);
    launch_axpy_dots(n, j + 1, V, n, h1, w, 0, s->d_lpart, h2, s->d_counters, s->st);
    launch_axpy_dots(n, j + 1, V, n, h2, w, 1, s->d_lpart, nrm2, s->d_counters, s->st);
    launch_lanczos_coef(j, h1, h2, nrm2, alpha, beta, scal, s->st);
    if (j + 1 < s->lan_max) launch_scale_dev(n, scal, w, V + size_t(j + 1) * n, s->st);
    if ((j + 1) % kCheck != 0 && j + 1 != s->lan_max) continue;
    HIPCHK(hipMemcpyAsync(s->h_small, alpha, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipMemcpyAsync(s->h_small + L, beta, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    // the first breakdown ends the basis
    k = j + 1;
    for (int i = 0; i <= j; ++i)
      if (s->h_small[L + i] <= 1e-14 * std::fabs(s->h_small[i])) {
        k = i + 1;
        break;
      }
    std::vector<double> a(s->h_small, s->h_small + k), b(s->h_small + L, s->h_small + L + std::max(k - 1, 0));
    std::vector<double> cur = tridiag_sqrt_e1(a, b);
    double diff = 0, nrm = 0;
    for (size_t i = 0; i < cur.size(); ++i) {
      const double d = cur[i] - (i < prev.size() ? prev[i] : 0.0);
      diff += d * d;
      nrm += cur[i] * cur[i];
    }
    prev.swap(cur);
    if (diff <= tol * tol * nrm || k <= j || j + 1 == s->lan_max) break;
  }
  std::vector<double> c(prev.size());
  for (size_t i = 0; i < c.size(); ++i) c[i] = b0 * prev[i];
  HIPCHK(hipMemcpyAsync(s->d_lc, c.data(), sizeof(double) * c.size(), hipMemcpyHostToDevice, s->st));
  launch_combine(n, int(c.size()), V, n, s->d_lc, out, s->st);
  HIPCHK(hipStreamSynchronize(s->st));  // c lives on the host stack
  return k;
}

// u_B = sqrt(2 kT / dt) (M_w^{1/2} psi_w + M_r^{1/2} psi_r) into d_ub (6 per bead) and
// F_B = sqrt(2 kT / dt) R_nf^{1/2} psi_nf into d_fb (3 per bead, translational)
void brownian_terms(fsd_system* s) {
  ensure_brownian(s);
  const size_t nb = s->nb;
  const double amp = std::sqrt(2.0 * s->p.kT / s->bdt);
  const NoiseKey kw{s->p.seed, s->bstream, 0, s->bstep}, kr{s->p.seed, s->bstream, 1, s->bstep},
      kn{s->p.seed, s->bstream, 2, s->bstep};
  // wave space: white noise on the grid through the square-root multiplier, interpolated
  double* grid = static_cast<double*>(s->d_grid);
  launch_noise_grid(s->wp.n, kw, s->psi_w_set ? s->d_psi_w : nullptr, grid, s->st);
  WaveParams wb = s->wp;
  wb.brownian = 1;
  for (int stage = 0; stage < 5; ++stage)
    launch_wave_fft<double>(grid, s->plan, s->d_tw64, wb, stage, s->st);
  launch_zero(s->d_ub, sizeof(double) * 6 * nb, s->st);
  mob_interp<double>(s, s->d_ub, nullptr, nullptr);  // the sheared grid's own interpolation when on
  // real space: Lanczos on the pair sum
  if (!s->psi_r_set) launch_normals(6 * nb, kr, s->d_psi_r, s->st);
  s->lan_its[0] = lanczos_sqrt(
      s, 6 * nb, [&](const double* in, double* out) { apply_mobility<double>(s, in, out, 1); }, s->d_psi_r,
      s->d_u6, s->p.lanczos_tol);
  launch_axpby(6 * nb, amp, s->d_u6, amp, s->d_ub, s->st);
  // near field: Lanczos on R_nf (the lubrication product returns -R_nf w)
  const bool lub = s->p.r_lub > 0 && s->nlub > 0;
  if (lub) {
    if (!s->psi_nf_set) launch_normals(3 * nb, kn, s->d_psi_nf, s->st);
    s->lan_its[1] = lanczos_sqrt(
        s, 3 * nb,
        [&](const double* in, double* out) {
          launch_lub_apply(s->nb, s->d_lrow, s->d_lcol, s->d_lcoef, in, out, s->st);
          launch_scale(3 * nb, -1.0, out, out, s->st);
        },
        s->d_psi_nf, s->d_fb, s->p.lanczos_tol);
    launch_scale(3 * nb, amp, s->d_fb, s->d_fb, s->st);
  } else {
    s->lan_its[1] = 0;
    launch_zero(s->d_fb, sizeof(double) * 3 * nb, s->st);
  }
}

void assemble_rhs(fsd_system* s) {
  const size_t nb6 = 6 * size_t(s->nb);
  const bool lub = s->p.r_lub > 0 && s->nlub > 0;
  const bool brown = s->p.kT > 0;
  if (brown) brownian_terms(s);
  launch_rhs(s->nb, s->na, s->d_offsets, s->d_body, s->d_r4, s->d_E, s->d_force, brown ? s->d_ub : nullptr, s->d_b,
             s->d_wt, s->st);
  if (lub) {
    // R_FE : E_inf = -Sigma f_e, f_e minus the near-field force on beads moving with the
    // ambient flow at their centroids; b2 = -(F_P + Sigma F_B + R_FE : E_inf)
    //    = -F_P + Sigma (f_e - F_B)
    launch_lub_strain(s->nb, s->d_pos4, s->d_r4, s->L, s->gam(), s->d_lrow, s->d_lcol, s->d_lcoef, s->d_E, s->d_fl,
                      s->st);
    if (brown) launch_axpby(3 * size_t(s->nb), -1.0, s->d_fb, 1.0, s->d_fl, s->st);
  }
  // conservative bead-pair forces join F_P through Sigma: b2 gains -Sigma f_c
  if (s->pair_forces)
    launch_pair_forces(s->nb, s->d_pos4, s->d_body, s->d_nrow, s->d_ncol, s->pf, s->d_fl, lub ? 1 : 0, s->st);
  launch_rhs_agg(s->na, s->d_offsets, s->d_r4, s->d_force, (lub || s->pair_forces) ? s->d_fl : nullptr,
                 s->d_b + nb6, s->st);
}

// ||v|| with a synchronisation (operator-access paths only)
double norm2(fsd_system* s, const double* v) {
  launch_dots(s->n, 1, v, s->n, v, s->d_part, s->d_h, s->d_counters, s->st);
  HIPCHK(hipMemcpyAsync(s->h_small, s->d_h, sizeof(double), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  return std::sqrt(s->h_small[0]);
}

// ---- GMRES segments (asynchronous; each ends with the control block copied to the host) ----
// Right-preconditioned restarted GMRES(m) with classical Gram-Schmidt applied twice
// (CGS2).  The Arnoldi bookkeeping, Givens rotations and stopping test run on the
// device; the host replays captured segments: a cycle start (true residual b - A x,
// beta, v0), batches of Arnoldi steps (kernels after the device stop flag return
// early), and a cycle end (x += P^-1 V y).  Every cycle starts from the recomputed
// residual, so the residual reported at convergence is a true one.

void seg_cycle_start(fsd_system* s) {
  auto& v = s->sv;
  const size_t n = s->n;
  const int m = s->m;
  double* hn2 = s->d_h + 2 * (m + 1);
  const int* stop = &s->d_ctl->stop;
  const double* b = v.b;
  double* x = v.x;
  const bool fp32 = v.fp32;
  (void)fp32;
  run_body(s, {0, 0, 0, 0, b, x}, [&] {
    // the true residual in FP64 at every cycle start: with FP32 Arnoldi matvecs
    // (mixed precision) each restart is an iterative-refinement step
    apply_saddle<double>(s, x, s->d_t);
    launch_sub(n, b, s->d_t, s->d_r, s->st);
    launch_dots(n, 1, s->d_r, n, s->d_r, s->d_part, hn2, s->d_counters, s->st);
    launch_gmres_begin(s->d_ctl, hn2, s->d_g, s->d_scal, s->st);
  });
  HIPCHK(hipMemcpyAsync(s->h_ctl, s->d_ctl, sizeof(GmresCtl), hipMemcpyDeviceToHost, s->st));
}

// Arnoldi steps per segment.  A timed run ends a segment after every step, so the host
// reads the stop flag before the next launch and no timed launch is one that returns at
// once after convergence (those would pull the per-kernel averages down).
int seg_len(const fsd_system* s) { return s->timing ? 1 : std::max(1, std::min(s->batch, s->m)); }

void seg_batch(fsd_system* s, int j0) {
  auto& v = s->sv;
  const size_t n = s->n;
  const int m = s->m;
  const int S = seg_len(s);
  const int cnt = std::min(S, m - j0);
  double* V = s->d_basis;
  double* h1 = s->d_h;
  double* h2 = s->d_h + (m + 1);
  double* hn2 = s->d_h + 2 * (m + 1);
  const int* stop = &s->d_ctl->stop;
  const bool fp32 = v.fp32;
  run_body(s, {1, j0, cnt, fp32 ? 1 : 0, nullptr, nullptr}, [&] {
    const size_t G = cgs_blocks(n);
    double *P0 = s->d_part, *P1 = s->d_part + 32 * G, *P2 = s->d_part + 64 * G;
    for (int j = j0; j < j0 + cnt; ++j) {
      // v_j = w / H[j, j-1] (r / beta for j = 0) is formed inside the preconditioner.  Inside
      // a segment the Arnoldi update of step j-1 rides in this launch (its ||w||^2 partials
      // are in P2); a segment's last step makes its update alone, so the host reads a current
      // stop flag after every segment.
      if (j > j0 && cgs_fits(j)) {
        Timed t(s, FSD_TIMER_PRECOND, 8.0 * n * 3 + 32.0 * s->nb + 312.0 * s->na);
        const ArnoldiArgs prev{j - 1, s->d_ctl, h1, h2, s->d_H, s->d_cs, s->d_sn, s->d_g, s->d_scal};
        launch_precond_arnoldi(s->nb, s->na, s->d_offsets, s->d_r4, s->d_lu, s->d_piv, s->drag_t, s->drag_r, s->d_w,
                               V + size_t(j) * n, s->d_z, prev, P2, int(G), hn2, s->st, stop);
      } else {
        apply_precond(s, j == 0 ? s->d_r : s->d_w, s->d_z, stop, s->d_scal, V + size_t(j) * n);
      }
      apply_saddle_p(s, s->d_z, s->d_w, fp32, stop);
      const ArnoldiArgs arn{j, s->d_ctl, h1, h2, s->d_H, s->d_cs, s->d_sn, s->d_g, s->d_scal};
      const int nq = j + 1;
      if (cgs_fits(nq)) {
        // fence-free chain: three partial arrays, each reduced by the next launch
        {
          Timed t(s, FSD_TIMER_CGS_DOT, 8.0 * n * (nq + 1));
          launch_cgs_chain(0, n, nq, V, n, nullptr, s->d_w, P0, nullptr, s->st, stop);
        }
        {
          Timed t(s, FSD_TIMER_CGS_UPDATE, 8.0 * n * (nq + 2));
          launch_cgs_chain(1, n, nq, V, n, P0, s->d_w, P1, h1, s->st, stop);
        }
        {
          Timed t(s, FSD_TIMER_CGS_NORM, 8.0 * n * (nq + 2));
          launch_cgs_chain(2, n, nq, V, n, P1, s->d_w, P2, h2, s->st, stop);
        }
        if (j == j0 + cnt - 1) launch_arnoldi_reduce(arn, P2, int(G), hn2, s->st);  // else folded into step j+1
      } else {
        {
          Timed t(s, FSD_TIMER_CGS_DOT, 8.0 * n * (nq + 1));
          launch_dots(n, nq, V, n, s->d_w, s->d_part, h1, s->d_counters, s->st, stop);
        }
        {
          Timed t(s, FSD_TIMER_CGS_UPDATE, 8.0 * n * (nq + 2));
          launch_axpy_dots(n, nq, V, n, h1, s->d_w, 0, s->d_part, h2, s->d_counters, s->st, stop);
        }
        {
          Timed t(s, FSD_TIMER_CGS_NORM, 8.0 * n * (nq + 2));
          launch_axpy_dots(n, nq, V, n, h2, s->d_w, 1, s->d_part, hn2, s->d_counters, s->st, stop);
        }
        launch_arnoldi_step(arn, hn2, s->st);
      }
    }
  });
  HIPCHK(hipMemcpyAsync(s->h_ctl, s->d_ctl, sizeof(GmresCtl), hipMemcpyDeviceToHost, s->st));
}

void seg_cycle_end(fsd_system* s) {
  auto& v = s->sv;
  const size_t n = s->n;
  const int m = s->m;
  double* x = v.x;
  run_body(s, {2, 0, 0, v.fp32 ? 1 : 0, v.b, x}, [&] {
    launch_gmres_solve(s->d_ctl, s->d_H, s->d_g, s->d_y, s->st);
    launch_basis_combine(n, m, s->d_basis, n, s->d_y, s->d_ctl, s->d_t, s->st);
    apply_precond(s, s->d_t, s->d_z);
    launch_axpby(n, 1.0, s->d_z, 1.0, x, s->st);
  });
}

// start a GMRES on (b, x) from x = 0
void gmres_launch(fsd_system* s, const double* b, double* x, double tol, bool fp32, int maxit) {
  auto& v = s->sv;
  v.b = b;
  v.x = x;
  v.tol = tol;
  v.fp32 = fp32;
  // initial guess: zero, or with warm starts the previous converged solution of a full
  // right-hand side (the first cycle forms the true residual b - A x either way)
  if (s->warm && s->nprev > 0 && v.rhs_kind == 0) {
    // x0 = sum_i c_i x_(n-i): the value at the next step of the polynomial through the last
    // q solutions (steps of equal length): q = 1: x_n; 2: 2 x_n - x_(n-1);
    // 3: 3 x_n - 3 x_(n-1) + x_(n-2)
    static const double coef[3][3] = {{1, 0, 0}, {2, -1, 0}, {3, -3, 1}};
    const int q = std::min(s->warm, s->nprev);
    HIPCHK(hipMemcpyAsync(x, s->d_xp[0], sizeof(double) * s->n, hipMemcpyDeviceToDevice, s->st));
    if (q > 1) launch_axpby(s->n, coef[q - 1][1], s->d_xp[1], coef[q - 1][0], x, s->st);
    if (q > 2) launch_axpby(s->n, coef[q - 1][2], s->d_xp[2], 1.0, x, s->st);
  } else {
    launch_zero(x, sizeof(double) * s->n, s->st);
  }
  double* bb = s->d_h + 2 * (s->m + 1) + 1;
  launch_dots(s->n, 1, b, s->n, b, s->d_part, bb, s->d_counters, s->st);
  launch_gmres_init(s->d_ctl, bb, tol, std::max(1, maxit), s->m, s->st);
  seg_cycle_start(s);
  v.phase = fsd_system::SolveState::START;
}

void finish_solve(fsd_system* s, bool ok) {
  const size_t nb6 = 6 * size_t(s->nb);
  if (s->sv.rhs_kind != 0) {  // U = V: no ambient flow in the drift solves
    launch_zero(s->d_U, sizeof(double) * 6 * s->na, s->st);
    launch_axpby(6 * size_t(s->na), 1.0, s->d_x + nb6, 1.0, s->d_U, s->st);
  } else {
    launch_add_ambient(s->na, s->d_x + nb6, s->d_com, s->d_G, s->d_W, s->d_U, s->st);
  }
  if (ok && s->warm && s->sv.rhs_kind == 0) {  // keep the newest `warm` solutions, newest first
    const int q = s->warm;
    for (int i = 0; i < q; ++i)
      if (!s->d_xp[i]) s->d_xp[i] = dalloc<double>(s->owned, s->n);
    double* last = s->d_xp[q - 1];
    for (int i = q - 1; i > 0; --i) s->d_xp[i] = s->d_xp[i - 1];
    s->d_xp[0] = last;
    HIPCHK(hipMemcpyAsync(s->d_xp[0], s->d_x, sizeof(double) * s->n, hipMemcpyDeviceToDevice, s->st));
    s->nprev = std::min(s->nprev + 1, q);
  }
  if (s->sv.rhs_kind == 0) s->solved = true;
  s->sv.converged = ok;
  s->sv.status = ok ? FSD_OK : FSD_ENOCONV;
  if (!ok) s->err = "GMRES did not reach the tolerance within gmres_maxit iterations";
  s->sv.phase = fsd_system::SolveState::DONE;
}

// the correction of one mixed-precision refinement lives after the Krylov basis

// begin a solve at the current configuration (asynchronous)
void solve_begin(fsd_system* s) {
  auto& v = s->sv;
  v = fsd_system::SolveState{};
  if (!s->prepared) {
    prepare_begin(s);
    v.phase = fsd_system::SolveState::PREP;
    return;
  }
  v.phase = fsd_system::SolveState::PREP;  // prepared: PREP only assembles the right-hand side
}

// Advance after the system stream has drained.  Returns false once the solve is done.
bool solve_advance(fsd_system* s) {
  auto& v = s->sv;
  using SS = fsd_system::SolveState;
  const bool mixed = s->p.precision == FSD_MIXED;
  switch (v.phase) {
    case SS::PREP: {
      if (!s->prepared) prepare_end(s);
      const size_t nb6 = 6 * size_t(s->nb);
      if (v.rhs_kind == 1) {  // b = (0, -dq)
        launch_zero(s->d_b, sizeof(double) * s->n, s->st);
        launch_axpby(6 * size_t(s->na), -1.0, s->d_dq, 1.0, s->d_b + nb6, s->st);
      } else if (v.rhs_kind == 2) {  // b = (u_B, -Sigma F_B) with the stored Brownian terms
        launch_zero(s->d_b, sizeof(double) * s->n, s->st);
        launch_axpby(nb6, 1.0, s->d_ub, 1.0, s->d_b, s->st);
        launch_zero(s->d_fl, sizeof(double) * 3 * s->nb, s->st);
        launch_axpby(3 * size_t(s->nb), -1.0, s->d_fb, 1.0, s->d_fl, s->st);
        launch_zero(s->d_vplus, sizeof(double) * 6 * s->na, s->st);  // no other force
        launch_rhs_agg(s->na, s->d_offsets, s->d_r4, s->d_vplus, s->d_fl, s->d_b + nb6, s->st);
      } else {
        assemble_rhs(s);
      }
      gmres_launch(s, s->d_b, s->d_x, s->p.gmres_tol, mixed, s->p.gmres_maxit);
      return true;
    }
    case SS::START: {
      check_flags(s);
      const GmresCtl& c = *s->h_ctl;
      if (c.resid <= v.tol || c.stop) {
        v.its += c.its;
        v.rel = c.resid;
        finish_solve(s, c.resid <= v.tol);
        return false;
      }
      v.j0 = 0;
      seg_batch(s, 0);
      v.phase = SS::BATCH;
      return true;
    }
    case SS::BATCH: {
      const GmresCtl& c = *s->h_ctl;
      const int S = seg_len(s);
      if (c.stop) {
        seg_cycle_end(s);
        ++v.restarts;
        if (mixed) ++v.outer;  // each FP64 residual replacement is one refinement
        seg_cycle_start(s);
        v.phase = SS::START;
      } else {
        v.j0 += S;
        seg_batch(s, v.j0);
      }
      return true;
    }
    default:
      return false;
  }
}

fsd_solve_info info_of(const fsd_system* s) {
  const auto& v = s->sv;
  fsd_solve_info inf{};
  inf.status = v.status;
  inf.iterations = v.its;
  inf.restarts = v.restarts;
  inf.refinements = s->p.precision == FSD_MIXED ? v.outer : 1;
  inf.rel_residual_fp64 = v.rel;
  return inf;
}

fsd_status solve_current(fsd_system* s, fsd_solve_info* info, int rhs_kind = 0) {
  solve_begin(s);
  s->sv.rhs_kind = rhs_kind;
  while (true) {
    HIPCHK(hipStreamSynchronize(s->st));
    if (!solve_advance(s)) break;
  }
  if (info) *info = info_of(s);
  return s->sv.status;
}

// ---- Brownian drift by random finite differences (Appendix A, Eq. `rfd`) ------------------
// kT (U+ - U-) / eps with U+- the aggregate velocities of the saddle solves at the
// configurations displaced by +-(eps/2) dq, each with right-hand side (0, -dq); dq is
// Gaussian (6 per aggregate, Philox purpose 3 of this step) unless dq_host is given.
// Leaves the drift in d_udrift and the configuration as it found it.
void ensure_drift(fsd_system* s) {
  if (s->d_dq) return;
  auto& o = s->owned;
  const size_t na = s->na;
  s->d_dq = dalloc<double>(o, 6 * na);
  s->d_udrift = dalloc<double>(o, 6 * na);
  s->d_vplus = dalloc<double>(o, 6 * na);
  s->d_umain = dalloc<double>(o, 6 * na);
  s->d_com0 = dalloc<double>(o, 3 * na);
  s->d_quat0 = dalloc<double>(o, 4 * na);
}

void rfd_drift(fsd_system* s, const double* dq_host) {
  ensure_drift(s);
  const size_t na = s->na;
  const double eps = s->drift_eps > 0 ? s->drift_eps : std::cbrt(s->p.gmres_tol) * s->p.radius;
  if (dq_host)
    HIPCHK(hipMemcpyAsync(s->d_dq, dq_host, sizeof(double) * 6 * na, hipMemcpyHostToDevice, s->st));
  else
    launch_normals(6 * na, NoiseKey{s->p.seed, s->bstream, 3, s->bstep}, s->d_dq, s->st);
  HIPCHK(hipMemcpyAsync(s->d_com0, s->d_com, sizeof(double) * 3 * na, hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(s->d_quat0, s->d_quat, sizeof(double) * 4 * na, hipMemcpyDeviceToDevice, s->st));
  const double c = s->p.kT / eps;
  fsd_status r = FSD_OK;
  for (int sign = 1; sign >= -1 && r == FSD_OK; sign -= 2) {
    launch_displace(int(na), s->d_com0, s->d_quat0, s->d_dq, 0.5 * sign * eps, s->L, s->gam(), s->d_com, s->d_quat,
                    s->st);
    s->prepared = false;
    r = solve_current(s, nullptr, 1);
    if (sign > 0) HIPCHK(hipMemcpyAsync(s->d_vplus, s->d_U, sizeof(double) * 6 * na, hipMemcpyDeviceToDevice, s->st));
  }
  HIPCHK(hipMemcpyAsync(s->d_com, s->d_com0, sizeof(double) * 3 * na, hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(s->d_quat, s->d_quat0, sizeof(double) * 4 * na, hipMemcpyDeviceToDevice, s->st));
  s->prepared = false;
  if (r != FSD_OK) throw ApiError(r, std::string("drift solve: ") + s->err);
  launch_zero(s->d_udrift, sizeof(double) * 6 * na, s->st);
  launch_axpby(6 * na, c, s->d_vplus, 1.0, s->d_udrift, s->st);
  launch_axpby(6 * na, -c, s->d_U, 1.0, s->d_udrift, s->st);
}

// Fixman's midpoint drift (Appendix A), after a solve at x that computed this step's
// Brownian terms (d_ub, d_fb) and left its velocities in d_U: U0 from those terms alone at
// x, U' from the same terms at x + (dt/m) U0, drift (m/2) (U' - U0) into d_udrift; the
// configuration is restored and d_U holds the first solve's velocities again.
void fixman_drift(fsd_system* s, double dt) {
  ensure_drift(s);
  const size_t na = s->na;
  const double m = s->drift_eps > 0 ? s->drift_eps : 100.0;
  HIPCHK(hipMemcpyAsync(s->d_umain, s->d_U, sizeof(double) * 6 * na, hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(s->d_com0, s->d_com, sizeof(double) * 3 * na, hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(s->d_quat0, s->d_quat, sizeof(double) * 4 * na, hipMemcpyDeviceToDevice, s->st));
  fsd_status r = solve_current(s, nullptr, 2);  // U0 (positions unchanged: still prepared)
  if (r == FSD_OK) {
    HIPCHK(hipMemcpyAsync(s->d_udrift, s->d_U, sizeof(double) * 6 * na, hipMemcpyDeviceToDevice, s->st));
    launch_integrate(int(na), s->d_U, dt / m, s->L, s->gam(), s->d_com, s->d_quat, s->st);
    s->prepared = false;
    r = solve_current(s, nullptr, 2);  // U'
  }
  HIPCHK(hipMemcpyAsync(s->d_com, s->d_com0, sizeof(double) * 3 * na, hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(s->d_quat, s->d_quat0, sizeof(double) * 4 * na, hipMemcpyDeviceToDevice, s->st));
  s->prepared = false;
  if (r != FSD_OK) throw ApiError(r, std::string("Fixman drift solve: ") + s->err);
  // d_udrift = (m/2) (U' - U0), d_U = the first solve's velocities
  launch_axpby(6 * na, 0.5 * m, s->d_U, -0.5 * m, s->d_udrift, s->st);
  HIPCHK(hipMemcpyAsync(s->d_U, s->d_umain, sizeof(double) * 6 * na, hipMemcpyDeviceToDevice, s->st));
}

// The parts of one time step around its solve (fsd_step and the batched step take the same
// path): the random-finite-difference drift before the solve; after it Fixman's drift, the
// drift added to the velocities, and the Euler update of Eqs. `EM1`-`EM3`.
void step_before_solve(fsd_system* s) {
  if (s->drift_mode == 1 && s->p.kT > 0) rfd_drift(s, nullptr);
}

void step_after_solve(fsd_system* s, double dt) {
  const bool rfd = s->drift_mode == 1 && s->p.kT > 0, fixman = s->drift_mode == 2 && s->p.kT > 0;
  if (fixman) {  // its solves leave their own state: the step reports the main solve's
    const auto main = s->sv;
    fixman_drift(s, dt);
    s->sv = main;
  }
  if (rfd || fixman) launch_axpby(6 * size_t(s->na), 1.0, s->d_udrift, 1.0, s->d_U, s->st);
  integrate_step(s, dt);
  s->prepared = false;
  ++s->bstep;
}

fsd_status check_ready(fsd_system* s) {
  if (!s) return FSD_EINVAL;
  if (!s->have_box || !s->have_agg) return fail(s, FSD_ESTATE, "call fsd_init_box and fsd_init_aggregates first");
  return FSD_OK;
}

// one launch of the kernel behind a timer class, on the scratch vectors of the system
template <typename R>
bool replay_one(fsd_system* s, int cls) {
  const size_t nb6 = 6 * size_t(s->nb);
  const bool lub = s->p.r_lub > 0 && s->nlub > 0;
  switch (cls) {
    case FSD_TIMER_REAL: mob_real<R>(s, s->d_z, s->d_t, s->st, nullptr); return true;
    case FSD_TIMER_SPREAD:  // the kernel a solve runs for this class
      if (spread_fuses(s->spread) && !s->le)
        mob_first<R>(s, s->d_z, s->d_t, nullptr);
      else
        mob_spread<R>(s, s->d_z, nullptr);
      return true;
    case FSD_TIMER_FFT_FIRST: mob_fft<R>(s, 0, nullptr); return true;
    case FSD_TIMER_FFT_Y: mob_fft<R>(s, 1, nullptr); return true;
    case FSD_TIMER_GREEN: mob_fft<R>(s, 2, nullptr); return true;
    case FSD_TIMER_FFT_LAST: mob_fft<R>(s, 4, nullptr); return true;
    case FSD_TIMER_INTERP: mob_interp<R>(s, s->d_t, nullptr, s->d_z + nb6); return true;
    case FSD_TIMER_RIGID:
      launch_agg_lub(s->na, s->d_offsets, s->d_body, s->d_r4, s->d_z, s->d_z + nb6, lub ? s->d_lrow : nullptr,
                     s->d_lcol, s->d_lcoef, s->d_t + nb6, s->st, nullptr);
      return true;
    case FSD_TIMER_PRECOND:
      launch_precond_fused(s->nb, s->na, s->d_offsets, s->d_r4, s->d_lu, s->d_piv, s->drag_t, s->drag_r, s->d_z,
                           nullptr, nullptr, s->d_t, s->st, nullptr);
      return true;
    default: return false;
  }
}
}  // namespace

// ==========================================================================================
// C ABI
// ==========================================================================================

extern "C" {

void fsd_default_params(fsd_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->eta = 1.0;
  p->radius = 1.0;
  p->kT = 0.0;
  p->xi = 0.0;
  p->ewald_tol = 1e-6;
  p->grid = 0;
  p->support = 0;
  p->r_lub = 3.0;
  p->r_precond = 2.1;
  p->lub_eps_min = 1e-3;
  p->gmres_tol = 1e-6;
  p->gmres_restart = 30;
  p->gmres_maxit = 1000;
  p->precision = FSD_FP64;
  p->lanczos_tol = 1e-4;
  p->seed = 2607251610ull;
  p->lanczos_maxit = 100;
}

fsd_status fsd_create(const fsd_params* p, void* hip_stream, fsd_system** out) {
  if (!p || !out) return FSD_EINVAL;
  if (!(p->eta > 0) || !(p->radius > 0) || !(p->ewald_tol > 0 && p->ewald_tol < 1) || !(p->gmres_tol > 0) ||
      p->gmres_restart < 1 || p->gmres_restart > 200 || p->gmres_maxit < 1 || p->grid < 0 || p->support < 0 ||
      p->support > 21 || p->r_lub < 0 || (p->precision != FSD_FP64 && p->precision != FSD_MIXED) ||
      !(p->lanczos_tol > 0 && p->lanczos_tol < 1) || p->kT < 0 || p->lanczos_maxit < 1 ||
      p->lanczos_maxit > 2000)
    return FSD_EINVAL;
  fsd_system* s = new (std::nothrow) fsd_system;
  if (!s) return FSD_ENOMEM;
  s->p = *p;
  s->m = p->gmres_restart;
  s->lan_max = p->lanczos_maxit;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return FSD_EDEVICE;
  }
  if (hip_stream) {
    s->st = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreate(&s->st) != hipSuccess) {
      delete s;
      return FSD_EDEVICE;
    }
    s->own_stream = true;
  }
  *out = s;
  return FSD_OK;
}

fsd_status fsd_init_box(fsd_system* s, double Lx, double Ly, double Lz) {
  if (!s) return FSD_EINVAL;
  if (!(Lx == Ly && Ly == Lz)) return fail(s, FSD_EINVAL, "the box must be a cube (Lx == Ly == Lz)");
  const double L = Lx;
  if (!(L > 4.0 * s->p.radius)) return fail(s, FSD_EINVAL, "box side must exceed 4a");
  if (s->have_agg) return fail(s, FSD_ESTATE, "the box is fixed once aggregates are set");
  s->L = L;
  s->have_box = true;
  return FSD_OK;
}

fsd_status fsd_init_aggregates(fsd_system* s, int32_t n_agg, const int32_t* off, const double* x_body,
                               const double* com, const double* quat) {
  if (!s) return FSD_EINVAL;
  if (!s->have_box) return fail(s, FSD_ESTATE, "call fsd_init_box first");
  if (s->have_agg) return fail(s, FSD_ESTATE, "aggregates already set");
  if (n_agg < 1 || !off || !x_body || !com || !quat) return fail(s, FSD_EINVAL, "null or empty input");
  if (off[0] != 0) return fail(s, FSD_EINVAL, "bead_offsets[0] must be 0");
  for (int j = 0; j < n_agg; ++j)
    if (off[j + 1] <= off[j]) return fail(s, FSD_EINVAL, "every aggregate needs at least one bead");
  const int nb = off[n_agg];
  if (nb >= (1 << 22)) return fail(s, FSD_EINVAL, "at most 4194303 beads");
  const double L = s->L;
  std::vector<double> xb(x_body, x_body + 3 * size_t(nb)), X(3 * size_t(n_agg)), q(4 * size_t(n_agg));
  for (int i = 0; i < 3 * nb; ++i)
    if (!std::isfinite(xb[i])) return fail(s, FSD_EINVAL, "non-finite body coordinates");
  for (int j = 0; j < n_agg; ++j) {
    double c[3] = {0, 0, 0};
    const int n = off[j + 1] - off[j];
    for (int i = off[j]; i < off[j + 1]; ++i)
      for (int d = 0; d < 3; ++d) c[d] += xb[3 * i + d] / n;
    for (int i = off[j]; i < off[j + 1]; ++i)
      for (int d = 0; d < 3; ++d) xb[3 * i + d] -= c[d];
    double nq = 0;
    for (int d = 0; d < 4; ++d) nq += quat[4 * j + d] * quat[4 * j + d];
    nq = std::sqrt(nq);
    if (!(nq > 0) || !std::isfinite(nq)) return fail(s, FSD_EINVAL, "zero or non-finite quaternion");
    for (int d = 0; d < 4; ++d) q[4 * j + d] = quat[4 * j + d] / nq;
    // the body-frame centroid shift moves the centroid in the lab frame by R(q) c
    const double w = q[4 * j], x = q[4 * j + 1], y = q[4 * j + 2], z = q[4 * j + 3];
    const double Rc[3] = {(1 - 2 * (y * y + z * z)) * c[0] + 2 * (x * y - w * z) * c[1] + 2 * (x * z + w * y) * c[2],
                          2 * (x * y + w * z) * c[0] + (1 - 2 * (x * x + z * z)) * c[1] + 2 * (y * z - w * x) * c[2],
                          2 * (x * z - w * y) * c[0] + 2 * (y * z + w * x) * c[1] + (1 - 2 * (x * x + y * y)) * c[2]};
    double v3[3];
    for (int d = 0; d < 3; ++d) {
      if (!std::isfinite(com[3 * j + d])) return fail(s, FSD_EINVAL, "non-finite centroid");
      v3[d] = com[3 * j + d] + Rc[d];
    }
    const double ny = std::floor((v3[1] + 0.5 * L) / L);  // y first on a sheared lattice
    v3[1] -= ny * L;
    v3[0] -= ny * s->gam() * L;
    for (int d = 0; d < 3; ++d) {
      double v = v3[d];
      v -= L * std::floor((v + 0.5 * L) / L);
      if (v >= 0.5 * L) v -= L;
      X[3 * j + d] = v;
    }
  }
  return guarded(s, [&]() -> fsd_status {
    s->nb = nb;
    s->na = n_agg;
    s->n = 6 * size_t(nb + n_agg);
    choose_parameters(s);
    std::vector<int> body(nb);
    for (int j = 0; j < n_agg; ++j)
      for (int i = off[j]; i < off[j + 1]; ++i) body[i] = j;
    s->h_offsets.assign(off, off + n_agg + 1);
    auto& o = s->owned;
    s->d_offsets = dalloc<int>(o, n_agg + 1);
    s->d_body = dalloc<int>(o, nb);
    s->d_xbody = dalloc<double>(o, 3 * size_t(nb));
    s->d_com = dalloc<double>(o, 3 * size_t(n_agg));
    s->d_quat = dalloc<double>(o, 4 * size_t(n_agg));
    s->d_r4 = dalloc<double>(o, 4 * size_t(nb));
    s->d_pos4 = dalloc<double>(o, 4 * size_t(nb));
    s->d_force = dalloc<double>(o, 6 * size_t(n_agg));
    s->d_G = dalloc<double>(o, 9);
    s->d_E = dalloc<double>(o, 9);
    s->d_W = dalloc<double>(o, 3);
    s->d_nrow = dalloc<int>(o, nb + 1);
    s->d_lrow = dalloc<int>(o, nb + 1);
    s->d_rdiag = dalloc<double>(o, 6 * size_t(nb));
    s->d_lu = dalloc<double>(o, 36 * size_t(n_agg));
    s->d_piv = dalloc<int>(o, 6 * size_t(n_agg));
    s->d_flags = dalloc<int>(o, 2);
    const size_t N = s->wp.n;
    s->d_grid = dalloc<double>(o, 3 * 2 * N * N * N);
    const size_t n = s->n;
    s->d_b = dalloc<double>(o, n);
    s->d_x = dalloc<double>(o, n);
    s->d_basis = dalloc<double>(o, size_t(s->m + 1) * n);
    s->d_z = dalloc<double>(o, n);
    s->d_w = dalloc<double>(o, n);
    s->d_t = dalloc<double>(o, n);
    s->d_r = dalloc<double>(o, n);
    s->d_wt = dalloc<double>(o, 3 * size_t(nb));
    s->d_fl = dalloc<double>(o, 3 * size_t(nb));
    s->d_h = dalloc<double>(o, 2 * size_t(s->m + 1) + 16);
    s->d_part = dalloc<double>(o, std::max(size_t(s->m + 2) * 1024, size_t(96) * cgs_blocks(n)));
    s->d_U = dalloc<double>(o, 6 * size_t(n_agg));
    // small read-backs: GMRES columns, and the Lanczos alpha and beta (lan_max + 2 each)
    HIPCHK(hipHostMalloc((void**)&s->h_small,
                         sizeof(double) * std::max(2 * size_t(s->m + 1) + 8, 2 * size_t(s->lan_max + 2))));
    HIPCHK(hipHostMalloc((void**)&s->h_ctl, sizeof(GmresCtl)));
    s->d_ctl = reinterpret_cast<GmresCtl*>(dalloc<double>(o, (sizeof(GmresCtl) + 7) / 8));
    s->d_H = dalloc<double>(o, size_t(s->m + 1) * s->m);
    s->d_cs = dalloc<double>(o, s->m);
    s->d_sn = dalloc<double>(o, s->m);
    s->d_g = dalloc<double>(o, s->m + 1);
    s->d_y = dalloc<double>(o, s->m);
    s->d_scal = dalloc<double>(o, 2);
    s->d_counters = reinterpret_cast<unsigned*>(dalloc<int>(o, 64));
    HIPCHK(hipMemset(s->d_counters, 0, 64 * sizeof(int)));
    HIPCHK(hipStreamCreateWithFlags(&s->st2, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming));
    s->nw = neighbor_work_create(nb);
    s->nwl = neighbor_work_create(nb);
    if (!s->nw || !s->nwl) throw ApiError(FSD_ENOMEM, "neighbour-list workspace allocation failed");
    HIPCHK(hipHostMalloc((void**)&s->h_flags, 2 * sizeof(int)));
    HIPCHK(hipHostMalloc((void**)&s->h_scal, 4 * sizeof(double)));
    s->h_flags[0] = s->h_flags[1] = 0;
    s->spread = spread_plan_create(nb, s->wp.n, s->wp.support);  // nullptr: grid not a multiple of 4
    upload_tables(s);
    HIPCHK(hipMemcpy(s->d_offsets, off, sizeof(int) * (n_agg + 1), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->d_body, body.data(), sizeof(int) * nb, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->d_xbody, xb.data(), sizeof(double) * 3 * nb, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->d_com, X.data(), sizeof(double) * 3 * n_agg, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->d_quat, q.data(), sizeof(double) * 4 * n_agg, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(s->d_force, 0, sizeof(double) * 6 * n_agg));
    HIPCHK(hipMemcpy(s->d_G, s->G, sizeof(double) * 9, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->d_E, s->E, sizeof(double) * 9, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->d_W, s->W, sizeof(double) * 3, hipMemcpyHostToDevice));
    // initial neighbour capacity from the expected pair count
    const double dens = nb / (L * L * L);
    const double rc = s->rp.r_cut;
    s->ncap = (long long)(nb * (4.19 * rc * rc * rc * dens * 1.3 + 64));
    s->d_ncol = dalloc<uint32_t>(o, size_t(s->ncap));
    if (s->p.r_lub > 0) {
      const double rl = s->p.r_lub;
      s->lcap = (long long)(nb * (4.19 * rl * rl * rl * dens * 2.0 + 16));
      s->d_lcol = dalloc<uint32_t>(o, size_t(s->lcap));
      s->d_lcoef = dalloc<double>(o, 5 * size_t(s->lcap));
      s->lcoef_cap = s->lcap;
    }
    s->have_agg = true;
    s->prepared = false;
    return FSD_OK;
  });
}

fsd_status fsd_set_forces(fsd_system* s, const double* ft) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!ft) return fail(s, FSD_EINVAL, "null forces");
  for (int i = 0; i < 6 * s->na; ++i)
    if (!std::isfinite(ft[i])) return fail(s, FSD_EINVAL, "non-finite force");
  return guarded(s, [&]() -> fsd_status {
    HIPCHK(hipMemcpyAsync(s->d_force, ft, sizeof(double) * 6 * s->na, hipMemcpyHostToDevice, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return FSD_OK;
  });
}

fsd_status fsd_set_bead_forces(fsd_system* s, const double* fb) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!fb) return fail(s, FSD_EINVAL, "null forces");
  for (int i = 0; i < 3 * s->nb; ++i)
    if (!std::isfinite(fb[i])) return fail(s, FSD_EINVAL, "non-finite force");
  return guarded(s, [&]() -> fsd_status {
    prepare(s);
    // Sigma F_P: forces summed, torques r x f, with r the current body vectors
    std::vector<double> r4(4 * size_t(s->nb)), ft(6 * size_t(s->na), 0.0);
    HIPCHK(hipMemcpyAsync(r4.data(), s->d_r4, sizeof(double) * 4 * s->nb, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    for (int j = 0; j < s->na; ++j)
      for (int i = s->h_offsets[j]; i < s->h_offsets[j + 1]; ++i) {
        const double* f = fb + 3 * i;
        const double* r = &r4[4 * size_t(i)];
        ft[6 * j] += f[0];
        ft[6 * j + 1] += f[1];
        ft[6 * j + 2] += f[2];
        ft[6 * j + 3] += r[1] * f[2] - r[2] * f[1];
        ft[6 * j + 4] += r[2] * f[0] - r[0] * f[2];
        ft[6 * j + 5] += r[0] * f[1] - r[1] * f[0];
      }
    HIPCHK(hipMemcpyAsync(s->d_force, ft.data(), sizeof(double) * 6 * s->na, hipMemcpyHostToDevice, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return FSD_OK;
  });
}

fsd_status fsd_set_shear(fsd_system* s, const double g[9]) {
  if (!s || !g) return FSD_EINVAL;
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(g[i])) return fail(s, FSD_EINVAL, "non-finite velocity gradient");
  if (std::fabs(g[0] + g[4] + g[8]) > 1e-12 * (1 + std::fabs(g[0]) + std::fabs(g[4]) + std::fabs(g[8])))
    return fail(s, FSD_EINVAL, "velocity gradient must be traceless");
  if (s->le)
    for (int i = 0; i < 9; ++i)
      if (i != 1 && g[i] != 0) return fail(s, FSD_EINVAL, "the sheared lattice takes simple shear u_x = G_xy y only");
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      s->G[3 * a + b] = g[3 * a + b];
      s->E[3 * a + b] = 0.5 * (g[3 * a + b] + g[3 * b + a]);
    }
  s->W[0] = 0.5 * (g[7] - g[5]);
  s->W[1] = 0.5 * (g[2] - g[6]);
  s->W[2] = 0.5 * (g[3] - g[1]);
  if (!s->have_agg) return FSD_OK;
  return guarded(s, [&]() -> fsd_status {
    HIPCHK(hipMemcpyAsync(s->d_G, s->G, sizeof(double) * 9, hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemcpyAsync(s->d_E, s->E, sizeof(double) * 9, hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemcpyAsync(s->d_W, s->W, sizeof(double) * 3, hipMemcpyHostToDevice, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return FSD_OK;
  });
}

fsd_status fsd_solve_dev(fsd_system* s, double* dU, double* dlam, fsd_solve_info* info) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!dU) return fail(s, FSD_EINVAL, "null output");
  return guarded(s, [&]() -> fsd_status {
    fsd_status r = solve_current(s, info);
    HIPCHK(hipMemcpyAsync(dU, s->d_U, sizeof(double) * 6 * s->na, hipMemcpyDeviceToDevice, s->st));
    if (dlam) HIPCHK(hipMemcpyAsync(dlam, s->d_x, sizeof(double) * 6 * s->nb, hipMemcpyDeviceToDevice, s->st));
    return r;
  });
}

fsd_status fsd_solve(fsd_system* s, double* U, double* lam, fsd_solve_info* info) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!U) return fail(s, FSD_EINVAL, "null output");
  return guarded(s, [&]() -> fsd_status {
    fsd_status r = solve_current(s, info);
    HIPCHK(hipMemcpyAsync(U, s->d_U, sizeof(double) * 6 * s->na, hipMemcpyDeviceToHost, s->st));
    if (lam) HIPCHK(hipMemcpyAsync(lam, s->d_x, sizeof(double) * 6 * s->nb, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return r;
  });
}

fsd_status fsd_step(fsd_system* s, double dt, int n_steps, fsd_solve_info* last) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!(dt > 0) || n_steps < 0) return fail(s, FSD_EINVAL, "dt must be positive and n_steps >= 0");
  return guarded(s, [&]() -> fsd_status {
    fsd_status r = FSD_OK;
    s->bdt = dt;
    for (int k = 0; k < n_steps; ++k) {
      step_before_solve(s);
      r = solve_current(s, last);
      if (r != FSD_OK) return r;
      step_after_solve(s, dt);
    }
    HIPCHK(hipStreamSynchronize(s->st));
    return r;
  });
}

fsd_status fsd_get_state(const fsd_system* cs, double* com, double* quat, double* x_bead) {
  fsd_system* s = const_cast<fsd_system*>(cs);
  fsd_status c = check_ready(s);
  if (c) return c;
  return guarded(s, [&]() -> fsd_status {
    if (com) HIPCHK(hipMemcpyAsync(com, s->d_com, sizeof(double) * 3 * s->na, hipMemcpyDeviceToHost, s->st));
    if (quat) HIPCHK(hipMemcpyAsync(quat, s->d_quat, sizeof(double) * 4 * s->na, hipMemcpyDeviceToHost, s->st));
    if (x_bead) {
      launch_bead_positions(s->nb, s->na, s->d_body, s->d_xbody, s->d_com, s->d_quat, s->L, s->gam(), s->d_r4,
                            s->d_pos4, s->st);
      std::vector<double> r4(4 * size_t(s->nb)), X(3 * size_t(s->na));
      HIPCHK(hipMemcpyAsync(r4.data(), s->d_r4, sizeof(double) * 4 * s->nb, hipMemcpyDeviceToHost, s->st));
      HIPCHK(hipMemcpyAsync(X.data(), s->d_com, sizeof(double) * 3 * s->na, hipMemcpyDeviceToHost, s->st));
      HIPCHK(hipStreamSynchronize(s->st));
      for (int j = 0; j < s->na; ++j)
        for (int i = s->h_offsets[j]; i < s->h_offsets[j + 1]; ++i)
          for (int d = 0; d < 3; ++d) x_bead[3 * i + d] = X[3 * j + d] + r4[4 * size_t(i) + d];
    }
    HIPCHK(hipStreamSynchronize(s->st));
    return FSD_OK;
  });
}

fsd_status fsd_get_velocities(const fsd_system* cs, double* U) {
  fsd_system* s = const_cast<fsd_system*>(cs);
  if (!s || !U) return FSD_EINVAL;
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!s->solved) return fail(s, FSD_ESTATE, "no solve has completed");
  return guarded(s, [&]() -> fsd_status {
    HIPCHK(hipMemcpyAsync(U, s->d_U, sizeof(double) * 6 * s->na, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return FSD_OK;
  });
}

fsd_status fsd_get_stresslets(fsd_system* s, double* S_agg, double* S_mean) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!S_agg && !S_mean) return fail(s, FSD_EINVAL, "fsd_get_stresslets: no output");
  if (!s->solved || !s->prepared || s->sv.rhs_kind != 0)
    return fail(s, FSD_ESTATE, "fsd_get_stresslets: needs a completed solve at the current configuration");
  return guarded(s, [&]() -> fsd_status {
    const int nb = s->nb, na = s->na;
    const size_t nb6 = 6 * size_t(nb);
    if (!s->d_fst) {
      s->d_fst = dalloc<double>(s->owned, 3 * size_t(nb));
      s->d_wst = dalloc<double>(s->owned, 3 * size_t(nb));
      s->d_sst = dalloc<double>(s->owned, 9 * size_t(na));
    }
    // the near-field force on the beads at the solved velocities:
    // -sum_k R_pair (w_i - w_k) - (the strain term), w the rigid-body bead velocities
    const bool lub = s->p.r_lub > 0 && s->nlub > 0;
    launch_zero(s->d_fst, sizeof(double) * 3 * nb, s->st);
    if (lub) {
      launch_bead_rigid_vel(nb, s->d_body, s->d_r4, s->d_x + nb6, s->d_wst, s->st);
      launch_lub_apply(nb, s->d_lrow, s->d_lcol, s->d_lcoef, s->d_wst, s->d_fst, s->st);
      launch_lub_strain(nb, s->d_pos4, s->d_r4, s->L, s->gam(), s->d_lrow, s->d_lcol, s->d_lcoef, s->d_E, s->d_wst,
                        s->st);
      launch_axpby(3 * size_t(nb), -1.0, s->d_wst, 1.0, s->d_fst, s->st);
    }
    // conservative pair forces (the kernel returns their negative) and the near-field
    // Brownian force of this solve
    if (s->pair_forces) {
      launch_pair_forces(nb, s->d_pos4, s->d_body, s->d_nrow, s->d_ncol, s->pf, s->d_wst, 0, s->st);
      launch_axpby(3 * size_t(nb), -1.0, s->d_wst, 1.0, s->d_fst, s->st);
    }
    if (s->p.kT > 0 && s->d_fb) launch_axpby(3 * size_t(nb), 1.0, s->d_fb, 1.0, s->d_fst, s->st);
    launch_stresslets(na, s->d_offsets, s->d_r4, s->d_x, s->d_fst, s->d_sst, s->st);
    std::vector<double> S(9 * size_t(na));
    HIPCHK(hipMemcpyAsync(S.data(), s->d_sst, sizeof(double) * S.size(), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    if (S_agg) std::copy(S.begin(), S.end(), S_agg);
    if (S_mean) {
      const double V = s->L * s->L * s->L;
      for (int k = 0; k < 9; ++k) {
        double t = 0;
        for (int j = 0; j < na; ++j) t += S[9 * size_t(j) + k];
        S_mean[k] = t / V;
      }
    }
    return FSD_OK;
  });
}

fsd_status fsd_get_info(const fsd_system* cs, fsd_info* info) {
  fsd_system* s = const_cast<fsd_system*>(cs);
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!info) return FSD_EINVAL;
  return guarded(s, [&]() -> fsd_status {
    prepare(s);
    info->L = s->L;
    info->xi = s->wp.xi;
    info->r_cut = s->rp.r_cut;
    info->h = s->wp.h;
    info->eta_tilde = s->wp.eta_t;
    info->self_t = s->rp.self_t;
    info->self_r = s->rp.self_r;
    info->grid = s->wp.n;
    info->support = s->wp.support;
    info->n_bead = s->nb;
    info->n_agg = s->na;
    info->nnz_real = s->nnz;
    info->n_lub_pairs = s->nlub;
    return FSD_OK;
  });
}

size_t fsd_estimate_bytes(const fsd_params* p, int32_t nb, int32_t na, double L) {
  if (!p || nb <= 0 || na <= 0 || !(L > 0)) return 0;
  const double a = p->radius;
  const double xi = pick_xi(*p, nb, L);
  const double lnt = std::sqrt(-std::log(p->ewald_tol));
  const double rc = 1.15 * lnt / xi;
  int N = p->grid > 0 ? p->grid : next_smooth(int(std::ceil((2.0 * lnt * xi + 1.0 / a) * L / M_PI)));
  const double dens = nb / (L * L * L);
  const double nnz = nb * (4.19 * rc * rc * rc * dens * 1.3 + 64);
  const double rl = p->r_lub;
  const double nl = rl > 0 ? nb * (4.19 * rl * rl * rl * dens * 2.0 + 16) : 0;
  const double n = 6.0 * (nb + na);
  const int m = p->gmres_restart;
  double bytes = 48.0 * double(N) * N * N + 4.0 * nnz + 44.0 * nl + 8.0 * n * (m + 9) + 200.0 * nb + 400.0 * na +
                 8.0 * (m + 2) * 1024 + 8.0 * 8 * 4100 + (1 << 20);
  if (p->kT > 0) {  // Lanczos basis and partials, Brownian vectors
    const double lm = p->lanczos_maxit > 0 ? p->lanczos_maxit : 100;
    bytes += 8.0 * nb * (6.0 * (lm + 1) + 24) + 8.0 * (lm + 2) * 1024;
  }
  // spreading plan: 3P weights per bead (FP64, FP32 and a staging copy) and up to 27 block
  // slots per bead (keys and values, sorted copies and the sort's temporary storage)
  const int P = p->support > 0 ? p->support : int(std::ceil(2.0 / M_PI * std::log(1.0 / p->ewald_tol))) + 2;
  bytes += double(nb) * (20.0 * 3 * P + 27.0 * 32.0);
  return size_t(bytes);
}

const char* fsd_last_error(const fsd_system* s) { return s ? s->err.c_str() : g_last_error.c_str(); }

void fsd_destroy(fsd_system* s) {
  if (!s) return;
  if (s->st) (void)hipStreamSynchronize(s->st);
  if (s->own_stream && s->st) (void)hipStreamDestroy(s->st);
  delete s;
}

fsd_status fsd_apply_mobility(fsd_system* s, const double* lam, double* u, int parts, int precision) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!lam || !u || parts < 1 || parts > 3) return fail(s, FSD_EINVAL, "bad arguments");
  return guarded(s, [&]() -> fsd_status {
    prepare(s);
    const size_t nb6 = 6 * size_t(s->nb);
    HIPCHK(hipMemcpyAsync(s->d_z, lam, sizeof(double) * nb6, hipMemcpyHostToDevice, s->st));
    if (precision == FSD_MIXED)
      apply_mobility<float>(s, s->d_z, s->d_w, parts);
    else
      apply_mobility<double>(s, s->d_z, s->d_w, parts);
    HIPCHK(hipMemcpyAsync(u, s->d_w, sizeof(double) * nb6, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return FSD_OK;
  });
}

fsd_status fsd_apply_saddle(fsd_system* s, const double* x, double* y, int precision) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!x || !y) return fail(s, FSD_EINVAL, "bad arguments");
  return guarded(s, [&]() -> fsd_status {
    prepare(s);
    HIPCHK(hipMemcpyAsync(s->d_z, x, sizeof(double) * s->n, hipMemcpyHostToDevice, s->st));
    apply_saddle_p(s, s->d_z, s->d_w, precision == FSD_MIXED);
    HIPCHK(hipMemcpyAsync(y, s->d_w, sizeof(double) * s->n, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return FSD_OK;
  });
}

fsd_status fsd_apply_precond(fsd_system* s, const double* r, double* z) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!r || !z) return fail(s, FSD_EINVAL, "bad arguments");
  return guarded(s, [&]() -> fsd_status {
    prepare(s);
    HIPCHK(hipMemcpyAsync(s->d_r, r, sizeof(double) * s->n, hipMemcpyHostToDevice, s->st));
    apply_precond(s, s->d_r, s->d_z);
    HIPCHK(hipMemcpyAsync(z, s->d_z, sizeof(double) * s->n, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return FSD_OK;
  });
}

fsd_status fsd_get_rhs(fsd_system* s, double* b) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!b) return fail(s, FSD_EINVAL, "bad arguments");
  return guarded(s, [&]() -> fsd_status {
    prepare(s);
    assemble_rhs(s);
    HIPCHK(hipMemcpyAsync(b, s->d_b, sizeof(double) * s->n, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return FSD_OK;
  });
}

fsd_status fsd_real_functions(fsd_system* s, int n, const double* r, double* out) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (n < 0 || (n > 0 && (!r || !out))) return fail(s, FSD_EINVAL, "bad arguments");
  // the same interpolation as the real-space kernel, evaluated on the host table
  for (int q = 0; q < n; ++q) {
    if (!(r[q] > 0) || r[q] >= s->rp.r_cut) return fail(s, FSD_EINVAL, "r outside (0, r_cut)");
    double o[5];
    rpy_free(r[q], s->p.radius, s->p.eta, o);
    const double t = r[q] * s->rp.inv_ht;
    const int it = int(t);
    const double f = t - it;
    const double w[4] = {-f * (f - 1) * (f - 2) / 6.0, (f + 1) * (f - 1) * (f - 2) / 2.0,
                         -(f + 1) * f * (f - 2) / 2.0, (f + 1) * f * (f - 1) / 6.0};
    for (int k = 0; k < 5; ++k) {
      double sv = 0;
      for (int m = 0; m < 4; ++m) sv += w[m] * s->h_tab[8 * size_t(it + m) + k];
      out[5 * q + k] = o[k] - sv;
    }
  }
  return FSD_OK;
}

fsd_status fsd_set_graphs(fsd_system* s, int enable, int batch) {
  if (!s || batch < 0 || batch > 64) return FSD_EINVAL;
  return guarded(s, [&]() -> fsd_status {
    HIPCHK(hipStreamSynchronize(s->st));
    s->drop_graphs();
    s->use_graphs = enable != 0;
    if (batch > 0) s->batch = batch;
    return FSD_OK;
  });
}

fsd_status fsd_set_timing(fsd_system* s, int enable) {
  if (!s) return FSD_EINVAL;
  return guarded(s, [&]() -> fsd_status {
    harvest_timers(s);
    for (int k = 0; k < FSD_TIMER_COUNT; ++k) {
      s->t_ms[k] = 0;
      s->t_n[k] = 0;
      s->t_bytes[k] = 0;
    }
    if ((enable != 0) != s->timing) {
      s->drop_graphs();
      launch_timing_mark(s->st);  // brackets the timed launches in a profiler trace
    }
    s->timing = enable != 0;
    return FSD_OK;
  });
}

fsd_status fsd_get_timers(fsd_system* s, double* total_ms, long long* launches, double* bytes) {
  if (!s || !total_ms || !launches) return FSD_EINVAL;
  return guarded(s, [&]() -> fsd_status {
    harvest_timers(s);
    for (int k = 0; k < FSD_TIMER_COUNT; ++k) {
      total_ms[k] = s->t_ms[k];
      launches[k] = s->t_n[k];
      if (bytes) bytes[k] = s->t_bytes[k];
    }
    return FSD_OK;
  });
}

fsd_status fsd_time_kernel(fsd_system* s, int timer, int reps, double* avg_ms) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!avg_ms || reps < 1 || timer < 0 || timer > FSD_TIMER_PRECOND)
    return fail(s, FSD_EINVAL, "fsd_time_kernel: reps >= 1 and a mobility, rigid or preconditioner timer class");
  return guarded(s, [&]() -> fsd_status {
    if (!s->prepared) {  // lists, plan and factors for the current positions
      prepare_begin(s);
      HIPCHK(hipStreamSynchronize(s->st));
      prepare_end(s);
    }
    const bool fp32 = s->p.precision == FSD_MIXED;
    hipEvent_t ev[2] = {nullptr, nullptr};
    HIPCHK(hipEventCreate(&ev[0]));
    HIPCHK(hipEventCreate(&ev[1]));
    float ms = 0;
    try {
      launch_timing_mark(s->st);
      HIPCHK(hipEventRecord(ev[0], s->st));
      for (int r = 0; r < reps; ++r) (void)(fp32 ? replay_one<float>(s, timer) : replay_one<double>(s, timer));
      HIPCHK(hipEventRecord(ev[1], s->st));
      launch_timing_mark(s->st);
      HIPCHK(hipStreamSynchronize(s->st));
      HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
    } catch (...) {
      (void)hipEventDestroy(ev[0]);
      (void)hipEventDestroy(ev[1]);
      throw;
    }
    HIPCHK(hipEventDestroy(ev[0]));
    HIPCHK(hipEventDestroy(ev[1]));
    *avg_ms = double(ms) / reps;
    return FSD_OK;
  });
}

}  // extern "C"

namespace {
// Splitting parameters worth timing in [lo, hi]: for every grid size the Section 3.2 rule
// gives there, the largest xi that still gives it (the cheapest wave space for that grid
// and the shortest real-space cutoff), plus lo itself.
std::vector<double> xi_candidates(const fsd_params& p, double L, double lo, double hi, bool le) {
  const double a = p.radius, lnt = std::sqrt(-std::log(p.ewald_tol));
  const double margin = le ? std::sqrt(1.25) : 1.0;
  auto grid_of = [&](double xi) { return next_smooth(int(std::ceil((2.0 * lnt * xi + 1.0 / a) * L / M_PI * margin))); };
  std::vector<double> out{lo};
  for (int N = grid_of(lo); N <= std::min(grid_of(hi), kMaxGrid); N = next_smooth(N + 1)) {
    double xi = std::min(hi, (N * M_PI / (L * margin) - 1.0 / a) / (2.0 * lnt));
    while (xi > lo && grid_of(xi) > N) xi *= 1.0 - 1e-12;
    if (xi > lo * (1.0 + 1e-9)) out.push_back(xi);
  }
  return out;
}

// average ms of one saddle-operator apply in the system's Arnoldi precision, replayed back to
// back on the system stream (lists and factors built first)
double time_saddle(fsd_system* s, int reps) {
  if (!s->prepared) {
    prepare_begin(s);
    HIPCHK(hipStreamSynchronize(s->st));
    prepare_end(s);
  }
  const bool fp32 = s->p.precision == FSD_MIXED;
  launch_zero(s->d_z, sizeof(double) * s->n, s->st);
  hipEvent_t ev[2] = {nullptr, nullptr};
  HIPCHK(hipEventCreate(&ev[0]));
  HIPCHK(hipEventCreate(&ev[1]));
  float ms = 0;
  try {
    apply_saddle_p(s, s->d_z, s->d_t, fp32);  // warm
    HIPCHK(hipEventRecord(ev[0], s->st));
    for (int r = 0; r < reps; ++r) apply_saddle_p(s, s->d_z, s->d_t, fp32);
    HIPCHK(hipEventRecord(ev[1], s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
  } catch (...) {
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    throw;
  }
  HIPCHK(hipEventDestroy(ev[0]));
  HIPCHK(hipEventDestroy(ev[1]));
  return double(ms) / reps;
}
}  // namespace

extern "C" {

fsd_status fsd_autotune_xi(fsd_system* s, double xi_lo, double xi_hi, int reps, double* xi_out, double* ms_out) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!xi_out || reps < 1 || !(xi_lo > 0) || !(xi_hi >= xi_lo))
    return fail(s, FSD_EINVAL, "fsd_autotune_xi: 0 < xi_lo <= xi_hi, reps >= 1");
  return guarded(s, [&]() -> fsd_status {
    const int na = s->na, nb = s->nb;
    std::vector<double> com(3 * size_t(na)), quat(4 * size_t(na)), xb(3 * size_t(nb));
    HIPCHK(hipMemcpyAsync(com.data(), s->d_com, sizeof(double) * com.size(), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipMemcpyAsync(quat.data(), s->d_quat, sizeof(double) * quat.size(), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipMemcpyAsync(xb.data(), s->d_xbody, sizeof(double) * xb.size(), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    double best = s->wp.xi, best_ms = 1e300;
    for (double xi : xi_candidates(s->p, s->L, xi_lo, xi_hi, s->le)) {
      fsd_params p = s->p;
      p.xi = xi;
      p.grid = 0;
      fsd_system* t = nullptr;
      if (fsd_create(&p, s->st, &t) != FSD_OK) continue;
      double ms = -1;
      if (fsd_init_box(t, s->L, s->L, s->L) == FSD_OK && (!s->le || fsd_set_lees_edwards(t, 1, s->strain) == FSD_OK) &&
          fsd_init_aggregates(t, na, s->h_offsets.data(), xb.data(), com.data(), quat.data()) == FSD_OK &&
          fsd_set_shear(t, s->G) == FSD_OK) {
        const fsd_status r = guarded(t, [&]() -> fsd_status {
          ms = time_saddle(t, reps);
          return FSD_OK;
        });
        if (r != FSD_OK) ms = -1;
      }
      fsd_destroy(t);
      if (ms > 0 && ms < best_ms) best_ms = ms, best = xi;
    }
    if (!(best_ms < 1e300)) throw ApiError(FSD_EINVAL, "fsd_autotune_xi: no candidate could be set up");
    *xi_out = best;
    if (ms_out) *ms_out = best_ms;
    return FSD_OK;
  });
}

fsd_status fsd_autotune_tiles(fsd_system* s, int reps, int* lines_b, int* green_g) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (reps < 1) return fail(s, FSD_EINVAL, "fsd_autotune_tiles: reps >= 1");
  return guarded(s, [&]() -> fsd_status {
    const int N = s->wp.n, rb = s->p.precision == FSD_MIXED ? 4 : 8;
    auto timed = [&](int cls) {
      double ms = 0;
      const fsd_status r = fsd_time_kernel(s, cls, reps, &ms);
      if (r != FSD_OK) throw ApiError(r, s->err);
      return ms;
    };
    // the y pass stands for both line passes (same body, strides differ)
    int best_b = 0;
    double best = 1e300;
    for (int B : {1, 2, 4, 8, 16, 32, 64}) {
      if (!tile_b_fits(N, B, rb)) continue;
      s->wp.tile_b = B;
      const double ms = timed(FSD_TIMER_FFT_Y);
      if (ms < best) best = ms, best_b = B;
    }
    int best_g = 0;
    best = 1e300;
    for (int G : {1, 2, 3, 4, 6, 8}) {
      if (!tile_g_fits(N, G, rb)) continue;
      s->wp.tile_g = G;
      const double ms = timed(FSD_TIMER_GREEN);
      if (ms < best) best = ms, best_g = G;
    }
    s->wp.tile_b = best_b;
    s->wp.tile_g = best_g;
    s->drop_graphs();  // captured launches carry the old shapes
    if (lines_b) *lines_b = best_b;
    if (green_g) *green_g = best_g;
    return FSD_OK;
  });
}

fsd_status fsd_set_pair_forces(fsd_system* s, double k_n, double hamaker, double Z, double kappa, double h_c,
                               double r_cut) {
  fsd_status c = check_ready(s);
  if (c) return c;
  const double a = s->p.radius;
  const double v[6] = {k_n, hamaker, Z, kappa, h_c, r_cut};
  for (double x : v)
    if (!std::isfinite(x)) return fail(s, FSD_EINVAL, "non-finite pair-force parameter");
  if (k_n == 0 && hamaker == 0 && Z == 0) {
    s->pair_forces = false;
    return FSD_OK;
  }
  if (k_n < 0 || hamaker < 0) return fail(s, FSD_EINVAL, "k_n and the Hamaker constant must be >= 0");
  if (hamaker > 0 && !(h_c > 0)) return fail(s, FSD_EINVAL, "the van der Waals term needs h_c > 0");
  if (Z != 0 && !(kappa > 0)) return fail(s, FSD_EINVAL, "the double layer needs kappa > 0");
  if (!(r_cut >= 2 * a) || r_cut > s->rp.r_cut)
    return fail(s, FSD_EINVAL, "r_cut must lie in [2a, the real-space cutoff]");
  s->pf = PairForceParams{k_n, hamaker, Z, kappa, h_c, r_cut, a, s->L, s->gam()};
  s->pair_forces = true;
  return FSD_OK;
}

fsd_status fsd_set_roughness(fsd_system* s, double alpha, double h0) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!std::isfinite(alpha) || !std::isfinite(h0)) return fail(s, FSD_EINVAL, "non-finite roughness parameter");
  if (alpha < 0) return fail(s, FSD_EINVAL, "the roughness strength must be >= 0");
  if (alpha > 0) {
    if (!(s->p.r_lub > 0)) return fail(s, FSD_EINVAL, "roughness acts through lubrication, which is off");
    if (!(h0 > 0) || 2 * s->p.radius + h0 > s->p.r_lub)
      return fail(s, FSD_EINVAL, "h0 must lie in (0, r_lub - 2a]");
  }
  const double ra = alpha > 0 ? alpha : 0.0, rh = alpha > 0 ? h0 : 0.0;
  if (ra != s->rough_alpha || rh != s->rough_h0) {
    s->rough_alpha = ra;
    s->rough_h0 = rh;
    s->prepared = false;  // the lubrication coefficients and the preconditioner change
  }
  return FSD_OK;
}

fsd_status fsd_set_lees_edwards(fsd_system* s, int enable, double strain) {
  if (!s) return FSD_EINVAL;
  if (!std::isfinite(strain)) return fail(s, FSD_EINVAL, "non-finite strain");
  if (enable) {
    if (!s->le && s->have_agg) return fail(s, FSD_ESTATE, "switch the sheared lattice on before fsd_init_aggregates");
    for (int i = 0; i < 9; ++i)
      if (i != 1 && s->G[i] != 0) return fail(s, FSD_EINVAL, "the sheared lattice takes simple shear u_x = G_xy y only");
  }
  const double g = strain - std::floor(strain + 0.5);  // the lattice repeats with period 1
  if (bool(enable) != s->le || (enable && g != s->strain)) {
    // centroids need no refolding: bead positions are folded into the lattice at every
    // preparation, and the next step folds the centroids
    s->le = enable != 0;
    s->strain = s->le ? g : 0.0;
    s->prepared = false;
  }
  return FSD_OK;
}

fsd_status fsd_set_warm_start(fsd_system* s, int mode) {
  if (!s) return FSD_EINVAL;
  if (mode < 0 || mode > 3) return fail(s, FSD_EINVAL, "warm-start mode 0 to 3");
  if (mode != s->warm) s->nprev = 0;
  s->warm = mode;
  return FSD_OK;
}

fsd_status fsd_get_strain(const fsd_system* s, double* strain) {
  if (!s || !strain) return FSD_EINVAL;
  *strain = s->le ? s->strain : 0.0;
  return FSD_OK;
}

fsd_status fsd_get_pair_forces(fsd_system* s, double* f_bead) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!f_bead) return fail(s, FSD_EINVAL, "null output");
  return guarded(s, [&]() -> fsd_status {
    prepare(s);
    const size_t n3 = 3 * size_t(s->nb);
    if (!s->pair_forces) {
      std::fill(f_bead, f_bead + n3, 0.0);
      return FSD_OK;
    }
    launch_pair_forces(s->nb, s->d_pos4, s->d_body, s->d_nrow, s->d_ncol, s->pf, s->d_t, 0, s->st);
    HIPCHK(hipMemcpyAsync(f_bead, s->d_t, sizeof(double) * n3, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    for (size_t i = 0; i < n3; ++i) f_bead[i] = -f_bead[i];
    return FSD_OK;
  });
}

fsd_status fsd_set_drift(fsd_system* s, int mode, double eps) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (mode < 0 || mode > 2 || !std::isfinite(eps)) return fail(s, FSD_EINVAL, "drift mode 0, 1 or 2, finite eps");
  s->drift_mode = mode;
  s->drift_eps = eps;
  return FSD_OK;
}

fsd_status fsd_rfd_drift(fsd_system* s, const double* dq, double* u_drift) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!u_drift) return fail(s, FSD_EINVAL, "null output");
  if (dq)
    for (int i = 0; i < 6 * s->na; ++i)
      if (!std::isfinite(dq[i])) return fail(s, FSD_EINVAL, "non-finite dq");
  return guarded(s, [&]() -> fsd_status {
    rfd_drift(s, dq);
    HIPCHK(hipMemcpyAsync(u_drift, s->d_udrift, sizeof(double) * 6 * s->na, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return FSD_OK;
  });
}

fsd_status fsd_set_brownian(fsd_system* s, double dt, uint64_t step, uint64_t stream) {
  if (!s) return FSD_EINVAL;
  if (!(dt > 0)) return fail(s, FSD_EINVAL, "dt must be positive");
  s->bdt = dt;
  s->bstep = step;
  s->bstream = stream;
  return FSD_OK;
}

fsd_status fsd_set_noise(fsd_system* s, const double* psi_w, const double* psi_r, const double* psi_nf) {
  fsd_status c = check_ready(s);
  if (c) return c;
  return guarded(s, [&]() -> fsd_status {
    prepare(s);
    ensure_brownian(s);
    const size_t nb = s->nb, n3 = size_t(s->wp.n) * s->wp.n * s->wp.n;
    if (psi_w && !s->d_psi_w) s->d_psi_w = dalloc<double>(s->owned, 3 * n3);
    if (psi_w) HIPCHK(hipMemcpyAsync(s->d_psi_w, psi_w, sizeof(double) * 3 * n3, hipMemcpyHostToDevice, s->st));
    if (psi_r) HIPCHK(hipMemcpyAsync(s->d_psi_r, psi_r, sizeof(double) * 6 * nb, hipMemcpyHostToDevice, s->st));
    if (psi_nf) HIPCHK(hipMemcpyAsync(s->d_psi_nf, psi_nf, sizeof(double) * 3 * nb, hipMemcpyHostToDevice, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    s->psi_w_set = psi_w != nullptr;
    s->psi_r_set = psi_r != nullptr;
    s->psi_nf_set = psi_nf != nullptr;
    return FSD_OK;
  });
}

fsd_status fsd_brownian_terms(fsd_system* s, double* u_B, double* f_B, int* lanczos_steps) {
  fsd_status c = check_ready(s);
  if (c) return c;
  if (!u_B || !f_B) return fail(s, FSD_EINVAL, "null output");
  return guarded(s, [&]() -> fsd_status {
    prepare(s);
    brownian_terms(s);
    HIPCHK(hipMemcpyAsync(u_B, s->d_ub, sizeof(double) * 6 * s->nb, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipMemcpyAsync(f_B, s->d_fb, sizeof(double) * 3 * s->nb, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    if (lanczos_steps) {
      lanczos_steps[0] = s->lan_its[0];
      lanczos_steps[1] = s->lan_its[1];
    }
    return FSD_OK;
  });
}

fsd_status fsd_philox4x64(uint64_t k0, uint64_t k1, const uint64_t counter[4], int n_blocks, uint64_t* out) {
  if (!counter || !out || n_blocks < 1) return FSD_EINVAL;
  std::vector<void*> owned;
  fsd_status rc = FSD_OK;
  try {
    uint64_t* d = reinterpret_cast<uint64_t*>(dalloc<double>(owned, 4 * size_t(n_blocks)));
    launch_philox_raw(k0, k1, counter, n_blocks, d, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpy(out, d, sizeof(uint64_t) * 4 * size_t(n_blocks), hipMemcpyDeviceToHost));
  } catch (const ApiError& e) {
    rc = e.code;
    g_last_error = e.what();
  } catch (const std::exception& e) {
    rc = FSD_EDEVICE;
    g_last_error = e.what();
  }
  for (void* q : owned) (void)hipFree(q);
  return rc;
}

fsd_status fsd_normals(uint64_t k0, uint64_t k1, uint64_t purpose, uint64_t step, size_t n, double* out) {
  if (!out || n == 0) return FSD_EINVAL;
  std::vector<void*> owned;
  fsd_status rc = FSD_OK;
  try {
    double* d = dalloc<double>(owned, n);
    launch_normals(n, NoiseKey{k0, k1, purpose, step}, d, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpy(out, d, sizeof(double) * n, hipMemcpyDeviceToHost));
  } catch (const ApiError& e) {
    rc = e.code;
    g_last_error = e.what();
  } catch (const std::exception& e) {
    rc = FSD_EDEVICE;
    g_last_error = e.what();
  }
  for (void* q : owned) (void)hipFree(q);
  return rc;
}

fsd_status fsd_fft3d(int n, int sign, double* data) {
  if (!data || (sign != 1 && sign != -1)) return FSD_EINVAL;
  FftPlan plan;
  if (!make_plan(n, plan) || n > 512) return FSD_EINVAL;
  std::vector<void*> owned;
  fsd_status rc = FSD_OK;
  try {
    const size_t count = 2 * size_t(n) * n * n;
    double* d = dalloc<double>(owned, count);
    double* tw = dalloc<double>(owned, 2 * size_t(n));
    std::vector<double> h(2 * n);
    for (int t = 0; t < n; ++t) {
      h[2 * t] = std::cos(2.0 * M_PI * t / n);
      h[2 * t + 1] = -std::sin(2.0 * M_PI * t / n);
    }
    HIPCHK(hipMemcpy(tw, h.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(d, data, sizeof(double) * count, hipMemcpyHostToDevice));
    launch_fft3d<double>(d, 1, count, plan, tw, sign, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpy(data, d, sizeof(double) * count, hipMemcpyDeviceToHost));
  } catch (const ApiError& e) {
    rc = e.code;
    g_last_error = e.what();
  } catch (const std::exception& e) {
    rc = FSD_EDEVICE;
    g_last_error = e.what();
  }
  for (void* q : owned) (void)hipFree(q);
  return rc;
}

fsd_status fsd_fft3d_noalloc(int n, int sign, double* d_data, void* hip_stream) {
  if (!d_data || (sign != 1 && sign != -1)) {
    g_last_error = "fsd_fft3d_noalloc: a device buffer and sign +-1";
    return FSD_EINVAL;
  }
  FftPlan plan;
  if (n > kNoAllocFftMax || !make_plan(n, plan)) {
    g_last_error = "fsd_fft3d_noalloc: n must be a product of 2, 3 and 5 of at most " +
                   std::to_string(kNoAllocFftMax) + " (the size of its fixed twiddle array)";
    return FSD_EINVAL;
  }
  const hipError_t e = launch_fft3d_noalloc(n, sign, d_data, plan, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) {
    g_last_error = std::string("fsd_fft3d_noalloc: ") + hipGetErrorString(e);
    return FSD_EDEVICE;
  }
  return FSD_OK;
}

}  // extern "C"

// ==========================================================================================
// batches of independent systems
// ==========================================================================================

struct fsd_batch {
  size_t budget = 0, used = 0;
  std::vector<fsd_system*> slot;
  std::vector<size_t> bytes;
  std::vector<fsd_solve_info> last;
  std::string err;
  // multi-system launches (fused mode): descriptor and block tables on the device and
  // a stream of their own
  bool fused = true;
  // captured lock-step segments (j0, cnt) of the current tables; recaptured whenever the
  // tables are uploaded again (another set of systems, other block counts or LDS)
  struct SegGraph {
    int j0, cnt;
    hipGraphExec_t exec;
  };
  bool use_graphs = true;
  std::vector<SegGraph> seg_graphs;
  // the systems' stop flags gathered after each segment and read back in one copy
  int* d_stop = nullptr;
  int* h_stop = nullptr;  // pinned
  int stop_cap = 0;
  unsigned long long table_version = 0, graphs_version = ~0ull;
  void drop_graphs() {
    for (auto& g : seg_graphs) (void)hipGraphExecDestroy(g.exec);
    seg_graphs.clear();
  }
  hipStream_t st = nullptr;
  bool own_stream = false;
  BatchDesc* d_desc = nullptr;
  int* d_off = nullptr;
  int cap = 0;
  std::vector<BatchDesc> h_desc;
  std::vector<int> h_off;  // BK_COUNT x (cap + 1)
  int nsys = 0, prec = 0;
  int total[BK_COUNT] = {0};
  size_t shm[BK_COUNT] = {0};
  std::vector<fsd_system*> cyc;  // the systems of the tables, in table order
  std::vector<char> active;      // cyc[k] still iterating in the current cycle (timing only)
  // LDS per workgroup allowed to the z/y line passes and to the x+Green pass (0: no cap).
  // A multi-system launch reserves the largest system's LDS for every workgroup, so one
  // system's wide tile lowers the occupancy of all; fsd_batch_autotune_tiles measures these.
  size_t lds_cap[2] = {0, 0};
  // event timing of the multi-system launches (fsd_batch_set_timing)
  struct Pend {
    int cls;
    double bytes;
    hipEvent_t a, b;
  };
  bool timing = false;
  double t_ms[FSD_TIMER_COUNT] = {0}, t_bytes[FSD_TIMER_COUNT] = {0};
  long long t_n[FSD_TIMER_COUNT] = {0};
  std::vector<hipEvent_t> ev_pool;
  size_t ev_next = 0;
  std::vector<Pend> pending;
  ~fsd_batch() {
    drop_graphs();
    if (d_stop) (void)hipFree(d_stop);
    if (h_stop) (void)hipHostFree(h_stop);
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    if (d_desc) (void)hipFree(d_desc);
    if (d_off) (void)hipFree(d_off);
    if (st && own_stream) (void)hipStreamDestroy(st);
  }
};

namespace {
size_t system_bytes(const fsd_system* s) {
  fsd_params p = s->p;
  p.grid = s->wp.n;  // the grid it holds (larger on a sheared lattice than the rule gives)
  return fsd_estimate_bytes(&p, s->nb, s->na, s->L);
}

// One solve (and optionally an Euler step) for every admitted system.  Each system
// runs on its own stream; the host advances their state machines round-robin, so
// while it waits on one system the others keep the GPU busy.
fsd_status batch_run_streams(fsd_batch* b, const std::vector<fsd_system*>& act, double dt, bool integrate) {
  fsd_status worst = FSD_OK;
  std::vector<char> done(act.size(), 0);
  for (size_t k = 0; k < act.size(); ++k) {
    fsd_system* s = act[k];
    if (integrate) s->bdt = dt;
    fsd_status r = guarded(s, [&]() -> fsd_status {
      if (integrate) step_before_solve(s);
      solve_begin(s);
      return FSD_OK;
    });
    if (r != FSD_OK) {
      done[k] = 1;
      s->sv.status = r;
      worst = r;
    }
  }
  size_t remaining = 0;
  for (char d : done) remaining += d ? 0 : 1;
  // poll: advance whichever system's stream has drained; block only when none has
  while (remaining > 0) {
    bool progressed = false;
    for (size_t k = 0; k < act.size(); ++k) {
      if (done[k]) continue;
      fsd_system* s = act[k];
      const hipError_t q = hipStreamQuery(s->st);
      if (q == hipErrorNotReady) continue;
      progressed = true;
      bool more = false;
      fsd_status r = guarded(s, [&]() -> fsd_status {
        HIPCHK(q);
        more = solve_advance(s);
        return FSD_OK;
      });
      if (r != FSD_OK) {
        s->sv.status = r;  // a failure retires only this system's solve
        more = false;
      }
      if (!more) {
        done[k] = 1;
        --remaining;
        if (s->sv.status != FSD_OK && worst == FSD_OK) worst = s->sv.status;
        if (integrate && s->sv.status == FSD_OK) {
          const fsd_status ri = guarded(s, [&]() -> fsd_status {
            step_after_solve(s, dt);
            return FSD_OK;
          });
          if (ri != FSD_OK) {
            s->sv.status = ri;
            if (worst == FSD_OK) worst = ri;
          }
        }
      }
    }
    if (!progressed) {
      for (size_t k = 0; k < act.size(); ++k)
        if (!done[k]) {
          (void)hipStreamSynchronize(act[k]->st);
          break;
        }
    }
  }
  for (auto* s : act) (void)hipStreamSynchronize(s->st);
  return worst;
}
}  // namespace

namespace {
BatchDesc make_desc(fsd_system* s, int prec) {
  BatchDesc d{};
  const bool lub = s->p.r_lub > 0 && s->nlub > 0;
  const int N = s->wp.n;
  d.nb = s->nb;
  d.na = s->na;
  d.n = s->n;
  d.pos4 = s->d_pos4;
  d.r4 = s->d_r4;
  d.body = s->d_body;
  d.offsets = s->d_offsets;
  d.nrow = s->d_nrow;
  d.ncol = s->d_ncol;
  d.tab64 = s->d_tab64;
  d.tab32 = s->d_tab32;
  d.rp = s->rp;
  d.wp = s->wp;
  d.plan = s->plan;
  d.tw64 = s->d_tw64;
  d.tw32 = s->d_tw32;
  d.grid = s->d_grid;
  d.bl = lines_b_of(s->wp, prec ? 4 : 8);
  d.bg = green_g_of(s->wp);
  spread_plan_desc(s->spread, prec, d);
  d.lrow = lub ? s->d_lrow : nullptr;
  d.lcol = s->d_lcol;
  d.lcoef = s->d_lcoef;
  d.lu = s->d_lu;
  d.piv = s->d_piv;
  d.drag_t = s->drag_t;
  d.drag_r = s->drag_r;
  d.basis = s->d_basis;
  d.z = s->d_z;
  d.w = s->d_w;
  d.r = s->d_r;
  d.scal = s->d_scal;
  d.part = s->d_part;
  d.h1 = s->d_h;
  d.h2 = s->d_h + (s->m + 1);
  d.hn2 = s->d_h + 2 * (s->m + 1);
  d.H = s->d_H;
  d.gcs = s->d_cs;
  d.gsn = s->d_sn;
  d.g = s->d_g;
  d.counters = s->d_counters;
  d.ctl = s->d_ctl;
  d.ncgs = cgs_blocks(s->n);
  return d;
}

// can these systems share multi-system launches? (same precision and restart length,
// CGS in registers, gather spreading on 8^3 blocks, no per-launch timing)
bool fusable(const std::vector<fsd_system*>& act) {
  if (act.empty()) return false;
  const int prec = act[0]->p.precision, m = act[0]->m;
  for (auto* s : act) {
    if (s->p.precision != prec || s->m != m || !cgs_fits(m + 1) || s->timing || s->le) return false;
    if (!s->spread || s->wp.n % 8 || !s->wp.gtab) return false;
  }
  return true;
}

// upload descriptors and block tables for the systems in cyc (skipped when unchanged)
void set_tables(fsd_batch* b, const std::vector<fsd_system*>& cyc, int prec) {
  const int ns = int(cyc.size());
  std::vector<BatchDesc> desc(ns);
  for (int k = 0; k < ns; ++k) {
    BatchDesc& d = desc[k];
    d = make_desc(cyc[k], prec);
    // narrower tiles (fewer lines, fewer row pairs) within the batch's LDS caps
    if (b->lds_cap[0])
      while (d.bl > 1 && batch_shm(d, BK_FFT_OUTER, prec) > b->lds_cap[0]) d.bl /= 2;
    if (b->lds_cap[1])
      while (d.bg > 1 && batch_shm(d, BK_FFT_GREEN, prec) > b->lds_cap[1]) --d.bg;
  }
  std::vector<int> off(size_t(BK_COUNT) * (ns + 1), 0);
  int total[BK_COUNT];
  size_t shm[BK_COUNT];
  for (int kind = 0; kind < BK_COUNT; ++kind) {
    int acc = 0;
    size_t mx = 0;
    for (int k = 0; k < ns; ++k) {
      off[size_t(kind) * (ns + 1) + k] = acc;
      acc += batch_blocks(desc[k], kind);
      mx = std::max(mx, batch_shm(desc[k], kind, prec));
    }
    off[size_t(kind) * (ns + 1) + ns] = acc;
    total[kind] = acc;
    shm[kind] = mx;
  }
  b->cyc = cyc;
  b->active.assign(ns, 1);
  const bool same = ns == b->nsys && prec == b->prec && off == b->h_off &&
                    std::memcmp(desc.data(), b->h_desc.data(), sizeof(BatchDesc) * ns) == 0;
  if (same) return;
  ++b->table_version;  // captured segments hold the old block counts and LDS sizes
  if (ns > b->cap) {
    if (b->d_desc) HIPCHK(hipFree(b->d_desc));
    if (b->d_off) HIPCHK(hipFree(b->d_off));
    b->d_desc = nullptr;
    b->d_off = nullptr;
    HIPCHK(hipMalloc(&b->d_desc, sizeof(BatchDesc) * ns));
    HIPCHK(hipMalloc(&b->d_off, sizeof(int) * BK_COUNT * (ns + 1)));
    b->cap = ns;
  }
  HIPCHK(hipMemcpyAsync(b->d_desc, desc.data(), sizeof(BatchDesc) * ns, hipMemcpyHostToDevice, b->st));
  HIPCHK(hipMemcpyAsync(b->d_off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice, b->st));
  HIPCHK(hipStreamSynchronize(b->st));
  b->h_desc.swap(desc);
  b->h_off.swap(off);
  b->nsys = ns;
  b->prec = prec;
  std::copy(total, total + BK_COUNT, b->total);
  std::copy(shm, shm + BK_COUNT, b->shm);
}

// algorithmic HBM bytes of one system's share of a multi-system launch of timer class cls
// (as the single-system launches count them; nq basis vectors in the Gram-Schmidt passes)
double batch_share_bytes(const fsd_system* s, int cls, int prec, int nq) {
  const double full = prec ? grid_bytes<float>(s) : grid_bytes<double>(s), beads = 80.0 * s->nb;
  const double n = double(s->n);
  switch (cls) {
    case FSD_TIMER_PRECOND: return 8.0 * n * 3 + 32.0 * s->nb + 312.0 * s->na;
    case FSD_TIMER_REAL: return real_bytes(s);
    case FSD_TIMER_SPREAD: return full + beads;
    case FSD_TIMER_FFT_FIRST:
    case FSD_TIMER_FFT_Y:
    case FSD_TIMER_GREEN:
    case FSD_TIMER_FFT_LAST: return 2.0 * full;
    case FSD_TIMER_INTERP: return full + beads + 80.0 * s->nb + 48.0 * s->na;
    case FSD_TIMER_RIGID: return rigid_bytes(s);
    case FSD_TIMER_CGS_DOT: return 8.0 * n * (nq + 1);
    case FSD_TIMER_CGS_UPDATE:
    case FSD_TIMER_CGS_NORM: return 8.0 * n * (nq + 2);
    default: return 0.0;
  }
}

hipEvent_t batch_event(fsd_batch* b) {
  if (b->ev_next == b->ev_pool.size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    b->ev_pool.push_back(e);
  }
  return b->ev_pool[b->ev_next++];
}

// after the batch stream has drained: add the timed launches to the accumulators
void batch_harvest(fsd_batch* b) {
  if (b->pending.empty()) return;
  HIPCHK(hipStreamSynchronize(b->st));
  for (auto& p : b->pending) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
    b->t_ms[p.cls] += ms;
    b->t_n[p.cls] += 1;
    b->t_bytes[p.cls] += p.bytes;
  }
  b->pending.clear();
  b->ev_next = 0;
}

// one multi-system launch; with timing on it is bracketed by events on the batch stream and
// counts the bytes of the systems still iterating
template <typename L>
void batch_launch(fsd_batch* b, int cls, int nq, L&& launch) {
  if (!b->timing) {
    launch();
    return;
  }
  hipEvent_t ea = batch_event(b), eb = batch_event(b);
  HIPCHK(hipEventRecord(ea, b->st));
  launch();
  HIPCHK(hipEventRecord(eb, b->st));
  double by = 0;
  for (size_t k = 0; k < b->cyc.size(); ++k)
    if (b->active[k]) by += batch_share_bytes(b->cyc[k], cls, b->prec, nq);
  b->pending.push_back({cls, by, ea, eb});
}

// Arnoldi steps j0 .. j0 + cnt - 1 of every system in the tables, one launch per kernel
void batch_segment_body(fsd_batch* b, int j0, int cnt) {
  const int ns = b->nsys, prec = b->prec;
  auto off = [&](int kind) { return b->d_off + size_t(kind) * (ns + 1); };
  auto mob = [&](int cls, int kind, int stage) {
    batch_launch(b, cls, 0, [&] {
      launch_batch_mobility(kind, prec, stage, b->d_desc, off(kind), ns, b->total[kind], b->shm[kind], b->st);
    });
  };
  for (int j = j0; j < j0 + cnt; ++j) {
    // inside a segment the Arnoldi update of step j-1 rides in the preconditioner of step j;
    // the segment's last step makes its update alone (kb_arnoldi_reduce), so the host reads
    // current stop flags after every segment
    batch_launch(b, FSD_TIMER_PRECOND, 0, [&] {
      launch_batch_solver(j > j0 ? BK_PRECOND_ARNOLDI : BK_PRECOND, j, 0, b->d_desc, off(BK_PRECOND), ns,
                          b->total[BK_PRECOND], b->st);
    });
    mob(FSD_TIMER_REAL, BK_REAL, 0);
    mob(FSD_TIMER_SPREAD, BK_SPREAD, 0);
    static const int cls_of[5] = {FSD_TIMER_FFT_FIRST, FSD_TIMER_FFT_Y, FSD_TIMER_GREEN, FSD_TIMER_FFT_Y,
                                  FSD_TIMER_FFT_LAST};
    for (int stage = 0; stage < 5; ++stage) {
      const int kind = (stage == 0 || stage == 4) ? BK_FFT_OUTER : (stage == 2 ? BK_FFT_GREEN : BK_FFT_MID);
      mob(cls_of[stage], kind, stage);
    }
    mob(FSD_TIMER_INTERP, BK_INTERP, 0);
    batch_launch(b, FSD_TIMER_RIGID, 0, [&] {
      launch_batch_solver(BK_AGG, j, 0, b->d_desc, off(BK_AGG), ns, b->total[BK_AGG], b->st);
    });
    static const int cgs_cls[3] = {FSD_TIMER_CGS_DOT, FSD_TIMER_CGS_UPDATE, FSD_TIMER_CGS_NORM};
    for (int mode = 0; mode < 3; ++mode)
      batch_launch(b, cgs_cls[mode], j + 1, [&] {
        launch_batch_solver(BK_CGS, j, mode, b->d_desc, off(BK_CGS), ns, b->total[BK_CGS], b->st);
      });
    if (j == j0 + cnt - 1) launch_batch_solver(BK_ARNOLDI, j, 0, b->d_desc, nullptr, ns, ns, b->st);
  }
}

// One lock-step segment.  Without timing it replays a captured graph of the segment's
// launches, captured on first use for the current tables: the first cycle of every time
// step runs the same systems with the same tables, so its segments are captured once.
void batch_segment(fsd_batch* b, int j0, int cnt) {
  if (!b->use_graphs || b->timing) {
    batch_segment_body(b, j0, cnt);
    HIPCHK(hipGetLastError());
    return;
  }
  if (b->graphs_version != b->table_version) {
    b->drop_graphs();
    b->graphs_version = b->table_version;
  }
  hipGraphExec_t exec = nullptr;
  for (auto& g : b->seg_graphs)
    if (g.j0 == j0 && g.cnt == cnt) exec = g.exec;
  if (!exec) {
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
    try {
      batch_segment_body(b, j0, cnt);
    } catch (...) {
      (void)hipStreamEndCapture(b->st, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    HIPCHK(hipStreamEndCapture(b->st, &graph));
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) throw HipError(std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    b->seg_graphs.push_back({j0, cnt, exec});
  }
  HIPCHK(hipGraphLaunch(exec, b->st));
}

// Advances every solve in sys to its end, each on its own stream with its captured GMRES
// segments, polling whichever stream has drained (a failure ends only that solve).
void advance_solves(const std::vector<fsd_system*>& sys) {
  std::vector<char> live(sys.size(), 1);
  size_t left = sys.size();
  while (left > 0) {
    bool progressed = false;
    for (size_t k = 0; k < sys.size(); ++k) {
      if (!live[k]) continue;
      fsd_system* s = sys[k];
      const hipError_t q = hipStreamQuery(s->st);
      if (q == hipErrorNotReady) continue;
      progressed = true;
      bool more = false;
      const fsd_status r = guarded(s, [&]() -> fsd_status {
        HIPCHK(q);
        more = solve_advance(s);
        return FSD_OK;
      });
      if (r != FSD_OK) {
        s->sv.status = r;
        more = false;
      }
      if (!more) {
        live[k] = 0;
        --left;
      }
    }
    if (!progressed)
      for (size_t k = 0; k < sys.size(); ++k)
        if (live[k]) {
          (void)hipStreamSynchronize(sys[k]->st);
          break;
        }
  }
}

// at most this many systems still iterating: they leave the lock step and finish alone
constexpr size_t kSoloTail = 4;

// Lock-step solve of all admitted systems with multi-system launches.  Preparation,
// right-hand sides and GMRES cycle starts/ends run per system on the systems' own
// streams (they overlap); the Arnoldi steps of all systems whose cycle is running are
// one launch per kernel on the batch stream.  Systems that converge drop out at the
// next cycle boundary; the others restart together (equal restart length).  Once no
// more than kSoloTail systems are left after a cycle (the slow tail of an uneven
// batch), they finish on their own streams with captured segments, where a launch over a
// few small systems would cost its launch latency; the timing pass keeps them in the
// lock step.
fsd_status batch_run_fused(fsd_batch* b, const std::vector<fsd_system*>& act, double dt, bool integrate) {
  using SS = fsd_system::SolveState;
  const size_t na = act.size();
  std::vector<char> done(na, 0);
  fsd_status worst = FSD_OK;
  auto fail_one = [&](size_t k, fsd_status r) {
    act[k]->sv.status = r;
    act[k]->sv.phase = SS::DONE;
    done[k] = 1;
    if (worst == FSD_OK) worst = r;
  };
  for (size_t k = 0; k < na; ++k) {
    fsd_system* s = act[k];
    if (integrate) s->bdt = dt;
    fsd_status r = guarded(s, [&]() -> fsd_status {
      if (integrate) step_before_solve(s);
      solve_begin(s);
      return FSD_OK;
    });
    if (r != FSD_OK) fail_one(k, r);
  }
  for (size_t k = 0; k < na; ++k) {  // PREP: lists, right-hand side, first cycle start
    if (done[k]) continue;
    fsd_system* s = act[k];
    fsd_status r = guarded(s, [&]() -> fsd_status {
      HIPCHK(hipStreamSynchronize(s->st));
      (void)solve_advance(s);
      return FSD_OK;
    });
    if (r != FSD_OK) fail_one(k, r);
  }
  const int S = b->timing ? 1 : std::max(1, std::min(act[0]->batch, act[0]->m));
  const int prec = act[0]->p.precision == FSD_MIXED ? 1 : 0;
  int cycles = 0;  // lock-step cycles run
  while (true) {
    std::vector<fsd_system*> cyc;
    for (size_t k = 0; k < na; ++k) {  // cycle starts drained: finish or join the cycle
      if (done[k]) continue;
      fsd_system* s = act[k];
      bool more = false;
      fsd_status r = guarded(s, [&]() -> fsd_status {
        HIPCHK(hipStreamSynchronize(s->st));
        check_flags(s);
        const GmresCtl& c = *s->h_ctl;
        auto& v = s->sv;
        if (c.resid <= v.tol || c.stop) {
          v.its += c.its;
          v.rel = c.resid;
          finish_solve(s, c.resid <= v.tol);
          return FSD_OK;
        }
        more = true;
        return FSD_OK;
      });
      if (r != FSD_OK) {
        fail_one(k, r);
        continue;
      }
      if (more)
        cyc.push_back(s);
      else
        done[k] = 1;
    }
    if (cyc.empty()) break;
    if (!b->timing && cycles > 0 && cyc.size() <= kSoloTail) {
      advance_solves(cyc);
      break;
    }
    ++cycles;
    fsd_status r = guarded(cyc[0], [&]() -> fsd_status {
      set_tables(b, cyc, prec);
      for (int j0 = 0;; j0 += S) {
        const int cnt = std::min(S, cyc[0]->m - j0);
        batch_segment(b, j0, cnt);
        const int ns = int(cyc.size());
        if (ns > b->stop_cap) {
          if (b->d_stop) HIPCHK(hipFree(b->d_stop));
          if (b->h_stop) HIPCHK(hipHostFree(b->h_stop));
          b->d_stop = nullptr;
          b->h_stop = nullptr;
          b->stop_cap = 0;
          HIPCHK(hipMalloc(&b->d_stop, sizeof(int) * ns));
          HIPCHK(hipHostMalloc(&b->h_stop, sizeof(int) * ns));
          b->stop_cap = ns;
        }
        launch_batch_gather_stop(b->d_desc, ns, b->d_stop, b->st);
        HIPCHK(hipMemcpyAsync(b->h_stop, b->d_stop, sizeof(int) * ns, hipMemcpyDeviceToHost, b->st));
        HIPCHK(hipStreamSynchronize(b->st));
        bool all = true;
        for (int k = 0; k < ns; ++k) {
          b->active[k] = !b->h_stop[k];
          all = all && b->h_stop[k];
        }
        if (all || j0 + cnt >= cyc[0]->m) break;
      }
      for (auto* s : cyc) {  // cycle end and the next cycle start, per system
        seg_cycle_end(s);
        ++s->sv.restarts;
        if (s->p.precision == FSD_MIXED) ++s->sv.outer;
        seg_cycle_start(s);
        s->sv.phase = SS::START;
      }
      return FSD_OK;
    });
    if (r != FSD_OK) {
      for (size_t k = 0; k < na; ++k)
        if (!done[k]) fail_one(k, r);
      break;
    }
  }
  for (size_t k = 0; k < na; ++k) {
    fsd_system* s = act[k];
    if (integrate && s->sv.status == FSD_OK) {
      fsd_status r = guarded(s, [&]() -> fsd_status {
        step_after_solve(s, dt);
        return FSD_OK;
      });
      if (r != FSD_OK) {
        s->sv.status = r;
        if (worst == FSD_OK) worst = r;
      }
    }
    if (s->sv.status != FSD_OK && worst == FSD_OK) worst = s->sv.status;
  }
  for (auto* s : act) (void)hipStreamSynchronize(s->st);
  batch_harvest(b);
  return worst;
}

// one solve (and optionally an Euler step) for every admitted system: multi-system
// launches when the systems allow them, otherwise one stream per system
// counts (per slot, may be null: one each): the solves (and steps) each slot makes in this
// call.  Rounds of multi-system launches (or streams) run until every slot has made its
// count; a slot whose solve fails stops there.
fsd_status batch_run(fsd_batch* b, double dt, bool integrate, const int* counts = nullptr) {
  std::vector<int> left(b->slot.size(), 0);
  for (size_t q = 0; q < b->slot.size(); ++q)
    if (b->slot[q]) left[q] = counts ? std::max(counts[q], 0) : 1;
  fsd_status worst = FSD_OK;
  while (true) {
    std::vector<fsd_system*> act;
    std::vector<size_t> qs;
    for (size_t q = 0; q < b->slot.size(); ++q)
      if (b->slot[q] && left[q] > 0) {
        act.push_back(b->slot[q]);
        qs.push_back(q);
      }
    if (act.empty()) break;
    const fsd_status r = (b->fused && fusable(act)) ? batch_run_fused(b, act, dt, integrate)
                                                    : batch_run_streams(b, act, dt, integrate);
    for (size_t k = 0; k < act.size(); ++k) {
      b->last[qs[k]] = info_of(act[k]);
      left[qs[k]] = act[k]->sv.status == FSD_OK ? left[qs[k]] - 1 : 0;
    }
    if (worst == FSD_OK) worst = r;
  }
  return worst;
}
}  // namespace

extern "C" {

fsd_status fsd_batch_create(size_t mem_budget_bytes, int max_slots, void* hip_stream, fsd_batch** out) {
  if (!out || max_slots < 1 || max_slots > 4096) return FSD_EINVAL;
  auto* b = new (std::nothrow) fsd_batch;
  if (!b) return FSD_ENOMEM;
  b->budget = mem_budget_bytes;
  if (hip_stream) {
    b->st = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return FSD_EDEVICE;
    }
    b->own_stream = true;
  }
  b->slot.assign(max_slots, nullptr);
  b->bytes.assign(max_slots, 0);
  b->last.assign(max_slots, fsd_solve_info{});
  *out = b;
  return FSD_OK;
}

fsd_status fsd_batch_admit(fsd_batch* b, fsd_system* s, int* slot) {
  if (!b || !s || !slot) return FSD_EINVAL;
  if (!s->have_agg) return FSD_ESTATE;
  for (auto* q : b->slot)
    if (q == s) return FSD_EINVAL;
  const size_t need = system_bytes(s);
  if (b->used + need > b->budget) {
    b->err = "memory budget exhausted";
    return FSD_EBUSY;
  }
  for (size_t q = 0; q < b->slot.size(); ++q)
    if (!b->slot[q]) {
      b->slot[q] = s;
      b->bytes[q] = need;
      b->used += need;
      b->last[q] = fsd_solve_info{};
      *slot = int(q);
      return FSD_OK;
    }
  b->err = "no free slot";
  return FSD_EBUSY;
}

fsd_status fsd_batch_retire(fsd_batch* b, int slot) {
  if (!b || slot < 0 || slot >= int(b->slot.size()) || !b->slot[slot]) return FSD_EINVAL;
  b->used -= b->bytes[slot];
  b->slot[slot] = nullptr;
  b->bytes[slot] = 0;
  return FSD_OK;
}

fsd_status fsd_batch_solve(fsd_batch* b) {
  if (!b) return FSD_EINVAL;
  return batch_run(b, 0.0, false);
}

fsd_status fsd_batch_step(fsd_batch* b, double dt) {
  if (!b || !(dt > 0)) return FSD_EINVAL;
  return batch_run(b, dt, true);
}

fsd_status fsd_batch_step_counts(fsd_batch* b, double dt, const int* n_steps) {
  if (!b || !(dt > 0) || !n_steps) return FSD_EINVAL;
  for (size_t q = 0; q < b->slot.size(); ++q)
    if (n_steps[q] < 0) return FSD_EINVAL;
  return batch_run(b, dt, true, n_steps);
}

fsd_status fsd_batch_slot_info(const fsd_batch* b, int slot, fsd_solve_info* info) {
  if (!b || !info || slot < 0 || slot >= int(b->slot.size())) return FSD_EINVAL;
  *info = b->last[slot];
  return FSD_OK;
}

size_t fsd_batch_used_bytes(const fsd_batch* b) { return b ? b->used : 0; }

fsd_status fsd_batch_set_fused(fsd_batch* b, int enable) {
  if (!b) return FSD_EINVAL;
  b->fused = enable != 0;
  return FSD_OK;
}

fsd_status fsd_batch_set_graphs(fsd_batch* b, int enable) {
  if (!b) return FSD_EINVAL;
  b->use_graphs = enable != 0;
  if (!b->use_graphs) b->drop_graphs();
  return FSD_OK;
}

fsd_status fsd_batch_set_timing(fsd_batch* b, int enable) {
  if (!b) return FSD_EINVAL;
  try {
    batch_harvest(b);
  } catch (const std::exception& e) {
    b->err = e.what();
    return FSD_EDEVICE;
  }
  b->timing = enable != 0;
  std::fill(b->t_ms, b->t_ms + FSD_TIMER_COUNT, 0.0);
  std::fill(b->t_bytes, b->t_bytes + FSD_TIMER_COUNT, 0.0);
  std::fill(b->t_n, b->t_n + FSD_TIMER_COUNT, 0LL);
  return FSD_OK;
}

fsd_status fsd_batch_get_timers(fsd_batch* b, double* total_ms, long long* launches, double* bytes) {
  if (!b || !total_ms || !launches) return FSD_EINVAL;
  try {
    batch_harvest(b);
  } catch (const std::exception& e) {
    b->err = e.what();
    return FSD_EDEVICE;
  }
  for (int k = 0; k < FSD_TIMER_COUNT; ++k) {
    total_ms[k] = b->t_ms[k];
    launches[k] = b->t_n[k];
    if (bytes) bytes[k] = b->t_bytes[k];
  }
  return FSD_OK;
}

fsd_status fsd_batch_time_kernel(fsd_batch* b, int timer, int reps, double* avg_ms, double* bytes_per_launch) {
  if (!b || !avg_ms || reps < 1 || timer < 0 || timer > FSD_TIMER_PRECOND) return FSD_EINVAL;
  std::vector<fsd_system*> act;
  for (auto* s : b->slot)
    if (s) act.push_back(s);
  if (act.empty() || !fusable(act)) {
    b->err = "fsd_batch_time_kernel: needs admitted systems that share multi-system launches";
    return FSD_ESTATE;
  }
  fsd_system* s0 = act[0];
  return guarded(s0, [&]() -> fsd_status {
    for (auto* s : act)
      if (!s->prepared) {  // lists, plan and factors for the current positions
        prepare_begin(s);
        HIPCHK(hipStreamSynchronize(s->st));
        prepare_end(s);
      }
    for (auto* s : act) HIPCHK(hipStreamSynchronize(s->st));
    const int prec = s0->p.precision == FSD_MIXED ? 1 : 0;
    set_tables(b, act, prec);
    // every system iterating: the kernels return early for a raised stop flag
    for (auto* s : act) HIPCHK(hipMemsetAsync(&s->d_ctl->stop, 0, sizeof(int), b->st));
    const int ns = b->nsys;
    auto off = [&](int kind) { return b->d_off + size_t(kind) * (ns + 1); };
    auto one = [&]() {
      switch (timer) {
        case FSD_TIMER_PRECOND:
          launch_batch_solver(BK_PRECOND, 0, 0, b->d_desc, off(BK_PRECOND), ns, b->total[BK_PRECOND], b->st);
          break;
        case FSD_TIMER_RIGID:
          launch_batch_solver(BK_AGG, 0, 0, b->d_desc, off(BK_AGG), ns, b->total[BK_AGG], b->st);
          break;
        default: {
          int kind = BK_REAL, stage = 0;
          if (timer == FSD_TIMER_SPREAD) kind = BK_SPREAD;
          if (timer == FSD_TIMER_FFT_FIRST) kind = BK_FFT_OUTER;
          if (timer == FSD_TIMER_FFT_LAST) kind = BK_FFT_OUTER, stage = 4;
          if (timer == FSD_TIMER_FFT_Y) kind = BK_FFT_MID, stage = 1;
          if (timer == FSD_TIMER_GREEN) kind = BK_FFT_GREEN, stage = 2;
          if (timer == FSD_TIMER_INTERP) kind = BK_INTERP;
          launch_batch_mobility(kind, prec, stage, b->d_desc, off(kind), ns, b->total[kind], b->shm[kind], b->st);
        }
      }
    };
    hipEvent_t ev[2] = {nullptr, nullptr};
    HIPCHK(hipEventCreate(&ev[0]));
    HIPCHK(hipEventCreate(&ev[1]));
    float ms = 0;
    try {
      one();  // warm
      launch_timing_mark(b->st);
      HIPCHK(hipEventRecord(ev[0], b->st));
      for (int r = 0; r < reps; ++r) one();
      HIPCHK(hipEventRecord(ev[1], b->st));
      launch_timing_mark(b->st);
      HIPCHK(hipStreamSynchronize(b->st));
      HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
    } catch (...) {
      (void)hipEventDestroy(ev[0]);
      (void)hipEventDestroy(ev[1]);
      throw;
    }
    HIPCHK(hipEventDestroy(ev[0]));
    HIPCHK(hipEventDestroy(ev[1]));
    // the stop flags raised again: the next solve starts its own cycles
    const int one_flag = 1;
    for (auto* s : act) HIPCHK(hipMemcpyAsync(&s->d_ctl->stop, &one_flag, sizeof(int), hipMemcpyHostToDevice, b->st));
    HIPCHK(hipStreamSynchronize(b->st));
    *avg_ms = double(ms) / reps;
    if (bytes_per_launch) {
      double by = 0;
      for (auto* s : act) by += batch_share_bytes(s, timer, prec, 0);
      *bytes_per_launch = by;
    }
    return FSD_OK;
  });
}

fsd_status fsd_batch_set_lds_caps(fsd_batch* b, size_t lines_lds, size_t green_lds) {
  if (!b) return FSD_EINVAL;
  b->lds_cap[0] = lines_lds;
  b->lds_cap[1] = green_lds;
  return FSD_OK;
}

fsd_status fsd_batch_autotune_tiles(fsd_batch* b, int reps, size_t* lines_lds, size_t* green_lds) {
  if (!b || reps < 1) return FSD_EINVAL;
  constexpr size_t kCaps[] = {16u << 10, 24u << 10, 32u << 10, 40u << 10, 48u << 10, 0};
  const int timers[2] = {FSD_TIMER_FFT_Y, FSD_TIMER_GREEN};
  const size_t keep[2] = {b->lds_cap[0], b->lds_cap[1]};
  for (int w = 0; w < 2; ++w) {
    double best = 1e300;
    size_t best_cap = 0;
    for (size_t cap : kCaps) {
      b->lds_cap[w] = cap;
      double ms = 0;
      const fsd_status r = fsd_batch_time_kernel(b, timers[w], reps, &ms, nullptr);
      if (r != FSD_OK) {
        b->lds_cap[0] = keep[0];
        b->lds_cap[1] = keep[1];
        return r;
      }
      if (ms < best) best = ms, best_cap = cap;
    }
    b->lds_cap[w] = best_cap;
  }
  if (lines_lds) *lines_lds = b->lds_cap[0];
  if (green_lds) *green_lds = b->lds_cap[1];
  return FSD_OK;
}

void fsd_batch_destroy(fsd_batch* b) { delete b; }

}  // extern "C"
