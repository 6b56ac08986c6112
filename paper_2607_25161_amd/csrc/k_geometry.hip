// Geometry kernels: rigid-body kinematics, neighbour lists, lubrication pair
// coefficients and the per-aggregate factorisation of the preconditioner.
#include <hipcub/hipcub.hpp>

#include "fsd_impl.hpp"
#include "pair_code.hpp"

namespace fsd {

namespace {
constexpr int kThreads = 256;
inline int nblocks(long long n, int t = kThreads) { return int((n + t - 1) / t); }

__device__ inline void quat_rotate(const double* q, const double* v, double* out) {
  // rotation matrix of the unit quaternion (w, x, y, z) applied to v
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  out[0] = (1 - 2 * (y * y + z * z)) * v[0] + 2 * (x * y - w * z) * v[1] + 2 * (x * z + w * y) * v[2];
  out[1] = 2 * (x * y + w * z) * v[0] + (1 - 2 * (x * x + z * z)) * v[1] + 2 * (y * z - w * x) * v[2];
  out[2] = 2 * (x * z - w * y) * v[0] + 2 * (y * z + w * x) * v[1] + (1 - 2 * (x * x + y * y)) * v[2];
}

__device__ inline double wrap01(double p, double L) {
  double q = p - L * floor(p / L);
  return (q >= L) ? q - L : q;
}

// fold a centroid into [-L/2, L/2)^3 of the lattice of strain gam: y first, each period of
// y moving x by gam L, then x and z
__device__ inline void fold_centroid(double* c, double L, double gam) {
  const double ny = floor((c[1] + 0.5 * L) / L);
  c[1] -= ny * L;
  c[0] -= ny * gam * L;
  for (int d = 0; d < 3; ++d) {
    double x = c[d];
    x -= L * floor((x + 0.5 * L) / L);
    if (x >= 0.5 * L) x -= L;
    c[d] = x;
  }
}
}  // namespace

// Eq. `EM3`: x_i = X_j + R(q_j) x_body,i.  r4 holds the body vector R x_body,
// pos4 the bead centre in sheared coordinates (x - gam y, y, z), each folded into [0, L)
// (the Cartesian position itself when gam = 0).
__global__ void k_bead_positions(int nb, const int* __restrict__ body, const double* __restrict__ xbody,
                                 const double* __restrict__ com, const double* __restrict__ quat, double L,
                                 double gam, double4* __restrict__ r4, double4* __restrict__ pos4) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const int j = body[i];
  double r[3];
  quat_rotate(quat + 4 * j, xbody + 3 * i, r);
  r4[i] = make_double4(r[0], r[1], r[2], 0.0);
  const double x = com[3 * j] + r[0], y = com[3 * j + 1] + r[1], z = com[3 * j + 2] + r[2];
  pos4[i] = make_double4(wrap01(x - gam * y, L), wrap01(y, L), wrap01(z, L), 0.0);
}

void launch_bead_positions(int nb, int na, const int* body, const double* xbody, const double* com,
                           const double* quat, double L, double gam, double* r4, double* pos4, hipStream_t st) {
  (void)na;
  k_bead_positions<<<nblocks(nb), kThreads, 0, st>>>(nb, body, xbody, com, quat, L, gam, (double4*)r4,
                                                     (double4*)pos4);
}

// Eqs. `EM1` and `EM2`: X += U dt; q += (dt/2) (0, W) (x) q, normalised; X folded
// into [-L/2, L/2)^3 of the lattice of strain gam.
__global__ void k_integrate(int na, const double* __restrict__ U, double dt, double L, double gam,
                            double* __restrict__ com, double* __restrict__ quat) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= na) return;
  double c3[3];
  for (int c = 0; c < 3; ++c) c3[c] = com[3 * j + c] + U[6 * j + c] * dt;
  fold_centroid(c3, L, gam);
  for (int c = 0; c < 3; ++c) com[3 * j + c] = c3[c];
  const double ox = U[6 * j + 3], oy = U[6 * j + 4], oz = U[6 * j + 5];
  double w = quat[4 * j], x = quat[4 * j + 1], y = quat[4 * j + 2], z = quat[4 * j + 3];
  // (0, o) (x) (w, v) = (-o.v, w o + o x v)
  const double h = 0.5 * dt;
  const double dw = -(ox * x + oy * y + oz * z);
  const double dx = w * ox + (oy * z - oz * y);
  const double dy = w * oy + (oz * x - ox * z);
  const double dz = w * oz + (ox * y - oy * x);
  w += h * dw;
  x += h * dx;
  y += h * dy;
  z += h * dz;
  const double inv = 1.0 / sqrt(w * w + x * x + y * y + z * z);
  quat[4 * j] = w * inv;
  quat[4 * j + 1] = x * inv;
  quat[4 * j + 2] = y * inv;
  quat[4 * j + 3] = z * inv;
}

// Displaced configuration of the random finite differences for the Brownian drift
// (Appendix A, Eq. `rfd`): centroid com0 + h dq_t (wrapped as by the integrator) and
// orientation r(h dq_r) (x) quat0, with the exact rotation quaternion
// r(phi) = (cos(|phi|/2), sin(|phi|/2) phi / |phi|).
__global__ void k_displace(int na, const double* __restrict__ com0, const double* __restrict__ quat0,
                           const double* __restrict__ dq, double h, double L, double gam, double* __restrict__ com,
                           double* __restrict__ quat) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= na) return;
  double c3[3];
  for (int c = 0; c < 3; ++c) c3[c] = com0[3 * j + c] + h * dq[6 * j + c];
  fold_centroid(c3, L, gam);
  for (int c = 0; c < 3; ++c) com[3 * j + c] = c3[c];
  const double px = h * dq[6 * j + 3], py = h * dq[6 * j + 4], pz = h * dq[6 * j + 5];
  const double ang = sqrt(px * px + py * py + pz * pz);
  const double rw = cos(0.5 * ang), sc = ang > 0 ? sin(0.5 * ang) / ang : 0.0;
  const double rx = sc * px, ry = sc * py, rz = sc * pz;
  const double w = quat0[4 * j], x = quat0[4 * j + 1], y = quat0[4 * j + 2], z = quat0[4 * j + 3];
  // (rw, r) (x) (w, v) = (rw w - r.v, rw v + w r + r x v)
  double qw = rw * w - (rx * x + ry * y + rz * z);
  double qx = rw * x + w * rx + (ry * z - rz * y);
  double qy = rw * y + w * ry + (rz * x - rx * z);
  double qz = rw * z + w * rz + (rx * y - ry * x);
  const double inv = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  quat[4 * j] = qw * inv;
  quat[4 * j + 1] = qx * inv;
  quat[4 * j + 2] = qy * inv;
  quat[4 * j + 3] = qz * inv;
}

void launch_displace(int na, const double* com0, const double* quat0, const double* dq, double h, double L,
                     double gam, double* com, double* quat, hipStream_t st) {
  k_displace<<<nblocks(na), kThreads, 0, st>>>(na, com0, quat0, dq, h, L, gam, com, quat);
}

void launch_integrate(int na, const double* U, double dt, double L, double gam, double* com, double* quat,
                      hipStream_t st) {
  k_integrate<<<nblocks(na), kThreads, 0, st>>>(na, U, dt, L, gam, com, quat);
}

// ------------------------------------------------------------------------------------------
// neighbour lists
// ------------------------------------------------------------------------------------------


struct NeighborWork {
  int nb = 0;
  int ncell_cap = 0;
  int nc = 0;  // cells per side of the last count phase
  int *keys_in = nullptr, *keys_out = nullptr, *vals_in = nullptr, *vals_out = nullptr;
  int *cell_start = nullptr, *cell_end = nullptr, *counts = nullptr;
  void* temp = nullptr;
  size_t temp_bytes = 0;
  int* total = nullptr;  // pinned host, row count of the last build
};

NeighborWork* neighbor_work_create(int nb) {
  auto* w = new NeighborWork;
  w->nb = nb;
  bool ok = hipMalloc(&w->keys_in, sizeof(int) * nb) == hipSuccess &&
            hipMalloc(&w->keys_out, sizeof(int) * nb) == hipSuccess &&
            hipMalloc(&w->vals_in, sizeof(int) * nb) == hipSuccess &&
            hipMalloc(&w->vals_out, sizeof(int) * nb) == hipSuccess &&
            hipMalloc(&w->counts, sizeof(int) * (nb + 1)) == hipSuccess &&
            hipHostMalloc(&w->total, sizeof(int)) == hipSuccess;
  size_t b1 = 0, b2 = 0;
  hipcub::DeviceRadixSort::SortPairs(nullptr, b1, w->keys_in, w->keys_out, w->vals_in, w->vals_out, nb);
  hipcub::DeviceScan::ExclusiveSum(nullptr, b2, w->counts, w->counts, nb + 1);
  w->temp_bytes = b1 > b2 ? b1 : b2;
  ok = ok && hipMalloc(&w->temp, w->temp_bytes) == hipSuccess;
  if (!ok) {
    neighbor_work_destroy(w);
    return nullptr;
  }
  return w;
}

void neighbor_work_destroy(NeighborWork* w) {
  if (!w) return;
  (void)hipFree(w->keys_in);
  (void)hipFree(w->keys_out);
  (void)hipFree(w->vals_in);
  (void)hipFree(w->vals_out);
  (void)hipFree(w->counts);
  (void)hipFree(w->cell_start);
  (void)hipFree(w->cell_end);
  (void)hipFree(w->temp);
  if (w->total) (void)hipHostFree(w->total);
  delete w;
}

__global__ void k_cell_keys(int nb, const double4* __restrict__ pos, double cs, int nc, int* keys, int* vals) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const double4 p = pos[i];
  int cx = min(nc - 1, int(p.x / cs)), cy = min(nc - 1, int(p.y / cs)), cz = min(nc - 1, int(p.z / cs));
  keys[i] = (cz * nc + cy) * nc + cx;
  vals[i] = i;
}

// [start, end) of every cell c in the sorted keys, by binary search (empty cells get
// start == end), so no clearing of the two arrays is needed
__global__ void k_cell_bounds(int nb, int ncell, const int* __restrict__ keys, int* start, int* end) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  int lo = 0, hi = nb;  // first key >= c
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (keys[mid] < c) lo = mid + 1; else hi = mid;
  }
  int e = lo, h2 = nb;  // first key > c
  while (e < h2) {
    const int mid = (e + h2) >> 1;
    if (keys[mid] <= c) e = mid + 1; else h2 = mid;
  }
  start[c] = lo;
  end[c] = e;
}

// One wavefront per bead scans the 27 surrounding cells (nc >= 3, so each cell is visited
// once and the minimum image is unique), its lanes testing 64 candidates of a cell at a
// time; a ballot gives each hit its place, so a row lists its pairs cell by cell in sorted
// order whatever the wavefront width.  Cells live in sheared coordinates; their side covers
// the cutoff sphere's sheared extent r_c sqrt(1 + gam^2), and distances are Cartesian.
template <bool FILL>
__global__ __launch_bounds__(256) void k_cell_pairs(int nb, const double4* __restrict__ pos,
                                                    const int* __restrict__ body, double L, double gam, double cs,
                                                    int nc, double rc2, int exclude_same_body,
                                                    const int* __restrict__ start, const int* __restrict__ end,
                                                    const int* __restrict__ sorted, int* counts,
                                                    const int* __restrict__ rowptr, uint32_t* __restrict__ col) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= nb) return;  // whole wavefronts leave together
  if (!FILL && i == 0 && lane == 0) counts[nb] = 0;  // the scan's last input: rowptr[nb] = total
  const double4 p = pos[i];
  const int bi = body[i];
  const int cx = min(nc - 1, int(p.x / cs)), cy = min(nc - 1, int(p.y / cs)), cz = min(nc - 1, int(p.z / cs));
  const unsigned long long below = (1ull << lane) - 1ull;
  int cnt = 0;
  const int base = FILL ? rowptr[i] : 0;
  for (int dz = -1; dz <= 1; ++dz) {
    const int z = (cz + dz + nc) % nc;
    for (int dy = -1; dy <= 1; ++dy) {
      const int y = (cy + dy + nc) % nc;
      for (int dx = -1; dx <= 1; ++dx) {
        const int x = (cx + dx + nc) % nc;
        const int c = (z * nc + y) * nc + x;
        const int k1 = end[c];
        for (int k0 = start[c]; k0 < k1; k0 += 64) {
          const int k = k0 + lane;
          bool hit = false;
          uint32_t entry = 0;
          if (k < k1) {
            const int j = sorted[k];
            if (j != i && !(exclude_same_body && body[j] == bi)) {
              const double4 q = pos[j];
              double ddx = p.x - q.x, ddy = p.y - q.y, ddz = p.z - q.z;
              const double sx = -rint(ddx / L), sy = -rint(ddy / L), sz = -rint(ddz / L);
              ddx += sx * L;
              ddy += sy * L;
              ddz += sz * L;
              ddx += gam * ddy;
              hit = ddx * ddx + ddy * ddy + ddz * ddz < rc2;
              if (FILL && hit) entry = pack_entry(j, int(sx), int(sy), int(sz));
            }
          }
          const unsigned long long m = __ballot(hit);
          if (FILL && hit) col[base + cnt + __popcll(m & below)] = entry;
          cnt += __popcll(m);
        }
      }
    }
  }
  if (!FILL && lane == 0) counts[i] = cnt;
}

// Small boxes (fewer than 3 cells per side): all pairs and all images within
// the cutoff, including images of a bead itself.
template <bool FILL>
__global__ void k_brute_pairs(int nb, const double4* __restrict__ pos, const int* __restrict__ body, double L,
                              double gam, double rc2, int nmax, int exclude_same_body, int* counts,
                              const int* __restrict__ rowptr, uint32_t* __restrict__ col) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  if (!FILL && i == 0) counts[nb] = 0;  // the scan's last input: rowptr[nb] = total
  const double4 p = pos[i];
  const int bi = body[i];
  int cnt = 0;
  const int base = FILL ? rowptr[i] : 0;
  for (int j = 0; j < nb; ++j) {
    if (exclude_same_body && body[j] == bi) continue;
    const double4 q = pos[j];
    for (int sz = -nmax; sz <= nmax; ++sz)
      for (int sy = -nmax; sy <= nmax; ++sy)
        for (int sx = -nmax; sx <= nmax; ++sx) {
          if (j == i && sx == 0 && sy == 0 && sz == 0) continue;
          const double ddy = p.y - q.y + sy * L, ddz = p.z - q.z + sz * L;
          const double ddx = p.x - q.x + sx * L + gam * ddy;
          if (ddx * ddx + ddy * ddy + ddz * ddz < rc2) {
            if (FILL) col[base + cnt] = pack_entry(j, sx, sy, sz);
            ++cnt;
          }
        }
  }
  if (!FILL) counts[i] = cnt;
}

// Count phase: per-bead pair counts, exclusive scan into rowptr, and an
// asynchronous copy of the total into pinned memory (valid once the stream drains).
hipError_t neighbors_count(NeighborWork* w, int nb, const double* pos4v, const int* body, double L, double gam,
                           double cutoff, bool exclude_same_body, int* rowptr, hipStream_t st) {
  const double4* pos = (const double4*)pos4v;
  const double rc2 = cutoff * cutoff;
  const double reach = cutoff * sqrt(1.0 + gam * gam);  // sheared extent of the cutoff sphere
  int nc = int(L / reach);
  if (nc > 1024) nc = 1024;
  w->nc = nc;
  hipError_t e;
  if (nc >= 3) {
    const double cs = L / nc;
    const int ncell = nc * nc * nc;
    if (ncell > w->ncell_cap) {
      (void)hipFree(w->cell_start);
      (void)hipFree(w->cell_end);
      w->cell_start = w->cell_end = nullptr;
      w->ncell_cap = 0;
      if ((e = hipMalloc(&w->cell_start, sizeof(int) * ncell)) != hipSuccess) return e;
      if ((e = hipMalloc(&w->cell_end, sizeof(int) * ncell)) != hipSuccess) return e;
      w->ncell_cap = ncell;
    }
    k_cell_keys<<<nblocks(nb), kThreads, 0, st>>>(nb, pos, cs, nc, w->keys_in, w->vals_in);
    int bits = 1;
    while ((1 << bits) < ncell) ++bits;
    size_t tb = w->temp_bytes;
    if ((e = hipcub::DeviceRadixSort::SortPairs(w->temp, tb, w->keys_in, w->keys_out, w->vals_in, w->vals_out, nb, 0,
                                                 bits, st)) != hipSuccess)
      return e;
    k_cell_bounds<<<nblocks(ncell), kThreads, 0, st>>>(nb, ncell, w->keys_out, w->cell_start, w->cell_end);
    k_cell_pairs<false><<<nblocks(nb, 4), kThreads, 0, st>>>(nb, pos, body, L, gam, cs, nc, rc2, exclude_same_body,
                                                           w->cell_start, w->cell_end, w->vals_out, w->counts,
                                                           nullptr, nullptr);
  } else {
    const int nmax = int(reach / L) + 1;
    k_brute_pairs<false><<<nblocks(nb), kThreads, 0, st>>>(nb, pos, body, L, gam, rc2, nmax, exclude_same_body,
                                                            w->counts, nullptr, nullptr);
  }
  if (nb == 0 && (e = hipMemsetAsync(w->counts, 0, sizeof(int), st)) != hipSuccess) return e;
  size_t tb = w->temp_bytes;
  if ((e = hipcub::DeviceScan::ExclusiveSum(w->temp, tb, w->counts, rowptr, nb + 1, st)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(w->total, rowptr + nb, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  return hipGetLastError();
}

long long neighbors_total(const NeighborWork* w) { return *w->total; }

// Fill phase (after the count phase has drained; col holds at least the total).
hipError_t neighbors_fill(NeighborWork* w, int nb, const double* pos4v, const int* body, double L, double gam,
                          double cutoff, bool exclude_same_body, const int* rowptr, uint32_t* col, hipStream_t st) {
  const double4* pos = (const double4*)pos4v;
  const double rc2 = cutoff * cutoff;
  const int nc = w->nc;
  if (nc >= 3) {
    const double cs = L / nc;
    k_cell_pairs<true><<<nblocks(nb, 4), kThreads, 0, st>>>(nb, pos, body, L, gam, cs, nc, rc2, exclude_same_body,
                                                          w->cell_start, w->cell_end, w->vals_out, nullptr, rowptr,
                                                          col);
  } else {
    const int nmax = int(cutoff * sqrt(1.0 + gam * gam) / L) + 1;
    k_brute_pairs<true><<<nblocks(nb), kThreads, 0, st>>>(nb, pos, body, L, gam, rc2, nmax, exclude_same_body, nullptr,
                                                           rowptr, col);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// lubrication pairs: the stated model (squeeze X and shear Y of two equal spheres,
// shifted to vanish at r = 3a) acting on translational disturbance velocities.  Surface
// roughness (Section 4.2, Eq. `tan_fric`) adds to Y, below the asperity height h0, the
// correction alpha (a/h0)(h0/h - 3h/h0 + 2h^2/h0^2) = alpha (a/h)(1 - t)^2 (1 + 2t), t = h/h0,
// with h = eps a the regularised gap
// ------------------------------------------------------------------------------------------

__global__ void k_lub_setup(int nb, const double4* __restrict__ pos, double L, double gam, const int* __restrict__ rowptr,
                            const uint32_t* __restrict__ col, double a, double eta, double eps_min, double r_pre,
                            double rough_alpha, double rough_h0, double* __restrict__ coef,
                            double* __restrict__ rdiag, int* overlap_flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const double4 p = pos[i];
  const double z = 6.0 * M_PI * eta * a;
  double d6[6] = {0, 0, 0, 0, 0, 0};  // xx yy zz xy xz yz
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const uint32_t c = col[e];
    const int j = int(c & 0x3FFFFFu);
    const double4 q = pos[j];
    const double dy = p.y - q.y + (int((c >> 25) & 7u) - 3) * L;
    const double dx = p.x - q.x + (int((c >> 22) & 7u) - 3) * L + gam * dy;
    const double dz = p.z - q.z + (int((c >> 28) & 7u) - 3) * L;
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (r < 1.5 * a) atomicOr(overlap_flag, 1);
    const double nx = dx / r, ny = dy / r, nz = dz / r;
    const double eps = fmax(r / a - 2.0, eps_min);
    const double lg = log(1.0 / eps);
    const double X = z * (0.25 / eps + 0.225 * lg + (3.0 / 112.0) * eps * lg - 0.25);
    double Y = z * (lg / 6.0);
    const double h = eps * a;
    if (h < rough_h0) {  // rough_h0 = 0 when roughness is off
      const double t = h / rough_h0, u = 1.0 - t;
      Y += z * rough_alpha * (a / h) * u * u * (1.0 + 2.0 * t);
    }
    coef[5 * e] = X;
    coef[5 * e + 1] = Y;
    coef[5 * e + 2] = nx;
    coef[5 * e + 3] = ny;
    coef[5 * e + 4] = nz;
    if (r < r_pre) {
      const double dXY = X - Y;
      d6[0] += Y + dXY * nx * nx;
      d6[1] += Y + dXY * ny * ny;
      d6[2] += Y + dXY * nz * nz;
      d6[3] += dXY * nx * ny;
      d6[4] += dXY * nx * nz;
      d6[5] += dXY * ny * nz;
    }
  }
  for (int k = 0; k < 6; ++k) rdiag[6 * i + k] = d6[k];
}

void launch_lub_setup(int nb, const double* pos4, double L, double gam, const int* rowptr, const uint32_t* col,
                      double a, double eta, double eps_min, double r_pre, double rough_alpha, double rough_h0,
                      double* coef, double* rdiag, int* overlap_flag, hipStream_t st) {
  k_lub_setup<<<nblocks(nb), kThreads, 0, st>>>(nb, (const double4*)pos4, L, gam, rowptr, col, a, eta, eps_min, r_pre,
                                                 rough_alpha, rough_h0, coef, rdiag, overlap_flag);
}

// Near-field force on beads that all move with the ambient flow at their aggregate's
// centroid (V = 0), the term R_FE : E_inf of Eq. `FH_agg` at the bead level: each pair
// resists w = (u_i - u_k) - W d, which for these beads is E (X_j - X_l) with
// X_j - X_l = d_ik - r_i + r_k the centroid separation of the pair's image, so the force
// on bead i is -sum_k R_pair E (d_ik - r_i + r_k).  Stored with the opposite sign,
// f_i = sum_k R_pair E (d_ik - r_i + r_k), as the aggregate right-hand side
// b2 = -F_P + Sigma f takes it.  One thread per bead, the separation rebuilt from the
// positions and image code as k_lub_setup does.
__global__ void k_lub_strain(int nb, const double4* __restrict__ pos, const double4* __restrict__ r4, double L,
                             double gam, const int* __restrict__ rowptr, const uint32_t* __restrict__ col,
                             const double* __restrict__ coef, const double* __restrict__ E, double* __restrict__ f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const double4 p = pos[i], ri = r4[i];
  double Em[9];
  for (int a = 0; a < 9; ++a) Em[a] = E[a];
  double ax = 0, ay = 0, az = 0;
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const uint32_t c = col[e];
    const int k = int(c & 0x3FFFFFu);
    const double4 q = pos[k], rk = r4[k];
    const double dy = p.y - q.y + (int((c >> 25) & 7u) - 3) * L;
    const double dx = p.x - q.x + (int((c >> 22) & 7u) - 3) * L + gam * dy;
    const double dz = p.z - q.z + (int((c >> 28) & 7u) - 3) * L;
    const double sx = dx - ri.x + rk.x, sy = dy - ri.y + rk.y, sz = dz - ri.z + rk.z;
    const double wx = Em[0] * sx + Em[1] * sy + Em[2] * sz;
    const double wy = Em[3] * sx + Em[4] * sy + Em[5] * sz;
    const double wz = Em[6] * sx + Em[7] * sy + Em[8] * sz;
    const double* cf = coef + 5 * e;
    const double nd = cf[2] * wx + cf[3] * wy + cf[4] * wz;
    const double g = (cf[0] - cf[1]) * nd;
    ax += cf[1] * wx + g * cf[2];
    ay += cf[1] * wy + g * cf[3];
    az += cf[1] * wz + g * cf[4];
  }
  f[3 * i] = ax;
  f[3 * i + 1] = ay;
  f[3 * i + 2] = az;
}

void launch_lub_strain(int nb, const double* pos4, const double* r4, double L, double gam, const int* rowptr,
                       const uint32_t* col, const double* coef, const double* E, double* f, hipStream_t st) {
  k_lub_strain<<<nblocks(nb), kThreads, 0, st>>>(nb, (const double4*)pos4, (const double4*)r4, L, gam, rowptr, col,
                                                  coef, E, f);
}

// ------------------------------------------------------------------------------------------
// preconditioner factor (Algorithm 1, step 1): A_j = sum_i Sigma_ji (M~^-1 + R~_ii) Sigma_ji^T,
// LU with partial pivoting in FP64, one thread per aggregate
// ------------------------------------------------------------------------------------------

__global__ void k_precond_factor(int na, const int* __restrict__ offsets, const double4* __restrict__ r4,
                                 const double* __restrict__ rdiag, double drag_t, double drag_r, double* __restrict__ lu,
                                 int* __restrict__ piv, int* singular) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= na) return;
  double A[6][6];
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b) A[a][b] = 0.0;
  for (int i = offsets[j]; i < offsets[j + 1]; ++i) {
    const double4 rv = r4[i];
    const double* d = rdiag + 6 * i;
    double D[3][3] = {{drag_t + d[0], d[3], d[4]}, {d[3], drag_t + d[1], d[5]}, {d[4], d[5], drag_t + d[2]}};
    const double X[3][3] = {{0, -rv.z, rv.y}, {rv.z, 0, -rv.x}, {-rv.y, rv.x, 0}};
    double XD[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) XD[a][b] = X[a][0] * D[0][b] + X[a][1] * D[1][b] + X[a][2] * D[2][b];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        A[a][b] += D[a][b];
        A[3 + a][b] += XD[a][b];
        A[b][3 + a] += XD[a][b];
        // X D X^T
        A[3 + a][3 + b] += XD[a][0] * X[b][0] + XD[a][1] * X[b][1] + XD[a][2] * X[b][2];
      }
    for (int a = 0; a < 3; ++a) A[3 + a][3 + a] += drag_r;
  }
  int bad = 0;
  for (int k = 0; k < 6; ++k) {
    int p = k;
    double best = fabs(A[k][k]);
    for (int i = k + 1; i < 6; ++i)
      if (fabs(A[i][k]) > best) {
        best = fabs(A[i][k]);
        p = i;
      }
    piv[6 * j + k] = p;
    if (p != k)
      for (int c = 0; c < 6; ++c) {
        const double t = A[k][c];
        A[k][c] = A[p][c];
        A[p][c] = t;
      }
    if (A[k][k] == 0.0) {
      bad = 1;
      continue;
    }
    const double inv = 1.0 / A[k][k];
    for (int i = k + 1; i < 6; ++i) {
      A[i][k] *= inv;
      for (int c = k + 1; c < 6; ++c) A[i][c] -= A[i][k] * A[k][c];
    }
  }
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b) lu[36 * j + 6 * a + b] = A[a][b];
  if (bad) atomicOr(singular, 1);
}

void launch_precond_factor(int na, const int* offsets, const double* r4, const double* rdiag, double drag_t,
                           double drag_r, double* lu, int* piv, int* singular, hipStream_t st) {
  k_precond_factor<<<nblocks(na, 128), 128, 0, st>>>(na, offsets, (const double4*)r4, rdiag, drag_t, drag_r, lu, piv,
                                                      singular);
}

}  // namespace fsd
