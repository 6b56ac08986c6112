// Far-field mobility M = M_real + M_wave of the positively split Ewald sum.
//
// Wave space (spectral Ewald, Gaussian spreading): bead (force, torque) are
// spread to three complex grids Z_c = F_c + i T_c (c = x, y, z), transformed,
// multiplied by the Hasimoto-damped FT-RPY Green's function, transformed back
// and interpolated to the beads, where the grid holds u_c + i w_c.
//
// Real space: per neighbour pair within the cutoff, the free-space RPY block
// minus the smooth inverse transform of the damped multiplier, read from a
// table by cubic interpolation.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <type_traits>

#include <mutex>

#include "fsd_impl.hpp"
#include "k_rigid.hpp"

namespace fsd {

namespace {
constexpr int kThreads = 256;
constexpr int kMaxP = 21;  // 3 * P weights computed by one 64-lane wavefront
inline int nblocks(long long n, int t = kThreads) { return int((n + t - 1) / t); }

template <typename R>
struct C2;
template <>
struct C2<double> {
  using T = double2;
};
template <>
struct C2<float> {
  using T = float2;
};

// Workgroups are dealt to the 8 XCDs round robin; map workgroup b of nblk so that each
// XCD gets one contiguous range of logical blocks (neighbouring beads or grid blocks
// then share that XCD's L2).  A bijection on [0, nblk).
__device__ inline int xcd_remap(int b, int nblk) {
  const int q = nblk >> 3, r = nblk & 7, x = b & 7, k = b >> 3;
  return x * q + min(x, r) + k;
}

template <typename R>
__device__ inline R wave_sum(R v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
}  // namespace

// Gather-spreading plan: beads binned by the grid block holding the first point of
// their support, in sorted order with their support starts and per-axis weights.
struct SpreadPlan {
  int nb = 0, BS = 0, nbin = 0, K = 0, P = 0;
  int *keys_in = nullptr, *keys_out = nullptr, *vals_in = nullptr, *perm = nullptr;
  int *bin_start = nullptr, *bin_end = nullptr;
  // 8^3 blocks: for every block, the sorted indices of exactly the beads whose support
  // reaches it (cand[blk_start[b] .. blk_end[b]), in bead order); each bead files kc^3 slots
  // (its blocks, then sentinels) that one stable sort groups by block
  int kc = 0;
  int *blk_start = nullptr, *blk_end = nullptr, *pk_in = nullptr, *pk_out = nullptr, *pv_in = nullptr,
      *cand = nullptr;
  void* ptemp = nullptr;
  size_t ptemp_bytes = 0;
  int4* starts = nullptr;   // (sx, sy, sz, bin) per bead, sorted order
  double* weights = nullptr;  // 3P weights per bead, sorted order
  float* weights32 = nullptr;  // the same in FP32
  double* wtmp = nullptr;
  int4* stmp = nullptr;
  void* temp = nullptr;
  size_t temp_bytes = 0;
  size_t rbytes = 0;
};

// ------------------------------------------------------------------------------------------
// real-space pair sum: one group of LPR lanes per bead row
// ------------------------------------------------------------------------------------------

template <typename R, int LPR>
__device__ __forceinline__ void real_sum_body(int nb, const double4* __restrict__ pos,
                                                  const double* __restrict__ lam, const int* __restrict__ rowptr,
                                                  const uint32_t* __restrict__ col, const R* __restrict__ tab,
                                                  RealParams rp, double* __restrict__ out, int accumulate,
                                                  const int* __restrict__ order, const int* __restrict__ skip, int bx_, int by_, int gx_) {
  if (skip && *skip) return;
  // with order (beads in spatially sorted order), rows are visited in that order and
  // each XCD takes one contiguous range of them
  const int nblk = gx_ > 0 ? gx_ : int((size_t(nb) * LPR + blockDim.x - 1) / blockDim.x);
  const int gt = (order ? xcd_remap(bx_, nblk) : bx_) * blockDim.x + threadIdx.x;
  const int rl = gt / LPR;
  const int lane = gt % LPR;
  if (rl >= nb) return;  // LPR divides the wavefront, so whole groups leave together
  const int row = order ? order[rl] : rl;
  const double4 pi = pos[row];
  const R a = R(rp.a);
  const R c8 = R(1.0 / (8.0 * M_PI * rp.eta));
  const R mt = R(1.0 / (6.0 * M_PI * rp.eta * rp.a));
  const R mr = R(1.0 / (8.0 * M_PI * rp.eta * rp.a * rp.a * rp.a));
  const R inv_ht = R(rp.inv_ht);
  const double gam = rp.gam ? *rp.gam : 0.0;
  R u0 = 0, u1 = 0, u2 = 0, w0 = 0, w1 = 0, w2 = 0;
  const int e1 = rowptr[row + 1];
  for (int e = rowptr[row] + lane; e < e1; e += LPR) {
    const uint32_t c = col[e];
    const int j = int(c & 0x3FFFFFu);
    const double4 pj = pos[j];
    const double dyd = pi.y - pj.y + (int((c >> 25) & 7u) - 3) * rp.L;  // Cartesian from sheared
    const R dx = R(pi.x - pj.x + (int((c >> 22) & 7u) - 3) * rp.L + gam * dyd);
    const R dy = R(dyd);
    const R dz = R(pi.z - pj.z + (int((c >> 28) & 7u) - 3) * rp.L);
    const R r = sqrt(dx * dx + dy * dy + dz * dz);
    const R ir = R(1) / r;
    const R ex = dx * ir, ey = dy * ir, ez = dz * ir;
    // free-space force-torque RPY (non-overlapping and overlapping branches)
    R tI, tR, rI, rR, cc;
    if (r >= R(2) * a) {
      const R ir2 = ir * ir, a2 = a * a;
      tI = c8 * ir * (R(1) + R(2.0 / 3.0) * a2 * ir2);
      tR = c8 * ir * (R(1) - R(2) * a2 * ir2);
      rI = R(-0.5) * c8 * ir * ir2;
      rR = R(1.5) * c8 * ir * ir2;
      cc = -c8 * ir2;
    } else {
      const R s = r / a;
      tI = mt * (R(1) - R(9.0 / 32.0) * s);
      tR = mt * R(3.0 / 32.0) * s;
      rI = mr * (R(1) - R(27.0 / 32.0) * s + R(5.0 / 64.0) * s * s * s);
      rR = mr * (R(9.0 / 32.0) * s - R(3.0 / 64.0) * s * s * s);
      cc = -R(0.5) * c8 / (a * a) * s * (R(1) - R(3.0 / 8.0) * s);
    }
    // minus the smooth part (cubic Lagrange on nodes it-1 .. it+2; table row 0 is r = -h)
    const R t = r * inv_ht;
    const int it = int(t);
    const R f = t - R(it);
    const R wa = -f * (f - 1) * (f - 2) * R(1.0 / 6.0);
    const R wb = (f + 1) * (f - 1) * (f - 2) * R(0.5);
    const R wc = -(f + 1) * f * (f - 2) * R(0.5);
    const R wd = (f + 1) * f * (f - 1) * R(1.0 / 6.0);
    const R* T0 = tab + 8 * it;
    tI -= wa * T0[0] + wb * T0[8] + wc * T0[16] + wd * T0[24];
    tR -= wa * T0[1] + wb * T0[9] + wc * T0[17] + wd * T0[25];
    rI -= wa * T0[2] + wb * T0[10] + wc * T0[18] + wd * T0[26];
    rR -= wa * T0[3] + wb * T0[11] + wc * T0[19] + wd * T0[27];
    cc -= wa * T0[4] + wb * T0[12] + wc * T0[20] + wd * T0[28];
    const double* lj = lam + 6 * j;
    const R fx = R(lj[0]), fy = R(lj[1]), fz = R(lj[2]);
    const R tx = R(lj[3]), ty = R(lj[4]), tz = R(lj[5]);
    const R fd = ex * fx + ey * fy + ez * fz;
    const R td = ex * tx + ey * ty + ez * tz;
    u0 += tI * fx + tR * fd * ex + cc * (ey * tz - ez * ty);
    u1 += tI * fy + tR * fd * ey + cc * (ez * tx - ex * tz);
    u2 += tI * fz + tR * fd * ez + cc * (ex * ty - ey * tx);
    w0 += rI * tx + rR * td * ex + cc * (ey * fz - ez * fy);
    w1 += rI * ty + rR * td * ey + cc * (ez * fx - ex * fz);
    w2 += rI * tz + rR * td * ez + cc * (ex * fy - ey * fx);
  }
#pragma unroll
  for (int o = LPR / 2; o >= 1; o >>= 1) {
    u0 += __shfl_xor(u0, o, LPR);
    u1 += __shfl_xor(u1, o, LPR);
    u2 += __shfl_xor(u2, o, LPR);
    w0 += __shfl_xor(w0, o, LPR);
    w1 += __shfl_xor(w1, o, LPR);
    w2 += __shfl_xor(w2, o, LPR);
  }
  if (lane == 0) {
    const double* li = lam + 6 * row;
    double* o = out + 6 * row;
    const double v[6] = {double(u0) + rp.self_t * li[0], double(u1) + rp.self_t * li[1],
                         double(u2) + rp.self_t * li[2], double(w0) + rp.self_r * li[3],
                         double(w1) + rp.self_r * li[4], double(w2) + rp.self_r * li[5]};
    if (accumulate)
      for (int k = 0; k < 6; ++k) o[k] += v[k];
    else
      for (int k = 0; k < 6; ++k) o[k] = v[k];
  }
}

template <typename R, int LPR>
__global__ __launch_bounds__(256) void k_real_sum(int nb, const double4* __restrict__ pos,
                                                  const double* __restrict__ lam, const int* __restrict__ rowptr,
                                                  const uint32_t* __restrict__ col, const R* __restrict__ tab,
                                                  RealParams rp, double* __restrict__ out, int accumulate,
                                                  const int* __restrict__ order, const int* __restrict__ skip) {
  real_sum_body<R, LPR>(nb, pos, lam, rowptr, col, tab, rp, out, accumulate, order, skip, blockIdx.x, blockIdx.y, gridDim.x);
}

template <typename R>
void launch_real_sum(int nb, const double* pos4, const double* lam, const int* rowptr, const uint32_t* col,
                     const R* table, const RealParams& rp, double* out, bool accumulate, int lpr, hipStream_t st,
                     const int* skip, const int* order) {
  const long long threads = (long long)nb * lpr;
  const int acc = accumulate ? 1 : 0;
  const double4* p = (const double4*)pos4;
#define FSD_REAL(L_)                                                                                    \
  launch_k(k_real_sum<R, L_>, nblocks(threads), kThreads, 0, st, nb, p, lam, rowptr, col, table, rp, out, acc, order, skip)
  switch (lpr) {
    case 1: FSD_REAL(1); break;
    case 2: FSD_REAL(2); break;
    case 4: FSD_REAL(4); break;
    case 8: FSD_REAL(8); break;
    case 16: FSD_REAL(16); break;
    case 32: FSD_REAL(32); break;
    default: FSD_REAL(64); break;
  }
#undef FSD_REAL
}

// ------------------------------------------------------------------------------------------
// Gaussian spreading and interpolation: one wavefront per bead
// ------------------------------------------------------------------------------------------

namespace {
// 1D weights exp(-alpha (x_m - p)^2) for the P support points of each axis.
template <typename R>
__device__ inline void axis_weights(const double4& p, const WaveParams& wp, int lane, R* w, int* st) {
  const int P = wp.support;
  if (lane < 3 * P) {
    const int d = lane / P, k = lane % P;
    const double pd = d == 0 ? p.x : (d == 1 ? p.y : p.z);
    const double u = pd / wp.h;
    const int s = int(ceil(u - 0.5 * P));
    const double xm = (s + k) * wp.h - pd;
    w[d * kMaxP + k] = R(exp(-wp.alpha * xm * xm));
    if (k == 0) st[d] = s;
  }
}

__device__ inline int wrapi(int m, int n) {
  m %= n;
  return m < 0 ? m + n : m;
}
}  // namespace

template <typename R>
__global__ __launch_bounds__(256) void k_spread(int nb, const double4* __restrict__ pos,
                                                const double* __restrict__ lam, WaveParams wp, R* __restrict__ grid,
                                                size_t cs, const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ R wts[4][3 * kMaxP];
  __shared__ int sta[4][3];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + wv;
  const bool live = i < nb;
  const double4 p = live ? pos[i] : make_double4(0, 0, 0, 0);
  if (live) axis_weights<R>(p, wp, lane, wts[wv], sta[wv]);
  __syncthreads();
  if (!live) return;
  const int P = wp.support, N = wp.n;
  const double* li = lam + 6 * i;
  const R f0 = R(li[0]), f1 = R(li[1]), f2 = R(li[2]);
  const R t0 = R(li[3]), t1 = R(li[4]), t2 = R(li[5]);
  const int sx = sta[wv][0], sy = sta[wv][1], sz = sta[wv][2];
  const R* wx = wts[wv];
  const R* wy = wts[wv] + kMaxP;
  const R* wz = wts[wv] + 2 * kMaxP;
  const int P3 = P * P * P;
  for (int idx = lane; idx < P3; idx += 64) {
    const int kx = idx % P, ky = (idx / P) % P, kz = idx / (P * P);
    const R w = wx[kx] * wy[ky] * wz[kz];
    const size_t m = (size_t(wrapi(sz + kz, N)) * N + wrapi(sy + ky, N)) * N + wrapi(sx + kx, N);
    R* g = grid + 2 * m;
    atomicAdd(g, w * f0);
    atomicAdd(g + 1, w * t0);
    atomicAdd(g + cs, w * f1);
    atomicAdd(g + cs + 1, w * t1);
    atomicAdd(g + 2 * cs, w * f2);
    atomicAdd(g + 2 * cs + 1, w * t2);
  }
}

template <typename R>
void launch_spread(int nb, const double* pos4, const double* lam, const WaveParams& wp, R* grid, hipStream_t st,
                   const int* skip) {
  const size_t cs = 2 * size_t(wp.n) * wp.n * wp.n;
  launch_k(k_spread<R>, nblocks(nb, 4), kThreads, 0, st, nb, (const double4*)pos4, lam, wp, grid, cs, skip);
}

// ---- sheared lattice: one wavefront per bead, grid row j shifted along x -------------------
namespace {
// Weights of bead p in sheared coordinates: y and z as on the cube; for each of the P rows
// ky the start sxr[ky] and P x-weights, centred at p_x - gam (y_m - p_y), y_m = (sy + ky) h.
template <typename R>
__device__ inline void sheared_weights(const double4& p, const WaveParams& wp, int lane, R* wyz, int* st, R* wxr,
                                       int* sxr) {
  const int P = wp.support;
  const double h = wp.h, gam = wp.gam ? *wp.gam : 0.0;
  const int sy = int(ceil(p.y / h - 0.5 * P)), sz = int(ceil(p.z / h - 0.5 * P));
  if (lane < 2 * P) {
    const int d = lane / P, k = lane % P;
    const double xm = d == 0 ? (sy + k) * h - p.y : (sz + k) * h - p.z;
    wyz[d * kMaxP + k] = R(exp(-wp.alpha * xm * xm));
  }
  if (lane == 0) {
    st[0] = sy;
    st[1] = sz;
  }
  for (int t = lane; t < P * P; t += 64) {
    const int ky = t / P, kx = t - ky * P;
    const double cx = p.x - gam * ((sy + ky) * h - p.y);  // the row's centre along x
    const int sx = int(ceil(cx / h - 0.5 * P));
    const double xm = (sx + kx) * h - cx;
    wxr[ky * kMaxP + kx] = R(exp(-wp.alpha * xm * xm));
    if (kx == 0) sxr[ky] = sx;
  }
}
}  // namespace

template <typename R>
__global__ __launch_bounds__(256) void k_spread_sheared(int nb, const double4* __restrict__ pos,
                                                        const double* __restrict__ lam, WaveParams wp,
                                                        R* __restrict__ grid, size_t cs, const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ R wyz[4][2 * kMaxP];
  __shared__ R wxr[4][kMaxP * kMaxP];
  __shared__ int sxr[4][kMaxP];
  __shared__ int sta[4][2];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + wv;
  const bool live = i < nb;
  if (live) sheared_weights<R>(pos[i], wp, lane, wyz[wv], sta[wv], wxr[wv], sxr[wv]);
  __syncthreads();
  if (!live) return;
  const int P = wp.support, N = wp.n;
  const double* li = lam + 6 * i;
  const R f0 = R(li[0]), f1 = R(li[1]), f2 = R(li[2]);
  const R t0 = R(li[3]), t1 = R(li[4]), t2 = R(li[5]);
  const int sy = sta[wv][0], sz = sta[wv][1];
  const int P3 = P * P * P;
  for (int idx = lane; idx < P3; idx += 64) {
    const int kx = idx % P, ky = (idx / P) % P, kz = idx / (P * P);
    const R w = wxr[wv][ky * kMaxP + kx] * wyz[wv][ky] * wyz[wv][kMaxP + kz];
    const size_t m = (size_t(wrapi(sz + kz, N)) * N + wrapi(sy + ky, N)) * N + wrapi(sxr[wv][ky] + kx, N);
    R* g = grid + 2 * m;
    atomicAdd(g, w * f0);
    atomicAdd(g + 1, w * t0);
    atomicAdd(g + cs, w * f1);
    atomicAdd(g + cs + 1, w * t1);
    atomicAdd(g + 2 * cs, w * f2);
    atomicAdd(g + 2 * cs + 1, w * t2);
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_interp_sheared(int nb, const double4* __restrict__ pos,
                                                        const R* __restrict__ grid, size_t cs, WaveParams wp,
                                                        double* __restrict__ out, const int* __restrict__ skip,
                                                        const int* __restrict__ body, const double4* __restrict__ r4,
                                                        const double* __restrict__ V) {
  if (skip && *skip) return;
  __shared__ R wyz[4][2 * kMaxP];
  __shared__ R wxr[4][kMaxP * kMaxP];
  __shared__ int sxr[4][kMaxP];
  __shared__ int sta[4][2];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + wv;
  const bool live = i < nb;
  if (live) sheared_weights<R>(pos[i], wp, lane, wyz[wv], sta[wv], wxr[wv], sxr[wv]);
  __syncthreads();
  if (!live) return;
  const int P = wp.support, N = wp.n;
  const int sy = sta[wv][0], sz = sta[wv][1];
  R a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0;
  for (int pq = lane; pq < P * P; pq += 64) {  // lane -> (kx, ky) column, walking z
    const int ky = pq / P, kx = pq - ky * P;
    const int x = wrapi(sxr[wv][ky] + kx, N), y = wrapi(sy + ky, N);
    const R wxy = wxr[wv][ky * kMaxP + kx] * wyz[wv][ky];
    for (int kz = 0; kz < P; ++kz) {
      const R w = wxy * wyz[wv][kMaxP + kz];
      const R* g = grid + 2 * ((size_t(wrapi(sz + kz, N)) * N + y) * N + x);
      a0 += w * g[0];
      a3 += w * g[1];
      a1 += w * g[cs];
      a4 += w * g[cs + 1];
      a2 += w * g[2 * cs];
      a5 += w * g[2 * cs + 1];
    }
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  a2 = wave_sum(a2);
  a3 = wave_sum(a3);
  a4 = wave_sum(a4);
  a5 = wave_sum(a5);
  if (lane == 0) {
    double* o = out + 6 * size_t(i);
    double add[6] = {double(a0), double(a1), double(a2), double(a3), double(a4), double(a5)};
    if (V) {  // Sigma^T V: (U + W x r, W) of the bead's body
      const double* v = V + 6 * body[i];
      const double4 r = r4[i];
      add[0] += v[0] + (v[4] * r.z - v[5] * r.y);
      add[1] += v[1] + (v[5] * r.x - v[3] * r.z);
      add[2] += v[2] + (v[3] * r.y - v[4] * r.x);
      add[3] += v[3];
      add[4] += v[4];
      add[5] += v[5];
    }
    for (int k = 0; k < 6; ++k) o[k] += add[k];
  }
}

template <typename R>
void launch_spread_sheared(int nb, const double* pos4, const double* lam, const WaveParams& wp, R* grid,
                           hipStream_t st, const int* skip) {
  const size_t cs = 2 * size_t(wp.n) * wp.n * wp.n;
  launch_k(k_spread_sheared<R>, nblocks(nb, 4), kThreads, 0, st, nb, (const double4*)pos4, lam, wp, grid, cs, skip);
}

template <typename R>
void launch_interp_sheared(int nb, const double* pos4, const R* grid, const WaveParams& wp, double* out,
                           hipStream_t st, const int* skip, const int* body, const double* r4, const double* V) {
  const size_t cs = 2 * size_t(wp.n) * wp.n * wp.n;
  launch_k(k_interp_sheared<R>, nblocks(nb, 4), kThreads, 0, st, nb, (const double4*)pos4, grid, cs, wp, out, skip,
           body, (const double4*)r4, V);
}

// Global-memory accesses through a 32-bit element index i from a base the workgroup shares
// (the caller keeps i sizeof(R) below 2^32), so a load or store takes a 32-bit offset
// instead of a 64-bit address.  stg2 stores the pair p[i], p[i + 1] (i even); ldg4 loads
// p[i .. i + 3] (i a multiple of 4, aligned); ldg2 loads the pair p[i], p[i + 1].
template <typename R>
__device__ __forceinline__ void stg2(R* p, unsigned i, R a, R b) {
  typedef R V2 __attribute__((ext_vector_type(2)));
  const unsigned bytes = i * unsigned(sizeof(R));
  V2 v;
  v.x = a;
  v.y = b;
  *(__attribute__((address_space(1))) V2*)((__attribute__((address_space(1))) char*)p + bytes) = v;
}

template <typename R>
__device__ __forceinline__ void ldg4(const R* p, unsigned i, R& a, R& b, R& c, R& d) {
  typedef R V4 __attribute__((ext_vector_type(4)));
  const unsigned bytes = i * unsigned(sizeof(R));
  const V4 v = *(__attribute__((address_space(1))) const V4*)((__attribute__((address_space(1))) const char*)p + bytes);
  a = v.x;
  b = v.y;
  c = v.z;
  d = v.w;
}

template <typename R>
__device__ __forceinline__ void ldg2(const R* p, unsigned i, R& a, R& b) {
  typedef R V2 __attribute__((ext_vector_type(2)));
  const unsigned bytes = i * unsigned(sizeof(R));
  const V2 v = *(__attribute__((address_space(1))) const V2*)((__attribute__((address_space(1))) const char*)p + bytes);
  a = v.x;
  b = v.y;
}

template <typename R>
__device__ __forceinline__ void interp_body(int nb, const double4* __restrict__ pos,
                                                const R* __restrict__ grid, size_t cs, WaveParams wp,
                                                double* __restrict__ out, const int* __restrict__ skip,
                                                const int* __restrict__ body, const double4* __restrict__ r4,
                                                const double* __restrict__ V, const int* __restrict__ order,
                                                const int4* __restrict__ ostart, const R* __restrict__ ow,
                                                int bx_, int by_, int gx_) {
  if (skip && *skip) return;
  // one wavefront per bead.  With order (the spreading plan's sorted beads, their
  // support starts and weights), beads are visited in spatial order, each XCD taking one
  // contiguous range, and the weights come from the plan instead of being recomputed.
  __shared__ R wts[4][3 * kMaxP];
  __shared__ int sta[4][3];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nblk = gx_ > 0 ? gx_ : (nb + 3) / 4;
  const int k = (order ? xcd_remap(bx_, nblk) : bx_) * 4 + wv;
  const bool live = k < nb;
  const int i = live ? (order ? order[k] : k) : 0;
  if (live) {
    if (order) {
      const int P = wp.support;
      if (lane < 3 * P) wts[wv][(lane / P) * kMaxP + lane % P] = ow[size_t(k) * 3 * P + lane];
      if (lane == 0) {
        const int4 s4 = ostart[k];
        sta[wv][0] = s4.x;
        sta[wv][1] = s4.y;
        sta[wv][2] = s4.z;
      }
    } else {
      axis_weights<R>(pos[i], wp, lane, wts[wv], sta[wv]);
    }
  }
  __syncthreads();
  if (!live) return;
  const int P = wp.support, N = wp.n;
  const int sx = sta[wv][0], sy = sta[wv][1], sz = sta[wv][2];
  const R* wx = wts[wv];
  const R* wy = wts[wv] + kMaxP;
  const R* wz = wts[wv] + 2 * kMaxP;
  R a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0;
  // lane -> (x pair, ky) of the support, each lane walking its two columns along z: the
  // pairs (2m, 2m + 1) that cover the support's P x values (P/2 + 1 of them at most, the
  // points outside the support weighted 0), so each load brings two grid points in one
  // aligned 16-byte (FP32) or 32-byte (FP64) read; for even N no pair straddles the
  // periodic wrap.  The grid is read through 32-bit offsets from the three component bases
  // (2 N^3 < 2^31 for N <= 256), in two runs split where the columns wrap in z.
  const int sxw = wrapi(sx, N), syw = wrapi(sy, N), szw = wrapi(sz, N);
  const unsigned plane = 2 * N * N;
  const int n1 = min(P, N - szw), half = N >> 1, m0 = sxw >> 1;
  const int npx = ((sxw + P - 1) >> 1) - m0 + 1;
  const R* g0 = grid;
  const R* g1 = grid + cs;
  const R* g2 = grid + 2 * cs;
  // an odd grid side (set by the caller) keeps one column per lane: its pairs would
  // straddle the wrap and lose the alignment.  So does FP64, where the pairs' registers
  // (128 VGPRs against 70) cost more occupancy than the wider loads gain (the 4096x20
  // system: 267 us against 233 per launch)
  const bool paired = sizeof(R) == 4 && !(N & 1);
  for (int pq = lane; !paired && pq < P * P; pq += 64) {
    const int ky = pq / P, kx = pq - ky * P;
    int x = sxw + kx, y = syw + ky;
    x -= x >= N ? N : 0;
    y -= y >= N ? N : 0;
    const R wxy = wx[kx] * wy[ky];
    const unsigned col = 2 * (y * N + x);
    unsigned off = col + szw * plane;
    for (int kz = 0; kz < P; ++kz) {
      if (kz == n1) off = col;
      const R w = wxy * wz[kz];
      R v0, v1, v2, v3, v4, v5;
      ldg2(g0, off, v0, v3);
      ldg2(g1, off, v1, v4);
      ldg2(g2, off, v2, v5);
      a0 += w * v0;
      a3 += w * v3;
      a1 += w * v1;
      a4 += w * v4;
      a2 += w * v2;
      a5 += w * v5;
      off += plane;
    }
  }
  for (int pq = lane; paired && pq < npx * P; pq += 64) {
    const int ky = pq / npx, mp = pq - ky * npx;
    int m = m0 + mp, y = syw + ky;
    m -= m >= half ? half : 0;
    y -= y >= N ? N : 0;
    const int kx0 = 2 * (m0 + mp) - sxw;  // support offset of the pair's first point (>= -1)
    const R wyk = wy[ky];
    const R wp0 = kx0 >= 0 ? wx[kx0] * wyk : R(0);
    const R wp1 = kx0 + 1 < P ? wx[kx0 + 1] * wyk : R(0);
    const unsigned col = 2 * (y * N + 2 * m);
    unsigned off = col + szw * plane;
    for (int kz = 0; kz < P; ++kz) {
      if (kz == n1) off = col;  // the columns wrap to z = 0
      const R w = wz[kz], u0 = wp0 * w, u1 = wp1 * w;
      R b0, b1, b2, b3;
      ldg4(g0, off, b0, b1, b2, b3);
      a0 += u0 * b0 + u1 * b2;
      a3 += u0 * b1 + u1 * b3;
      ldg4(g1, off, b0, b1, b2, b3);
      a1 += u0 * b0 + u1 * b2;
      a4 += u0 * b1 + u1 * b3;
      ldg4(g2, off, b0, b1, b2, b3);
      a2 += u0 * b0 + u1 * b2;
      a5 += u0 * b1 + u1 * b3;
      off += plane;
    }
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  a2 = wave_sum(a2);
  a3 = wave_sum(a3);
  a4 = wave_sum(a4);
  a5 = wave_sum(a5);
  if (lane == 0) {
    double* o = out + 6 * size_t(i);
    double add[6] = {double(a0), double(a1), double(a2), double(a3), double(a4), double(a5)};
    if (V) {  // Sigma^T V: (U + W x r, W) of the bead's body
      const double* v = V + 6 * body[i];
      const double4 r = r4[i];
      add[0] += v[0] + (v[4] * r.z - v[5] * r.y);
      add[1] += v[1] + (v[5] * r.x - v[3] * r.z);
      add[2] += v[2] + (v[3] * r.y - v[4] * r.x);
      add[3] += v[3];
      add[4] += v[4];
      add[5] += v[5];
    }
    for (int k = 0; k < 6; ++k) o[k] += add[k];
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_interp(int nb, const double4* __restrict__ pos,
                                                const R* __restrict__ grid, size_t cs, WaveParams wp,
                                                double* __restrict__ out, const int* __restrict__ skip,
                                                const int* __restrict__ body, const double4* __restrict__ r4,
                                                const double* __restrict__ V,
                                                const int* __restrict__ order, const int4* __restrict__ ostart,
                                                const R* __restrict__ ow) {
  interp_body<R>(nb, pos, grid, cs, wp, out, skip, body, r4, V, order, ostart, ow, blockIdx.x, blockIdx.y, gridDim.x);
}

template <typename R>
void launch_interp(int nb, const double* pos4, const R* grid, const WaveParams& wp, double* out, hipStream_t st,
                   const int* skip, const int* body, const double* r4, const double* V, const SpreadPlan* sp) {
  const size_t cs = 2 * size_t(wp.n) * wp.n * wp.n;
  const R* ow = nullptr;
  if (sp) {
    if (std::is_same<R, double>::value)
      ow = reinterpret_cast<const R*>(sp->weights);
    else
      ow = reinterpret_cast<const R*>(sp->weights32);
  }
  launch_k(k_interp<R>, nblocks(nb, 4), kThreads, 0, st, nb, (const double4*)pos4, grid, cs, wp, out, skip, body,
                                                   (const double4*)r4, V, sp ? sp->perm : nullptr,
                                                   sp ? sp->starts : nullptr, ow);
}

const int* spread_plan_order(const SpreadPlan* sp) { return sp ? sp->perm : nullptr; }

// ------------------------------------------------------------------------------------------
// Gaussian spreading as a gather: beads are binned by the grid block that holds
// the first point of their support (sorted once per configuration); a workgroup
// owns one BS^3 block of grid points and sums the contributions of every bead
// whose support reaches it.  No atomics, deterministic, each grid value written
// once.
// ------------------------------------------------------------------------------------------



namespace {
int pick_block(int N) {
  if (N % 8 == 0) return 8;
  if (N % 4 == 0) return 4;
  return 0;
}
}  // namespace

SpreadPlan* spread_plan_create(int nb, int N, int P) {
  const int BS = pick_block(N);
  if (BS == 0) return nullptr;
  auto* sp = new SpreadPlan;
  sp->nb = nb;
  sp->BS = BS;
  sp->nbin = N / BS;
  sp->P = P;
  sp->K = std::min(1 + (P - 1 + BS - 1) / BS, sp->nbin);
  const int nbins = sp->nbin * sp->nbin * sp->nbin;
  bool ok = hipMalloc(&sp->keys_in, sizeof(int) * nb) == hipSuccess &&
            hipMalloc(&sp->keys_out, sizeof(int) * nb) == hipSuccess &&
            hipMalloc(&sp->vals_in, sizeof(int) * nb) == hipSuccess &&
            hipMalloc(&sp->perm, sizeof(int) * nb) == hipSuccess &&
            hipMalloc(&sp->bin_start, sizeof(int) * nbins) == hipSuccess &&
            hipMalloc(&sp->bin_end, sizeof(int) * nbins) == hipSuccess &&
            hipMalloc(&sp->starts, sizeof(int4) * nb) == hipSuccess &&
            hipMalloc(&sp->stmp, sizeof(int4) * nb) == hipSuccess &&
            hipMalloc(&sp->weights, sizeof(double) * 3 * P * size_t(nb)) == hipSuccess &&
            hipMalloc(&sp->weights32, sizeof(float) * 3 * P * size_t(nb)) == hipSuccess &&
            hipMalloc(&sp->wtmp, sizeof(double) * 3 * P * size_t(nb)) == hipSuccess;
  size_t b = 0;
  hipcub::DeviceRadixSort::SortPairs(nullptr, b, sp->keys_in, sp->keys_out, sp->vals_in, sp->perm, nb);
  sp->temp_bytes = b;
  ok = ok && hipMalloc(&sp->temp, b) == hipSuccess;
  if (ok && BS == 8) {
    sp->kc = std::min(sp->K, sp->nbin);
    const size_t slots = size_t(nb) * sp->kc * sp->kc * sp->kc;
    ok = hipMalloc(&sp->blk_start, sizeof(int) * nbins) == hipSuccess &&
         hipMalloc(&sp->blk_end, sizeof(int) * nbins) == hipSuccess &&
         hipMalloc(&sp->pk_in, sizeof(int) * slots) == hipSuccess &&
         hipMalloc(&sp->pk_out, sizeof(int) * slots) == hipSuccess &&
         hipMalloc(&sp->pv_in, sizeof(int) * slots) == hipSuccess &&
         hipMalloc(&sp->cand, sizeof(int) * slots) == hipSuccess;
    size_t pb = 0;
    hipcub::DeviceRadixSort::SortPairs(nullptr, pb, sp->pk_in, sp->pk_out, sp->pv_in, sp->cand, int(slots));
    sp->ptemp_bytes = pb;
    ok = ok && hipMalloc(&sp->ptemp, pb) == hipSuccess;
  }
  if (!ok) {
    spread_plan_destroy(sp);
    return nullptr;
  }
  return sp;
}

void spread_plan_destroy(SpreadPlan* sp) {
  if (!sp) return;
  (void)hipFree(sp->keys_in);
  (void)hipFree(sp->keys_out);
  (void)hipFree(sp->vals_in);
  (void)hipFree(sp->perm);
  (void)hipFree(sp->bin_start);
  (void)hipFree(sp->bin_end);
  (void)hipFree(sp->starts);
  (void)hipFree(sp->stmp);
  (void)hipFree(sp->weights);
  (void)hipFree(sp->weights32);
  (void)hipFree(sp->wtmp);
  (void)hipFree(sp->temp);
  (void)hipFree(sp->blk_start);
  (void)hipFree(sp->blk_end);
  (void)hipFree(sp->pk_in);
  (void)hipFree(sp->pk_out);
  (void)hipFree(sp->pv_in);
  (void)hipFree(sp->cand);
  (void)hipFree(sp->ptemp);
  delete sp;
}

__global__ void k_bead_prep(int nb, const double4* __restrict__ pos, WaveParams wp, int BS, int nbin,
                            double* __restrict__ w, int4* __restrict__ st, int* __restrict__ keys, int* __restrict__ vals) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const int P = wp.support, N = wp.n;
  const double4 p = pos[i];
  int sm[3];
  for (int d = 0; d < 3; ++d) {
    const double pd = d == 0 ? p.x : (d == 1 ? p.y : p.z);
    const int s = int(ceil(pd / wp.h - 0.5 * P));
    for (int k = 0; k < P; ++k) {
      const double xm = (s + k) * wp.h - pd;
      w[size_t(i) * 3 * P + d * P + k] = exp(-wp.alpha * xm * xm);
    }
    sm[d] = ((s % N) + N) % N;
  }
  const int bin = ((sm[2] / BS) * nbin + sm[1] / BS) * nbin + sm[0] / BS;
  st[i] = make_int4(sm[0], sm[1], sm[2], bin);
  keys[i] = bin;
  vals[i] = i;
}

// one thread per copied weight: consecutive threads move consecutive weights of a bead
__global__ void k_bead_permute(int nb, int P3, const int* __restrict__ perm, const double* __restrict__ w_in,
                               const int4* __restrict__ s_in, double* __restrict__ w_out, float* __restrict__ w32,
                               int4* __restrict__ s_out) {
  const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= size_t(nb) * P3) return;
  const int k = int(t / P3), q = int(t - size_t(k) * P3);
  const int i = perm[k];
  const double v = w_in[size_t(i) * P3 + q];
  w_out[t] = v;
  w32[t] = float(v);
  if (q == 0) s_out[k] = s_in[i];
}

__global__ void k_bin_bounds(int nb, const int* __restrict__ keys, int* start, int* end) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb) return;
  const int c = keys[k];
  if (k == 0 || keys[k - 1] != c) start[c] = k;
  if (k == nb - 1 || keys[k + 1] != c) end[c] = k + 1;
}

// the kc^3 slots of sorted bead k: the blocks its support reaches (their index as the key,
// k as the value), the remaining slots a sentinel key past the last block
__global__ void k_block_slots(int nb, const int4* __restrict__ starts, int P, int nbin, int kc,
                              int* __restrict__ keys, int* __restrict__ vals) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb) return;
  const int4 s = starts[k];
  const int cnt[3] = {min(((s.x & 7) + P - 1) / 8 + 1, nbin), min(((s.y & 7) + P - 1) / 8 + 1, nbin),
                      min(((s.z & 7) + P - 1) / 8 + 1, nbin)};
  const int b0[3] = {s.x >> 3, s.y >> 3, s.z >> 3};
  const int per = kc * kc * kc, sentinel = nbin * nbin * nbin;
  int q = 0;
  for (int jz = 0; jz < cnt[2]; ++jz)
    for (int jy = 0; jy < cnt[1]; ++jy)
      for (int jx = 0; jx < cnt[0]; ++jx) {
        const int bz = (b0[2] + jz) % nbin, by = (b0[1] + jy) % nbin, bx = (b0[0] + jx) % nbin;
        keys[size_t(k) * per + q] = (bz * nbin + by) * nbin + bx;
        vals[size_t(k) * per + q] = k;
        ++q;
      }
  for (; q < per; ++q) {
    keys[size_t(k) * per + q] = sentinel;
    vals[size_t(k) * per + q] = k;
  }
}

// list bounds per block from the sorted slot keys (sentinels ignored)
__global__ void k_block_bounds(int n, int nblk, const int* __restrict__ keys, int* start, int* end) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int c = keys[p];
  if (c >= nblk) return;
  if (p == 0 || keys[p - 1] != c) start[c] = p;
  if (p == n - 1 || keys[p + 1] != c) end[c] = p + 1;
}

hipError_t spread_plan_update(SpreadPlan* sp, const double* pos4, const WaveParams& wp, hipStream_t st) {
  const int nb = sp->nb;
  double* w = sp->wtmp;
  k_bead_prep<<<nblocks(nb), kThreads, 0, st>>>(nb, (const double4*)pos4, wp, sp->BS, sp->nbin, w, sp->stmp,
                                                   sp->keys_in, sp->vals_in);
  int bits = 1;
  const int nbins = sp->nbin * sp->nbin * sp->nbin;
  while ((1 << bits) < nbins) ++bits;
  size_t tb = sp->temp_bytes;
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(sp->temp, tb, sp->keys_in, sp->keys_out, sp->vals_in, sp->perm,
                                                    nb, 0, bits, st);
  if (e != hipSuccess) return e;
  if ((e = hipMemsetAsync(sp->bin_start, 0, sizeof(int) * nbins, st)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(sp->bin_end, 0, sizeof(int) * nbins, st)) != hipSuccess) return e;
  k_bin_bounds<<<nblocks(nb), kThreads, 0, st>>>(nb, sp->keys_out, sp->bin_start, sp->bin_end);
  k_bead_permute<<<nblocks((long long)nb * 3 * sp->P), kThreads, 0, st>>>(nb, 3 * sp->P, sp->perm, w, sp->stmp,
                                                                         sp->weights,
                                                   sp->weights32, sp->starts);
  if (sp->BS == 8) {  // the candidate list of every block
    const int kc = sp->kc, slots = nb * kc * kc * kc;
    k_block_slots<<<nblocks(nb), kThreads, 0, st>>>(nb, sp->starts, sp->P, sp->nbin, kc, sp->pk_in, sp->pv_in);
    int pbits = 1;
    while ((1 << pbits) <= nbins) ++pbits;  // the sentinel nbins included
    size_t pb = sp->ptemp_bytes;
    if ((e = hipcub::DeviceRadixSort::SortPairs(sp->ptemp, pb, sp->pk_in, sp->pk_out, sp->pv_in, sp->cand, slots, 0,
                                                pbits, st)) != hipSuccess)
      return e;
    if ((e = hipMemsetAsync(sp->blk_start, 0, sizeof(int) * nbins, st)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(sp->blk_end, 0, sizeof(int) * nbins, st)) != hipSuccess) return e;
    k_block_bounds<<<nblocks(slots), kThreads, 0, st>>>(slots, nbins, sp->pk_out, sp->blk_start, sp->blk_end);
  }
  return hipGetLastError();
}

namespace {
constexpr int kChunk = 64;
}

template <typename R, int BS>
__global__ __launch_bounds__(BS* BS* BS) void k_spread_gather(const int* __restrict__ bin_start,
                                                               const int* __restrict__ bin_end,
                                                               const int* __restrict__ perm,
                                                               const int4* __restrict__ starts,
                                                               const R* __restrict__ weights,
                                                               const double* __restrict__ lam, WaveParams wp,
                                                               int nbin, int K, R* __restrict__ grid, size_t cs,
                                                               const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int NT = BS * BS * BS;
  __shared__ int4 sh_s[kChunk];
  __shared__ R sh_w[kChunk * 3 * kMaxP];
  __shared__ R sh_l[kChunk * 6];
  __shared__ int rb0[2 * 8 * 8], rlen[2 * 8 * 8], roff[2 * 8 * 8 + 1];
  const int P = wp.support, N = wp.n, P3 = 3 * P;
  const int bx = blockIdx.x % nbin, by = (blockIdx.x / nbin) % nbin, bz = blockIdx.x / (nbin * nbin);
  const int t = threadIdx.x;
  const int mx = bx * BS + t % BS, my = by * BS + (t / BS) % BS, mz = bz * BS + t / (BS * BS);
  // candidate beads: per (kz, ky) one or two contiguous runs of the sorted bead array
  // (bins bx-K+1 .. bx along x, split where they wrap); thread r computes run r
  const int x0 = bx - K + 1;
  const int nparts = x0 >= 0 ? 1 : 2;
  const int nruns = K * K * nparts;
  for (int rr = t; rr < nruns; rr += NT) {
    const int part = rr % nparts, ky = (rr / nparts) % K, kz = rr / (nparts * K);
    const int cz = (bz - kz + nbin) % nbin, cy = (by - ky + nbin) % nbin;
    int lo, hi;
    if (x0 >= 0) {
      lo = x0;
      hi = bx;
    } else if (part == 0) {
      lo = 0;
      hi = bx;
    } else {
      lo = x0 + nbin;
      hi = nbin - 1;
    }
    const int row = (cz * nbin + cy) * nbin;
    int b0 = 0, b1 = 0;
    bool any = false;
    for (int c = lo; c <= hi; ++c) {
      const int e0 = bin_start[row + c], e1 = bin_end[row + c];
      if (e1 > e0) {
        if (!any) b0 = e0;
        b1 = e1;
        any = true;
      }
    }
    rb0[rr] = b0;
    rlen[rr] = any ? b1 - b0 : 0;
  }
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int r = 0; r < nruns; ++r) {
      roff[r] = acc;
      acc += rlen[r];
    }
    roff[nruns] = acc;
  }
  __syncthreads();
  const int total = roff[nruns];
  R a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0;
  for (int c0 = 0; c0 < total; c0 += kChunk) {
    const int n = min(kChunk, total - c0);
    if (c0 > 0) __syncthreads();
    // stage candidates c0 .. c0+n-1 (run-major order) in LDS
    for (int q = t; q < n * (P3 + 7); q += NT) {
      const int cand = q / (P3 + 7), f = q % (P3 + 7);
      const int gidx = c0 + cand;
      int r = 0;
      while (roff[r + 1] <= gidx) ++r;
      const int k = rb0[r] + (gidx - roff[r]);
      if (f < P3) {
        sh_w[cand * P3 + f] = weights[size_t(k) * P3 + f];
      } else if (f == P3) {
        sh_s[cand] = starts[k];
      } else {
        sh_l[6 * cand + (f - P3 - 1)] = R(lam[6 * size_t(perm[k]) + (f - P3 - 1)]);
      }
    }
    __syncthreads();
    for (int q = 0; q < n; ++q) {
      const int4 s = sh_s[q];
      int ix = mx - s.x, iy = my - s.y, iz = mz - s.z;
      ix += ix < 0 ? N : 0;
      iy += iy < 0 ? N : 0;
      iz += iz < 0 ? N : 0;
      if (ix < P && iy < P && iz < P) {
        const R* wq = sh_w + q * P3;
        const R w = wq[ix] * wq[P + iy] * wq[2 * P + iz];
        const R* l = sh_l + 6 * q;
        a0 += w * l[0];
        a1 += w * l[1];
        a2 += w * l[2];
        a3 += w * l[3];
        a4 += w * l[4];
        a5 += w * l[5];
      }
    }
  }
  const size_t m = (size_t(mz) * N + my) * N + mx;
  R* g = grid + 2 * m;
  g[0] = a0;
  g[1] = a3;
  g[cs] = a1;
  g[cs + 1] = a4;
  g[2 * cs] = a2;
  g[2 * cs + 1] = a5;
}

// Gather spreading on 8^3 blocks with the candidates split among the four wavefronts:
// lane (x, y) owns one grid column and all 8 planes of the block; wavefront w takes
// every fourth candidate of the block's list (the beads whose support reaches it, built
// with the plan) and forms the x-y weight once per lane, reusing it over the planes.  The
// four partial blocks are added through LDS in a fixed order (deterministic).  Candidates
// are staged in LDS in chunks of C (dynamic shared memory): the sorted bead index, then
// the weights with independent loads in flight, then start cells and force moments.
constexpr int kSplitRedBytes64 = 2 * 48 * 64 * 8;  // LDS of the two-step reduction (FP64)

template <typename R>
__device__ __forceinline__ void spread_split_body(const int* __restrict__ blk_start,
                                                               const int* __restrict__ blk_end,
                                                               const int* __restrict__ cand,
                                                               const int* __restrict__ perm,
                                                               const int4* __restrict__ starts,
                                                               const R* __restrict__ weights,
                                                               const double* __restrict__ lam, WaveParams wp,
                                                               int nbin, int C, R* __restrict__ grid,
                                                               size_t cs, const int* __restrict__ skip, int bx_, int by_, int gx_) {
  if (skip && *skip) return;
  constexpr int BS = 8, NT = 256, ZW = 8, NW = NT / 64;
  const int P = wp.support, N = wp.n, P3 = 3 * P;
  extern __shared__ unsigned char smem_raw[];
  R* sh_w = reinterpret_cast<R*>(smem_raw);                 // C * 3P
  R* sh_l = sh_w + size_t(C) * P3;                           // C * 6
  int4* sh_s = reinterpret_cast<int4*>(sh_l + size_t(C) * 6); // C
  int* sh_k = reinterpret_cast<int*>(sh_s + C);              // C
  const int bl = xcd_remap(bx_, nbin * nbin * nbin);  // each XCD takes a contiguous slab of blocks
  const int bx = bl % nbin, by = (bl / nbin) % nbin, bz = bl / (nbin * nbin);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int x0 = bx * BS, y0 = by * BS, z0 = bz * BS;
  const int mx = x0 + (lane & 7), my = y0 + (lane >> 3);
  const int cb = blk_start[bl], total = blk_end[bl] - cb;
  R a[ZW][6];
#pragma unroll
  for (int zz = 0; zz < ZW; ++zz)
#pragma unroll
    for (int c = 0; c < 6; ++c) a[zz][c] = 0;
  for (int c0 = 0; c0 < total; c0 += C) {
    const int n = min(C, total - c0);
    if (c0 > 0) __syncthreads();
    for (int c = t; c < n; c += NT) sh_k[c] = cand[cb + c0 + c];
    __syncthreads();
    const int nw = n * P3;
    for (int q0 = t; q0 < nw; q0 += 4 * NT) {
      R v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q0 + u * NT;
        if (q < nw) {
          const int cq = q / P3;
          v[u] = weights[size_t(sh_k[cq]) * P3 + (q - cq * P3)];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (q0 + u * NT < nw) sh_w[q0 + u * NT] = v[u];
    }
    for (int c = t; c < n; c += NT) {
      const int k = sh_k[c];
      sh_s[c] = starts[k];
      const double* l = lam + 6 * size_t(perm[k]);
#pragma unroll
      for (int f = 0; f < 6; ++f) sh_l[6 * c + f] = R(l[f]);
    }
    __syncthreads();
    for (int q = wave; q < n; q += NW) {
      const int4 s = sh_s[q];
      // offsets of the block (or the wave's planes) from the support start, mod N
      int ox = x0 - s.x, oy = y0 - s.y, oz = z0 - s.z;
      ox += ox < 0 ? N : 0;
      oy += oy < 0 ? N : 0;
      oz += oz < 0 ? N : 0;
      if (!((ox < P || ox > N - BS) && (oy < P || oy > N - BS) && (oz < P || oz > N - ZW))) continue;
      int ix = mx - s.x, iy = my - s.y;
      ix += ix < 0 ? N : 0;
      iy += iy < 0 ? N : 0;
      if (ix < P && iy < P) {
        const R* wq = sh_w + q * P3;
        const R wxy = wq[ix] * wq[P + iy];
        const R* l = sh_l + 6 * q;
        const R l0 = l[0], l1 = l[1], l2 = l[2], l3 = l[3], l4 = l[4], l5 = l[5];
        // the planes zz of the block inside the support, (oz + zz) mod N < P: before the
        // wrap zz < P - oz, after it N - oz <= zz < N - oz + P; the same in every lane, so
        // the mask goes to a scalar register and the plane tests are scalar branches
        const int hi1 = min(max(P - oz, 0), ZW), lo2 = min(N - oz, ZW), hi2 = min(N - oz + P, ZW);
        const unsigned zmask = __builtin_amdgcn_readfirstlane(
            int(((1u << hi1) - 1u) | (((1u << hi2) - 1u) & ~((1u << lo2) - 1u))));
#pragma unroll
        for (int zz = 0; zz < ZW; ++zz) {
          if (zmask & (1u << zz)) {
            int iz = oz + zz;
            iz -= iz >= N ? N : 0;
            const R w = wxy * wq[2 * P + iz];
            a[zz][0] += w * l0;
            a[zz][1] += w * l1;
            a[zz][2] += w * l2;
            a[zz][3] += w * l3;
            a[zz][4] += w * l4;
            a[zz][5] += w * l5;
          }
        }
      }
    }
  }
  // partial blocks of waves 2, 3 -> added by waves 0, 1; then wave 1 -> wave 0
  __syncthreads();
  R* red = reinterpret_cast<R*>(smem_raw);  // [2][48][64], reusing the staging area
  if (wave >= 2)
#pragma unroll
    for (int zz = 0; zz < ZW; ++zz)
#pragma unroll
      for (int c = 0; c < 6; ++c) red[((wave - 2) * 48 + zz * 6 + c) * 64 + lane] = a[zz][c];
  __syncthreads();
  if (wave < 2)
#pragma unroll
    for (int zz = 0; zz < ZW; ++zz)
#pragma unroll
      for (int c = 0; c < 6; ++c) a[zz][c] += red[(wave * 48 + zz * 6 + c) * 64 + lane];
  __syncthreads();
  if (wave == 1)
#pragma unroll
    for (int zz = 0; zz < ZW; ++zz)
#pragma unroll
      for (int c = 0; c < 6; ++c) red[(zz * 6 + c) * 64 + lane] = a[zz][c];
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int zz = 0; zz < ZW; ++zz)
#pragma unroll
    for (int c = 0; c < 6; ++c) a[zz][c] += red[(zz * 6 + c) * 64 + lane];
#pragma unroll
  for (int zz = 0; zz < ZW; ++zz) {
    const size_t m = (size_t(z0 + zz) * N + my) * N + mx;
    R* g = grid + 2 * m;
    g[0] = a[zz][0];
    g[1] = a[zz][3];
    g[cs] = a[zz][1];
    g[cs + 1] = a[zz][4];
    g[2 * cs] = a[zz][2];
    g[2 * cs + 1] = a[zz][5];
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_spread_split(const int* __restrict__ blk_start, const int* __restrict__ blk_end,
                                                      const int* __restrict__ cand, const int* __restrict__ perm,
                                                      const int4* __restrict__ starts, const R* __restrict__ weights,
                                                      const double* __restrict__ lam, WaveParams wp, int nbin, int C,
                                                      R* __restrict__ grid, size_t cs, const int* __restrict__ skip) {
  spread_split_body<R>(blk_start, blk_end, cand, perm, starts, weights, lam, wp, nbin, C, grid, cs, skip, blockIdx.x,
                       blockIdx.y, gridDim.x);
}


namespace {
template <typename R>
const R* plan_weights(const SpreadPlan* sp);
template <>
const double* plan_weights<double>(const SpreadPlan* sp) {
  return sp->weights;
}
template <>
const float* plan_weights<float>(const SpreadPlan* sp) {
  return sp->weights32;
}
}  // namespace

template <typename R>
void launch_spread_gather(const SpreadPlan* sp, const double* lam, const WaveParams& wp, R* grid, hipStream_t st,
                          const int* skip) {
  const size_t cs = 2 * size_t(wp.n) * wp.n * wp.n;
  const int nblk = sp->nbin * sp->nbin * sp->nbin;
  if (sp->BS == 8) {
    // candidates per LDS chunk: at most 128, within 60 KB of dynamic shared memory (the
    // static arrays take the rest of 64 KB)
    const size_t per = sizeof(R) * (3 * size_t(wp.support) + 6) + sizeof(int4) + sizeof(int);
    const int C = int(std::min<size_t>(128, (size_t(60) << 10) / per)) & ~3;  // int4 array stays 16-byte aligned
    const size_t shm = std::max(per * C, size_t(kSplitRedBytes64) / sizeof(double) * sizeof(R));
    launch_k(k_spread_split<R>, nblk, 256, shm, st, sp->blk_start, sp->blk_end, sp->cand, sp->perm, sp->starts,
             plan_weights<R>(sp), lam, wp, sp->nbin, C, grid, cs, skip);
  }
  else
    launch_k(k_spread_gather<R, 4>, nblk, 64, 0, st, sp->bin_start, sp->bin_end, sp->perm, sp->starts,
                                                plan_weights<R>(sp), lam, wp, sp->nbin, sp->K, grid, cs, skip);
}

// First pass of the saddle operator in one launch.  The Sigma/lubrication reduction, the
// real-space sum and the gather spreading all read only the input vector, so instead of
// three dependent launches (or a fork onto a second stream) they take three block ranges
// of one grid: the reduction first, then the real-space rows, then the 8^3 spreading
// blocks.  The two short ranges are padded to multiples of 8 blocks, so every spreading
// block keeps the XCD (block index mod 8) its slab mapping assumes, and they finish early,
// leaving their slots to the longer spreading blocks.
template <typename R, int LPR>
__global__ __launch_bounds__(256) void k_spread_fused(const int* __restrict__ blk_start, const int* __restrict__ blk_end,
                                                      const int* __restrict__ cand, const int* __restrict__ perm,
                                                      const int4* __restrict__ starts,
                                                      const R* __restrict__ weights, const double* __restrict__ lam,
                                                      WaveParams wp, int nbin, int C, R* __restrict__ grid,
                                                      size_t cs, const R* __restrict__ tab, RealArgs ra, RigidArgs ga,
                                                      int na_blk, int nr_blk, const int* __restrict__ skip) {
  int b = blockIdx.x;
  if (b < na_blk) {
    agg_lub_body(ga.na, ga.offsets, ga.body, ga.r4, lam, ga.V, ga.lrow, ga.lcol, ga.coef, ga.y2, skip, b, 0, na_blk);
    return;
  }
  b -= na_blk;
  if (b < nr_blk) {
    real_sum_body<R, LPR>(ra.nb, ra.pos, lam, ra.rowptr, ra.col, tab, ra.rp, ra.out, 0, ra.order, skip, b, 0, nr_blk);
    return;
  }
  spread_split_body<R>(blk_start, blk_end, cand, perm, starts, weights, lam, wp, nbin, C, grid, cs, skip, b - nr_blk, 0,
                       0);
}

bool spread_fuses(const SpreadPlan* sp) { return sp && sp->BS == 8; }

template <typename R>
void launch_spread_fused(const SpreadPlan* sp, const double* lam, const WaveParams& wp, R* grid, const R* table,
                         int lpr, const RealArgs& ra, const RigidArgs& ga, hipStream_t st, const int* skip) {
  const size_t cs = 2 * size_t(wp.n) * wp.n * wp.n;
  const int nblk = sp->nbin * sp->nbin * sp->nbin;
  const size_t per = sizeof(R) * (3 * size_t(wp.support) + 6) + sizeof(int4) + sizeof(int);
  const int C = int(std::min<size_t>(128, (size_t(60) << 10) / per)) & ~3;  // as launch_spread_gather
  const size_t shm = std::max(per * C, size_t(kSplitRedBytes64) / sizeof(double) * sizeof(R));
  auto pad8 = [](long long n) { return int((n + 7) / 8 * 8); };
  const int na_blk = pad8((ga.na + 3) / 4), nr_blk = pad8(((long long)ra.nb * lpr + 255) / 256);
  const int total = na_blk + nr_blk + nblk;
#define FSD_FUSED(L_)                                                                                       \
  launch_k(k_spread_fused<R, L_>, total, 256, shm, st, sp->blk_start, sp->blk_end, sp->cand, sp->perm,        \
           sp->starts, plan_weights<R>(sp), lam, wp, sp->nbin, C, grid, cs, table, ra, ga, na_blk, nr_blk, skip)
  switch (lpr) {
    case 1: FSD_FUSED(1); break;
    case 2: FSD_FUSED(2); break;
    case 4: FSD_FUSED(4); break;
    case 8: FSD_FUSED(8); break;
    case 16: FSD_FUSED(16); break;
    case 32: FSD_FUSED(32); break;
    default: FSD_FUSED(64); break;
  }
#undef FSD_FUSED
}

// ------------------------------------------------------------------------------------------
// 3D FFT: three passes of batched 1D transforms, each line staged in LDS and
// transformed by mixed-radix (4, 2, 3, 5) Stockham stages.
// ------------------------------------------------------------------------------------------

namespace {
template <typename T>
__device__ inline T cmul(T a, T b) {
  T r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename T>
__device__ inline T cadd(T a, T b) {
  T r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <typename T>
__device__ inline T csub(T a, T b) {
  T r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}
// Quotient and remainder by a divisor known only at run time, for dividends below 2^21:
// the product with the FP32 reciprocal (v_rcp_f32, within 1 ulp) is within 1/4 of the true
// quotient, so truncating it and one correction step give the exact result (a hardware
// integer division sequence costs about 25 instructions per use in these index loops).
struct FastDiv {
  int d;
  float inv;
  __device__ explicit FastDiv(int d_) : d(d_), inv(__frcp_rn(float(d_))) {}
  __device__ __forceinline__ int div(int a) const {
    int q = int(float(a) * inv);
    const int r = a - q * d;
    q += (r >= d) - (r < 0);
    return q;
  }
  __device__ __forceinline__ void divmod(int a, int& q, int& r) const {
    q = div(a);
    r = a - q * d;
  }
};

// multiply by -i*sign... rot(v, s) = s * i * v
template <typename T>
__device__ inline T rot(T v, int s) {
  T r;
  r.x = -s * v.y;
  r.y = s * v.x;
  return r;
}
}  // namespace

namespace {
// One radix-Rd butterfly of a Stockham stage: reads Rd inputs nbf apart, twiddles them by
// w^(r k tstride) (w = exp(s 2 pi i / N), the table tw), transforms and writes them Ns apart.
template <typename T, typename R, int Rd>
__device__ __forceinline__ void butterfly(const T* li, T* lo, const T* tw, int b, int nbf, int k, int Ns, int tstride,
                                          int od, int s) {
  T v[Rd];
#pragma unroll
  for (int r = 0; r < Rd; ++r) v[r] = li[b + r * nbf];
  if (Ns > 1) {
#pragma unroll
    for (int r = 1; r < Rd; ++r) v[r] = cmul(v[r], tw[r * k * tstride]);
  }
  if (Rd == 8) {
    // even and odd halves by 4-point transforms, joined by w^k = exp(s 2 pi i k / 8)
    const T es02 = cadd(v[0], v[4]), ed02 = csub(v[0], v[4]), es13 = cadd(v[2], v[6]),
            ed13 = rot(csub(v[2], v[6]), s);
    const T os02 = cadd(v[1], v[5]), od02 = csub(v[1], v[5]), os13 = cadd(v[3], v[7]),
            od13 = rot(csub(v[3], v[7]), s);
    const T e0 = cadd(es02, es13), e1 = cadd(ed02, ed13), e2 = csub(es02, es13), e3 = csub(ed02, ed13);
    const T o0 = cadd(os02, os13), o1 = cadd(od02, od13), o2 = csub(os02, os13), o3 = csub(od02, od13);
    const R h8 = R(0.70710678118654752440), sr = R(s);
    T t1, t3;
    t1.x = h8 * (o1.x - sr * o1.y);  // w o1, w = (1 + s i) / sqrt 2
    t1.y = h8 * (o1.y + sr * o1.x);
    t3.x = -h8 * (o3.x + sr * o3.y);  // w^3 o3, w^3 = (-1 + s i) / sqrt 2
    t3.y = h8 * (sr * o3.x - o3.y);
    const T t2 = rot(o2, s);
    lo[od] = cadd(e0, o0);
    lo[od + 4 * Ns] = csub(e0, o0);
    lo[od + Ns] = cadd(e1, t1);
    lo[od + 5 * Ns] = csub(e1, t1);
    lo[od + 2 * Ns] = cadd(e2, t2);
    lo[od + 6 * Ns] = csub(e2, t2);
    lo[od + 3 * Ns] = cadd(e3, t3);
    lo[od + 7 * Ns] = csub(e3, t3);
  } else if (Rd == 4) {
    const T s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]), s13 = cadd(v[1], v[3]), d13 = rot(csub(v[1], v[3]), s);
    lo[od] = cadd(s02, s13);
    lo[od + Ns] = cadd(d02, d13);
    lo[od + 2 * Ns] = csub(s02, s13);
    lo[od + 3 * Ns] = csub(d02, d13);
  } else if (Rd == 2) {
    lo[od] = cadd(v[0], v[1]);
    lo[od + Ns] = csub(v[0], v[1]);
  } else if (Rd == 3) {
    const R c3 = R(-0.5), s3 = R(0.86602540378443864676);
    const T sm = cadd(v[1], v[2]), jd = rot(csub(v[1], v[2]), s);  // s i (v1 - v2)
    T m1, y1, y2;
    m1.x = v[0].x + c3 * sm.x;
    m1.y = v[0].y + c3 * sm.y;
    y1.x = m1.x + s3 * jd.x;
    y1.y = m1.y + s3 * jd.y;
    y2.x = m1.x - s3 * jd.x;
    y2.y = m1.y - s3 * jd.y;
    lo[od] = cadd(v[0], sm);
    lo[od + Ns] = y1;
    lo[od + 2 * Ns] = y2;
  } else {  // radix 5: cos and sin of 2 pi / 5 and 4 pi / 5
    const R c1 = R(0.30901699437494742410), c2 = R(-0.80901699437494742410);
    const R s1 = R(0.95105651629515357212), s2 = R(0.58778525229247312917);
    const T t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    const T t3 = rot(csub(v[1], v[4]), s), t4 = rot(csub(v[2], v[3]), s);  // s i (v1 - v4), s i (v2 - v3)
    T m1, m2, p1, p2;
    m1.x = v[0].x + c1 * t1.x + c2 * t2.x;
    m1.y = v[0].y + c1 * t1.y + c2 * t2.y;
    m2.x = v[0].x + c2 * t1.x + c1 * t2.x;
    m2.y = v[0].y + c2 * t1.y + c1 * t2.y;
    p1.x = s1 * t3.x + s2 * t4.x;
    p1.y = s1 * t3.y + s2 * t4.y;
    p2.x = s2 * t3.x - s1 * t4.x;
    p2.y = s2 * t3.y - s1 * t4.y;
    lo[od] = cadd(v[0], cadd(t1, t2));
    lo[od + Ns] = cadd(m1, p1);
    lo[od + 2 * Ns] = cadd(m2, p2);
    lo[od + 3 * Ns] = csub(m2, p2);
    lo[od + 4 * Ns] = csub(m1, p1);
  }
}

// Stockham stages (radices 8, 4, 2, 3, 5) on `nl` lines of length N held in LDS `ls`
// elements apart (`in`, scratch `out`); returns the buffer holding the result.  The
// radices come from the plan's packed code (4 bits per stage), so the stage loop indexes
// no array.
template <typename T, typename R>
__device__ __forceinline__ T* stockham(T* in, T* out, const T* tw, int N, int ls, int nl, const FftPlan& plan,
                                       int s) {
  int Ns = 1;
  const unsigned long long code = plan.rcode;
  for (int stg = 0; stg < plan.nstage; ++stg) {
    const int Rd = int((code >> (4 * stg)) & 15ull);
    const int nbf = N / Rd;
    const int tstride = N / (Ns * Rd);
    const FastDiv dbf(nbf), dns(Ns);
    for (int t = threadIdx.x; t < nl * nbf; t += blockDim.x) {
      int l, b, j, k;
      dbf.divmod(t, l, b);
      dns.divmod(b, j, k);
      const T* li = in + l * ls;
      T* lo = out + l * ls;
      const int od = j * Ns * Rd + k;
      if (Rd == 8)
        butterfly<T, R, 8>(li, lo, tw, b, nbf, k, Ns, tstride, od, s);
      else if (Rd == 4)
        butterfly<T, R, 4>(li, lo, tw, b, nbf, k, Ns, tstride, od, s);
      else if (Rd == 2)
        butterfly<T, R, 2>(li, lo, tw, b, nbf, k, Ns, tstride, od, s);
      else if (Rd == 3)
        butterfly<T, R, 3>(li, lo, tw, b, nbf, k, Ns, tstride, od, s);
      else
        butterfly<T, R, 5>(li, lo, tw, b, nbf, k, Ns, tstride, od, s);
    }
    __syncthreads();
    T* tmp = in;
    in = out;
    out = tmp;
    Ns *= Rd;
  }
  return in;
}

// Stockham stages on B lines (B a power of two, 2^lb) held S elements apart, with the
// line as the fastest thread index: t -> (line t & (B - 1), butterfly t >> lb).  Lanes
// that differ in the line meet distinct banks (the stride of fft_line_stride), and the
// mapping needs one division per butterfly (by the stage's Ns) instead of two.
// As stockham_lines for any number of lines nl (held S apart, S odd so that consecutive
// lines start on distinct banks): t -> (line t mod nl, butterfly t / nl).
template <typename T, typename R>
__device__ __forceinline__ T* stockham_lm(T* in, T* out, const T* tw, int N, int S, int nl, const FftPlan& plan,
                                          int s) {
  int Ns = 1;
  const unsigned long long code = plan.rcode;
  const FastDiv dnl(nl);
  for (int stg = 0; stg < plan.nstage; ++stg) {
    const int Rd = int((code >> (4 * stg)) & 15ull);
    const int nbf = N / Rd;
    const int tstride = N / (Ns * Rd);
    const FastDiv dns(Ns);
    for (int t = threadIdx.x; t < nl * nbf; t += blockDim.x) {
      int b, l, j, k;
      dnl.divmod(t, b, l);
      dns.divmod(b, j, k);
      const T* li = in + l * S;
      T* lo = out + l * S;
      const int od = j * Ns * Rd + k;
      if (Rd == 8)
        butterfly<T, R, 8>(li, lo, tw, b, nbf, k, Ns, tstride, od, s);
      else if (Rd == 4)
        butterfly<T, R, 4>(li, lo, tw, b, nbf, k, Ns, tstride, od, s);
      else if (Rd == 2)
        butterfly<T, R, 2>(li, lo, tw, b, nbf, k, Ns, tstride, od, s);
      else if (Rd == 3)
        butterfly<T, R, 3>(li, lo, tw, b, nbf, k, Ns, tstride, od, s);
      else
        butterfly<T, R, 5>(li, lo, tw, b, nbf, k, Ns, tstride, od, s);
    }
    __syncthreads();
    T* tmp = in;
    in = out;
    out = tmp;
    Ns *= Rd;
  }
  return in;
}

template <typename T, typename R>
__device__ __forceinline__ T* stockham_lines(T* in, T* out, const T* tw, int N, int S, int B, int lb,
                                             const FftPlan& plan, int s) {
  int Ns = 1;
  const unsigned long long code = plan.rcode;
  for (int stg = 0; stg < plan.nstage; ++stg) {
    const int Rd = int((code >> (4 * stg)) & 15ull);
    const int nbf = N / Rd;
    const int tstride = N / (Ns * Rd);
    const FastDiv dns(Ns);
    for (int t = threadIdx.x; t < (nbf << lb); t += blockDim.x) {
      const int l = t & (B - 1), b = t >> lb;
      int j, k;
      dns.divmod(b, j, k);
      const T* li = in + l * S;
      T* lo = out + l * S;
      const int od = j * Ns * Rd + k;
      if (Rd == 8)
        butterfly<T, R, 8>(li, lo, tw, b, nbf, k, Ns, tstride, od, s);
      else if (Rd == 4)
        butterfly<T, R, 4>(li, lo, tw, b, nbf, k, Ns, tstride, od, s);
      else if (Rd == 2)
        butterfly<T, R, 2>(li, lo, tw, b, nbf, k, Ns, tstride, od, s);
      else if (Rd == 3)
        butterfly<T, R, 3>(li, lo, tw, b, nbf, k, Ns, tstride, od, s);
      else
        butterfly<T, R, 5>(li, lo, tw, b, nbf, k, Ns, tstride, od, s);
    }
    __syncthreads();
    T* tmp = in;
    in = out;
    out = tmp;
    Ns *= Rd;
  }
  return in;
}

// stockham_lines for a grid side N known at compile time: the radices (8s, then 4, 2, 3s,
// 5s), the butterfly counts, the divisions by Ns and the LDS offsets of every stage fold
// into constants.  Used for the common grid sides; others take stockham_lines.
template <int Rem>
constexpr int pick_radix() {
  return Rem % 8 == 0 ? 8 : Rem % 4 == 0 ? 4 : Rem % 2 == 0 ? 2 : Rem % 3 == 0 ? 3 : 5;
}

template <typename T, typename R, int N, int Ns, int Rem>
__device__ __forceinline__ T* stockham_n(T* in, T* out, const T* tw, int S, int B, int lb, int s) {
  if constexpr (Rem == 1) {
    return in;
  } else {
    constexpr int Rd = pick_radix<Rem>(), nbf = N / Rd, tstride = N / (Ns * Rd);
    for (int t = threadIdx.x; t < (nbf << lb); t += blockDim.x) {
      const int l = t & (B - 1), b = t >> lb;
      const int j = b / Ns, k = b - j * Ns;
      butterfly<T, R, Rd>(in + l * S, out + l * S, tw, b, nbf, k, Ns, tstride, j * Ns * Rd + k, s);
    }
    __syncthreads();
    return stockham_n<T, R, N, Ns * Rd, Rem / Rd>(out, in, tw, S, B, lb, s);
  }
}

// stockham_lm for a compile-time grid side (nl lines, dnl its divider)
template <typename T, typename R, int N, int Ns, int Rem>
__device__ __forceinline__ T* stockham_lm_n(T* in, T* out, const T* tw, int S, int nl, const FastDiv& dnl, int s) {
  if constexpr (Rem == 1) {
    return in;
  } else {
    constexpr int Rd = pick_radix<Rem>(), nbf = N / Rd, tstride = N / (Ns * Rd);
    for (int t = threadIdx.x; t < nl * nbf; t += blockDim.x) {
      int b, l;
      dnl.divmod(t, b, l);
      const int j = b / Ns, k = b - j * Ns;
      butterfly<T, R, Rd>(in + l * S, out + l * S, tw, b, nbf, k, Ns, tstride, j * Ns * Rd + k, s);
    }
    __syncthreads();
    return stockham_lm_n<T, R, N, Ns * Rd, Rem / Rd>(out, in, tw, S, nl, dnl, s);
  }
}

template <typename T, typename R>
__device__ __forceinline__ T* stockham_lm_any(T* in, T* out, const T* tw, int N, int S, int nl, const FftPlan& plan,
                                              int s) {
  const FastDiv dnl(nl);
  switch (N) {
    case 32: return stockham_lm_n<T, R, 32, 1, 32>(in, out, tw, S, nl, dnl, s);
    case 40: return stockham_lm_n<T, R, 40, 1, 40>(in, out, tw, S, nl, dnl, s);
    case 48: return stockham_lm_n<T, R, 48, 1, 48>(in, out, tw, S, nl, dnl, s);
    case 64: return stockham_lm_n<T, R, 64, 1, 64>(in, out, tw, S, nl, dnl, s);
    case 72: return stockham_lm_n<T, R, 72, 1, 72>(in, out, tw, S, nl, dnl, s);
    case 80: return stockham_lm_n<T, R, 80, 1, 80>(in, out, tw, S, nl, dnl, s);
    case 96: return stockham_lm_n<T, R, 96, 1, 96>(in, out, tw, S, nl, dnl, s);
    case 120: return stockham_lm_n<T, R, 120, 1, 120>(in, out, tw, S, nl, dnl, s);
    case 128: return stockham_lm_n<T, R, 128, 1, 128>(in, out, tw, S, nl, dnl, s);
    default: return stockham_lm<T, R>(in, out, tw, N, S, nl, plan, s);
  }
}

// stockham_lines with the grid side dispatched to a compile-time instance where there is one
template <typename T, typename R>
__device__ __forceinline__ T* stockham_lines_any(T* in, T* out, const T* tw, int N, int S, int B, int lb,
                                                 const FftPlan& plan, int s) {
  switch (N) {
    case 32: return stockham_n<T, R, 32, 1, 32>(in, out, tw, S, B, lb, s);
    case 40: return stockham_n<T, R, 40, 1, 40>(in, out, tw, S, B, lb, s);
    case 48: return stockham_n<T, R, 48, 1, 48>(in, out, tw, S, B, lb, s);
    case 64: return stockham_n<T, R, 64, 1, 64>(in, out, tw, S, B, lb, s);
    case 72: return stockham_n<T, R, 72, 1, 72>(in, out, tw, S, B, lb, s);
    case 80: return stockham_n<T, R, 80, 1, 80>(in, out, tw, S, B, lb, s);
    case 96: return stockham_n<T, R, 96, 1, 96>(in, out, tw, S, B, lb, s);
    case 120: return stockham_n<T, R, 120, 1, 120>(in, out, tw, S, B, lb, s);
    case 128: return stockham_n<T, R, 128, 1, 128>(in, out, tw, S, B, lb, s);
    default: return stockham_lines<T, R>(in, out, tw, N, S, B, lb, plan, s);
  }
}

}  // namespace

template <typename R, int DIR>
__global__ __launch_bounds__(256) void k_fft_pass(R* __restrict__ data, size_t cs, FftPlan plan,
                                                  const R* __restrict__ twiddle, int sign, int B, const int* __restrict__ skip) {
  if (skip && *skip) return;
  using T = typename C2<R>::T;
  extern __shared__ unsigned char smem_raw[];
  const int N = plan.n;
  const int S = fft_line_stride(N, B, int(sizeof(T)));
  T* buf0 = reinterpret_cast<T*>(smem_raw);
  T* buf1 = buf0 + B * S;
  T* tw = buf1 + B * S;
  T* base = reinterpret_cast<T*>(data + blockIdx.y * cs);
  const int line0 = blockIdx.x * B;
  const T* twg = reinterpret_cast<const T*>(twiddle);
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    T w = twg[t];
    if (sign > 0) w.y = -w.y;
    tw[t] = w;
  }
  for (int t = threadIdx.x; t < B * N; t += blockDim.x) {
    int l, e;
    if (DIR == 0) {
      l = t / N;
      e = t % N;
    } else {
      l = t % B;
      e = t / B;
    }
    const size_t gl = size_t(line0 + l);
    size_t off;
    if (DIR == 0)
      off = gl * N + e;
    else if (DIR == 1)
      off = ((gl / N) * N + e) * N + (gl % N);
    else
      off = (size_t(e) * N + (gl / N)) * N + (gl % N);
    buf0[l * S + e] = base[off];
  }
  __syncthreads();
  const T* in = stockham<T, R>(buf0, buf1, tw, N, S, B, plan, sign > 0 ? 1 : -1);
  for (int t = threadIdx.x; t < B * N; t += blockDim.x) {
    int l, e;
    if (DIR == 0) {
      l = t / N;
      e = t % N;
    } else {
      l = t % B;
      e = t / B;
    }
    const size_t gl = size_t(line0 + l);
    size_t off;
    if (DIR == 0)
      off = gl * N + e;
    else if (DIR == 1)
      off = ((gl / N) * N + e) * N + (gl % N);
    else
      off = (size_t(e) * N + (gl / N)) * N + (gl % N);
    base[off] = in[l * S + e];
  }
}

namespace {
int lines_per_block(int N) {
  int B = 1;
  while (B * 2 * N <= 1024 && (N % (B * 2)) == 0) B *= 2;
  return B;
}
}  // namespace

template <typename R>
void launch_fft3d(R* grid, int ncomp, size_t comp_stride, const FftPlan& plan, const R* twiddle, int sign,
                  hipStream_t st, int pass, const int* skip) {
  using T = typename C2<R>::T;
  const int N = plan.n;
  const int B = lines_per_block(N);
  const size_t shm = sizeof(T) * (2 * size_t(B) * fft_line_stride(N, B, int(sizeof(T))) + N);
  dim3 g(N * N / B, ncomp);
  if (pass < 0 || pass == 0) k_fft_pass<R, 0><<<g, kThreads, shm, st>>>(grid, comp_stride, plan, twiddle, sign, B, skip);
  if (pass < 0 || pass == 1) k_fft_pass<R, 1><<<g, kThreads, shm, st>>>(grid, comp_stride, plan, twiddle, sign, B, skip);
  if (pass < 0 || pass == 2) k_fft_pass<R, 2><<<g, kThreads, shm, st>>>(grid, comp_stride, plan, twiddle, sign, B, skip);
}

namespace {
// Block-wide copy of `count` elements, t -> store(t, load(t)), with U loads in flight per
// thread: each thread issues its next U loads before it writes any of them, so one wait
// covers U memory latencies (a plain strided loop waits once per element).
template <int U, typename T, typename Load, typename Store>
__device__ __forceinline__ void staged_copy(int count, Load&& load, Store&& store) {
  for (int t0 = threadIdx.x; t0 < count; t0 += U * int(blockDim.x)) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * int(blockDim.x);
      if (t < count) v[u] = load(t);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * int(blockDim.x);
      if (t < count) store(t, v[u]);
    }
  }
}

template <typename T>
__device__ inline void load_twiddles(T* tw, const T* twg, int N, int sign) {
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    T w = twg[t];
    if (sign > 0) w.y = -w.y;
    tw[t] = w;
  }
}
}  // namespace

namespace {
__device__ inline void sinc_jv_d(double x, double& s, double& j) {
  if (x < 0.5) {
    const double x2 = x * x;
    s = 1.0 - x2 / 6.0 * (1.0 - x2 / 20.0 * (1.0 - x2 / 42.0 * (1.0 - x2 / 72.0 * (1.0 - x2 / 110.0))));
    j = 1.0 - x2 / 10.0 * (1.0 - x2 / 28.0 * (1.0 - x2 / 54.0 * (1.0 - x2 / 88.0 * (1.0 - x2 / 130.0))));
  } else {
    double sn, cn;
    sincos(x, &sn, &cn);
    s = sn / x;
    j = 3.0 * (sn - x * cn) / (x * x * x);
  }
}
}  // namespace

// ------------------------------------------------------------------------------------------
// Coalesced wave-space pipeline for N <= 256 (5 passes, in place on the three packed
// complex grids Z_c = F_c + i T_c):
//   z, y  : transforms along z, then y; a workgroup takes B consecutive x of B lines,
//           so every load and store is a run of B contiguous complex values
//   x+G   : one workgroup per pair of rows (ky, kz) and (-ky, -kz) of all three grids:
//           forward x transform, split of the packed spectra by Hermitian symmetry
//           (F^(k) = (Z(k) + conj Z(-k)) / 2, T^(k) = (Z(k) - conj Z(-k)) / 2i, the -k
//           partner lies in the paired row), Green's-function scaling, repacking as
//           Y^ = U^ + i W^, inverse x transform
//   y, z  : inverse transforms
// The product is the same linear operator as the half-spectrum pipeline.
// ------------------------------------------------------------------------------------------

template <typename R, int DIR>
__device__ __forceinline__ void fft_lines_body(R* __restrict__ grid, size_t cs, FftPlan plan,
                                               const R* __restrict__ twiddle, int sign, int B,
                                               const int* __restrict__ skip, int bx_, int by_, int gx_) {
  if (skip && *skip) return;
  using T = typename C2<R>::T;
  extern __shared__ unsigned char smem_raw[];
  const int N = plan.n;
  const int S = fft_line_stride(N, B, int(sizeof(T)));
  T* buf0 = reinterpret_cast<T*>(smem_raw);
  T* buf1 = buf0 + B * S;
  T* tw = buf1 + B * S;
  T* base = reinterpret_cast<T*>(grid + by_ * cs);
  const int line0 = bx_ * B;  // line gl = o N + x: B consecutive x of one o (B divides N)
  const int o = line0 / N, x0 = line0 - o * N;
  const int lb = __ffs(B) - 1;  // B is a power of two
  // element e of line l sits at g[e * es + l]: a workgroup-uniform base and a 32-bit
  // offset (its byte offset stays below 2 N^3 sizeof(R) <= 2^28 for N <= 256)
  R* g = reinterpret_cast<R*>(base + (DIR == 1 ? size_t(o) * N * N : size_t(o) * N) + x0);
  const unsigned es = DIR == 1 ? N : N * N;
  load_twiddles(tw, reinterpret_cast<const T*>(twiddle), N, sign);
  staged_copy<8, T>(
      B * N,
      [&](int t) {
        T v;
        ldg2(g, 2 * (unsigned(t >> lb) * es + unsigned(t & (B - 1))), v.x, v.y);
        return v;
      },
      [&](int t, const T& v) { buf0[(t & (B - 1)) * S + (t >> lb)] = v; });
  __syncthreads();
  const T* Y = stockham_lines_any<T, R>(buf0, buf1, tw, N, S, B, lb, plan, sign);
  for (int t = threadIdx.x; t < B * N; t += blockDim.x) {
    const int l = t & (B - 1), e = t >> lb;
    const T y = Y[l * S + e];
    stg2(g, 2 * (unsigned(e) * es + unsigned(l)), y.x, y.y);
  }
}

template <typename R, int DIR>
__global__ __launch_bounds__(256) void k_fft_lines(R* __restrict__ grid, size_t cs, FftPlan plan,
                                                   const R* __restrict__ twiddle, int sign, int B,
                                                   const int* __restrict__ skip) {
  fft_lines_body<R, DIR>(grid, cs, plan, twiddle, sign, B, skip, blockIdx.x, blockIdx.y, gridDim.x);
}

// TABLE: the cube, multipliers read from the table by |m|^2; otherwise (the sheared lattice)
// computed per mode.  Two instantiations keep the per-mode FP64 arithmetic out of the
// cube's register budget.
// LDS of the x+Green pass with G row slots and complex values of tb bytes: two buffers of
// 6 G lines (stride N | 1) and the twiddles, then (16-byte aligned) the 2 G row descriptors
__host__ __device__ inline size_t xgreen_rows_offset(int N, int G, int tb) {
  return (size_t(tb) * (12 * size_t(G) * (N | 1) + N) + 15) & ~size_t(15);
}
__host__ __device__ inline size_t xgreen_shm(int N, int G, int tb) {
  return xgreen_rows_offset(N, G, tb) + 2 * size_t(G) * sizeof(int4);
}

template <typename R, bool TABLE>
__device__ __forceinline__ void fft_xgreen_body(R* __restrict__ grid, size_t cs, FftPlan plan,
                                                const R* __restrict__ twiddle, WaveParams wp, int G,
                                                const int* __restrict__ skip, int bx_, int by_, int gx_) {
  if (skip && *skip) return;
  using T = typename C2<R>::T;
  extern __shared__ unsigned char smem_raw[];
  const int N = plan.n, NN = N * N;
  // G row slots per workgroup; slot g takes the pair number p = bx G + g of the
  // N^2/2 + 2 pairs {r, rp} (r = kz N + ky, rp = its (-kz, -ky) partner, r <= rp; the
  // four self-paired rows have rp == r).  Line (g, c, q) = component c of row q (0: r,
  // 1: rp) sits at (6 g + 2 c + q) N; lines of idle slots are zero.
  const int NL = 6 * G, S = N | 1;  // lines S apart: an odd stride spreads them over the banks
  T* buf0 = reinterpret_cast<T*>(smem_raw);
  T* buf1 = buf0 + NL * S;
  T* tw = buf1 + NL * S;
  int4* rows = reinterpret_cast<int4*>(smem_raw + xgreen_rows_offset(N, G, int(sizeof(T))));
  const int H = N / 2, npair = NN / 2 + 2;
  const FastDiv dn(N);
  auto row_of = [N, H](int p) {  // pair number -> its first row r
    if (p <= H) return p;                        // kz = 0, ky = 0 .. N/2
    p -= H + 1;
    if (p < (H - 1) * N) return N + p;           // kz = 1 .. N/2 - 1, all ky
    return H * N + (p - (H - 1) * N);            // kz = N/2, ky = 0 .. N/2
  };
  // one descriptor per (slot g, row q), index 2 g + q: x = the row's (kz, ky) packed with
  // bit 31 set (0: no row), y, z = LDS offsets of its line and of its partner's line
  // (component 0), w = the row's index in the grid (-1: none)
  for (int i = threadIdx.x; i < 2 * G; i += blockDim.x) {
    const int g = i >> 1, q = i & 1, pn = bx_ * G + g;
    int4 v = make_int4(0, 0, 0, -1);
    if (pn < npair) {
      const int r = row_of(pn);
      int kz, ky;
      dn.divmod(r, kz, ky);
      const int rp = (kz ? N - kz : 0) * N + (ky ? N - ky : 0);  // the row of (-kz, -ky)
      if (q == 0 || rp != r) {
        if (q) dn.divmod(rp, kz, ky);
        const int qm = rp == r ? 0 : 1 - q;
        v.x = int(0x80000000u | (unsigned(kz) << 15) | unsigned(ky));
        v.y = (6 * g + q) * S;
        v.z = (6 * g + qm) * S;
        v.w = q ? rp : r;
      }
    }
    rows[i] = v;
  }
  load_twiddles(tw, reinterpret_cast<const T*>(twiddle), N, -1);
  __syncthreads();
  staged_copy<8, T>(
      NL * N,
      [&](int t) {
        int line, x;
        dn.divmod(t, line, x);
        const int g = line / 6, c = (line % 6) >> 1, q = line & 1;
        const int row = rows[2 * g + q].w;
        T v;
        v.x = 0;
        v.y = 0;
        if (row >= 0) ldg2(grid, unsigned(c * cs) + 2 * unsigned(row * N + x), v.x, v.y);
        return v;
      },
      [&](int t, const T& v) {
        int line, x;
        dn.divmod(t, line, x);
        buf0[line * S + x] = v;
      });
  __syncthreads();
  T* X = stockham_lm_any<T, R>(buf0, buf1, tw, N, S, NL, plan, -1);
  T* O = (X == buf0) ? buf1 : buf0;
  const double tp = 2.0 * M_PI / wp.L, gam = (!TABLE && wp.gam) ? *wp.gam : 0.0;
  // items (row 2 g + q, x mode kx), kx fastest; each thread steps blockDim.x items at a time
  int gq, kx;
  dn.divmod(int(threadIdx.x), gq, kx);
  const int dq = int(blockDim.x) / N, dr = int(blockDim.x) - dq * N;
  for (; gq < 2 * G; gq += dq, kx += dr) {
    if (kx >= N) {
      kx -= N;
      if (++gq >= 2 * G) break;
    }
    const int4 ri = rows[gq];
    if (ri.x >= 0) continue;  // no row
    const int kz = (ri.x >> 15) & 0x7fff, ky = ri.x & 0x7fff;
    const int kxm = kx ? N - kx : 0;
    const int o = ri.y + kx, om = ri.z + kxm;  // this mode and its (-k) partner, component 0
    const bool nyq = (N % 2 == 0) && (kx == N / 2 || ky == N / 2 || kz == N / 2);
    if (nyq || (kx == 0 && ky == 0 && kz == 0)) {
      for (int c = 0; c < 3; ++c) {
        O[o + 2 * c * S].x = 0;
        O[o + 2 * c * S].y = 0;
      }
      continue;
    }
    // the per-mode arithmetic runs in the grid's precision R (the multipliers are tabulated
    // in FP64 and rounded once).  F, T below are twice the split spectra
    // F^ = (Z(k) + conj Z(-k)) / 2, T^ = (Z(k) - conj Z(-k)) / 2i; the halving moves into the
    // scalar factor Bk (exact: the products scale by powers of two)
    R Fr[3], Fi[3], Tr[3], Ti[3];
    for (int c = 0; c < 3; ++c) {
      const T z = X[o + 2 * c * S], zm = X[om + 2 * c * S];
      Fr[c] = z.x + zm.x;
      Fi[c] = z.y - zm.y;
      Tr[c] = z.y + zm.y;
      Ti[c] = zm.x - z.x;
    }
    // Cartesian wave vector of grid mode m: (2 pi / L)(m_x, m_y - gam m_x, m_z) (the
    // reciprocal lattice of the sheared lattice; gam = 0 for the cube)
    // signed mode numbers in [-N/2, N/2] (an even N's N/2 modes were zeroed above; an odd N
    // keeps the symmetric range), so |m|^2 <= 3 (N/2)^2 indexes the multiplier table
    const int mx = kx <= N / 2 ? kx : kx - N, my = ky <= N / 2 ? ky : ky - N, mz = kz <= N / 2 ? kz : kz - N;
    const R k[3] = {R(tp * mx), R(tp * (my - gam * mx)), R(tp * mz)};
    R sk, jk, Bk, ikn;
    if (TABLE) {  // the multipliers depend on the integer |m|^2 alone
      const int m2 = mx * mx + my * my + mz * mz;
      if constexpr (sizeof(R) == 4) {  // the FP32 copy of the table (the same roundings)
        const float4 g4 = *reinterpret_cast<const float4*>(wp.gtab32 + 8 * m2);
        sk = g4.x;
        jk = g4.y;
        Bk = wp.brownian ? g4.w : g4.z;
        ikn = wp.gtab32[8 * m2 + 4];
      } else {
        const double* gt = wp.gtab + 5 * m2;
        sk = R(gt[0]);
        jk = R(gt[1]);
        Bk = R(wp.brownian ? gt[3] : gt[2]);
        ikn = R(gt[4]);
      }
    } else {
      const double kd[3] = {tp * mx, tp * (my - gam * mx), tp * mz};
      const double k2 = kd[0] * kd[0] + kd[1] * kd[1] + kd[2] * kd[2];
      const double kn = sqrt(k2);
      double skd, jkd;
      sinc_jv_d(kn * wp.a, skd, jkd);
      const double qq = k2 / (4.0 * wp.xi * wp.xi);
      const double damp = (1.0 + qq) * exp(-(1.0 - wp.eta_t) * qq) / wp.eta;
      sk = R(skd);
      jk = R(jkd);
      ikn = R(1.0 / kn);
      Bk = R(wp.brownian ? sqrt(wp.scale / (double(N) * N * N) * damp) / kn : wp.scale * damp / k2);
    }
    Bk *= R(0.5);
    const R hjk = R(0.5) * jk;
    const R kh[3] = {k[0] * ikn, k[1] * ikn, k[2] * ikn};
    R gr[3], gi[3];
    if (wp.brownian) {
      for (int a = 0; a < 3; ++a) {
        gr[a] = Fr[a];
        gi[a] = Fi[a];
      }
    } else {
      const R cxr[3] = {k[1] * Tr[2] - k[2] * Tr[1], k[2] * Tr[0] - k[0] * Tr[2], k[0] * Tr[1] - k[1] * Tr[0]};
      const R cxi[3] = {k[1] * Ti[2] - k[2] * Ti[1], k[2] * Ti[0] - k[0] * Ti[2], k[0] * Ti[1] - k[1] * Ti[0]};
      for (int a = 0; a < 3; ++a) {
        gr[a] = sk * Fr[a] - hjk * cxi[a];
        gi[a] = sk * Fi[a] + hjk * cxr[a];
      }
    }
    const R pr = kh[0] * gr[0] + kh[1] * gr[1] + kh[2] * gr[2];
    const R pim = kh[0] * gi[0] + kh[1] * gi[1] + kh[2] * gi[2];
    R ur[3], ui[3];
    for (int a = 0; a < 3; ++a) {
      ur[a] = Bk * (gr[a] - pr * kh[a]);
      ui[a] = Bk * (gi[a] - pim * kh[a]);
    }
    // U^ = sinc u^, W^ = (i/2) jv (k x u^); Y^ = U^ + i W^
    const R kur[3] = {k[1] * ur[2] - k[2] * ur[1], k[2] * ur[0] - k[0] * ur[2], k[0] * ur[1] - k[1] * ur[0]};
    const R kui[3] = {k[1] * ui[2] - k[2] * ui[1], k[2] * ui[0] - k[0] * ui[2], k[0] * ui[1] - k[1] * ui[0]};
    for (int c = 0; c < 3; ++c) {
      const R Ur = sk * ur[c], Ui = sk * ui[c];
      const R Wr = -hjk * kui[c], Wi = hjk * kur[c];
      T y;
      y.x = Ur - Wi;
      y.y = Ui + Wr;
      O[o + 2 * c * S] = y;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < N; t += blockDim.x) tw[t].y = -tw[t].y;
  __syncthreads();
  const T* Y = stockham_lm_any<T, R>(O, X, tw, N, S, NL, plan, +1);
  for (int t = threadIdx.x; t < NL * N; t += blockDim.x) {
    int line, x;
    dn.divmod(t, line, x);
    const int g = line / 6, c = (line % 6) >> 1, q = line & 1;
    const int row = rows[2 * g + q].w;
    if (row < 0) continue;
    const T y = Y[line * S + x];
    stg2(grid, unsigned(c * cs) + 2 * unsigned(row * N + x), y.x, y.y);
  }
}

template <typename R, bool TABLE>
__global__ __launch_bounds__(256) void k_fft_xgreen(R* __restrict__ grid, size_t cs, FftPlan plan,
                                                    const R* __restrict__ twiddle, WaveParams wp, int G,
                                                    const int* __restrict__ skip) {
  fft_xgreen_body<R, TABLE>(grid, cs, plan, twiddle, wp, G, skip, blockIdx.x, blockIdx.y, gridDim.x);
}

// row slots per workgroup of the x+Green pass (measured: 2 is fastest at 64^3 and 128^3)
int fft_green_rows(int N) { return N >= 256 ? 1 : N >= 64 ? 2 : 256 / N; }

bool tile_b_fits(int N, int B, int rbytes) {
  return B >= 1 && (B & (B - 1)) == 0 && N % B == 0 &&
         size_t(2 * rbytes) * (2 * size_t(B) * fft_line_stride(N, B, 2 * rbytes) + N) <= (size_t(64) << 10);
}

bool tile_g_fits(int N, int G, int rbytes) {
  return G >= 1 && G <= 16 && xgreen_shm(N, G, 2 * rbytes) <= (size_t(64) << 10);
}

// lines per workgroup of the coalesced y/z passes: largest B in {16, 8, 4, 2, 1} dividing N
// whose two LDS buffers and twiddles fit in 64 KB
int fft_lines_b(int N, int rbytes) {
  for (int B = 16; B > 1; B /= 2)
    if (tile_b_fits(N, B, rbytes)) return B;
  return 1;
}

int lines_b_of(const WaveParams& wp, int rbytes) {
  return wp.tile_b > 0 && tile_b_fits(wp.n, wp.tile_b, rbytes) ? wp.tile_b : fft_lines_b(wp.n, rbytes);
}

int green_g_of(const WaveParams& wp) {
  return wp.tile_g > 0 && tile_g_fits(wp.n, wp.tile_g, 8) ? wp.tile_g : fft_green_rows(wp.n);
}

template <typename R>
void launch_wave_fft(R* grid, const FftPlan& plan, const R* twiddle, const WaveParams& wp, int stage,
                     hipStream_t st, const int* skip) {
  using T = typename C2<R>::T;
  const int N = plan.n;
  const size_t cs = 2 * size_t(N) * N * N;
  if (stage == 2) {
    const int G = green_g_of(wp);
    const size_t shm = xgreen_shm(N, G, int(sizeof(T)));
    const int nblk = (N * N / 2 + 2 + G - 1) / G;
    if (wp.gtab && !wp.gam)  // the cube: tabulated multipliers
      launch_k(k_fft_xgreen<R, true>, nblk, kThreads, shm, st, grid, cs, plan, twiddle, wp, G, skip);
    else
      launch_k(k_fft_xgreen<R, false>, nblk, kThreads, shm, st, grid, cs, plan, twiddle, wp, G, skip);
  } else {
    const int B = lines_b_of(wp, sizeof(R));
    const size_t shm = sizeof(T) * (2 * size_t(B) * fft_line_stride(N, B, int(sizeof(T))) + N);
    dim3 g(N * N / B, 3);
    const int sign = stage < 2 ? -1 : +1;
    if (stage == 0 || stage == 4)
      launch_k(k_fft_lines<R, 2>, g, kThreads, shm, st, grid, cs, plan, twiddle, sign, B, skip);
    else
      launch_k(k_fft_lines<R, 1>, g, kThreads, shm, st, grid, cs, plan, twiddle, sign, B, skip);
  }
}

// ------------------------------------------------------------------------------------------
// multi-system launches: block -> (system, local block) by the prefix table, then the
// single-system body with that system's pointers (the Arnoldi step maps z -> w)
// ------------------------------------------------------------------------------------------

namespace {
__device__ inline int batch_sys(const int* __restrict__ off, int nsys, int b) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <typename R>
__device__ inline const R* pick(const double* a, const float* b);
template <>
__device__ inline const double* pick<double>(const double* a, const float*) {
  return a;
}
template <>
__device__ inline const float* pick<float>(const double*, const float* b) {
  return b;
}

constexpr int kBatchLpr = 16;  // lanes per bead row of the batched real-space sum
}  // namespace

template <typename R>
__global__ __launch_bounds__(256) void kb_real(const BatchDesc* __restrict__ D, const int* __restrict__ off,
                                              int nsys) {
  const int s = batch_sys(off, nsys, blockIdx.x);
  const BatchDesc& d = D[s];
  real_sum_body<R, kBatchLpr>(d.nb, (const double4*)d.pos4, d.z, d.nrow, d.ncol, pick<R>(d.tab64, d.tab32), d.rp,
                              d.w, 0, d.perm, &d.ctl->stop, blockIdx.x - off[s], 0, 0);
}

template <typename R>
__global__ __launch_bounds__(256) void kb_spread(const BatchDesc* __restrict__ D, const int* __restrict__ off,
                                                int nsys) {
  const int s = batch_sys(off, nsys, blockIdx.x);
  const BatchDesc& d = D[s];
  const size_t cs = 2 * size_t(d.wp.n) * d.wp.n * d.wp.n;
  spread_split_body<R>(d.blk_start, d.blk_end, d.cand, d.perm, d.starts, pick<R>(d.w64, d.w32), d.z, d.wp, d.nbin,
                       d.C, static_cast<R*>(d.grid), cs, &d.ctl->stop, blockIdx.x - off[s], 0, 0);
}

template <typename R, int STAGE>
__global__ __launch_bounds__(256) void kb_fft(const BatchDesc* __restrict__ D, const int* __restrict__ off,
                                             int nsys) {
  const int s = batch_sys(off, nsys, blockIdx.x);
  const BatchDesc& d = D[s];
  const int lb = blockIdx.x - off[s];
  const int N = d.plan.n;
  const size_t cs = 2 * size_t(N) * N * N;
  R* grid = static_cast<R*>(d.grid);
  const R* tw = pick<R>(d.tw64, d.tw32);
  const int* stop = &d.ctl->stop;
  if (STAGE == 2) {  // multi-system launches hold cubic systems only (fusable)
    fft_xgreen_body<R, true>(grid, cs, d.plan, tw, d.wp, d.bg, stop, lb, 0, 0);
  } else {
    const int gx = N * N / d.bl;
    if (STAGE == 0 || STAGE == 4)
      fft_lines_body<R, 2>(grid, cs, d.plan, tw, STAGE == 0 ? -1 : +1, d.bl, stop, lb % gx, lb / gx, gx);
    else
      fft_lines_body<R, 1>(grid, cs, d.plan, tw, STAGE == 1 ? -1 : +1, d.bl, stop, lb % gx, lb / gx, gx);
  }
}

template <typename R>
__global__ __launch_bounds__(256) void kb_interp(const BatchDesc* __restrict__ D, const int* __restrict__ off,
                                                int nsys) {
  const int s = batch_sys(off, nsys, blockIdx.x);
  const BatchDesc& d = D[s];
  const size_t cs = 2 * size_t(d.wp.n) * d.wp.n * d.wp.n;
  interp_body<R>(d.nb, (const double4*)d.pos4, static_cast<const R*>(d.grid), cs, d.wp, d.w, &d.ctl->stop, d.body,
                 (const double4*)d.r4, d.z + 6 * size_t(d.nb), d.perm, d.starts, pick<R>(d.w64, d.w32),
                 blockIdx.x - off[s], 0, 0);
}

// spreading fields of a batch descriptor (bin_start == nullptr: no gather plan)
void spread_plan_desc(const SpreadPlan* sp, int prec, BatchDesc& d) {
  if (!sp || sp->BS != 8) {
    d.blk_start = d.blk_end = d.cand = nullptr;
    d.bin_start = d.bin_end = d.perm = nullptr;
    d.starts = nullptr;
    d.w64 = nullptr;
    d.w32 = nullptr;
    d.nbin = d.K = d.C = 0;
    return;
  }
  d.bin_start = sp->bin_start;
  d.bin_end = sp->bin_end;
  d.blk_start = sp->blk_start;
  d.blk_end = sp->blk_end;
  d.cand = sp->cand;
  d.perm = sp->perm;
  d.starts = sp->starts;
  d.w64 = sp->weights;
  d.w32 = sp->weights32;
  d.nbin = sp->nbin;
  d.K = sp->K;
  const size_t rb = prec ? sizeof(float) : sizeof(double);
  const size_t per = rb * (3 * size_t(d.wp.support) + 6) + sizeof(int4) + sizeof(int);
  d.C = int(std::min<size_t>(128, (size_t(60) << 10) / per)) & ~3;  // as launch_spread_gather
}

int batch_blocks(const BatchDesc& d, int kind) {
  const int N = d.plan.n;
  switch (kind) {
    case BK_PRECOND:
    case BK_AGG:
      return (d.na + 3) / 4;
    case BK_REAL:
      return int((size_t(d.nb) * kBatchLpr + kThreads - 1) / kThreads);
    case BK_SPREAD:
      return d.bin_start ? d.nbin * d.nbin * d.nbin : 0;
    case BK_FFT_OUTER:
    case BK_FFT_MID:
      return N * N / d.bl * 3;
    case BK_FFT_GREEN:
      return (N * N / 2 + 2 + d.bg - 1) / d.bg;
    case BK_INTERP:
      return (d.nb + 3) / 4;
    case BK_CGS:
      return d.ncgs;
    default:
      return 0;
  }
}

size_t batch_shm(const BatchDesc& d, int kind, int prec) {
  const size_t rb = prec ? sizeof(float) : sizeof(double), tb = 2 * rb;
  const size_t N = d.plan.n;
  switch (kind) {
    case BK_SPREAD:
      return std::max((rb * (3 * size_t(d.wp.support) + 6) + sizeof(int4) + sizeof(int)) * d.C,
                      size_t(kSplitRedBytes64) / sizeof(double) * rb);
    case BK_FFT_OUTER:
    case BK_FFT_MID:
      return tb * (2 * size_t(d.bl) * fft_line_stride(int(N), d.bl, int(tb)) + N);
    case BK_FFT_GREEN:
      return xgreen_shm(int(N), d.bg, int(tb));
    default:
      return 0;
  }
}

namespace {
template <typename R>
void batch_mobility(int kind, int stage, const BatchDesc* D, const int* off, int nsys, int total, size_t shm,
                    hipStream_t st) {
  switch (kind) {
    case BK_REAL:
      kb_real<R><<<total, kThreads, 0, st>>>(D, off, nsys);
      break;
    case BK_SPREAD:
      kb_spread<R><<<total, 256, shm, st>>>(D, off, nsys);
      break;
    case BK_FFT_OUTER:
      if (stage == 0)
        kb_fft<R, 0><<<total, kThreads, shm, st>>>(D, off, nsys);
      else
        kb_fft<R, 4><<<total, kThreads, shm, st>>>(D, off, nsys);
      break;
    case BK_FFT_MID:
      if (stage == 1)
        kb_fft<R, 1><<<total, kThreads, shm, st>>>(D, off, nsys);
      else
        kb_fft<R, 3><<<total, kThreads, shm, st>>>(D, off, nsys);
      break;
    case BK_FFT_GREEN:
      kb_fft<R, 2><<<total, kThreads, shm, st>>>(D, off, nsys);
      break;
    case BK_INTERP:
      kb_interp<R><<<total, kThreads, 0, st>>>(D, off, nsys);
      break;
    default:
      break;
  }
}
}  // namespace

void launch_batch_mobility(int kind, int prec, int stage, const BatchDesc* D, const int* off, int nsys, int total,
                           size_t shm, hipStream_t st) {
  if (total <= 0) return;
  if (prec)
    batch_mobility<float>(kind, stage, D, off, nsys, total, shm, st);
  else
    batch_mobility<double>(kind, stage, D, off, nsys, total, shm, st);
}

template void launch_wave_fft<double>(double*, const FftPlan&, const double*, const WaveParams&, int, hipStream_t,
                                      const int*);
template void launch_wave_fft<float>(float*, const FftPlan&, const float*, const WaveParams&, int, hipStream_t,
                                     const int*);
template void launch_spread_gather<double>(const SpreadPlan*, const double*, const WaveParams&, double*, hipStream_t, const int*);
template void launch_spread_gather<float>(const SpreadPlan*, const double*, const WaveParams&, float*, hipStream_t, const int*);
template void launch_spread_fused<double>(const SpreadPlan*, const double*, const WaveParams&, double*, const double*,
                                          int, const RealArgs&, const RigidArgs&, hipStream_t, const int*);
template void launch_spread_fused<float>(const SpreadPlan*, const double*, const WaveParams&, float*, const float*, int,
                                         const RealArgs&, const RigidArgs&, hipStream_t, const int*);
template void launch_real_sum<double>(int, const double*, const double*, const int*, const uint32_t*, const double*,
                                      const RealParams&, double*, bool, int, hipStream_t, const int*, const int*);
template void launch_real_sum<float>(int, const double*, const double*, const int*, const uint32_t*, const float*,
                                     const RealParams&, double*, bool, int, hipStream_t, const int*, const int*);
template void launch_spread<double>(int, const double*, const double*, const WaveParams&, double*, hipStream_t, const int*);
template void launch_spread<float>(int, const double*, const double*, const WaveParams&, float*, hipStream_t, const int*);
template void launch_interp<double>(int, const double*, const double*, const WaveParams&, double*, hipStream_t, const int*,
                                    const int*, const double*, const double*, const SpreadPlan*);
template void launch_interp<float>(int, const double*, const float*, const WaveParams&, double*, hipStream_t, const int*,
                                   const int*, const double*, const double*, const SpreadPlan*);
template void launch_spread_sheared<double>(int, const double*, const double*, const WaveParams&, double*, hipStream_t,
                                            const int*);
template void launch_spread_sheared<float>(int, const double*, const double*, const WaveParams&, float*, hipStream_t,
                                           const int*);
template void launch_interp_sheared<double>(int, const double*, const double*, const WaveParams&, double*, hipStream_t,
                                            const int*, const int*, const double*, const double*);
template void launch_interp_sheared<float>(int, const double*, const float*, const WaveParams&, double*, hipStream_t,
                                           const int*, const int*, const double*, const double*);
// ------------------------------------------------------------------------------------------
// the allocation-free transform (fsd_fft3d_noalloc): its twiddle table lives in file-scope
// device memory, one copy per GPU held until the process ends, sized for the largest n
// ------------------------------------------------------------------------------------------

static __device__ __align__(256) double scratch[2 * kNoAllocFftMax];

// exp(-2 pi i t / n) for t < n, interleaved (re, im)
__global__ void k_twiddles(int n, double* __restrict__ tw) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double sv, cv;
  sincospi(2.0 * double(t) / double(n), &sv, &cv);
  tw[2 * t] = cv;
  tw[2 * t + 1] = -sv;
}

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {nullptr};
}  // namespace

// the device address of this GPU's copy of `scratch`, looked up once per device
hipError_t noalloc_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_fft3d_noalloc(int n, int sign, double* data, const FftPlan& plan, hipStream_t st) {
  double* tw = nullptr;
  hipError_t e = noalloc_scratch(&tw);
  if (e != hipSuccess) return e;
  k_twiddles<<<(n + 255) / 256, 256, 0, st>>>(n, tw);
  launch_fft3d<double>(data, 1, 2 * size_t(n) * n * n, plan, tw, sign, st);
  return hipGetLastError();
}

template void launch_fft3d<double>(double*, int, size_t, const FftPlan&, const double*, int, hipStream_t, int, const int*);
template void launch_fft3d<float>(float*, int, size_t, const FftPlan&, const float*, int, hipStream_t, int, const int*);

}  // namespace fsd
