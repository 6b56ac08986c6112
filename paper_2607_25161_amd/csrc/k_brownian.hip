// Brownian terms of Eq. `SP2` (Algorithm 1 step 3): counter-based Gaussian noise,
// the wave-space noise grid, and the vector kernels of the Lanczos square roots.
//
// Noise comes from Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC 2011): a 256-bit counter is enciphered under a
// 128-bit key by ten rounds of two 64x64 -> 128-bit multiplications, with the key
// bumped by the Weyl constants between rounds.  Uniforms take the top 53 bits,
// shifted to the open interval (0, 1); Box-Muller turns each pair into two normals.
#include "fsd_impl.hpp"

namespace fsd {

namespace {
constexpr int kThreads = 256;
inline int nblocks(long long n, int t = kThreads) { return int((n + t - 1) / t); }

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;  // golden ratio
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;  // sqrt(3) - 1

__device__ inline void philox_round(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
  const uint64_t lo0 = kPhiloxM0 * c[0], hi0 = __umul64hi(kPhiloxM0, c[0]);
  const uint64_t lo1 = kPhiloxM1 * c[2], hi1 = __umul64hi(kPhiloxM1, c[2]);
  const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}
}  // namespace

__device__ void philox4x64_10(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    philox_round(c, k0, k1);
  }
}

namespace {
__device__ inline double unit_open(uint64_t x) { return (double(x >> 11) + 0.5) * 0x1.0p-53; }

// four normals of block b of stream (key, purpose, step): counter (b + 1, purpose, step, 0)
__device__ inline void normals4(const NoiseKey& nk, uint64_t b, double (&z)[4]) {
  uint64_t c[4] = {b + 1, nk.purpose, nk.step, 0};
  philox4x64_10(c, nk.k0, nk.k1);
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const double u1 = unit_open(c[2 * p]), u2 = unit_open(c[2 * p + 1]);
    const double r = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    z[2 * p] = r * cs;
    z[2 * p + 1] = r * sn;
  }
}
}  // namespace

__global__ void k_philox_raw(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, int nblk,
                             uint64_t* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblk) return;
  uint64_t c[4] = {c0 + uint64_t(b), c1, c2, c3};
  philox4x64_10(c, k0, k1);
  for (int q = 0; q < 4; ++q) out[4 * size_t(b) + q] = c[q];
}

void launch_philox_raw(uint64_t k0, uint64_t k1, const uint64_t ctr[4], int nblk, uint64_t* out, hipStream_t st) {
  k_philox_raw<<<nblocks(nblk), kThreads, 0, st>>>(k0, k1, ctr[0], ctr[1], ctr[2], ctr[3], nblk, out);
}

// out[e] = normal e of the stream, e < n
__global__ void k_normals(size_t n, NoiseKey nk, double* __restrict__ out) {
  const size_t b = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (4 * b >= n) return;
  double z[4];
  normals4(nk, b, z);
  for (int q = 0; q < 4; ++q)
    if (4 * b + q < n) out[4 * b + q] = z[q];
}

void launch_normals(size_t n, const NoiseKey& nk, double* out, hipStream_t st) {
  k_normals<<<nblocks((long long)((n + 3) / 4)), kThreads, 0, st>>>(n, nk, out);
}

// Real white noise on the grid for the wave-space square root: component c of grid
// point m is normal c N^3 + m of the stream (or src[c N^3 + m] when src != nullptr);
// it fills the real part of complex grid c (the imaginary parts, the torque slots of
// the packed transform, are zero).
__global__ void k_noise_grid(size_t n3, NoiseKey nk, const double* __restrict__ src, double* __restrict__ grid,
                             size_t cs) {
  const size_t b = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t total = 3 * n3;
  if (4 * b >= total) return;
  double z[4];
  if (src) {
    for (int q = 0; q < 4; ++q) z[q] = 4 * b + q < total ? src[4 * b + q] : 0.0;
  } else {
    normals4(nk, b, z);
  }
  for (int q = 0; q < 4; ++q) {
    const size_t e = 4 * b + q;
    if (e >= total) break;
    const size_t c = e / n3, m = e % n3;
    grid[c * cs + 2 * m] = z[q];
    grid[c * cs + 2 * m + 1] = 0.0;
  }
}

void launch_noise_grid(int N, const NoiseKey& nk, const double* src, double* grid, hipStream_t st) {
  const size_t n3 = size_t(N) * N * N;
  const size_t cs = 2 * n3;
  k_noise_grid<<<nblocks((long long)((3 * n3 + 3) / 4)), kThreads, 0, st>>>(n3, nk, src, grid, cs);
}

// y = a x
__global__ void k_scale(size_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

void launch_scale(size_t n, double a, const double* x, double* y, hipStream_t st) {
  k_scale<<<nblocks((long long)n), kThreads, 0, st>>>(n, a, x, y);
}

// out = sum_q c[q] V_q (q < k), c on the device
__global__ void k_combine(size_t n, int k, const double* __restrict__ V, size_t ldv, const double* __restrict__ c,
                          double* __restrict__ out) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int q = 0; q < k; ++q) s += c[q] * V[size_t(q) * ldv + i];
  out[i] = s;
}

void launch_combine(size_t n, int k, const double* V, size_t ldv, const double* c, double* out, hipStream_t st) {
  k_combine<<<nblocks((long long)n), kThreads, 0, st>>>(n, k, V, ldv, c, out);
}

// translational parts of 6-per-bead vectors: t[3 i + a] = v[6 i + a]; and back (rotations 0)
__global__ void k_take_trans(int nb, const double* __restrict__ v6, double* __restrict__ t3) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  for (int a = 0; a < 3; ++a) t3[3 * i + a] = v6[6 * i + a];
}

void launch_take_trans(int nb, const double* v6, double* t3, hipStream_t st) {
  k_take_trans<<<nblocks(nb), kThreads, 0, st>>>(nb, v6, t3);
}

}  // namespace fsd
