// Device bodies shared by the solver kernels and the fused first pass of the mobility
// kernels (included by both translation units).
#pragma once
#include "fsd_impl.hpp"

namespace fsd {

// sum over the 64 lanes of a wavefront
__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// y2_j = Sigma_j (lambda + f_lub) with f_lub,i = -sum_k R_ik (u_i - u_k) and u the rigid
// translational velocities of V (neighbour velocities rebuilt from V and body vectors)
__device__ __forceinline__ void agg_lub_body(int na, const int* __restrict__ offsets, const int* __restrict__ body,
                                                 const double4* __restrict__ r4, const double* __restrict__ lam,
                                                 const double* __restrict__ V, const int* __restrict__ lrow,
                                                 const uint32_t* __restrict__ lcol, const double* __restrict__ coef,
                                                 double* __restrict__ y2, const int* __restrict__ skip, int bx_, int by_, int gx_) {
  if (skip && *skip) return;
  const int j = bx_ * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (j >= na) return;
  double F0 = 0, F1 = 0, F2 = 0, T0 = 0, T1 = 0, T2 = 0;
  for (int i = offsets[j] + lane; i < offsets[j + 1]; i += 64) {
    const double* l = lam + 6 * size_t(i);
    double fx = l[0], fy = l[1], fz = l[2];
    const double4 r = r4[i];
    if (lrow) {
      const double* v = V + 6 * j;
      const double ux = v[0] + (v[4] * r.z - v[5] * r.y);
      const double uy = v[1] + (v[5] * r.x - v[3] * r.z);
      const double uz = v[2] + (v[3] * r.y - v[4] * r.x);
      for (int e = lrow[i]; e < lrow[i + 1]; ++e) {
        const int k = int(lcol[e] & 0x3FFFFFu);
        const double* vk = V + 6 * body[k];
        const double4 rk = r4[k];
        const double dx = ux - (vk[0] + (vk[4] * rk.z - vk[5] * rk.y));
        const double dy = uy - (vk[1] + (vk[5] * rk.x - vk[3] * rk.z));
        const double dz = uz - (vk[2] + (vk[3] * rk.y - vk[4] * rk.x));
        const double* c = coef + 5 * size_t(e);
        const double nd = c[2] * dx + c[3] * dy + c[4] * dz;
        const double g = (c[0] - c[1]) * nd;
        fx -= c[1] * dx + g * c[2];
        fy -= c[1] * dy + g * c[3];
        fz -= c[1] * dz + g * c[4];
      }
    }
    F0 += fx;
    F1 += fy;
    F2 += fz;
    T0 += l[3] + (r.y * fz - r.z * fy);
    T1 += l[4] + (r.z * fx - r.x * fz);
    T2 += l[5] + (r.x * fy - r.y * fx);
  }
  F0 = wsum(F0);
  F1 = wsum(F1);
  F2 = wsum(F2);
  T0 = wsum(T0);
  T1 = wsum(T1);
  T2 = wsum(T2);
  if (lane == 0) {
    double* y = y2 + 6 * size_t(j);
    y[0] = F0;
    y[1] = F1;
    y[2] = F2;
    y[3] = T0;
    y[4] = T1;
    y[5] = T2;
  }
}

}  // namespace fsd
