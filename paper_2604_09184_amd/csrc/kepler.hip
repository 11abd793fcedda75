// H_A drift (eq. Ha, Kepler part) and H_C jump (eq. Hc).
//
// The drift advances each body on its two-body orbit about mu = G m0 with the f and g functions
// in universal variables (Stumpff functions c_k), solved with the Laguerre-Conway iteration; one
// body per lane, binary64 throughout. The jump shifts every position by h * P / m0; P is reduced
// deterministically from per-64-body partial sums by every workgroup in the same order.
#include "internal.hpp"
#include "kepler_core.hpp"

namespace nbk {
using namespace nbd;

// One wave per workgroup: the per-body Kepler solve is long and latency-bound, so small n still
// spreads over every compute unit. Momentum partials: one per 64 bodies (a wave butterfly).
__global__ __launch_bounds__(64) void k_momentum(const double4 *__restrict__ xm,
                                                 const double4 *__restrict__ v, int n,
                                                 double4 *__restrict__ mom) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  double P[3] = {0.0, 0.0, 0.0};
  if (i < n) {
    const double m = xm[i].w;
    const double4 q = v[i];
    P[0] = m * q.x; P[1] = m * q.y; P[2] = m * q.z;
  }
  wave_sum<3>(P);
  if (threadIdx.x == 0) mom[blockIdx.x] = make_double4(P[0], P[1], P[2], 0.0);
}

// x_rec (may be null) receives a copy of the new positions.
__global__ __launch_bounds__(64) void k_jump(double4 *__restrict__ xm,
                                             const double4 *__restrict__ mom, int nb, int n,
                                             double h, double m0, double4 *__restrict__ x_rec) {
  double P[3];
  partials_total_wave(mom, nb, P);
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  const double sx = h * (P[0] / m0), sy = h * (P[1] / m0), sz = h * (P[2] / m0);
  double4 p = xm[i];
  p.x = p.x + sx; p.y = p.y + sy; p.z = p.z + sz;
  xm[i] = p;
  if (x_rec) x_rec[i] = p;
}

// Momentum and jump of up to kJumpSmall bodies in one workgroup (16 waves): the per-64-body
// partials of k_momentum (the same wave butterfly) into LDS, then every wave sums them as k_jump
// does, so the positions come out bit for bit as from the two launches.
__global__ __launch_bounds__(1024) void k_momentum_jump_small(double4 *__restrict__ xm,
                                                              const double4 *__restrict__ v, int n,
                                                              double h, double m0) {
  __shared__ double4 mom[kJumpSmall / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int nb = (n + 63) / 64;
  // block b = w + 16 u holds body t + 1024 u: the positions read for the momentum are the ones
  // this thread jumps, kept in registers
  constexpr int kPer = kJumpSmall / 1024;
  double4 pos[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int b = w + 16 * u;
    if (b >= nb) break;
    const int i = b * 64 + lane;
    double P[3] = {0.0, 0.0, 0.0};
    if (i < n) {
      pos[u] = xm[i];
      const double m = pos[u].w;
      const double4 q = v[i];
      P[0] = m * q.x; P[1] = m * q.y; P[2] = m * q.z;
    }
    wave_sum<3>(P);
    if (lane == 0) mom[b] = make_double4(P[0], P[1], P[2], 0.0);
  }
  __syncthreads();
  double P[3];
  partials_total_wave(mom, nb, P);
  const double sx = h * (P[0] / m0), sy = h * (P[1] / m0), sz = h * (P[2] / m0);
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = t + 1024 * u;
    if (i >= n) break;
    double4 p = pos[u];
    p.x = p.x + sx; p.y = p.y + sy; p.z = p.z + sz;
    xm[i] = p;
  }
}

// x_rec / v_rec (may be null) receive the positions after the jump (before the drift) and the
// velocities after the drift. skip (may be null): bodies with skip[i] != 0 get the jump but not
// the Kepler drift (their drift is the close-encounter integration).
__global__ __launch_bounds__(64) void k_jump_drift(double4 *__restrict__ xm,
                                                   double4 *__restrict__ v,
                                                   const double4 *__restrict__ mom_in, int nb,
                                                   int n, double hjump, double dt, double m0,
                                                   double mu, uint32_t *__restrict__ status,
                                                   double4 *__restrict__ mom_out,
                                                   double4 *__restrict__ x_rec,
                                                   double4 *__restrict__ v_rec,
                                                   const int *__restrict__ skip) {
  double P[3];
  partials_total_wave(mom_in, nb, P);
  const int i = blockIdx.x * 64 + threadIdx.x;
  double Q[3] = {0.0, 0.0, 0.0};
  if (i < n) {
    const double sx = hjump * (P[0] / m0), sy = hjump * (P[1] / m0), sz = hjump * (P[2] / m0);
    double4 p = xm[i];
    double4 q = v[i];
    p.x = p.x + sx; p.y = p.y + sy; p.z = p.z + sz;
    if (x_rec) x_rec[i] = p;
    const int st = (skip && skip[i]) ? 0 : kepler_advance(p.x, p.y, p.z, q.x, q.y, q.z, mu, dt);
    xm[i] = p;
    v[i] = q;
    if (v_rec) v_rec[i] = q;
    if (status) status[i] |= (uint32_t)st;
    Q[0] = p.w * q.x; Q[1] = p.w * q.y; Q[2] = p.w * q.z;
  }
  wave_sum<3>(Q);
  if (threadIdx.x == 0) mom_out[blockIdx.x] = make_double4(Q[0], Q[1], Q[2], 0.0);
}

// skip (may be null): bodies with skip[i] != 0 are left alone.
__global__ __launch_bounds__(64) void k_drift(double4 *__restrict__ xm, double4 *__restrict__ v,
                                              int n, double dt, double mu,
                                              uint32_t *__restrict__ status,
                                              const int *__restrict__ skip) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= n || (skip && skip[i])) return;
  double4 p = xm[i];
  double4 q = v[i];
  const int st = kepler_advance(p.x, p.y, p.z, q.x, q.y, q.z, mu, dt);
  xm[i] = p;
  v[i] = q;
  if (status) status[i] = (uint32_t)st;
}

hipError_t launch_momentum(const double4 *xm, const double4 *v, int n, double4 *mom, hipStream_t st) {
  hipLaunchKernelGGL(k_momentum, dim3(fin_blocks(n)), dim3(64), 0, st, xm, v, n, mom);
  return hipGetLastError();
}

hipError_t launch_momentum_jump_small(double4 *xm, const double4 *v, int n, double h, double m0,
                                     hipStream_t st) {
  hipLaunchKernelGGL(k_momentum_jump_small, dim3(1), dim3(1024), 0, st, xm, v, n, h, m0);
  return hipGetLastError();
}

hipError_t launch_jump(double4 *xm, const double4 *mom, int nb, int n, double h, double m0,
                       hipStream_t st, double4 *x_rec) {
  hipLaunchKernelGGL(k_jump, dim3(fin_blocks(n)), dim3(64), 0, st, xm, mom, nb, n, h, m0, x_rec);
  return hipGetLastError();
}

hipError_t launch_jump_drift(double4 *xm, double4 *v, const double4 *mom_in, int nb, int n,
                             double hjump, double dt, double m0, double mu, uint32_t *status,
                             double4 *mom_out, hipStream_t st, double4 *x_rec, double4 *v_rec,
                             const int *skip) {
  hipLaunchKernelGGL(k_jump_drift, dim3(fin_blocks(n)), dim3(64), 0, st, xm, v, mom_in, nb, n,
                     hjump, dt, m0, mu, status, mom_out, x_rec, v_rec, skip);
  return hipGetLastError();
}

hipError_t launch_drift(double4 *xm, double4 *v, int n, double dt, double mu, uint32_t *status,
                        hipStream_t st, const int *skip) {
  hipLaunchKernelGGL(k_drift, dim3(fin_blocks(n)), dim3(64), 0, st, xm, v, n, dt, mu, status, skip);
  return hipGetLastError();
}

}  // namespace nbk
