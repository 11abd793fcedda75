// Device helpers shared by the kernels of this library: threshold words, the exact close-encounter
// predicate, the changeover weight, r^-3 and deterministic block reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace nbk {
constexpr int kBlock = 256;   // threads per workgroup of the body-parallel kernels (4 wave64)
}  // namespace nbk

// ------------------------------------------------------------------ device helpers
namespace nbd {

__device__ __forceinline__ uint32_t hiword(double x) {
  return (uint32_t)((unsigned long long)__double_as_longlong(x) >> 32);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    uint32_t w = (uint32_t)__shfl_xor((int)v, o, 64);
    v = v > w ? v : w;
  }
  return v;
}

// Critical radius and thresholds of one body (the library's definition, see nbody.h):
// {rc, H, V, T}, T bounding every r^2 that H or V can flag.
__device__ __forceinline__ double4 body_thresholds(double4 p, double4 q, double m0, double cH,
                                                   double cV, double n1, double n2dt) {
  const double r2 = fma(p.z, p.z, fma(p.y, p.y, p.x * p.x));
  const double mu = p.w / m0;
  const double vv = fma(q.z, q.z, fma(q.y, q.y, q.x * q.x));
  const double H = (cH * ((r2 * r2) * r2)) * (mu * mu);
  const double V = cV * vv;
  const double rhill = sqrt(r2) * cbrt(mu / 3.0);
  const double a = n1 * rhill, b = n2dt * sqrt(vv);
  const double rc = a > b ? a : b;
  const double c = cbrt(H);
  const double T = (V > c ? V : c) * (1.0 + 0x1p-30);
  return make_double4(rc, H, V, T);
}

// Exact binary64 close-encounter predicate (the library's definition, see nbody.h).
__device__ __forceinline__ bool close_exact(double r2, double Hi, double Hj, double Vi, double Vj) {
  const double H = Hi > Hj ? Hi : Hj;
  const double V = Vi > Vj ? Vi : Vj;
  return ((r2 * r2) * r2 < H) || (r2 < V);
}

// Pair weight for a close pair: w = K/r^3 - K'(r)/r^2 with the changeover
// K(y) = y^2/(2y^2-2y+1), y = clamp((r - f_in rc)/((1-f_in) rc), 0, 1).
__device__ __forceinline__ double close_weight(double r2, double rcij, double f_in) {
  const double r = sqrt(r2);
  const double r3 = r2 * r;
  const double span = (1.0 - f_in) * rcij;
  double y = (r - f_in * rcij) / span;
  if (y <= 0.0) return 0.0;
  if (y >= 1.0) return 1.0 / r3;
  const double D = 2.0 * y * y - 2.0 * y + 1.0;
  const double K = y * y / D;
  const double dKdy = 2.0 * y * (1.0 - y) / (D * D);
  return K / r3 - (dKdy / span) / r2;
}

// As close_weight for a pair inside the changeover span (y < 1): stores w and returns true. At
// y >= 1 the pair has the far weight 1/r^3 and the function returns false, so that the caller
// keeps its own far-pair value: a pair flagged only by thresholds widened beyond rc (the list
// margin of the changeover levels) then gets exactly the bits of an unflagged pair.
__device__ __forceinline__ bool close_weight_inner(double r2, double rcij, double f_in, double &w) {
  const double r = sqrt(r2);
  const double span = (1.0 - f_in) * rcij;
  const double y = (r - f_in * rcij) / span;
  if (y >= 1.0) return false;
  if (y <= 0.0) {
    w = 0.0;
    return true;
  }
  const double r3 = r2 * r;
  const double D = 2.0 * y * y - 2.0 * y + 1.0;
  const double K = y * y / D;
  const double dKdy = 2.0 * y * (1.0 - y) / (D * D);
  w = K / r3 - (dKdy / span) / r2;
  return true;
}

// m * r^-3 from the hardware reciprocal-square-root seed y and the first-order correction of
// (1 - e)^(-3/2) = 1 + 1.5 e + 1.875 e^2 + ..., e = 1 - r2 y^2. The terms left out make the result
// smaller than m r^-3 by 1.875 e^2 (1 + O(e)) relative: at most 1.1e-13 for a seed within the
// documented 2^-23 of r^-1, and 2.1e-14 for the largest |e| = 1.06e-7 measured on gfx950 over
// 4.3e9 arguments; rounding adds a few ulp. c15 = 1.5 arrives as a kernel argument and is kept in
// a loop-invariant register (no literal operands in 64-bit VOP3 on gfx9).
__device__ __forceinline__ double m_rinv3(double r2, double m, double c15) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double t = y * y;
  const double e = fma(-r2, t, 1.0);
  const double my3 = (m * y) * t;
  return fma(my3 * e, c15, my3);
}

// r^-3 alone (equal-mass systems multiply by m once after the sum).
__device__ __forceinline__ double rinv3(double r2, double c15) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double t = y * y;
  const double e = fma(-r2, t, 1.0);
  const double y3 = y * t;
  return fma(y3 * e, c15, y3);
}

// Split precision: r^-3 in binary32 (offsets and r^2 stay binary64), scaled by m in binary64.
__device__ __forceinline__ double m_rinv3_split(double r2, double m) {
  const float f = (float)r2;
  const float y = __builtin_amdgcn_rsqf(f);
  const float y3 = (y * y) * y;
  return m * (double)y3;
}


// Deterministic workgroup sum of NV doubles per thread (fixed tree order); every thread gets the
// totals. lds must hold NV * kBlock doubles.
template <int NV>
__device__ __forceinline__ void block_sum(double (&x)[NV], double *lds) {
  constexpr int B = nbk::kBlock;
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < NV; ++k) lds[k * B + t] = x[k];
  __syncthreads();
  for (int s = B / 2; s > 0; s >>= 1) {
    if (t < s) {
#pragma unroll
      for (int k = 0; k < NV; ++k) lds[k * B + t] += lds[k * B + t + s];
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) x[k] = lds[k * B];
  __syncthreads();
}

// Wave minimum / maximum of a double, returned as a wave-uniform (scalar register) value.
__device__ __forceinline__ double uniform_f64(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double wave_min_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return uniform_f64(v);
}

__device__ __forceinline__ double wave_max_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return uniform_f64(v);
}

// Sum over the 64 lanes of a wave by butterfly: every lane ends with the same bits.
template <int NV>
__device__ __forceinline__ void wave_sum(double (&x)[NV]) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int k = 0; k < NV; ++k) x[k] += __shfl_xor(x[k], o, 64);
}

// Total of nb momentum partials, read by a one-wave workgroup: lane l sums partials l, l+64, ...
// in order, then the wave butterfly; the same bits in every workgroup.
__device__ __forceinline__ void partials_total_wave(const double4 *__restrict__ mom, int nb,
                                                    double (&P)[3]) {
  P[0] = P[1] = P[2] = 0.0;
  for (int b = threadIdx.x & 63; b < nb; b += 64) {
    const double4 q = mom[b];
    P[0] += q.x; P[1] += q.y; P[2] += q.z;
  }
  wave_sum<3>(P);
}

// Total momentum from per-block partials, summed in the same order by every workgroup.
__device__ __forceinline__ void momentum_total(const double4 *__restrict__ mom, int nb, double (&P)[3],
                                               double *lds) {
  P[0] = P[1] = P[2] = 0.0;
  for (int b = threadIdx.x; b < nb; b += nbk::kBlock) {
    const double4 q = mom[b];
    P[0] += q.x; P[1] += q.y; P[2] += q.z;
  }
  block_sum<3>(P, lds);
}

}  // namespace nbd
