// Reverse-mode derivatives (vector-Jacobian products) of the kick (eq. Hb), the jump (eq. Hc)
// and the Kepler drift (eq. Ha), with the critical radii held fixed.
//
// Adjoint arrays mirror the state layout: lam_x [n][4] = dL/d{x, y, z, m}, lam_v [n][4] = dL/dv.
//
// Kick  v' = v + h a(x, m), a_i = G sum_j m_j w(r_ij) d_ij, d_ij = x_j - x_i. With lam_a = h lam_v':
//   lam_x_k += G sum_{j != k} J(d_kj) (m_k lam_a_j - m_j lam_a_k),  J(d) = w I + (w'(r)/r) d d^T,
//   lam_m_k += -G sum_{j != k} w(r_kj) lam_a_j . d_kj.
// Jump  x' = x + h P / m0, P = sum_j m_j v_j. With Lam = sum_i lam_x'_i:
//   lam_v_j += (h/m0) m_j Lam,  lam_m_j += (h/m0) v_j . Lam.
// Drift (x', v') = (f x + g v, fd x + gd v) with f, g, fd, gd from the universal Kepler equation
//   r0 G1(s) + u G2(s) + mu G3(s) = dt (s implicit): reverse sweep through the scalars, with
//   ds = -(G1 dr0 + G2 du + F_beta dbeta) / r and dG_k/dbeta = (k G_{k+2} - s G_{k+1}) / 2.
#include "internal.hpp"
#include "kepler_core.hpp"

namespace nbk {
using namespace nbd;

// ------------------------------------------------------------------ kick VJP pair kernel
// For the kick a_k = G sum_j m_j w(r_kj) d_kj (d_kj = x_j - x_k), the derivative contracted with
// lam_a gives, per body k (before the factor G; the kernel contracts with lam_v, and h, the other
// factor of lam_a = h lam_v, is applied with G in the finalize),
//   g_k = sum_j [ w b + (w'/r) (d . b) d ],   b = m_k lam_j - m_j lam_k,
//   dL/dm_k part = -sum_j w (lam_j . d).
// The sum is split so that b is never formed per pair:
//   sum_j w b      = m_k A - lam_k B,        A = sum_j w lam_j,   B = sum_j m_j w,
//   sum_j q d      with q = (w'/r) (m_k (lam_j . d) - m_j (lam_k . d)).
// Far from the changeover w = r^-3 and w'/r = -3 r^-5; the loop accumulates r^-5 (d . b) d and
// the factor -3 is applied once at the end (close pairs store their w'/r divided by -3).
// One body k per lane, wave-uniform j-bodies (x, m) and their lam_v through scalar loads, and the
// block screen of the forward pair kernel in front of the per-pair prefilter.
// perm (may be null) maps lanes to bodies; as in the forward pair kernel it changes no result.
// uni (may be null) = {1, m} when all masses are equal: m_j leaves the loop.
template <bool UNI>
__device__ __forceinline__ void vjp_pair(const double4 *__restrict__ thr, const double4 &pk,
                                         const double4 &lk, const double4 &pj, const double4 &lj,
                                         int ii, uint32_t tw, int j, bool screened, double f_in,
                                         double (&A)[3], double &B, double (&C)[3], double &gm) {
  const double dx = pj.x - pk.x, dy = pj.y - pk.y, dz = pj.z - pk.z;
  const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
  // 1/r to full precision from the hardware seed (second-order correction)
  const double y0 = __builtin_amdgcn_rsq(r2);
  const double e = fma(-r2, y0 * y0, 1.0);
  const double ri = fma(y0 * e, fma(e, 0.375, 0.5), y0);
  const double ri2 = ri * ri;
  double w = ri2 * ri;       // 1/r^3
  double wq = w * ri2;       // (w'/r) / (-3) = 1/r^5
  if (screened) {
    const uint32_t tj = hiword(thr[j].w);
    const uint32_t U = tw > tj ? tw : tj;
    if (hiword(r2) <= U) {
      if (j == ii) {
        w = 0.0;
        wq = 0.0;
      } else {
        const double4 ti = thr[ii];
        const double4 tq = thr[j];
        if (close_exact(r2, ti.y, tq.y, ti.z, tq.z)) {
          const double rcij = ti.x > tq.x ? ti.x : tq.x;
          const double r = sqrt(r2);
          const double span = (1.0 - f_in) * rcij;
          const double y = (r - f_in * rcij) / span;
          if (y <= 0.0) {
            w = 0.0;
            wq = 0.0;
          } else if (y < 1.0) {
            const double D = 2.0 * y * y - 2.0 * y + 1.0;
            const double K = y * y / D;
            const double K1 = 2.0 * y * (1.0 - y) / (D * D) / span;                        // dK/dr
            const double K2 = 2.0 * (1.0 - 2.0 * y) * (1.0 + 2.0 * y - 2.0 * y * y) /
                              (D * D * D) / (span * span);                                 // d2K/dr2
            const double r3 = r2 * r;
            w = K / r3 - K1 / r2;
            wq = (3.0 * K1 / r3 - 3.0 * K / (r3 * r) - K2 / r2) / r / -3.0;
          }
        }
      }
    }
  }
  const double ld = fma(lj.z, dz, fma(lj.y, dy, lj.x * dx));     // lam_j . d
  const double lkd = fma(lk.z, dz, fma(lk.y, dy, lk.x * dx));    // lam_k . d
  const double db = UNI ? ld - lkd : fma(pk.w, ld, -pj.w * lkd);
  const double q = wq * db;
  C[0] = fma(q, dx, C[0]);
  C[1] = fma(q, dy, C[1]);
  C[2] = fma(q, dz, C[2]);
  A[0] = fma(w, lj.x, A[0]);
  A[1] = fma(w, lj.y, A[1]);
  A[2] = fma(w, lj.z, A[2]);
  B = UNI ? B + w : fma(pj.w, w, B);
  gm = fma(-w, ld, gm);
}

template <bool UNI>
__device__ __forceinline__ void vjp_loop(const double4 *__restrict__ xm, const double4 *__restrict__ thr,
                                         const double4 *__restrict__ lam_v, const double4 &pk,
                                         const double4 &lk, int ii, uint32_t tw, int j0, int j1,
                                         double f_in, double (&A)[3], double &B, double (&C)[3],
                                         double &gm) {
  const int lane = threadIdx.x & 63;
  const double bx0 = wave_min_f64(pk.x), bx1 = wave_max_f64(pk.x);
  const double by0 = wave_min_f64(pk.y), by1 = wave_max_f64(pk.y);
  const double bz0 = wave_min_f64(pk.z), bz1 = wave_max_f64(pk.z);
  for (int jb = j0; jb < j1; jb += 64) {
    const int jl = jb + lane;
    bool near = false;
    if (jl < j1) {
      const double4 q = xm[jl];
      const uint32_t tq = hiword(thr[jl].w);
      const uint32_t U = tw > tq ? tw : tq;
      const double ex = fmax(fmax(bx0 - q.x, q.x - bx1), 0.0);
      const double ey = fmax(fmax(by0 - q.y, q.y - by1), 0.0);
      const double ez = fmax(fmax(bz0 - q.z, q.z - bz1), 0.0);
      const double d2 = fma(ez, ez, fma(ey, ey, ex * ex));
      near = !(hiword(d2) >= U + 2u);
    }
    const unsigned long long mask = __ballot(near);
    const int je = min(j1, jb + 64);
    // j-bodies fetched two at a time, so their scalar loads overlap
    int j = jb;
    for (; j + 2 <= je; j += 2) {
      const double4 p0 = xm[j], p1 = xm[j + 1], l0 = lam_v[j], l1 = lam_v[j + 1];
      vjp_pair<UNI>(thr, pk, lk, p0, l0, ii, tw, j, (mask >> (j - jb)) & 1ull, f_in, A, B, C, gm);
      vjp_pair<UNI>(thr, pk, lk, p1, l1, ii, tw, j + 1, (mask >> (j + 1 - jb)) & 1ull, f_in, A, B, C,
                    gm);
    }
    if (j < je)
      vjp_pair<UNI>(thr, pk, lk, xm[j], lam_v[j], ii, tw, j, (mask >> (j - jb)) & 1ull, f_in, A, B,
                    C, gm);
  }
}

__global__ __launch_bounds__(kBlock) void k_kick_vjp(const double4 *__restrict__ xm,
                                                     const double4 *__restrict__ thr,
                                                     const int *__restrict__ perm,
                                                     const double2 *__restrict__ uni,
                                                     const double4 *__restrict__ lam_v, int n,
                                                     int chunk, double f_in,
                                                     double4 *__restrict__ part) {
  const int lane_body = blockIdx.x * kBlock + threadIdx.x;
  const bool valid = lane_body < n;
  const int lb = valid ? lane_body : n - 1;
  const int ii = perm ? perm[lb] : lb;
  const double4 pk = xm[ii];
  const double4 lk = lam_v[ii];
  const uint32_t tw = __builtin_amdgcn_readfirstlane(wave_max_u32(hiword(thr[ii].w)));
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  double A[3] = {0.0, 0.0, 0.0}, C[3] = {0.0, 0.0, 0.0};
  double B = 0.0, gm = 0.0;
  const bool uniform = uni && uni[0].x != 0.0;
  if (uniform) vjp_loop<true>(xm, thr, lam_v, pk, lk, ii, tw, j0, j1, f_in, A, B, C, gm);
  else vjp_loop<false>(xm, thr, lam_v, pk, lk, ii, tw, j0, j1, f_in, A, B, C, gm);
  if (!valid) return;
  if (uniform) {
    // equal masses: the loop summed sum_j w and (lam_j - lam_k) . d without the common mass
    const double m = uni[0].y;
    B *= m;
    C[0] *= m; C[1] *= m; C[2] *= m;
  }
  // g = m_k A - lam_k B - 3 C
  const double gx = fma(pk.w, A[0], fma(-lk.x, B, -3.0 * C[0]));
  const double gy = fma(pk.w, A[1], fma(-lk.y, B, -3.0 * C[1]));
  const double gz = fma(pk.w, A[2], fma(-lk.z, B, -3.0 * C[2]));
  part[(size_t)blockIdx.y * n + ii] = make_double4(gx, gy, gz, gm);
}

// lam_x += Gh * sum of partials (component 3 accumulates dL/dm), napply times: two consecutive
// kick derivatives at the same positions with the same lam_v give the same increment, so adding
// one evaluation twice equals evaluating twice, bit for bit. Same partial-sum layout as
// k_finalize: 64 bodies per workgroup, four waves over the chunks, added in wave order.
__global__ __launch_bounds__(kBlock) void k_vjp_finalize(const double4 *__restrict__ part, int S, int n,
                                                         double Gh, int napply,
                                                         double4 *__restrict__ lam_x) {
  constexpr int W = kBlock / 64;
  __shared__ double red[W - 1][4][64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i = blockIdx.x * 64 + lane;
  const int cs = (S + W - 1) / W;
  const int s0 = w * cs, s1 = min(S, s0 + cs);
  double g[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < n) {
    int s = s0;
    for (; s + 8 <= s1; s += 8) {
      double4 q[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) q[k] = part[(size_t)(s + k) * n + i];
#pragma unroll
      for (int k = 0; k < 8; ++k) { g[0] += q[k].x; g[1] += q[k].y; g[2] += q[k].z; g[3] += q[k].w; }
    }
    for (; s < s1; ++s) {
      const double4 q = part[(size_t)s * n + i];
      g[0] += q.x; g[1] += q.y; g[2] += q.z; g[3] += q.w;
    }
  }
  if (w > 0)
    for (int k = 0; k < 4; ++k) red[w - 1][k][lane] = g[k];
  __syncthreads();
  if (w > 0 || i >= n) return;
  for (int q = 0; q < W - 1; ++q)
    for (int k = 0; k < 4; ++k) g[k] += red[q][k][lane];
  double4 l = lam_x[i];
  for (int k = 0; k < napply; ++k) {
    l.x += Gh * g[0]; l.y += Gh * g[1]; l.z += Gh * g[2]; l.w += Gh * g[3];
  }
  lam_x[i] = l;
}

// The derivative is linear in lam_v = h lam_v: the pair kernel runs on lam_v and the factor h joins
// G in the finalize.
hipError_t launch_kick_vjp(const double4 *xm, const double4 *thr, const int *perm, const double2 *uni,
                           const double4 *lam_v, double h, double G, double f_in, int n, int S,
                           int chunk, int napply, double4 *part, double4 *lam_x, hipStream_t st) {
  hipLaunchKernelGGL(k_kick_vjp, dim3(nblocks(n), S), dim3(kBlock), 0, st, xm, thr, perm, uni, lam_v,
                     n, chunk, f_in, part);
  hipLaunchKernelGGL(k_vjp_finalize, dim3(fin_blocks(n)), dim3(kBlock), 0, st, part, S, n, G * h,
                     napply, lam_x);
  return hipGetLastError();
}

// ------------------------------------------------------------------ jump VJP
__global__ __launch_bounds__(kBlock) void k_sum_lam(const double4 *__restrict__ lam_x, int n,
                                                    double4 *__restrict__ parts) {
  __shared__ double lds[3 * kBlock];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double L[3] = {0.0, 0.0, 0.0};
  if (i < n) {
    const double4 l = lam_x[i];
    L[0] = l.x; L[1] = l.y; L[2] = l.z;
  }
  block_sum<3>(L, lds);
  if (threadIdx.x == 0) parts[blockIdx.x] = make_double4(L[0], L[1], L[2], 0.0);
}

__global__ __launch_bounds__(kBlock) void k_jump_vjp(const double4 *__restrict__ xm,
                                                     const double4 *__restrict__ v,
                                                     const double4 *__restrict__ parts, int nb, int n,
                                                     double h, double m0, double4 *__restrict__ lam_x,
                                                     double4 *__restrict__ lam_v) {
  __shared__ double lds[3 * kBlock];
  double L[3];
  momentum_total(parts, nb, L, lds);
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double c = h / m0;
  const double m = xm[i].w;
  const double4 q = v[i];
  double4 lv = lam_v[i];
  lv.x += c * m * L[0];
  lv.y += c * m * L[1];
  lv.z += c * m * L[2];
  lam_v[i] = lv;
  double4 lx = lam_x[i];
  lx.w += c * (q.x * L[0] + q.y * L[1] + q.z * L[2]);
  lam_x[i] = lx;
}

hipError_t launch_jump_vjp(const double4 *xm, const double4 *v, double h, double m0, int n,
                           double4 *parts, double4 *lam_x, double4 *lam_v, hipStream_t st) {
  const int nb = nblocks(n);
  hipLaunchKernelGGL(k_sum_lam, dim3(nb), dim3(kBlock), 0, st, lam_x, n, parts);
  hipLaunchKernelGGL(k_jump_vjp, dim3(nb), dim3(kBlock), 0, st, xm, v, parts, nb, n, h, m0, lam_x,
                     lam_v);
  return hipGetLastError();
}

// ------------------------------------------------------------------ drift VJP
// Stumpff functions c0..c5 (argument quartering, series, quadrupling; for c4, c5:
// c4(4z) = c3 (1 + c1) / 8 and c5(4z) = (c4 + c5 + c2/6 - z c2 c5) / 16).
__device__ void stumpff6(double z, double c[6]) {
  int k = 0;
  while (fabs(z) > 0.1 && k < 64) {
    z *= 0.25;
    ++k;
  }
  double c2 = 0.5 - z * (1.0 / 24 - z * (1.0 / 720 - z * (1.0 / 40320 - z * (1.0 / 3628800 - z * (1.0 / 479001600)))));
  double c3 = 1.0 / 6 - z * (1.0 / 120 - z * (1.0 / 5040 - z * (1.0 / 362880 - z * (1.0 / 39916800 - z * (1.0 / 6227020800.0)))));
  double c4 = 1.0 / 24 - z * (1.0 / 720 - z * (1.0 / 40320 - z * (1.0 / 3628800 - z * (1.0 / 479001600 - z * (1.0 / 87178291200.0)))));
  double c5 = 1.0 / 120 - z * (1.0 / 5040 - z * (1.0 / 362880 - z * (1.0 / 39916800 - z * (1.0 / 6227020800.0 - z * (1.0 / 1307674368000.0)))));
  double c1 = 1.0 - z * c3;
  double c0 = 1.0 - z * c2;
  for (; k > 0; --k) {
    const double n5 = (c4 + c5 + c2 / 6.0 - z * c2 * c5) / 16.0;
    const double n4 = c3 * (1.0 + c1) / 8.0;
    const double n3 = (c2 + c0 * c3) * 0.25;
    const double n2 = 0.5 * c1 * c1;
    const double n1 = c0 * c1;
    const double n0 = 2.0 * c0 * c0 - 1.0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3; c4 = n4; c5 = n5;
    z *= 4.0;
  }
  c[0] = c0; c[1] = c1; c[2] = c2; c[3] = c3; c[4] = c4; c[5] = c5;
}

__global__ __launch_bounds__(kBlock) void k_drift_vjp(const double4 *__restrict__ xm,
                                                      const double4 *__restrict__ v, int n, double dt,
                                                      double mu, double4 *__restrict__ lam_x,
                                                      double4 *__restrict__ lam_v) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double4 P = xm[i];
  const double4 Q = v[i];
  const double x[3] = {P.x, P.y, P.z};
  const double vv[3] = {Q.x, Q.y, Q.z};
  const double r0 = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  const double v2 = vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2];
  const double u = x[0] * vv[0] + x[1] * vv[1] + x[2] * vv[2];
  const double beta = 2.0 * mu / r0 - v2;
  int status;
  const double s = kepler_solve(r0, u, beta, mu, dt, &status);   // same iteration as the drift
  double c[6];
  stumpff6(beta * s * s, c);
  const double s2 = s * s, s3 = s2 * s;
  const double G0 = c[0], G1 = s * c[1], G2 = s2 * c[2], G3 = s3 * c[3], G4 = s2 * s2 * c[4],
               G5 = s3 * s2 * c[5];
  const double r = r0 * G0 + u * G1 + mu * G2;
  const double f = 1.0 - mu * G2 / r0;
  const double g = dt - mu * G3;
  const double fd = -mu * G1 / (r0 * r);
  const double gd = 1.0 - mu * G2 / r;
  const double4 LX = lam_x[i];
  const double4 LV = lam_v[i];
  const double lx[3] = {LX.x, LX.y, LX.z};
  const double lv[3] = {LV.x, LV.y, LV.z};
  double ox[3], ov[3];
  double lf = 0.0, lg = 0.0, lfd = 0.0, lgd = 0.0;
  for (int k = 0; k < 3; ++k) {
    ox[k] = f * lx[k] + fd * lv[k];
    ov[k] = g * lx[k] + gd * lv[k];
    lf += lx[k] * x[k];
    lg += lx[k] * vv[k];
    lfd += lv[k] * x[k];
    lgd += lv[k] * vv[k];
  }
  double lr0 = lf * mu * G2 / (r0 * r0) + lfd * mu * G1 / (r0 * r0 * r);
  double lr = lfd * mu * G1 / (r0 * r * r) + lgd * mu * G2 / (r * r);
  double lG1 = -lfd * mu / (r0 * r);
  double lG2 = -lf * mu / r0 - lgd * mu / r;
  const double lG3 = -lg * mu;
  double lG0 = 0.0;
  // r = r0 G0 + u G1 + mu G2
  lr0 += lr * G0;
  double lu = lr * G1;
  lG0 += lr * r0;
  lG1 += lr * u;
  lG2 += lr * mu;
  // G_k(s, beta)
  const double dG0b = -0.5 * s * G1;
  const double dG1b = 0.5 * (G3 - s * G2);
  const double dG2b = 0.5 * (2.0 * G4 - s * G3);
  const double dG3b = 0.5 * (3.0 * G5 - s * G4);
  const double ls = lG0 * (-beta * G1) + lG1 * G0 + lG2 * G1 + lG3 * G2;
  double lb = lG0 * dG0b + lG1 * dG1b + lG2 * dG2b + lG3 * dG3b;
  // s implicit in r0 G1 + u G2 + mu G3 = dt
  const double Fb = r0 * dG1b + u * dG2b + mu * dG3b;
  lr0 += -ls * G1 / r;
  lu += -ls * G2 / r;
  lb += -ls * Fb / r;
  // beta = 2 mu / r0 - v2
  lr0 += -lb * 2.0 * mu / (r0 * r0);
  const double lv2 = -lb;
  for (int k = 0; k < 3; ++k) {
    ox[k] += lr0 * x[k] / r0 + lu * vv[k];
    ov[k] += lu * x[k] + 2.0 * lv2 * vv[k];
  }
  lam_x[i] = make_double4(ox[0], ox[1], ox[2], LX.w);
  lam_v[i] = make_double4(ov[0], ov[1], ov[2], LV.w);
}

hipError_t launch_drift_vjp(const double4 *xm, const double4 *v, int n, double dt, double mu,
                            double4 *lam_x, double4 *lam_v, hipStream_t st) {
  hipLaunchKernelGGL(k_drift_vjp, dim3(nblocks(n)), dim3(kBlock), 0, st, xm, v, n, dt, mu, lam_x, lam_v);
  return hipGetLastError();
}

}  // namespace nbk
