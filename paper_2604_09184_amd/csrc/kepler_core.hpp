// Kepler two-body advance in universal variables (shared by the drift and its derivative).
#pragma once
#include <hip/hip_runtime.h>

namespace nbd {

// Stumpff functions c0..c3 at z: argument quartered until |z| <= 0.1, series there, then the
// quadrupling relations c0(4z) = 2c0^2 - 1, c1(4z) = c0 c1, c2(4z) = c1^2/2,
// c3(4z) = (c2 + c0 c3)/4.
__device__ __forceinline__ void stumpff(double z, double &c0, double &c1, double &c2, double &c3) {
  int k = 0;
  while (fabs(z) > 0.1 && k < 64) {
    z *= 0.25;
    ++k;
  }
  c2 = 0.5 - z * (1.0 / 24 - z * (1.0 / 720 - z * (1.0 / 40320 - z * (1.0 / 3628800 - z * (1.0 / 479001600)))));
  c3 = 1.0 / 6 - z * (1.0 / 120 - z * (1.0 / 5040 - z * (1.0 / 362880 - z * (1.0 / 39916800 - z * (1.0 / 6227020800.0)))));
  c1 = 1.0 - z * c3;
  c0 = 1.0 - z * c2;
  for (; k > 0; --k) {
    c3 = (c2 + c0 * c3) * 0.25;
    c2 = 0.5 * c1 * c1;
    c1 = c0 * c1;
    c0 = 2.0 * c0 * c0 - 1.0;
  }
}

// Universal anomaly s of the Kepler equation r0 G1(s) + u G2(s) + mu G3(s) = dt,
// G_k(s) = s^k c_k(beta s^2), beta = 2 mu / r0 - v^2, by the Laguerre-Conway iteration.
// F(s) is increasing (F' = r > 0), so the iteration keeps a sign bracket and bisects whenever a
// step would leave it. For unbound orbits the first guess comes from the exponential asymptote
// of the G-functions, ks = ln(2 |dt| k^3 / (r0 k^2 +- u k + mu)), k = sqrt(-beta).
// *status = 0 when converged, 1 otherwise.
__device__ __forceinline__ double kepler_solve(double r0, double u, double beta, double mu, double dt,
                                               int *status) {
  double s = dt / r0;
  if (beta < 0.0) {
    const double k = sqrt(-beta);
    const double sg = dt >= 0.0 ? 1.0 : -1.0;
    const double D = r0 * k * k + sg * u * k + mu;
    const double arg = 2.0 * fabs(dt) * k * k * k / D;
    if (D > 0.0 && arg > 1.0) {
      const double sh = sg * log(arg) / k;
      if (fabs(sh) < fabs(s)) s = sh;
    }
  }
  double lo = -INFINITY, hi = INFINITY;
  if (dt >= 0.0) lo = 0.0; else hi = 0.0;   // F(0) = -dt
  double c0, c1, c2, c3;
  double prev = INFINITY;
  *status = 1;
  for (int it = 0; it < 60; ++it) {
    stumpff(beta * s * s, c0, c1, c2, c3);
    const double G1 = s * c1, G2 = s * s * c2, G3 = s * s * s * c3;
    const double F = r0 * G1 + u * G2 + mu * G3 - dt;
    if (F == 0.0) {
      *status = 0;
      break;
    }
    if (F > 0.0) hi = fmin(hi, s); else lo = fmax(lo, s);
    const double Fp = r0 * c0 + u * G1 + mu * G2;
    const double Fpp = (mu - beta * r0) * G1 + u * c0;
    const double disc = fabs(16.0 * Fp * Fp - 20.0 * F * Fpp);
    const double den = Fp + (Fp >= 0.0 ? 1.0 : -1.0) * sqrt(disc);
    double sn = s - 5.0 * F / den;
    if (!(sn > lo && sn < hi)) {
      if (isfinite(lo) && isfinite(hi)) sn = 0.5 * (lo + hi);
      else sn = isfinite(lo) ? fmax(2.0 * s, s + 1.0) : fmin(2.0 * s, s - 1.0);
    }
    const double a = fabs(sn - s);
    s = sn;
    // converged: a correction at the last-bits level, or corrections that no longer shrink
    // once they are down to rounding noise (cubic convergence has then already finished)
    if (a <= 1e-15 * fabs(s) || (a >= prev && a <= 1e-11 * fabs(s))) {
      *status = 0;
      break;
    }
    prev = a;
  }
  return s;
}

// Advance (x, v) by dt on the Kepler orbit about mu. Returns 0, or 1 if not converged.
__device__ __forceinline__ int kepler_advance(double &x, double &y, double &z, double &vx, double &vy,
                                              double &vz, double mu, double dt) {
  const double r0 = sqrt(x * x + y * y + z * z);
  const double v2 = vx * vx + vy * vy + vz * vz;
  const double u = x * vx + y * vy + z * vz;
  const double beta = 2.0 * mu / r0 - v2;
  int status;
  const double s = kepler_solve(r0, u, beta, mu, dt, &status);
  double c0, c1, c2, c3;
  stumpff(beta * s * s, c0, c1, c2, c3);
  const double G1 = s * c1, G2 = s * s * c2, G3 = s * s * s * c3;
  const double r = r0 * c0 + u * G1 + mu * G2;
  const double f = 1.0 - mu * G2 / r0;
  const double g = dt - mu * G3;
  const double fd = -mu * G1 / (r0 * r);
  const double gd = 1.0 - mu * G2 / r;
  const double nx = f * x + g * vx, ny = f * y + g * vy, nz = f * z + g * vz;
  const double nvx = fd * x + gd * vx, nvy = fd * y + gd * vy, nvz = fd * z + gd * vz;
  x = nx; y = ny; z = nz;
  vx = nvx; vy = nvy; vz = nvz;
  return status;
}


}  // namespace nbd
