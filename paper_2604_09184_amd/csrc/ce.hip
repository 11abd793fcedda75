// Close-encounter drift: the H_A part of the step (eq. Ha) in full, including the [1 - K] pair
// term, for the bodies of close-encounter groups; bodies in no group keep the Kepler drift.
//
// Within a group the equations of motion are
//   dx_i/dt = v_i,
//   dv_i/dt = -G m0 x_i/|x_i|^3 + G sum_{j in group, j != i} m_j ((1 - K)/r^3 + K'(r)/r^2) d_ij,
// d_ij = x_j - x_i: minus the gradient of the [1 - K] part of the pair potential, which vanishes
// for r >= rc_ij. They are integrated with the Gragg-Bulirsch-Stoer method: modified-midpoint
// sweeps with 2, 4, ..., 16 substeps over a macro step H, extrapolated to zero substep length as a
// polynomial in (H/n)^2 (Aitken-Neville); a macro step is accepted when the last two extrapolants
// agree to the tolerance relative to the group's largest position and velocity, and halved
// otherwise.
//
// One wave per group of at most 64 bodies: lane l holds one body, the pair sums visit the members
// in ascending body index (the same order whatever lane holds which body), the positions of the
// others arrive by lane shuffles, and every step-size decision is taken on wave-wide maxima, so the
// whole integration is uniform across the wave and deterministic.
#include "internal.hpp"
#include "kepler_core.hpp"

namespace nbk {
using namespace nbd;

// ------------------------------------------------------------------ group member lists
// in[i] = 1 for a body that shares its group with another body; gsize[root] counts them.
__global__ __launch_bounds__(kBlock) void k_gmark(const int *__restrict__ label, int n,
                                                  int *__restrict__ mark, int *__restrict__ gsize,
                                                  int *__restrict__ gfill, int *__restrict__ counter) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    mark[i] = 0;
    gsize[i] = 0;
    gfill[i] = 0;
  }
  if (i == 0) *counter = 0;
}

__global__ __launch_bounds__(kBlock) void k_gmark2(const int *__restrict__ label, int n,
                                                   int *__restrict__ mark) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n && label[i] != i) mark[label[i]] = 1;
}

__global__ __launch_bounds__(kBlock) void k_gsize(const int *__restrict__ label,
                                                  const int *__restrict__ mark, int n,
                                                  int *__restrict__ in, int *__restrict__ gsize) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int r = label[i];
  const int g = (r != i) || mark[i];
  in[i] = g;
  if (g) atomicAdd(gsize + r, 1);
}

// Exclusive prefix sum of gsize over n roots (one workgroup; each thread a contiguous segment).
__global__ __launch_bounds__(1024) void k_gscan(const int *__restrict__ gsize, int n,
                                                int *__restrict__ gstart) {
  __shared__ int lds[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int b0 = t * per, b1 = min(n, b0 + per);
  int s = 0;
  for (int b = b0; b < b1; ++b) s += gsize[b];
  lds[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int add = t >= o ? lds[t - o] : 0;
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  int run = lds[t] - s;
  for (int b = b0; b < b1; ++b) {
    gstart[b] = run;
    run += gsize[b];
  }
}

// Members into their group's slots (slot order is arbitrary; the integrator orders them by body
// index) and the roots of the groups into a list.
__global__ __launch_bounds__(kBlock) void k_gfill(const int *__restrict__ label,
                                                  const int *__restrict__ in, int n,
                                                  const int *__restrict__ gstart,
                                                  int *__restrict__ gfill, int *__restrict__ gmem,
                                                  int *__restrict__ groot, int *__restrict__ counter) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n || !in[i]) return;
  const int r = label[i];
  const int slot = atomicAdd(gfill + r, 1);
  gmem[gstart[r] + slot] = i;
  if (r == i) groot[atomicAdd(counter, 1)] = i;
}

// ------------------------------------------------------------------ integrator
// Work layout. A group of k <= 64 bodies is integrated by one workgroup of kCeWaves = 4 waves.
// The eight modified-midpoint sweeps of a macro step (n = 2, 4, ..., 16 substeps) are independent
// of one another, so wave w runs the sweeps n = 2w + 2 and n = 16 - 2w: 20 evaluations of the
// right-hand side per wave, against 80 for all eight in a row. Their end values meet in LDS, and
// every wave then forms the same extrapolation tableau, takes the same decision and updates the
// same state, so the waves stay in step without further exchange.
//
// Within a wave, body slot s (0 <= s < k) sits on the lanes s + kp r, r = 0 .. 64/kp - 1, with kp
// the power of two at or above k: replica r sums the pair terms of every (64/kp)-th member, and the
// replicas' partial sums meet in a butterfly over lane distances kp, 2 kp, ... (commutative
// additions, so every replica ends with the same bits). Small groups thus spread their pair sums
// over the whole wave.
constexpr int kCeWaves = 4;
constexpr int kMaxMacroSteps = 20000;

__device__ __forceinline__ double wave_max_d(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

// Per-member constants in ascending body order: G m, rc, 1/((1 - f_in) rc).
struct CeMember {
  double Gm, rc, ispan, pad;
};

// f = (v, a) of this lane's body at the state z. The pair coefficient is
// G m_j ((1 - K)/r^3 + K'(r)/r^2) for r < rc_ij and zero beyond; with y the changeover variable and
// D = 2y^2 - 2y + 1, K = y^2/D, 1 - K = (1 - y)^2/D and K'(r) = 2y(1 - y)/(D^2 (1 - f_in) rc_ij).
__device__ __forceinline__ void ce_rhs(const double (&z)[6], int k, int iters, int P, int rep,
                                       int slot, const int *owner, const CeMember *mem,
                                       double rc, double ispan, double Gm0, double f_in,
                                       int kp, double (&f)[6]) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int it = 0; it < iters; ++it) {
    const int q = rep + it * P;
    const bool valid = q < k;
    const int qq = valid ? q : 0;
    const int src = owner[qq];
    const double xj = __shfl(z[0], src, 64), yj = __shfl(z[1], src, 64),
                 zj = __shfl(z[2], src, 64);
    const CeMember mj = mem[qq];
    const double dx = xj - z[0], dy = yj - z[1], dz = zj - z[2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double rcij = rc > mj.rc ? rc : mj.rc;
    if (valid && src != slot && r2 < rcij * rcij) {
      const double r = sqrt(r2);
      const double ir = 1.0 / r;
      const double isp = rc > mj.rc ? ispan : mj.ispan;
      const double y = (r - f_in * rcij) * isp;
      double c = ir * ir * ir;
      if (y > 0.0) {
        const double iD = 1.0 / (2.0 * y * y - 2.0 * y + 1.0);
        const double omy = 1.0 - y;
        c = ir * ir * (omy * omy * iD * ir + 2.0 * y * omy * iD * iD * isp);
      }
      c *= mj.Gm;
      a0 += c * dx;
      a1 += c * dy;
      a2 += c * dz;
    }
  }
  for (int o = kp; o < 64; o <<= 1) {
    a0 += __shfl_xor(a0, o, 64);
    a1 += __shfl_xor(a1, o, 64);
    a2 += __shfl_xor(a2, o, 64);
  }
  const double r2 = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
  const double s = -Gm0 / (r2 * sqrt(r2));
  f[0] = z[3]; f[1] = z[4]; f[2] = z[5];
  f[3] = s * z[0] + a0;
  f[4] = s * z[1] + a1;
  f[5] = s * z[2] + a2;
}

// Modified-midpoint sweep of ns substeps over H from y: the end value (z_n + z_{n-1} + hs f(z_n))/2.
__device__ __forceinline__ void ce_sweep(const double (&y)[6], double H, int ns, int k, int iters,
                                         int P, int rep, int slot, const int *owner,
                                         const CeMember *mem, double rc, double ispan, double Gm0,
                                         double f_in, int kp, double (&est)[6]) {
  const double hs = H / ns;
  double zm[6], zc[6], f[6];
  ce_rhs(y, k, iters, P, rep, slot, owner, mem, rc, ispan, Gm0, f_in, kp, f);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    zm[i] = y[i];
    zc[i] = y[i] + hs * f[i];
  }
  for (int s = 1; s < ns; ++s) {
    ce_rhs(zc, k, iters, P, rep, slot, owner, mem, rc, ispan, Gm0, f_in, kp, f);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const double zn = zm[i] + 2.0 * hs * f[i];
      zm[i] = zc[i];
      zc[i] = zn;
    }
  }
  ce_rhs(zc, k, iters, P, rep, slot, owner, mem, rc, ispan, Gm0, f_in, kp, f);
#pragma unroll
  for (int i = 0; i < 6; ++i) est[i] = 0.5 * (zc[i] + zm[i] + hs * f[i]);
}

// Aitken-Neville over the eight sweeps (substep counts 2c + 2) of one component: T[c][0] = e[c],
// T[c][j] = T[c][j-1] + (T[c][j-1] - T[c-1][j-1]) / ((n_c/n_{c-j})^2 - 1). Returns T[want][want]
// and, in err[c], max(err[c], |T[c][c] - T[c][c-1]| iscale) for c >= 2.
__device__ __forceinline__ double ce_tableau(const double (&e)[8], double iscale, int want,
                                             double (&err)[8]) {
  double prev[8], cur[8], out = e[0];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    cur[0] = e[c];
#pragma unroll
    for (int j = 1; j <= c; ++j) {
      const double ratio = (double)(c + 1) / (double)(c + 1 - j);
      cur[j] = cur[j - 1] + (cur[j - 1] - prev[j - 1]) / (ratio * ratio - 1.0);
    }
    if (c >= 2) err[c] = fmax(err[c], fabs(cur[c] - cur[c - 1]) * iscale);
    if (c == want) out = cur[c];
#pragma unroll
    for (int j = 0; j <= c; ++j) prev[j] = cur[j];
  }
  return out;
}

// stats (device uint64 [6]): [0] groups integrated, [1] largest group, [2] bodies in groups, [3]
// groups above 64 bodies (drifted on Kepler orbits only), [4] groups whose integration did not
// finish (step halved 60 times in a row, or too many macro steps).
//
// Step control: a macro step is accepted at the first column c >= 2 whose last two extrapolants
// agree to tol (|T[c][c] - T[c][c-1]|, relative to the group's largest |x| and |v|); after
// acceptance at c <= 3 the next H is 4 H, at c = 4 it is 2 H, otherwise H; a rejected step is
// halved.
__global__ __launch_bounds__(64 * kCeWaves) void k_ce_drift(
    double4 *__restrict__ xm, double4 *__restrict__ v, const double4 *__restrict__ thr,
    const int *__restrict__ gmem, const int *__restrict__ gstart, const int *__restrict__ gsize,
    const int *__restrict__ groot, const int *__restrict__ ngroups, double G, double m0,
    double f_in, double h, double tol, unsigned long long *__restrict__ stats) {
  __shared__ double est_s[2][8][6][64];
  __shared__ int owner[64];
  __shared__ CeMember mem[64];
  const int w = blockIdx.x;
  if (w >= *ngroups) return;
  const int r = groot[w];
  const int k = gsize[r];
  const int base = gstart[r];
  const double Gm0 = G * m0;
  if (k > 64) {
    // too large for one wave: Kepler orbits only, and reported
    for (int q = threadIdx.x; q < k; q += 64 * kCeWaves) {
      const int b = gmem[base + q];
      double4 p = xm[b], u = v[b];
      kepler_advance(p.x, p.y, p.z, u.x, u.y, u.z, Gm0, h);
      xm[b] = p;
      v[b] = u;
    }
    if (threadIdx.x == 0) atomicAdd(stats + 3, 1ull);
    return;
  }
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  int kp = 1;
  while (kp < k) kp <<= 1;
  const int P = 64 / kp;
  const int slot = lane & (kp - 1), rep = lane / kp;
  const int iters = (k + P - 1) / P;
  const bool act = slot < k;
  const int b = gmem[base + (act ? slot : 0)];
  const double4 p0 = xm[b], u0 = v[b];
  const double rc = thr[b].x;
  const double ispan = 1.0 / ((1.0 - f_in) * rc);
  if (wv == 0 && rep == 0 && act) {
    int rank = 0;
    for (int q = 0; q < k; ++q) rank += gmem[base + q] < b;
    owner[rank] = slot;
    mem[rank] = CeMember{G * p0.w, rc, ispan, 0.0};
  }
  __syncthreads();
  double y[6] = {p0.x, p0.y, p0.z, u0.x, u0.y, u0.z};
  double t = 0.0, H = h;
  int halvings = 0, macro = 0, status = 0, buf = 0;
  while (fabs(h - t) > 0.0) {
    if (++macro > kMaxMacroSteps) { status = 1; break; }
    if (fabs(H) > fabs(h - t)) H = h - t;
    const double sx = wave_max_d(act ? fmax(fabs(y[0]), fmax(fabs(y[1]), fabs(y[2]))) : 0.0);
    const double sv = wave_max_d(act ? fmax(fabs(y[3]), fmax(fabs(y[4]), fabs(y[5]))) : 0.0);
    const double isx = 1.0 / sx, isv = 1.0 / sv;
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
      const int c = cc == 0 ? wv : 7 - wv;
      double est[6];
      ce_sweep(y, H, 2 * c + 2, k, iters, P, rep, slot, owner, mem, rc, ispan, Gm0, f_in, kp, est);
      if (rep == 0)
#pragma unroll
        for (int i = 0; i < 6; ++i) est_s[buf][c][i][slot] = est[i];
    }
    __syncthreads();
    // tableau of every component; the first pass finds the accepted column
    double err[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      double e[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) e[c] = est_s[buf][c][i][slot];
      (void)ce_tableau(e, i < 3 ? isx : isv, -1, err);
    }
    int accepted = -1;
#pragma unroll
    for (int c = 2; c < 8; ++c)
      if (accepted < 0 && __ballot(act && !(err[c] <= tol)) == 0) accepted = c;
    if (accepted < 0) {
      buf ^= 1;
      H = H / 2.0;
      if (++halvings > 60) { status = 1; break; }
      continue;
    }
    halvings = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      double e[8], dummy[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int c = 0; c < 8; ++c) e[c] = est_s[buf][c][i][slot];
      y[i] = ce_tableau(e, 1.0, accepted, dummy);
    }
    buf ^= 1;
    if (t + H == t) break;   // the remaining interval is below the resolution of t
    t = t + H;
    if (accepted <= 3) H = H * 4.0;
    else if (accepted == 4) H = H * 2.0;
  }
  if (wv == 0 && rep == 0 && act) {
    xm[b] = make_double4(y[0], y[1], y[2], p0.w);
    v[b] = make_double4(y[3], y[4], y[5], u0.w);
  }
  if (threadIdx.x == 0) {
    atomicAdd(stats + 0, 1ull);
    atomicMax(stats + 1, (unsigned long long)k);
    atomicAdd(stats + 2, (unsigned long long)k);
    if (status) atomicAdd(stats + 4, 1ull);
  }
}

// stats[5] += 1 when an encounter list was truncated (count > cap): its groups are incomplete.
__global__ void k_list_overflow(const int64_t *__restrict__ count, int64_t cap,
                                unsigned long long *__restrict__ stats) {
  if (threadIdx.x == 0 && *count > cap) atomicAdd(stats + 5, 1ull);
}

hipError_t launch_list_overflow(const int64_t *count, int64_t cap, unsigned long long *stats,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_list_overflow, dim3(1), dim3(64), 0, st, count, cap, stats);
  return hipGetLastError();
}

hipError_t launch_group_lists(const int *label, int n, int *mark, int *in, int *gsize, int *gstart,
                              int *gfill, int *gmem, int *groot, int *counter, hipStream_t st) {
  hipLaunchKernelGGL(k_gmark, dim3(nblocks(n)), dim3(kBlock), 0, st, label, n, mark, gsize, gfill,
                     counter);
  hipLaunchKernelGGL(k_gmark2, dim3(nblocks(n)), dim3(kBlock), 0, st, label, n, mark);
  hipLaunchKernelGGL(k_gsize, dim3(nblocks(n)), dim3(kBlock), 0, st, label, mark, n, in, gsize);
  hipLaunchKernelGGL(k_gscan, dim3(1), dim3(1024), 0, st, gsize, n, gstart);
  hipLaunchKernelGGL(k_gfill, dim3(nblocks(n)), dim3(kBlock), 0, st, label, in, n, gstart, gfill,
                     gmem, groot, counter);
  return hipGetLastError();
}

hipError_t launch_ce_drift(double4 *xm, double4 *v, const double4 *thr, const int *gmem,
                           const int *gstart, const int *gsize, const int *groot,
                           const int *ngroups, int max_groups, double G, double m0, double f_in,
                           double h, double tol, unsigned long long *stats, hipStream_t st) {
  if (max_groups > 0)
    hipLaunchKernelGGL(k_ce_drift, dim3(max_groups), dim3(64 * kCeWaves), 0, st, xm, v, thr, gmem,
                       gstart, gsize,
                       groot, ngroups, G, m0, f_in, h, tol, stats);
  return hipGetLastError();
}

}  // namespace nbk
