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
__device__ __forceinline__ double wave_max_d(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

// Pair coefficient of the close-encounter force: G m_j ((1 - K)/r^3 + K'(r)/r^2) for r < rc_ij,
// zero beyond.
__device__ __forceinline__ double ce_coef(double r2, double rcij, double f_in, double Gmj) {
  const double r = sqrt(r2);
  const double span = (1.0 - f_in) * rcij;
  const double y = (r - f_in * rcij) / span;
  if (y >= 1.0) return 0.0;
  double K = 0.0, dKdr = 0.0;
  if (y > 0.0) {
    const double D = 2.0 * y * y - 2.0 * y + 1.0;
    K = y * y / D;
    dKdr = 2.0 * y * (1.0 - y) / (D * D) / span;
  }
  return Gmj * ((1.0 - K) / (r2 * r) + dKdr / r2);
}

// f = (v, a) for this lane's body at the group state z; owner[q] = lane holding the q-th member
// in ascending body index.
__device__ __forceinline__ void ce_rhs(const double (&z)[6], int k, const int *owner, int lane,
                                       double m, double rc, double Gm0, double G, double f_in,
                                       double (&f)[6]) {
  const double r2 = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
  const double s = -Gm0 / (r2 * sqrt(r2));
  double a0 = s * z[0], a1 = s * z[1], a2 = s * z[2];
  for (int q = 0; q < k; ++q) {
    const int src = owner[q];
    const double xj = __shfl(z[0], src, 64), yj = __shfl(z[1], src, 64), zj = __shfl(z[2], src, 64);
    const double mj = __shfl(m, src, 64), rcj = __shfl(rc, src, 64);
    if (src == lane) continue;
    const double dx = xj - z[0], dy = yj - z[1], dz = zj - z[2];
    const double c = ce_coef(dx * dx + dy * dy + dz * dz, rc > rcj ? rc : rcj, f_in, G * mj);
    a0 += c * dx;
    a1 += c * dy;
    a2 += c * dz;
  }
  f[0] = z[3]; f[1] = z[4]; f[2] = z[5];
  f[3] = a0; f[4] = a1; f[5] = a2;
}

constexpr int kMaxMacroSteps = 20000;

// One wave per group. stats (device uint64 [6]): [0] groups integrated, [1] largest group,
// [2] bodies in groups, [3] groups above 64 bodies (drifted on Kepler orbits only), [4] groups
// whose integration did not finish (step halved 60 times in a row, or too many macro steps).
__global__ __launch_bounds__(64) void k_ce_drift(double4 *__restrict__ xm, double4 *__restrict__ v,
                                                 const double4 *__restrict__ thr,
                                                 const int *__restrict__ gmem,
                                                 const int *__restrict__ gstart,
                                                 const int *__restrict__ gsize,
                                                 const int *__restrict__ groot,
                                                 const int *__restrict__ ngroups, double G,
                                                 double m0, double f_in, double h, double tol,
                                                 unsigned long long *__restrict__ stats) {
  __shared__ int owner[64];
  const int w = blockIdx.x;
  if (w >= *ngroups) return;
  const int lane = threadIdx.x;
  const int r = groot[w];
  const int k = gsize[r];
  const int base = gstart[r];
  const double Gm0 = G * m0;
  if (k > 64) {
    // too large for one wave: Kepler orbits only, and reported
    for (int q = lane; q < k; q += 64) {
      const int b = gmem[base + q];
      double4 p = xm[b], u = v[b];
      kepler_advance(p.x, p.y, p.z, u.x, u.y, u.z, Gm0, h);
      xm[b] = p;
      v[b] = u;
    }
    if (lane == 0) atomicAdd(stats + 3, 1ull);
    return;
  }
  const bool act = lane < k;
  const int b = gmem[base + (act ? lane : 0)];
  int rank = 0;
  for (int q = 0; q < k; ++q) rank += __shfl(b, q, 64) < b;
  if (act) owner[rank] = lane;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const double4 p0 = xm[b], u0 = v[b];
  const double m = p0.w, rc = thr[b].x;
  double y[6] = {p0.x, p0.y, p0.z, u0.x, u0.y, u0.z};
  const int seq[8] = {2, 4, 6, 8, 10, 12, 14, 16};
  double t = 0.0, H = h;
  int halvings = 0, macro = 0, status = 0;
  while (fabs(h - t) > 0.0) {
    if (++macro > kMaxMacroSteps) { status = 1; break; }
    if (fabs(H) > fabs(h - t)) H = h - t;
    const double sx = wave_max_d(act ? fmax(fabs(y[0]), fmax(fabs(y[1]), fabs(y[2]))) : 0.0);
    const double sv = wave_max_d(act ? fmax(fabs(y[3]), fmax(fabs(y[4]), fabs(y[5]))) : 0.0);
    double R[8][6];
    int accepted = -1;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (accepted < 0) {
        const double hs = H / seq[c];
        double zm[6], zc[6], f[6], est[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) zm[i] = y[i];
        ce_rhs(zm, k, owner, lane, m, rc, Gm0, G, f_in, f);
#pragma unroll
        for (int i = 0; i < 6; ++i) zc[i] = zm[i] + hs * f[i];
        for (int s = 1; s < seq[c]; ++s) {
          ce_rhs(zc, k, owner, lane, m, rc, Gm0, G, f_in, f);
#pragma unroll
          for (int i = 0; i < 6; ++i) {
            const double zn = zm[i] + 2.0 * hs * f[i];
            zm[i] = zc[i];
            zc[i] = zn;
          }
        }
        ce_rhs(zc, k, owner, lane, m, rc, Gm0, G, f_in, f);
#pragma unroll
        for (int i = 0; i < 6; ++i) est[i] = (zc[i] + zm[i] + hs * f[i]) / 2.0;
        // Aitken-Neville: row c from row c - 1
        double e = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          double cur = est[i];
#pragma unroll
          for (int j = 1; j <= c; ++j) {
            const double old = R[j - 1][i];
            R[j - 1][i] = cur;
            const double ratio = (double)seq[c] / (double)seq[c - j];
            cur = cur + (cur - old) / (ratio * ratio - 1.0);
          }
          R[c][i] = cur;
          if (c >= 2) e = fmax(e, fabs(R[c][i] - R[c - 1][i]) / (i < 3 ? sx : sv));
        }
        if (c >= 2 && wave_max_d(act ? e : 0.0) <= tol) accepted = c;
      }
    }
    if (accepted < 0) {
      H = H / 2.0;
      if (++halvings > 60) { status = 1; break; }
      continue;
    }
    halvings = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (c == accepted)
#pragma unroll
        for (int i = 0; i < 6; ++i) y[i] = R[c][i];
    if (t + H == t) break;   // the remaining interval is below the resolution of t
    t = t + H;
    if (accepted <= 4) H = H * 2.0;
  }
  if (act) {
    xm[b] = make_double4(y[0], y[1], y[2], p0.w);
    v[b] = make_double4(y[3], y[4], y[5], u0.w);
  }
  if (lane == 0) {
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
    hipLaunchKernelGGL(k_ce_drift, dim3(max_groups), dim3(64), 0, st, xm, v, thr, gmem, gstart, gsize,
                       groot, ngroups, G, m0, f_in, h, tol, stats);
  return hipGetLastError();
}

}  // namespace nbk
