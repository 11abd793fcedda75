// Multi-level changeover (the paper's intermediate levels between the symplectic step and the
// direct close-encounter integrator; section "The hybrid symplectic integrator"). Level l has the
// time step dt / s^l and critical radii from eq. rcrit at that step. Above the deepest level a
// level-l drift over tau is s substeps of kick(tau/2s) drift_{l+1}(tau/s) kick(tau/2s), the kick
// acting on the step's close pairs with the potential -G m_i m_j W_l K_{l+1} / r,
// W_l = prod_{i <= l} [1 - K_i]. This file holds the kick and its bookkeeping; the orchestration
// is on the host and the deepest level runs the close-encounter integrator.
#include <algorithm>

#include "internal.hpp"

namespace nbk {

// ------------------------------------------------------------------ adjacency of a pair list
__global__ __launch_bounds__(kBlock) void k_adj_zero(int *__restrict__ deg, int *__restrict__ fill,
                                                     int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    deg[i] = 0;
    fill[i] = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_adj_count(const int32_t *__restrict__ pairs, int64_t cap,
                                                      const int64_t *__restrict__ count, int n,
                                                      int *__restrict__ deg) {
  const int64_t np = min(*count, cap);
  for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < np; e += (int64_t)gridDim.x * kBlock) {
    const int i = pairs[2 * e], j = pairs[2 * e + 1];
    if (i < 0 || j < 0 || i >= n || j >= n || i == j) continue;
    atomicAdd(deg + i, 1);
    atomicAdd(deg + j, 1);
  }
}

__global__ __launch_bounds__(kBlock) void k_adj_fill(const int32_t *__restrict__ pairs, int64_t cap,
                                                     const int64_t *__restrict__ count, int n,
                                                     const int *__restrict__ off,
                                                     int *__restrict__ fill, int *__restrict__ adj) {
  const int64_t np = min(*count, cap);
  for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < np; e += (int64_t)gridDim.x * kBlock) {
    const int i = pairs[2 * e], j = pairs[2 * e + 1];
    if (i < 0 || j < 0 || i >= n || j >= n || i == j) continue;
    adj[off[i] + atomicAdd(fill + i, 1)] = j;
    adj[off[j] + atomicAdd(fill + j, 1)] = i;
  }
}

// Each row in ascending neighbour index (insertion sort: rows are short), so that the kicks sum
// in an order that does not depend on the atomics above.
__global__ __launch_bounds__(kBlock) void k_adj_sort(const int *__restrict__ off,
                                                     const int *__restrict__ deg, int n,
                                                     int *__restrict__ adj) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int *row = adj + off[i];
  const int d = deg[i];
  for (int a = 1; a < d; ++a) {
    const int key = row[a];
    int b = a - 1;
    while (b >= 0 && row[b] > key) {
      row[b + 1] = row[b];
      --b;
    }
    row[b + 1] = key;
  }
}

// ------------------------------------------------------------------ level kick
// Changeover K and dK/dr for a pair at distance r with critical radius rcij.
__device__ __forceinline__ void level_K(double r, double rcij, double f_in, double &K, double &dK) {
  const double span = (1.0 - f_in) * rcij;
  double y = (r - f_in * rcij) / span;
  y = fmin(fmax(y, 0.0), 1.0);
  const double D = 2.0 * y * y - 2.0 * y + 1.0;
  K = y * y / D;
  dK = 2.0 * y * (1.0 - y) / (D * D) / span;
}

// v_i += h G sum_j m_j (V/r^3 - V'(r)/r^2) d_ij over body i's listed partners (ascending j),
// V = W_{level-1} K_level.
__global__ __launch_bounds__(kBlock) void k_level_kick(const double4 *__restrict__ xm,
                                                       double4 *__restrict__ v,
                                                       const int *__restrict__ off,
                                                       const int *__restrict__ deg,
                                                       const int *__restrict__ adj, int n,
                                                       LevelThr lt, int level, double G,
                                                       double f_in, double h) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int d = deg[i];
  if (d == 0) return;
  const int *row = adj + off[i];
  const double4 p = xm[i];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int q = 0; q < d; ++q) {
    const int j = row[q];
    const double4 pj = xm[j];
    const double dx = pj.x - p.x, dy = pj.y - p.y, dz = pj.z - p.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double r = sqrt(r2);
    double W = 1.0, dW = 0.0;
    for (int l = 0; l < level; ++l) {
      const double rcij = fmax(lt.thr[l][i].x, lt.thr[l][j].x);
      double K, dK;
      level_K(r, rcij, f_in, K, dK);
      dW = dW * (1.0 - K) - W * dK;
      W = W * (1.0 - K);
    }
    double K, dK;
    level_K(r, fmax(lt.thr[level][i].x, lt.thr[level][j].x), f_in, K, dK);
    const double V = W * K, dV = dW * K + W * dK;
    const double c = G * pj.w * (V / (r2 * r) - dV / r2);
    a0 += c * dx;
    a1 += c * dy;
    a2 += c * dz;
  }
  double4 u = v[i];
  u.x += h * a0;
  u.y += h * a1;
  u.z += h * a2;
  v[i] = u;
}

__global__ __launch_bounds__(kBlock) void k_level_mask(const int *__restrict__ deg,
                                                       const int *__restrict__ in, int n,
                                                       int *__restrict__ skip) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  skip[i] = in ? !(deg[i] > 0 && !in[i]) : (deg[i] > 0);
}

// One workgroup's exclusive prefix sum (as for the group slices).
__global__ __launch_bounds__(1024) void k_adj_scan(const int *__restrict__ deg, int n,
                                                   int *__restrict__ off) {
  __shared__ int lds[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int b0 = t * per, b1 = min(n, b0 + per);
  int s = 0;
  for (int b = b0; b < b1; ++b) s += deg[b];
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
    off[b] = run;
    run += deg[b];
  }
}

hipError_t launch_adjacency(const int32_t *pairs, int64_t cap, const int64_t *count, int n, int *deg,
                            int *off, int *fill, int *adj, hipStream_t st) {
  const int blocks = (int)std::min<int64_t>(4096, (cap + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_adj_zero, dim3(nblocks(n)), dim3(kBlock), 0, st, deg, fill, n);
  if (blocks > 0)
    hipLaunchKernelGGL(k_adj_count, dim3(blocks), dim3(kBlock), 0, st, pairs, cap, count, n, deg);
  hipLaunchKernelGGL(k_adj_scan, dim3(1), dim3(1024), 0, st, deg, n, off);
  if (blocks > 0)
    hipLaunchKernelGGL(k_adj_fill, dim3(blocks), dim3(kBlock), 0, st, pairs, cap, count, n, off, fill, adj);
  hipLaunchKernelGGL(k_adj_sort, dim3(nblocks(n)), dim3(kBlock), 0, st, off, deg, n, adj);
  return hipGetLastError();
}

hipError_t launch_level_kick(const double4 *xm, double4 *v, const int *off, const int *deg,
                             const int *adj, int n, const LevelThr &lt, int level, double G,
                             double f_in, double h, hipStream_t st) {
  hipLaunchKernelGGL(k_level_kick, dim3(nblocks(n)), dim3(kBlock), 0, st, xm, v, off, deg, adj, n, lt,
                     level, G, f_in, h);
  return hipGetLastError();
}

hipError_t launch_level_mask(const int *deg, const int *in, int n, int *skip, hipStream_t st) {
  hipLaunchKernelGGL(k_level_mask, dim3(nblocks(n)), dim3(kBlock), 0, st, deg, in, n, skip);
  return hipGetLastError();
}

}  // namespace nbk
