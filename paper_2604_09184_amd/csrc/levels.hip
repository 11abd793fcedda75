// Multi-level changeover (the paper's intermediate levels between the symplectic step and the
// direct close-encounter integrator; section "The hybrid symplectic integrator"). Level l has the
// time step dt / s^l and critical radii from eq. rcrit at that step. Above the deepest level a
// level-l drift over tau is s substeps of kick(tau/2s) drift_{l+1}(tau/s) kick(tau/2s), the kick
// acting on the step's close pairs with the potential -G m_i m_j W_l K_{l+1} / r,
// W_l = prod_{i <= l} [1 - K_i]. This file holds the kick and its bookkeeping; the orchestration
// is on the host and the deepest level runs the close-encounter integrator.
#include "internal.hpp"
#include "kepler_core.hpp"

#include <algorithm>

namespace nbk {

// Lanes per body row of the level kick: one 16-lane DPP row, four body rows per wave (the rows of
// the close-pair adjacency hold about 20 entries on the planetesimal disks). Rows longer than
// kKickLong entries are left to a part of the same launch that gives each a whole wave (the
// longest rows of the 32768-body disk's list at 1.5 rc hold about 140 entries: nine passes of 16
// lanes, three of 64).
constexpr int kKickLanes = 16;
constexpr int kKickLong = 48;

// ------------------------------------------------------------------ adjacency of a pair list
__global__ __launch_bounds__(kBlock) void k_adj_zero(int *__restrict__ deg, int *__restrict__ fill,
                                                     int n, int *__restrict__ total) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    deg[i] = 0;
    fill[i] = 0;
  }
  if (i < 2) total[i] = 0;
}

// Row slots by atomic allocation: where a row sits does not matter (each row is used on its own);
// the rows longer than kKickLong also go to the list longv (total[1] of them, in any order).
__global__ __launch_bounds__(kBlock) void k_adj_alloc(const int *__restrict__ deg, int n,
                                                      int *__restrict__ off, int *__restrict__ total,
                                                      int *__restrict__ longv) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n || deg[i] == 0) return;
  off[i] = atomicAdd(total, deg[i]);
  if (deg[i] > kKickLong) longv[atomicAdd(total + 1, 1)] = i;
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

// adj[slot] = neighbour.
__global__ __launch_bounds__(kBlock) void k_adj_fill(const int32_t *__restrict__ pairs, int64_t cap,
                                                     const int64_t *__restrict__ count, int n,
                                                     const int *__restrict__ off,
                                                     int *__restrict__ fill, int *__restrict__ adj) {
  const int64_t np = min(*count, cap);
  for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < np; e += (int64_t)gridDim.x * kBlock) {
    const int i = pairs[2 * e], j = pairs[2 * e + 1];
    if (i < 0 || j < 0 || i >= n || j >= n || i == j) continue;
    const int si = off[i] + atomicAdd(fill + i, 1), sj = off[j] + atomicAdd(fill + j, 1);
    adj[si] = j;
    adj[sj] = i;
  }
}

// Each row in ascending neighbour index, so that the kicks sum in an order that does not depend on
// the atomics above: one wave per row; a row of up to 512 entries is placed by rank (the entries
// are distinct; lane l holds entries l, l + 64, ...), a longer one by insertion sort in one lane.
constexpr int kSortChunks = 8;
__global__ __launch_bounds__(kBlock) void k_adj_sort(const int *__restrict__ off,
                                                     const int *__restrict__ deg, int n,
                                                     int *__restrict__ adj) {
  const int i = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int d = deg[i];
  if (d < 2) return;
  int *row = adj + off[i];
  if (d <= 64 * kSortChunks) {
    int a[kSortChunks], rank[kSortChunks];
#pragma unroll
    for (int c = 0; c < kSortChunks; ++c) {
      a[c] = c * 64 + lane < d ? row[c * 64 + lane] : 0x7fffffff;
      rank[c] = 0;
    }
#pragma unroll
    for (int c2 = 0; c2 < kSortChunks; ++c2) {
      if (c2 * 64 >= d) break;
      const int lim = min(64, d - c2 * 64);
      for (int m = 0; m < lim; ++m) {
        const int x = __builtin_amdgcn_readlane(a[c2], m);   // m is wave-uniform: a broadcast
#pragma unroll
        for (int c = 0; c < kSortChunks; ++c) rank[c] += x < a[c];
      }
    }
#pragma unroll
    for (int c = 0; c < kSortChunks; ++c)
      if (c * 64 + lane < d) row[rank[c]] = a[c];
    return;
  }
  if (lane != 0) return;
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
// Changeover K and dK/dr for a pair at distance r with critical radius rcij, from refined hardware
// reciprocals (a few ulp; no division): y = (r - f_in rcij)/((1 - f_in) rcij) clamped to [0, 1],
// D = 2y^2 - 2y + 1 in [1/2, 1], K = y^2/D, dK/dr = 2y(1 - y)/(D^2 (1 - f_in) rcij).
__device__ __forceinline__ void level_K(double r, double rcij, double f_in, double &K, double &dK) {
  const double isp = recip_refined((1.0 - f_in) * rcij);
  const double y = fmin(fmax((r - f_in * rcij) * isp, 0.0), 1.0);
  const double iD = recip_refined((2.0 * y * y - 2.0 * y) + 1.0);
  K = y * y * iD;
  dK = 2.0 * y * (1.0 - y) * (iD * iD) * isp;
}

// One term of row i: v_i's acceleration from neighbour j, G m_j (V/r^3 - V'(r)/r^2) d_ij with
// V = W_{level-1} K_level; UNION: a pair (i < j) close under level `level`'s exact predicate is
// also joined in the forest parent.
template <bool UNION>
__device__ __forceinline__ void level_term(const double4 *__restrict__ xm, const LevelThr &lt,
                                           int level, double G, double f_in, int i,
                                           const double4 &p, const double4 &ti, int j, int *parent,
                                           double &a0, double &a1, double &a2) {
  const double4 pj = xm[j];
  const double dx = pj.x - p.x, dy = pj.y - p.y, dz = pj.z - p.z;
  const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
  if (UNION && j > i) {
    const double4 tj = lt.thr[level][j];
    if (nbd::close_exact(r2, ti.y, tj.y, ti.z, tj.z)) uf_unite(parent, i, j);
  }
  const double ir = rinv_refined(r2);
  const double r = r2 * ir;
  double W = 1.0, dW = 0.0, K, dK;
  for (int l = 0; l < level; ++l) {
    level_K(r, fmax(lt.thr[l][i].x, lt.thr[l][j].x), f_in, K, dK);
    dW = fma(dW, 1.0 - K, -(W * dK));
    W = W * (1.0 - K);
  }
  level_K(r, fmax(ti.x, lt.thr[level][j].x), f_in, K, dK);
  const double V = W * K, dV = fma(dW, K, W * dK);
  const double c = (G * pj.w) * (ir * ir) * fma(V, ir, -dV);
  a0 = fma(c, dx, a0);
  a1 = fma(c, dy, a1);
  a2 = fma(c, dz, a2);
}

// v_i += h times the sum of its row's terms. Blocks below nshort: lane l of the body's 16-lane row
// takes the terms l, l + 16, ... of the sorted row, then a butterfly of commutative additions
// inside the row (rows longer than kKickLong are skipped there). The blocks from nshort on: each
// wave takes long rows from the list longv (*nlong of them) in turn, lane l the terms l, l + 64,
// ..., then the butterfly inside each 16-lane row and the four row sums in row order.
template <bool UNION>
__global__ __launch_bounds__(kBlock) void k_level_kick(const double4 *__restrict__ xm,
                                                       const int *__restrict__ off,
                                                       const int *__restrict__ deg,
                                                       const int *__restrict__ adj, LevelThr lt,
                                                       int level, double G, double f_in, int n,
                                                       double h, double4 *__restrict__ v,
                                                       int *parent, const int *__restrict__ longv,
                                                       const int *__restrict__ nlong, int nshort) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if ((int)blockIdx.x < nshort) {
    const int i = blockIdx.x * (kBlock / kKickLanes) + (int)(threadIdx.x / kKickLanes);
    const int lane = threadIdx.x & (kKickLanes - 1);
    // both exits are uniform over a 16-lane row, so the row's DPP exchanges below see only its
    // own active lanes
    if (i >= n) return;
    const int d = deg[i];
    if (d == 0 || d > kKickLong) return;
    const int *row = adj + off[i];
    const double4 p = xm[i];
    const double4 ti = lt.thr[level][i];
    for (int q = lane; q < d; q += kKickLanes)
      level_term<UNION>(xm, lt, level, G, f_in, i, p, ti, row[q], parent, a0, a1, a2);
    a0 += dpp_f64<0xB1>(a0);    // quad_perm [1, 0, 3, 2]: lane xor 1
    a1 += dpp_f64<0xB1>(a1);
    a2 += dpp_f64<0xB1>(a2);
    a0 += dpp_f64<0x4E>(a0);    // quad_perm [2, 3, 0, 1]: lane xor 2
    a1 += dpp_f64<0x4E>(a1);
    a2 += dpp_f64<0x4E>(a2);
    a0 += dpp_f64<0x141>(a0);   // half-row mirror
    a1 += dpp_f64<0x141>(a1);
    a2 += dpp_f64<0x141>(a2);
    a0 += dpp_f64<0x140>(a0);   // row mirror
    a1 += dpp_f64<0x140>(a1);
    a2 += dpp_f64<0x140>(a2);
    if (lane == 0) {
      double4 u = v[i];
      u.x = fma(h, a0, u.x);
      u.y = fma(h, a1, u.y);
      u.z = fma(h, a2, u.z);
      v[i] = u;
    }
    return;
  }
  const int waves = (gridDim.x - nshort) * (kBlock / 64);
  const int lane = threadIdx.x & 63;
  const int count = *nlong;
  for (int r = (blockIdx.x - nshort) * (kBlock / 64) + (int)(threadIdx.x >> 6); r < count; r += waves) {
    const int i = longv[r];
    const int d = deg[i];
    const int *row = adj + off[i];
    const double4 p = xm[i];
    const double4 ti = lt.thr[level][i];
    a0 = a1 = a2 = 0.0;
    for (int q = lane; q < d; q += 64)
      level_term<UNION>(xm, lt, level, G, f_in, i, p, ti, row[q], parent, a0, a1, a2);
    a0 += dpp_f64<0xB1>(a0);
    a1 += dpp_f64<0xB1>(a1);
    a2 += dpp_f64<0xB1>(a2);
    a0 += dpp_f64<0x4E>(a0);
    a1 += dpp_f64<0x4E>(a1);
    a2 += dpp_f64<0x4E>(a2);
    a0 += dpp_f64<0x141>(a0);
    a1 += dpp_f64<0x141>(a1);
    a2 += dpp_f64<0x141>(a2);
    a0 += dpp_f64<0x140>(a0);
    a1 += dpp_f64<0x140>(a1);
    a2 += dpp_f64<0x140>(a2);
    // the four row sums (every lane of a row holds its row's), added in row order
    double rs[3][4];
    const double a[3] = {a0, a1, a2};
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const long long b = __double_as_longlong(a[k]);
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, 16 * q);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), 16 * q);
        rs[k][q] = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
      }
    if (lane == 0) {
      double4 u = v[i];
      u.x = fma(h, (rs[0][0] + rs[0][1]) + (rs[0][2] + rs[0][3]), u.x);
      u.y = fma(h, (rs[1][0] + rs[1][1]) + (rs[1][2] + rs[1][3]), u.y);
      u.z = fma(h, (rs[2][0] + rs[2][1]) + (rs[2][2] + rs[2][3]), u.z);
      v[i] = u;
    }
  }
}

// ------------------------------------------------------------------ deepest-level groups
// Every body with listed partners walks to its root (the unions have all completed; a value read
// while another thread flattens is the root or an ancestor on the way to it), takes it as its
// label and a slot in its root's slice; the second member to arrive registers the root as a group.
__global__ __launch_bounds__(kBlock) void k_level_groups(const int *__restrict__ deg, int n,
                                                         int *parent, int *__restrict__ gsize,
                                                         int *__restrict__ gstart,
                                                         int *__restrict__ gmem,
                                                         int *__restrict__ groot,
                                                         int *__restrict__ counter) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n || deg[i] == 0) return;
  int r = i;
  for (int pr = parent[r]; pr != r; pr = parent[r]) r = pr;
  parent[i] = r;
  const int pos = atomicAdd(gsize + r, 1);
  if (pos < kLevelSlice) gmem[(size_t)r * kLevelSlice + pos] = i;
  if (pos == 1) {
    gstart[r] = r * kLevelSlice;
    groot[atomicAdd(counter, 1)] = r;
  }
}

// Kepler drift of the bodies with listed partners that the close-encounter drift did not move
// (no group, or a group above 64 bodies), then the reset for the next deepest-level drift.
__global__ __launch_bounds__(kBlock) void k_level_drift(double4 *__restrict__ xm,
                                                        double4 *__restrict__ v, int n, double dt,
                                                        double mu, const int *__restrict__ deg,
                                                        int *__restrict__ parent,
                                                        const int *__restrict__ gsize,
                                                        int *__restrict__ gsize_next,
                                                        int *__restrict__ counter_next) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < kGroupCounters) counter_next[i] = 0;
  if (i >= n) return;
  const int k = gsize[parent[i]];   // read by this thread only, before its reset
  parent[i] = i;
  gsize_next[i] = 0;
  if (deg[i] == 0 || (k >= 2 && k <= 64)) return;
  double4 p = xm[i], q = v[i];
  nbd::kepler_advance(p.x, p.y, p.z, q.x, q.y, q.z, mu, dt);
  xm[i] = p;
  v[i] = q;
}

__global__ __launch_bounds__(kBlock) void k_level_mask(const int *__restrict__ deg,
                                                       const int *__restrict__ in, int n,
                                                       int *__restrict__ skip) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  skip[i] = in ? !(deg[i] > 0 && !in[i]) : (deg[i] > 0);
}

// Thresholds of the close-pair list with a margin: rc kept, H f6, V f2 and the prefilter bound T f2
// (f2 = (1 + margin)^2, f6 = f2^3).
__global__ __launch_bounds__(kBlock) void k_thr_scale(const double4 *__restrict__ thr, int n, double f2,
                                                      double f6, double4 *__restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double4 t = thr[i];
  out[i] = make_double4(t.x, t.y * f6, t.z * f2, t.w * f2);
}

hipError_t launch_thr_scale(const double4 *thr, int n, double f2, double f6, double4 *out, hipStream_t st) {
  hipLaunchKernelGGL(k_thr_scale, dim3(nblocks(n)), dim3(kBlock), 0, st, thr, n, f2, f6, out);
  return hipGetLastError();
}

hipError_t launch_adjacency(const int32_t *pairs, int64_t cap, const int64_t *count, int n,
                            const LevelAdj &g, hipStream_t st) {
  const int blocks = (int)std::min<int64_t>(4096, (cap + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_adj_zero, dim3(nblocks(n > 2 ? n : 2)), dim3(kBlock), 0, st, g.deg, g.fill, n, g.total);
  if (blocks > 0)
    hipLaunchKernelGGL(k_adj_count, dim3(blocks), dim3(kBlock), 0, st, pairs, cap, count, n, g.deg);
  hipLaunchKernelGGL(k_adj_alloc, dim3(nblocks(n)), dim3(kBlock), 0, st, g.deg, n, g.off, g.total, g.longv);
  if (blocks > 0)
    hipLaunchKernelGGL(k_adj_fill, dim3(blocks), dim3(kBlock), 0, st, pairs, cap, count, n, g.off, g.fill,
                       g.adj);
  hipLaunchKernelGGL(k_adj_sort, dim3((n + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0, st, g.off,
                     g.deg, n, g.adj);
  return hipGetLastError();
}

hipError_t launch_level_kick(const double4 *xm, double4 *v, const LevelAdj &g, int n, const LevelThr &lt,
                             int level, double G, double f_in, double h, hipStream_t st, int *parent) {
  // the short rows' blocks, then up to 1024 blocks (4096 waves) for the long rows
  const int nshort = (n + kBlock / kKickLanes - 1) / (kBlock / kKickLanes);
  const int nlongb = std::max(1, std::min(1024, n / 32));
  const dim3 grid(nshort + nlongb);
  if (parent)
    hipLaunchKernelGGL(k_level_kick<true>, grid, dim3(kBlock), 0, st, xm, g.off, g.deg, g.adj, lt, level, G,
                       f_in, n, h, v, parent, g.longv, g.total + 1, nshort);
  else
    hipLaunchKernelGGL(k_level_kick<false>, grid, dim3(kBlock), 0, st, xm, g.off, g.deg, g.adj, lt, level, G,
                       f_in, n, h, v, nullptr, g.longv, g.total + 1, nshort);
  return hipGetLastError();
}

hipError_t launch_level_groups(const int *deg, int n, int *parent, int *gsize, int *gstart, int *gmem,
                               int *groot, int *counter, hipStream_t st) {
  hipLaunchKernelGGL(k_level_groups, dim3(nblocks(n)), dim3(kBlock), 0, st, deg, n, parent, gsize, gstart,
                     gmem, groot, counter);
  return hipGetLastError();
}

hipError_t launch_level_drift(double4 *xm, double4 *v, int n, double dt, double mu, const int *deg,
                              int *parent, const int *gsize, int *gsize_next, int *counter_next,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_level_drift, dim3(nblocks(n > kGroupCounters ? n : kGroupCounters)), dim3(kBlock), 0,
                     st, xm, v, n, dt, mu, deg, parent, gsize, gsize_next, counter_next);
  return hipGetLastError();
}

hipError_t launch_level_mask(const int *deg, const int *in, int n, int *skip, hipStream_t st) {
  hipLaunchKernelGGL(k_level_mask, dim3(nblocks(n)), dim3(kBlock), 0, st, deg, in, n, skip);
  return hipGetLastError();
}

}  // namespace nbk
