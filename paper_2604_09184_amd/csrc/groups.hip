// Close-encounter groups: connected components of the graph whose edges are the close pairs of an
// encounter list (the bodies that the hybrid method's close-encounter integration treats together;
// section "The hybrid symplectic integrator"). Every body is labelled with the smallest index in
// its component.
//
// Lock-free union-find over the pair list: each pair joins the roots of its two bodies by hooking
// the larger root under the smaller one with a compare-and-swap, so a parent index is never larger
// than its child and every root is the smallest index of its set. Parent reads and path-halving
// writes inside the union phase are device-scope atomics (another workgroup's hook must be seen);
// the final flattening runs as its own kernel, when every hook has completed.
//
// Termination: parent[x] <= x at all times and a hook or a halving only lowers it, so every find
// walks a strictly decreasing chain; a failed compare-and-swap means another thread hooked the same
// root, which lowers it, so each pair retries at most as often as its roots are lowered.
#include "internal.hpp"

namespace nbk {

__device__ __forceinline__ int ld_parent(const int *p, int x) {
  return __hip_atomic_load(p + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int find_root(int *p, int x) {
  int px = ld_parent(p, x);
  while (px != x) {
    const int gx = ld_parent(p, px);
    if (gx != px)   // path halving: point x at its grandparent (still in its set, still smaller)
      __hip_atomic_store(p + x, gx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = px;
    px = gx;
  }
  return x;
}

// parent[i] = i; the group sizes and fill counters zeroed (when given), the outputs and the list
// counters zeroed (when given).
__global__ __launch_bounds__(kBlock) void k_groups_init(int *__restrict__ parent,
                                                        int *__restrict__ gsize,
                                                        int *__restrict__ gfill, int n,
                                                        unsigned long long *__restrict__ out,
                                                        int *__restrict__ counter) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    parent[i] = i;
    gsize[i] = 0;
    if (gfill) gfill[i] = 0;
  }
  if (out && i < 2) out[i] = 0;
  if (counter && i < kGroupCounters) counter[i] = 0;
}

// With xm and thr given, a listed pair is an edge only while it is close under thr's exact
// predicate at the positions xm (a deeper changeover level's thresholds).
__global__ __launch_bounds__(kBlock) void k_groups_union(const int32_t *__restrict__ pairs,
                                                         int64_t cap,
                                                         const int64_t *__restrict__ count, int n,
                                                         int *parent,
                                                         unsigned long long *__restrict__ out,
                                                         const double4 *__restrict__ xm,
                                                         const double4 *__restrict__ thr) {
  const int64_t np = min(*count, cap);
  unsigned long long bad = 0;
  for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < np;
       k += (int64_t)gridDim.x * kBlock) {
    const int i = pairs[2 * k], j = pairs[2 * k + 1];
    if (i < 0 || j < 0 || i >= n || j >= n || i == j) {
      ++bad;
      continue;
    }
    if (xm) {
      const double4 a = xm[i], b = xm[j], ta = thr[i], tb = thr[j];
      const double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
      const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
      if (!nbd::close_exact(r2, ta.y, tb.y, ta.z, tb.z)) continue;
    }
    int ri = find_root(parent, i), rj = find_root(parent, j);
    while (ri != rj) {
      const int lo = ri < rj ? ri : rj, hi = ri < rj ? rj : ri;
      const int old = atomicCAS(parent + hi, hi, lo);
      if (old == hi) break;
      // hi was hooked meanwhile: continue from the roots as they are now
      ri = find_root(parent, lo);
      rj = find_root(parent, old);
    }
  }
  if (bad && out) atomicAdd(out + 1, bad);
}

// Flatten every body onto its root and count the bodies of every root (gsize[root] >= 2: a group).
__global__ __launch_bounds__(kBlock) void k_groups_flatten(int *__restrict__ parent,
                                                           int *__restrict__ gsize, int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int r = i;
  while (parent[r] != r) r = parent[r];
  parent[i] = r;
  atomicAdd(gsize + r, 1);
}

__global__ __launch_bounds__(kBlock) void k_groups_count(const int *__restrict__ gsize, int n,
                                                         unsigned long long *__restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  unsigned long long c = (i < n && gsize[i] >= 2) ? 1ull : 0ull;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

hipError_t launch_groups(const int32_t *pairs, int64_t cap, const int64_t *count, int n,
                         int32_t *labels, int *gsize, int *gfill, int *counter, int64_t *out,
                         int union_blocks, hipStream_t st, const double4 *xm, const double4 *thr) {
  unsigned long long *o = (unsigned long long *)out;
  hipLaunchKernelGGL(k_groups_init, dim3(nblocks(n > kGroupCounters ? n : kGroupCounters)),
                     dim3(kBlock), 0, st, labels, gsize, gfill, n, o, counter);
  if (cap > 0)
    hipLaunchKernelGGL(k_groups_union, dim3(union_blocks), dim3(kBlock), 0, st, pairs, cap, count, n,
                       labels, o, xm, thr);
  hipLaunchKernelGGL(k_groups_flatten, dim3(nblocks(n)), dim3(kBlock), 0, st, labels, gsize, n);
  if (o) hipLaunchKernelGGL(k_groups_count, dim3(nblocks(n)), dim3(kBlock), 0, st, gsize, n, o);
  return hipGetLastError();
}

}  // namespace nbk
