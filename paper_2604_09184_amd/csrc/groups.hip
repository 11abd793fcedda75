// Close-encounter groups: connected components of the graph whose edges are the close pairs of an
// encounter list (the bodies that the hybrid method's close-encounter integration treats together;
// section "The hybrid symplectic integrator"). Every body is labelled with the smallest index in
// its component.
//
// Lock-free union-find over the pair list (uf_unite): each pair joins the roots of its two bodies
// by hooking the larger root under the smaller one, so every root is the smallest index of its
// set. The final flattening runs as its own kernel, when every hook has completed.
#include "internal.hpp"

namespace nbk {

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
    uf_unite(parent, i, j);
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

// ------------------------------------------------------------------ one-workgroup path
// For n <= kGroupsSmall the whole pipeline runs in one workgroup with the forest in LDS: union
// over the list, flattening (labels and group sizes) and, when lists are asked for, the member
// lists of the groups (in, gstart/gmem slices, the root list groot and counter[0..2]) as
// launch_group_lists builds them. The labels are the same as those of the multi-kernel path (the
// smallest index of each component); slices and roots are placed by LDS atomics, in an order that
// does not matter.
__device__ __forceinline__ int ld_lds(const int *p, int x) {
  return __hip_atomic_load(p + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int find_root_lds(int *p, int x) {
  int px = ld_lds(p, x);
  while (px != x) {
    const int gx = ld_lds(p, px);
    if (gx != px) __hip_atomic_store(p + x, gx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    x = px;
    px = gx;
  }
  return x;
}

__global__ __launch_bounds__(1024) void k_groups_small(
    const int32_t *__restrict__ pairs, int64_t cap, const int64_t *__restrict__ count, int n,
    int32_t *__restrict__ labels, int *__restrict__ gsize, unsigned long long *__restrict__ out,
    const double4 *__restrict__ xm, const double4 *__restrict__ thr, int *__restrict__ in,
    int *__restrict__ gstart, int *__restrict__ gmem, int *__restrict__ groot,
    int *__restrict__ counter, const int *__restrict__ deg, int *__restrict__ skip) {
  __shared__ int par[kGroupsSmall], gsz[kGroupsSmall], gst[kGroupsSmall], gfl[kGroupsSmall];
  __shared__ int ngroups, nmembers;
  __shared__ unsigned long long nbad;
  const int t = threadIdx.x;
  for (int i = t; i < n; i += 1024) {
    par[i] = i;
    gsz[i] = 0;
    gfl[i] = 0;
  }
  if (t == 0) {
    ngroups = 0;
    nmembers = 0;
    nbad = 0;
  }
  __syncthreads();
  const int64_t np = cap > 0 ? min(*count, cap) : 0;
  unsigned long long bad = 0;
  for (int64_t k = t; k < np; k += 1024) {
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
    int ri = find_root_lds(par, i), rj = find_root_lds(par, j);
    while (ri != rj) {
      const int lo = ri < rj ? ri : rj, hi = ri < rj ? rj : ri;
      const int old = atomicCAS(par + hi, hi, lo);
      if (old == hi) break;
      ri = find_root_lds(par, lo);
      rj = find_root_lds(par, old);
    }
  }
  if (bad) atomicAdd(&nbad, bad);
  __syncthreads();
  // flatten: every hook is done, a root's chain only shortens under the concurrent writes
  for (int i = t; i < n; i += 1024) {
    int r = i;
    while (ld_lds(par, r) != r) r = ld_lds(par, r);
    __hip_atomic_store(par + i, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    labels[i] = r;
    atomicAdd(gsz + r, 1);
  }
  __syncthreads();
  for (int i = t; i < n; i += 1024) {
    const int r = par[i];
    gsize[i] = r == i ? gsz[i] : 0;
    if (in) {
      in[i] = gsz[r] >= 2;
      if (skip) skip[i] = !(deg[i] > 0 && !(gsz[r] >= 2));
      if (r == i && gsz[i] >= 2) {
        const int s0 = atomicAdd(&nmembers, gsz[i]);
        gst[i] = s0;
        gstart[i] = s0;
        groot[atomicAdd(&ngroups, 1)] = i;
      }
    } else if (r == i && gsz[i] >= 2) {
      atomicAdd(&ngroups, 1);
    }
  }
  __syncthreads();
  if (in)
    for (int i = t; i < n; i += 1024) {
      const int r = par[i];
      if (gsz[r] >= 2) gmem[gst[r] + atomicAdd(gfl + r, 1)] = i;
    }
  if (t == 0) {
    if (counter) {
      counter[0] = ngroups;
      counter[1] = nmembers;
      for (int q = 2; q < kGroupCounters; ++q) counter[q] = 0;
    }
    if (out) {
      out[0] = (unsigned long long)ngroups;
      out[1] = nbad;
    }
  }
}

hipError_t launch_groups_small(const int32_t *pairs, int64_t cap, const int64_t *count, int n,
                               int32_t *labels, int *gsize, int64_t *out, hipStream_t st,
                               const double4 *xm, const double4 *thr, int *in, int *gstart,
                               int *gmem, int *groot, int *counter, const int *deg, int *skip) {
  hipLaunchKernelGGL(k_groups_small, dim3(1), dim3(1024), 0, st, pairs, cap, count, n, labels, gsize,
                     (unsigned long long *)out, xm, thr, in, gstart, gmem, groot, counter, deg, skip);
  return hipGetLastError();
}

hipError_t launch_groups_init(int *parent, int *gsize, int n, int *counter, hipStream_t st) {
  hipLaunchKernelGGL(k_groups_init, dim3(nblocks(n > kGroupCounters ? n : kGroupCounters)), dim3(kBlock), 0,
                     st, parent, gsize, nullptr, n, nullptr, counter);
  return hipGetLastError();
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
