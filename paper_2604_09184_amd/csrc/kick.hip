// Around the pair kernel of the H_B kick (eq. Hb): critical radius (eq. rcrit), equal-mass
// detection, lane permutation by position, the deterministic sum of the j-chunk partials, the
// close-encounter list and energy diagnostics.
#include "internal.hpp"

namespace nbk {
using namespace nbd;

// ------------------------------------------------------------------ critical radius (eq. rcrit)
__global__ __launch_bounds__(kBlock) void k_rcrit(const double4 *__restrict__ xm,
                                                  const double4 *__restrict__ v,
                                                  double4 *__restrict__ thr, int n, double m0,
                                                  double cH, double cV, double n1, double n2dt) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  thr[i] = body_thresholds(xm[i], v[i], m0, cH, cV, n1, n2dt);
}

hipError_t launch_rcrit(const double4 *xm, const double4 *v, double4 *thr, int n, double m0,
                        double cH, double cV, double n1, double n2dt, hipStream_t st) {
  hipLaunchKernelGGL(k_rcrit, dim3(nblocks(n)), dim3(kBlock), 0, st, xm, v, thr, n, m0, cH, cV, n1,
                     n2dt);
  return hipGetLastError();
}

// ------------------------------------------------------------------ equal-mass detection
__global__ __launch_bounds__(kBlock) void k_mass_range(const double4 *__restrict__ xm, int n,
                                                       double2 *__restrict__ part) {
  __shared__ double lo[kBlock], hi[kBlock];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const double m = i < n ? xm[i].w : xm[0].w;
  lo[threadIdx.x] = m;
  hi[threadIdx.x] = m;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + s]);
      hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = make_double2(lo[0], hi[0]);
}

__global__ __launch_bounds__(kBlock) void k_mass_flag(const double2 *__restrict__ part, int nb,
                                                      double2 *__restrict__ uni) {
  __shared__ double lo[kBlock], hi[kBlock];
  double a = part[0].x, b = part[0].y;
  for (int k = threadIdx.x; k < nb; k += kBlock) {
    a = fmin(a, part[k].x);
    b = fmax(b, part[k].y);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + s]);
      hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) uni[0] = lo[0] == hi[0] ? make_double2(1.0, lo[0]) : make_double2(0.0, 0.0);
}

hipError_t launch_mass_check(const double4 *xm, int n, double2 *part, double2 *uni, hipStream_t st) {
  const int nb = nblocks(n);
  hipLaunchKernelGGL(k_mass_range, dim3(nb), dim3(kBlock), 0, st, xm, n, part);
  hipLaunchKernelGGL(k_mass_flag, dim3(1), dim3(kBlock), 0, st, part, nb, uni);
  return hipGetLastError();
}

// ------------------------------------------------------------------ locality permutation
// Bodies are binned into 64 x 64 cells of (log r, azimuth), r and azimuth taken in the x-y
// plane, log r scaled to the call's range; cells are visited in Morton order and bodies within
// a cell in arbitrary order (atomic placement: the order of bodies cannot change any result).
constexpr int kCells = 4096;

__device__ __forceinline__ float body_logr(double4 p) {
  return logf(fmaxf((float)sqrt(p.x * p.x + p.y * p.y), 1e-30f));
}

__global__ __launch_bounds__(kBlock) void k_lr_range(const double4 *__restrict__ xm, int n,
                                                     float2 *__restrict__ part) {
  __shared__ float lo[kBlock], hi[kBlock];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  float v = i < n ? body_logr(xm[i]) : 0.f;
  lo[threadIdx.x] = i < n ? v : INFINITY;
  hi[threadIdx.x] = i < n ? v : -INFINITY;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      lo[threadIdx.x] = fminf(lo[threadIdx.x], lo[threadIdx.x + s]);
      hi[threadIdx.x] = fmaxf(hi[threadIdx.x], hi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = make_float2(lo[0], hi[0]);
}

__device__ __forceinline__ unsigned spread6(unsigned v) {
  unsigned r = 0;
  for (int b = 0; b < 6; ++b) r |= ((v >> b) & 1u) << (2 * b);
  return r;
}

__global__ __launch_bounds__(kBlock) void k_cells(const double4 *__restrict__ xm, int n,
                                                  const float2 *__restrict__ part, int nb,
                                                  unsigned short *__restrict__ cell,
                                                  unsigned *__restrict__ count) {
  __shared__ float lo[kBlock], hi[kBlock];
  float a = INFINITY, b = -INFINITY;
  for (int k = threadIdx.x; k < nb; k += kBlock) {
    a = fminf(a, part[k].x);
    b = fmaxf(b, part[k].y);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      lo[threadIdx.x] = fminf(lo[threadIdx.x], lo[threadIdx.x + s]);
      hi[threadIdx.x] = fmaxf(hi[threadIdx.x], hi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double4 p = xm[i];
  const float span = fmaxf(hi[0] - lo[0], 1e-6f);
  int ir = (int)((body_logr(p) - lo[0]) / span * 64.f);
  int ia = (int)((atan2f((float)p.y, (float)p.x) + 3.14159265f) * (64.f / 6.2831853f));
  ir = min(max(ir, 0), 63);
  ia = min(max(ia, 0), 63);
  const unsigned c = spread6((unsigned)ir) | (spread6((unsigned)ia) << 1);
  cell[i] = (unsigned short)c;
  atomicAdd(count + c, 1u);
}

// Exclusive scan of the cell counts (one workgroup of 1024 threads, 4 cells each).
__global__ __launch_bounds__(1024) void k_scan_cells(unsigned *__restrict__ count,
                                                     unsigned *__restrict__ cursor) {
  __shared__ unsigned lds[1024];
  const int t = threadIdx.x;
  unsigned v[4], s = 0;
  for (int k = 0; k < 4; ++k) { v[k] = count[4 * t + k]; s += v[k]; }
  lds[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    unsigned add = t >= o ? lds[t - o] : 0u;
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  unsigned run = lds[t] - s;
  for (int k = 0; k < 4; ++k) { cursor[4 * t + k] = run; run += v[k]; count[4 * t + k] = 0u; }
}

__global__ __launch_bounds__(kBlock) void k_place(const unsigned short *__restrict__ cell, int n,
                                                  unsigned *__restrict__ cursor,
                                                  int *__restrict__ perm) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const unsigned pos = atomicAdd(cursor + cell[i], 1u);
  perm[pos] = i;
}

// count must hold kCells zeros on entry and holds zeros again on return.
hipError_t launch_locality(const double4 *xm, int n, float2 *range_part, unsigned short *cell,
                           unsigned *count, unsigned *cursor, int *perm, hipStream_t st) {
  const int nb = nblocks(n);
  hipLaunchKernelGGL(k_lr_range, dim3(nb), dim3(kBlock), 0, st, xm, n, range_part);
  hipLaunchKernelGGL(k_cells, dim3(nb), dim3(kBlock), 0, st, xm, n, range_part, nb, cell, count);
  hipLaunchKernelGGL(k_scan_cells, dim3(1), dim3(1024), 0, st, count, cursor);
  hipLaunchKernelGGL(k_place, dim3(nb), dim3(kBlock), 0, st, cell, n, cursor, perm);
  return hipGetLastError();
}

int locality_cells() { return kCells; }

// ------------------------------------------------------------------ finalize: sum partials
// One workgroup per 64 bodies: wave w sums chunks [w cs, (w+1) cs) of each body's S partials in
// chunk order (cs = ceil(S/4)), and wave 0 adds the four sums in wave order. Four waves per body
// keep enough loads in flight when n is small. Momentum partials: one per 64 bodies.
// cnt (may be null): per-(chunk, body) numbers of close partners j > i; their total is added to
// *count_out (integer atomics: the total does not depend on the order). part may be null
// (counting only). v_rec (may be null) receives a copy of the updated velocities.
__global__ __launch_bounds__(kBlock) void k_finalize(const double4 *__restrict__ part,
                                                     const double4 *__restrict__ part_ce, int S,
                                                     int n, double G, double h, int napply,
                                                     const double4 *__restrict__ xm,
                                                     double4 *__restrict__ v,
                                                     double4 *__restrict__ acc,
                                                     double4 *__restrict__ acc_ce,
                                                     double4 *__restrict__ mom,
                                                     const int *__restrict__ cnt,
                                                     unsigned long long *__restrict__ count_out,
                                                     double4 *__restrict__ v_rec) {
  constexpr int W = kBlock / 64;
  __shared__ double red[2][W - 1][3][64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i = blockIdx.x * 64 + lane;
  const int cs = (S + W - 1) / W;
  const int s0 = w * cs, s1 = min(S, s0 + cs);
  if (cnt) {
    unsigned long long t = 0;
    if (i < n)
      for (int s = s0; s < s1; ++s) t += (unsigned)cnt[(size_t)s * n + i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (lane == 0 && t) atomicAdd(count_out, t);
  }
  if (!part) return;
  double a[3] = {0.0, 0.0, 0.0};
  double c[3] = {0.0, 0.0, 0.0};
  if (i < n) {
    int s = s0;
    for (; s + 8 <= s1; s += 8) {
      double4 q[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) q[k] = part[(size_t)(s + k) * n + i];
#pragma unroll
      for (int k = 0; k < 8; ++k) { a[0] += q[k].x; a[1] += q[k].y; a[2] += q[k].z; }
    }
    for (; s < s1; ++s) {
      const double4 q = part[(size_t)s * n + i];
      a[0] += q.x; a[1] += q.y; a[2] += q.z;
    }
    if (part_ce)
      for (s = s0; s < s1; ++s) {
        const double4 q = part_ce[(size_t)s * n + i];
        c[0] += q.x; c[1] += q.y; c[2] += q.z;
      }
  }
  if (w > 0)
    for (int k = 0; k < 3; ++k) { red[0][w - 1][k][lane] = a[k]; red[1][w - 1][k][lane] = c[k]; }
  __syncthreads();
  if (w > 0) return;
  for (int q = 0; q < W - 1; ++q)
    for (int k = 0; k < 3; ++k) { a[k] += red[0][q][k][lane]; c[k] += red[1][q][k][lane]; }
  double P[3] = {0.0, 0.0, 0.0};
  if (i < n) {
    const double ax = G * a[0], ay = G * a[1], az = G * a[2];
    if (acc) acc[i] = make_double4(ax, ay, az, 0.0);
    if (acc_ce) acc_ce[i] = make_double4(G * c[0], G * c[1], G * c[2], 0.0);
    if (v) {
      double4 q = v[i];
      for (int k = 0; k < napply; ++k) {
        q.x = q.x + h * ax;
        q.y = q.y + h * ay;
        q.z = q.z + h * az;
      }
      v[i] = q;
      if (v_rec) v_rec[i] = q;
      const double m = xm[i].w;
      P[0] = m * q.x; P[1] = m * q.y; P[2] = m * q.z;
    }
  }
  if (mom) {
    // butterfly: every lane ends with the same bits
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
      for (int k = 0; k < 3; ++k) P[k] += __shfl_xor(P[k], o, 64);
    if (lane == 0) mom[blockIdx.x] = make_double4(P[0], P[1], P[2], 0.0);
  }
}

hipError_t launch_finalize(const double4 *part, const double4 *part_ce, int S, int n, double G,
                           double h, int napply, const double4 *xm, double4 *v, double4 *acc,
                           double4 *acc_ce, double4 *mom, hipStream_t st, const int *cnt,
                           unsigned long long *count_out, double4 *v_rec) {
  hipLaunchKernelGGL(k_finalize, dim3(fin_blocks(n)), dim3(kBlock), 0, st, part, part_ce, S, n, G,
                     h, napply, xm, v, acc, acc_ce, mom, cnt, count_out, v_rec);
  return hipGetLastError();
}

// ------------------------------------------------------------------ encounter list emission
// Rows are emitted in ascending i; within a row the chunks are visited in ascending j and each
// chunk recorded its partners in ascending j, so the list comes out sorted by (i, j) without a
// sort. A row-chunk with more partners than the buffer holds is rescanned here.
// Row totals from the pair kernel's per-row sums when it kept them (rowsum, cleared here; the
// chunk masks too when no emission follows), else from the counts of every chunk.
__global__ __launch_bounds__(kBlock) void k_rowtot(const int *__restrict__ cnt, int S, int n,
                                                   int64_t *__restrict__ rowtot,
                                                   int64_t *__restrict__ bsum,
                                                   int *__restrict__ rowsum,
                                                   unsigned long long *__restrict__ rowmask,
                                                   bool clear_mask) {
  __shared__ int64_t lds[kBlock];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  int64_t t = 0;
  if (i < n && rowsum) {
    t = rowsum[i];
    rowsum[i] = 0;
    if (clear_mask)
      for (int w = 0; w < kRowMaskWords; ++w) rowmask[(size_t)i * kRowMaskWords + w] = 0;
  } else if (i < n) {
    for (int s = 0; s < S; ++s) t += cnt[(size_t)s * n + i];
  }
  if (i < n) rowtot[i] = t;
  lds[threadIdx.x] = t;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = lds[0];
}

// Exclusive scan of the block sums in one workgroup of 1024 threads; writes the total, and counts
// a list longer than cap in *overflow (when given).
__global__ __launch_bounds__(1024) void k_scan_bsum(int64_t *__restrict__ bsum, int nb,
                                                    int64_t *__restrict__ count, int64_t cap,
                                                    unsigned long long *__restrict__ overflow) {
  __shared__ int64_t lds[1024];
  const int t = threadIdx.x;
  const int per = (nb + 1023) / 1024;
  const int b0 = t * per, b1 = min(nb, b0 + per);
  int64_t s = 0;
  for (int b = b0; b < b1; ++b) s += bsum[b];
  lds[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int64_t add = t >= o ? lds[t - o] : 0;
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  int64_t run = lds[t] - s;  // exclusive prefix of this thread's segment
  for (int b = b0; b < b1; ++b) {
    const int64_t x = bsum[b];
    bsum[b] = run;
    run += x;
  }
  if (t == 1023) {
    *count = lds[1023];
    if (overflow && lds[1023] > cap) atomicAdd(overflow, 1ull);
  }
}

// The partners of row i in chunk s (c of them, c > 0) appended at off (up to cap): from the
// partner buffer, or by an exact rescan of the chunk when they did not fit in it.
__device__ __forceinline__ void emit_chunk(const double4 *__restrict__ xm,
                                           const double4 *__restrict__ thr, int n, int chunk,
                                           const int *__restrict__ rowbuf, int R, int i, int s, int c,
                                           int32_t *__restrict__ pairs, int64_t cap, int64_t &off) {
  if (c <= R) {
    for (int k = 0; k < c && off < cap; ++k, ++off) {
      pairs[2 * off] = i;
      pairs[2 * off + 1] = rowbuf[((size_t)s * R + k) * n + i];
    }
    return;
  }
  const double4 pi = xm[i];
  const double4 ti = thr[i];
  const int j0 = max(i + 1, s * chunk), j1 = min(n, (s + 1) * chunk);
  for (int j = j0; j < j1 && off < cap; ++j) {
    const double4 pj = xm[j];
    const double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    const double4 tq = thr[j];
    if (close_exact(r2, ti.y, tq.y, ti.z, tq.z)) {
      pairs[2 * off] = i;
      pairs[2 * off + 1] = j;
      ++off;
    }
  }
}

// The partners of row i in the chunks its mask m names, appended at off (up to cap) in chunk and
// slot order. Up to kBatch masked chunks at a time: their counts and their first kSlots slots are
// loaded together before anything is stored (a masked chunk has at least one recorded partner,
// and every slot below R lies inside the buffer, so the slots need not wait for the counts), so
// a row waits for one memory round trip per batch rather than one per chunk and per partner.
__device__ __forceinline__ void emit_row_masked(const double4 *__restrict__ xm,
                                                const double4 *__restrict__ thr, int n, int chunk,
                                                const int *__restrict__ cnt,
                                                const int *__restrict__ rowbuf, int R, int i,
                                                const unsigned long long (&m)[kRowMaskWords],
                                                int32_t *__restrict__ pairs, int64_t cap,
                                                int64_t &off) {
  constexpr int kBatch = 8, kSlots = 4;
  static_assert(kRowMaskWords == 4, "the word selection below");
  const int ks = R < kSlots ? R : kSlots;
  int w = 0;
  unsigned long long cur = m[0];
  while (off < cap) {
    int sidx[kBatch], c[kBatch], pj[kBatch][kSlots];
    int nb = 0;
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      while (cur == 0 && w < kRowMaskWords - 1) {
        ++w;
        cur = w == 1 ? m[1] : w == 2 ? m[2] : m[3];
      }
      sidx[b] = 0;
      if (cur != 0) {
        sidx[b] = 64 * w + __builtin_ctzll(cur);
        cur &= cur - 1;
        nb = b + 1;
      }
    }
    if (nb == 0) break;
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      c[b] = b < nb ? cnt[(size_t)sidx[b] * n + i] : 0;
#pragma unroll
      for (int k = 0; k < kSlots; ++k)
        pj[b][k] = (b < nb && k < ks) ? rowbuf[((size_t)sidx[b] * R + k) * n + i] : 0;
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      if (b >= nb) break;
      if (c[b] <= ks) {
#pragma unroll
        for (int k = 0; k < kSlots; ++k)
          if (k < c[b] && off < cap) {
            reinterpret_cast<int2 *>(pairs)[off] = make_int2(i, pj[b][k]);
            ++off;
          }
      } else {
        emit_chunk(xm, thr, n, chunk, rowbuf, R, i, sidx[b], c[b], pairs, cap, off);
      }
    }
  }
}

// One wave per workgroup, 64 rows: the row offsets come per kBlock rows (boff), so a wave adds
// the totals of the rows before its own within that block, then its own exclusive scan.
__global__ __launch_bounds__(64) void k_emit(const double4 *__restrict__ xm,
                                             const double4 *__restrict__ thr, int n, int S,
                                             int chunk, const int *__restrict__ cnt,
                                             const int *__restrict__ rowbuf, int R,
                                             const int64_t *__restrict__ rowtot,
                                             const int64_t *__restrict__ boff,
                                             int32_t *__restrict__ pairs, int64_t cap,
                                             unsigned long long *__restrict__ rowmask) {
  constexpr int kQuarters = kBlock / 64;
  const int t = threadIdx.x;
  const int i = blockIdx.x * 64 + t;
  const int blk = blockIdx.x / kQuarters, q = blockIdx.x % kQuarters;
  const int64_t mine = i < n ? rowtot[i] : 0;
  // the chunks with partners, from the pair kernel's mask (read and cleared) when it kept one
  unsigned long long m[kRowMaskWords] = {0, 0, 0, 0};
  if (rowmask && i < n)
    for (int w = 0; w < kRowMaskWords; ++w) {
      m[w] = rowmask[(size_t)i * kRowMaskWords + w];
      if (m[w]) rowmask[(size_t)i * kRowMaskWords + w] = 0;
    }
  // rows of the block before this wave's (all below n: only the last block is partial)
  int64_t before = 0;
  for (int qq = 0; qq < q; ++qq) before += rowtot[(size_t)blk * kBlock + qq * 64 + t];
  int64_t incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t up = __shfl_up(incl, o, 64);
    if (t >= o) incl += up;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) before += __shfl_xor(before, o, 64);
  if (i >= n || mine == 0) return;
  int64_t off = boff[blk] + before + incl - mine;
  if (rowmask) {
    emit_row_masked(xm, thr, n, chunk, cnt, rowbuf, R, i, m, pairs, cap, off);
    return;
  }
  for (int s = 0; s < S && off < cap; ++s) {
    const int c = cnt[(size_t)s * n + i];
    if (c != 0) emit_chunk(xm, thr, n, chunk, rowbuf, R, i, s, c, pairs, cap, off);
  }
}

// The one-workgroup emission for n <= kEmitSmall: row totals, their scan and the emission in one
// launch. The first pass reads the counts coalesced (thread t takes the rows t, t + 1024, ...,
// eight chunks of each in flight) and keeps, per row, the total and the mask of its chunks with
// partners in LDS; thread t then owns the rows [t per, (t + 1) per) for the scan and the emission,
// which reads only the counts of the masked chunks.
__global__ __launch_bounds__(1024) void k_emit_small(const double4 *__restrict__ xm,
                                                     const double4 *__restrict__ thr, int n, int S,
                                                     int chunk, const int *__restrict__ cnt,
                                                     const int *__restrict__ rowbuf, int R,
                                                     int32_t *__restrict__ pairs, int64_t cap,
                                                     int64_t *__restrict__ count,
                                                     unsigned long long *__restrict__ overflow,
                                                     int *__restrict__ rowsum,
                                                     unsigned long long *__restrict__ rowmask) {
  __shared__ unsigned long long mask[2][kEmitSmall];   // chunks 0..63 and 64..127
  __shared__ int rtot[kEmitSmall];
  __shared__ int64_t lds[16];
  const int t = threadIdx.x;
  for (int i = t; i < n; i += 1024) {
    unsigned long long m[2] = {0, 0};
    int tot = 0;
    if (rowsum) {
      // the pair kernel's per-row total and chunk mask (at most 128 chunks here), read and cleared
      tot = rowsum[i];
      if (tot) {
        rowsum[i] = 0;
        m[0] = rowmask[(size_t)i * kRowMaskWords];
        m[1] = rowmask[(size_t)i * kRowMaskWords + 1];
        rowmask[(size_t)i * kRowMaskWords] = 0;
        rowmask[(size_t)i * kRowMaskWords + 1] = 0;
      }
      mask[0][i] = m[0];
      mask[1][i] = m[1];
      rtot[i] = tot;
      continue;
    }
    for (int s0 = 0; s0 < S; s0 += 8) {
      int c[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) c[u] = s0 + u < S ? cnt[(size_t)(s0 + u) * n + i] : 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        tot += c[u];
        if (c[u] != 0) m[(s0 + u) >> 6] |= 1ull << ((s0 + u) & 63);
      }
    }
    mask[0][i] = m[0];
    mask[1][i] = m[1];
    rtot[i] = tot;
  }
  __syncthreads();
  const int per = (n + 1023) / 1024;
  const int i0 = min(n, t * per), i1 = min(n, i0 + per);
  int64_t mine = 0;
  for (int i = i0; i < i1; ++i) mine += rtot[i];
  // inclusive scan: within each wave by lane shifts, then over the sixteen wave totals
  const int lane = t & 63, w = t >> 6;
  int64_t inc = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t up = __shfl_up(inc, o, 64);
    if (lane >= o) inc += up;
  }
  if (lane == 63) lds[w] = inc;
  __syncthreads();
  if (t == 0) {
    int64_t run = 0;
    for (int q = 0; q < 16; ++q) {
      const int64_t x = lds[q];
      lds[q] = run;
      run += x;
    }
    *count = run;
    if (overflow && run > cap) atomicAdd(overflow, 1ull);
  }
  __syncthreads();
  if (!pairs || mine == 0) return;
  int64_t off = lds[w] + inc - mine;
  for (int i = i0; i < i1 && off < cap; ++i)
    for (int h = 0; h < 2; ++h) {
      unsigned long long m = mask[h][i];
      while (m && off < cap) {
        const int s = 64 * h + __builtin_ctzll(m);
        m &= m - 1;
        emit_chunk(xm, thr, n, chunk, rowbuf, R, i, s, cnt[(size_t)s * n + i], pairs, cap, off);
      }
    }
}

hipError_t launch_emit(const KickArgs &a, int32_t *pairs, int64_t cap, int64_t *count,
                       int64_t *rowtot, int64_t *bsum, hipStream_t st,
                       unsigned long long *overflow) {
  if (a.n <= kEmitSmall && a.nchunk <= 128) {
    hipLaunchKernelGGL(k_emit_small, dim3(1), dim3(1024), 0, st, a.xm, a.thr, a.n, a.nchunk, a.chunk,
                       a.cnt, a.rowbuf, a.R, cap > 0 ? pairs : nullptr, cap, count, overflow, a.rowsum,
                       a.rowmask);
    return hipGetLastError();
  }
  const int nb = nblocks(a.n);
  const bool emit = pairs && cap > 0;
  hipLaunchKernelGGL(k_rowtot, dim3(nb), dim3(kBlock), 0, st, a.cnt, a.nchunk, a.n, rowtot, bsum, a.rowsum,
                     a.rowmask, !emit);
  hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(1024), 0, st, bsum, nb, count, cap, overflow);
  if (emit)
    hipLaunchKernelGGL(k_emit, dim3((a.n + 63) / 64), dim3(64), 0, st, a.xm, a.thr, a.n, a.nchunk, a.chunk,
                       a.cnt, a.rowbuf, a.R, rowtot, bsum, pairs, cap, a.rowmask);
  return hipGetLastError();
}

// ------------------------------------------------------------------ input validation
// Problems are reported as key = (index << 3) | reason, folded with atomicMin: the smallest
// index wins, then the smallest reason, whatever the order in which threads find them.
__device__ __forceinline__ void report(unsigned long long *key, long long i, unsigned reason) {
  atomicMin(key, ((unsigned long long)i << 3) | reason);
}

__global__ __launch_bounds__(kBlock) void k_validate_bodies(const double4 *__restrict__ xm,
                                                            const double4 *__restrict__ v, int n,
                                                            unsigned long long *__restrict__ key) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double4 p = xm[i];
  const double4 q = v[i];
  const bool finite = isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(p.w) &&
                      isfinite(q.x) && isfinite(q.y) && isfinite(q.z);
  if (!finite) report(key, i, 1);
  else if (p.w < 0.0) report(key, i, 2);
  else if (p.x == 0.0 && p.y == 0.0 && p.z == 0.0) report(key, i, 3);
}

// Coincident bodies: lane i against the wave-uniform j of its chunk, j > i.
__global__ __launch_bounds__(kBlock) void k_validate_pairs(const double4 *__restrict__ xm, int n,
                                                           int chunk,
                                                           unsigned long long *__restrict__ key) {
  const int i0 = blockIdx.x * kBlock + threadIdx.x;
  const int i = i0 < n ? i0 : n - 1;
  const double4 p = xm[i];
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  bool hit = false;
  for (int j = j0; j < j1; ++j) {
    const double4 q = xm[j];
    hit |= (j > i) & (q.x == p.x) & (q.y == p.y) & (q.z == p.z);
  }
  if (hit && i0 < n) report(key, i, 4);
}

__global__ void k_validate_out(const unsigned long long *__restrict__ key, int64_t *__restrict__ out) {
  if (threadIdx.x != 0) return;
  const unsigned long long k = *key;
  out[0] = k == ~0ull ? -1 : (int64_t)(k >> 3);
  out[1] = k == ~0ull ? 0 : (int64_t)(k & 7);
}

hipError_t launch_validate(const double4 *xm, const double4 *v, int n, unsigned long long *key,
                           int64_t *out, hipStream_t st) {
  hipError_t e = hipMemsetAsync(key, 0xff, sizeof(unsigned long long), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_validate_bodies, dim3(nblocks(n)), dim3(kBlock), 0, st, xm, v, n, key);
  const int chunk = 1024;
  hipLaunchKernelGGL(k_validate_pairs, dim3(nblocks(n), (n + chunk - 1) / chunk), dim3(kBlock), 0, st,
                     xm, n, chunk, key);
  hipLaunchKernelGGL(k_validate_out, dim3(1), dim3(64), 0, st, key, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ energy diagnostics
// Per block: kinetic, star potential, Newtonian pair potential, K-weighted pair potential,
// angular momentum and momentum partial sums (10 doubles), then one block sums the partials.
__global__ __launch_bounds__(kBlock) void k_energy_parts(const double4 *__restrict__ xm,
                                                         const double4 *__restrict__ v,
                                                         const double4 *__restrict__ thr, int n,
                                                         double G, double m0, double f_in,
                                                         double *__restrict__ parts) {
  __shared__ double lds[10 * kBlock];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (i < n) {
    const double4 p = xm[i];
    const double4 q = v[i];
    const double4 ti = thr[i];
    double eN = 0.0, eK = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      const double4 pj = xm[j];
      const double dx = pj.x - p.x, dy = pj.y - p.y, dz = pj.z - p.z;
      const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
      const double r = sqrt(r2);
      const double e = pj.w / r;
      eN += e;
      const double4 tq = thr[j];
      if (close_exact(r2, ti.y, tq.y, ti.z, tq.z)) {
        const double rcij = ti.x > tq.x ? ti.x : tq.x;
        double y = (r - f_in * rcij) / ((1.0 - f_in) * rcij);
        double K = 1.0;
        if (y <= 0.0) K = 0.0;
        else if (y < 1.0) K = y * y / (2.0 * y * y - 2.0 * y + 1.0);
        eK += e * K;
      } else {
        eK += e;
      }
    }
    acc[0] = 0.5 * p.w * (q.x * q.x + q.y * q.y + q.z * q.z);
    acc[1] = -G * m0 * p.w / sqrt(p.x * p.x + p.y * p.y + p.z * p.z);
    acc[2] = -0.5 * G * p.w * eN;
    acc[3] = -0.5 * G * p.w * eK;
    acc[4] = p.w * (p.y * q.z - p.z * q.y);
    acc[5] = p.w * (p.z * q.x - p.x * q.z);
    acc[6] = p.w * (p.x * q.y - p.y * q.x);
    acc[7] = p.w * q.x;
    acc[8] = p.w * q.y;
    acc[9] = p.w * q.z;
  }
  block_sum<10>(acc, lds);
  if (threadIdx.x < 10) parts[(size_t)blockIdx.x * 10 + threadIdx.x] = acc[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_energy_final(const double *__restrict__ parts, int nb,
                                                         double m0, double *__restrict__ out) {
  __shared__ double lds[10 * kBlock];
  double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += kBlock)
    for (int k = 0; k < 10; ++k) acc[k] += parts[(size_t)b * 10 + k];
  block_sum<10>(acc, lds);
  if (threadIdx.x == 0) {
    const double hc = (acc[7] * acc[7] + acc[8] * acc[8] + acc[9] * acc[9]) / (2.0 * m0);
    out[0] = acc[0] + acc[1] + acc[2] + hc;
    out[1] = acc[0] + acc[1] + acc[3] + hc;
    for (int k = 0; k < 3; ++k) {
      out[2 + k] = acc[4 + k];
      out[5 + k] = acc[7 + k];
    }
  }
}

hipError_t launch_energy(const double4 *xm, const double4 *v, const double4 *thr, int n, double G,
                         double m0, double f_in, double4 *eparts, double *out, hipStream_t st) {
  const int nb = nblocks(n);
  double *parts = reinterpret_cast<double *>(eparts);
  hipLaunchKernelGGL(k_energy_parts, dim3(nb), dim3(kBlock), 0, st, xm, v, thr, n, G, m0, f_in,
                     parts);
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kBlock), 0, st, parts, nb, m0, out);
  return hipGetLastError();
}

}  // namespace nbk
